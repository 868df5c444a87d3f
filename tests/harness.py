"""Independent numpy/scipy checks for the oracle (third code base).

Nothing here is shared with the oracle or with the GPU library: the dense
Hamiltonian is assembled from Kronecker products of 1-D difference matrices
and the Pauli matrices typed in here, the free lattice propagator is applied
mode by mode after an FFT, and the Landau levels are the textbook closed form.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.integrate
import scipy.sparse as sp

SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
ID2 = np.eye(2, dtype=np.complex128)


def axes(prob):
    hx = (prob["x_max"] - prob["x_min"]) / prob["nx"]
    hy = (prob["y_max"] - prob["y_min"]) / prob["ny"]
    return (prob["x_min"] + hx * np.arange(prob["nx"]), prob["y_min"] + hy * np.arange(prob["ny"]),
            hx, hy)


def diff_1d(n, h, periodic):
    """Central first-derivative matrix (f[i+1]-f[i-1])/(2h)."""
    d = sp.lil_matrix((n, n), dtype=np.complex128)
    for i in range(n):
        for off, sgn in ((1, 1.0), (-1, -1.0)):
            j = i + off
            if 0 <= j < n:
                d[i, j] += sgn / (2 * h)
            elif periodic:
                d[i, j % n] += sgn / (2 * h)
    return d.tocsr()


def potential_grid(prob):
    x, y, _, _ = axes(prob)
    X, Y = np.meshgrid(x, y)
    r2 = X * X + Y * Y
    v = np.zeros_like(X)
    if prob.get("pot_kind", 0) == 1:
        v = -prob["pot_z"] / np.sqrt(r2 + prob["pot_a"] ** 2)
    elif prob.get("pot_kind", 0) == 2:
        z = prob["pot_z"]
        v = -1.5 * z / np.sqrt(r2 + 3.0 / (z * z))
    if prob.get("v_table") is not None:
        v = v + np.asarray(prob["v_table"])
    return v


def dense_h(prob, a_hom=(0.0, 0.0)):
    """Sparse matrix of H on the flattened (2, ny, nx) spinor."""
    nx, ny = prob["nx"], prob["ny"]
    x, y, hx, hy = axes(prob)
    q, c, m = prob.get("charge", -1.0), prob.get("c", 137.036), prob.get("mass", 1.0)
    bz = prob.get("bz", 0.0)
    Dx = sp.kron(sp.identity(ny), diff_1d(nx, hx, prob["bc_x"]))
    Dy = sp.kron(diff_1d(ny, hy, prob["bc_y"]), sp.identity(nx))
    X = sp.diags(np.tile(x, ny))
    Y = sp.diags(np.repeat(y, nx))
    Ieye = sp.identity(nx * ny)
    Ax = -0.5 * bz * Y + a_hom[0] * Ieye
    Ay = 0.5 * bz * X + a_hom[1] * Ieye
    PIx = -1j * Dx - q * Ax
    PIy = -1j * Dy - q * Ay
    V = sp.diags(potential_grid(prob).ravel())
    chi = -1.0 if prob.get("chirality", 0) < 0 else 1.0  # alpha2 = chi sigma2
    H = (c * (sp.kron(SX, PIx) + chi * sp.kron(SY, PIy)) + m * c * c * sp.kron(SZ, Ieye)
         + sp.kron(ID2, V))
    return H.tocsr()


def pulse_value(prob, t):
    """A_L(t) typed in from the workload definitions."""
    T = prob["t_pulse"]
    if prob.get("pulse_kind", 0) == 0 or t < 0 or t > T:
        return np.zeros(2)
    env2 = math.sin(math.pi * t / T) ** 2
    if prob["pulse_kind"] == 1:
        f = prob["a0"] * math.sin(prob["omega"] * t) * env2
        return f * np.asarray(prob["pulse_e"], dtype=float)
    w0 = 2 * math.pi / T
    cf = np.asarray(prob["coef"], dtype=float).reshape(-1, 4)
    ax = sum(cf[k, 0] * math.sin((k + 1) * w0 * t) + cf[k, 1] * math.cos((k + 1) * w0 * t)
             for k in range(len(cf)))
    ay = sum(cf[k, 2] * math.sin((k + 1) * w0 * t) + cf[k, 3] * math.cos((k + 1) * w0 * t)
             for k in range(len(cf)))
    return env2 * np.array([ax, ay])


def pulse_average_quad(prob, t0, dt):
    """(1/dt) integral over [t0, t0+dt] of A_L by adaptive quadrature."""
    if prob.get("pulse_kind", 0) == 0:
        return np.zeros(2)
    lo, hi = min(t0, t0 + dt), max(t0, t0 + dt)
    out = np.zeros(2)
    for comp in range(2):
        val, _ = scipy.integrate.quad(lambda t: pulse_value(prob, t)[comp], lo, hi,
                                      epsabs=1e-15, epsrel=1e-14, limit=200,
                                      points=[prob["t_pulse"]] if lo < prob["t_pulse"] < hi else None)
        out[comp] = val / abs(dt)
    return out


def lattice_energy(prob, kx, ky, a_hom=(0.0, 0.0)):
    """Closed form: plane-wave eigenvalues +-sqrt(m^2c^4 + c^2 |sin(kh)/h - qA|^2)."""
    _, _, hx, hy = axes(prob)
    q, c, m = prob.get("charge", -1.0), prob.get("c", 137.036), prob.get("mass", 1.0)
    px = math.sin(kx * hx) / hx - q * a_hom[0]
    py = math.sin(ky * hy) / hy - q * a_hom[1]
    e = math.sqrt((m * c * c) ** 2 + c * c * (px * px + py * py))
    return e, px, py


def free_propagate_fft(prob, psi, t):
    """Exact solution of the free periodic lattice problem: each DFT mode evolves
    with exp(-i H0(k) t) = cos(Et) - i sin(Et) H0/E."""
    _, _, hx, hy = axes(prob)
    c, m = prob.get("c", 137.036), prob.get("mass", 1.0)
    kx = np.sin(2 * np.pi * np.fft.fftfreq(prob["nx"])) / hx
    ky = np.sin(2 * np.pi * np.fft.fftfreq(prob["ny"])) / hy
    KX, KY = np.meshgrid(kx, ky)
    mc2 = m * c * c
    E = np.sqrt(mc2 ** 2 + c * c * (KX ** 2 + KY ** 2))
    f0, f1 = np.fft.fft2(psi[0]), np.fft.fft2(psi[1])
    h0 = mc2 * f0 + c * (KX - 1j * KY) * f1
    h1 = c * (KX + 1j * KY) * f0 - mc2 * f1
    cs, sn = np.cos(E * t), np.sin(E * t)
    g0 = cs * f0 - 1j * sn * h0 / E
    g1 = cs * f1 - 1j * sn * h1 / E
    return np.stack([np.fft.ifft2(g0), np.fft.ifft2(g1)])


def landau_levels(prob, n_max):
    """Relativistic Landau levels sqrt(m^2c^4 + 2 n c^2 |qB|), n = 1..n_max."""
    c, m, q, b = prob.get("c", 137.036), prob.get("mass", 1.0), prob.get("charge", -1.0), prob["bz"]
    return np.array([math.sqrt((m * c * c) ** 2 + 2 * n * c * c * abs(q * b))
                     for n in range(1, n_max + 1)])


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def dense_h4(prob, a_hom=(0.0, 0.0)):
    """Four-component H = c alpha.(p - qA) + beta m c^2 + V on the flattened
    (4, ny, nx) spinor, standard Dirac representation alpha_i = [[0, s_i],
    [s_i, 0]], beta = diag(1, 1, -1, -1), no z motion."""
    nx, ny = prob["nx"], prob["ny"]
    x, y, hx, hy = axes(prob)
    per_x, per_y = prob["bc_x"] == 1, prob["bc_y"] == 1
    Dx = sp.kron(sp.identity(ny), diff_1d(nx, hx, per_x))
    Dy = sp.kron(diff_1d(ny, hy, per_y), sp.identity(nx))
    X, Y = np.meshgrid(x, y)
    q, c, m = prob["charge"], prob["c"], prob["mass"]
    ax = (-0.5 * prob.get("bz", 0.0) * Y + a_hom[0]).ravel()
    ay = (0.5 * prob.get("bz", 0.0) * X + a_hom[1]).ravel()
    PIx = -1j * Dx - q * sp.diags(ax)
    PIy = -1j * Dy - q * sp.diags(ay)
    V = sp.diags(potential_grid(prob).ravel())
    Z2 = np.zeros((2, 2), dtype=np.complex128)
    ax4 = np.block([[Z2, SX], [SX, Z2]])
    ay4 = np.block([[Z2, SY], [SY, Z2]])
    b4 = np.diag([1.0, 1.0, -1.0, -1.0]).astype(np.complex128)
    Ieye = sp.identity(nx * ny)
    H = c * (sp.kron(ax4, PIx) + sp.kron(ay4, PIy)) + m * c * c * sp.kron(b4, Ieye) + sp.kron(np.eye(4), V)
    return H.tocsr()


def lanczos_dense(A, psi, k):
    """Textbook Lanczos on a dense Hermitian matrix with full
    reorthogonalisation (numpy): returns (alpha[k], beta[k], Q) with beta[k-1]
    = ||A q_k - alpha_k q_k - beta_{k-1} q_{k-1}|| (the residual norm that
    multiplies the last Krylov coefficient in the step error estimate)."""
    A = np.asarray(A)
    v = np.asarray(psi, dtype=np.complex128).ravel()
    q = v / np.linalg.norm(v)
    Q = [q]
    al, be = [], []
    prev, bprev = np.zeros_like(q), 0.0
    for i in range(k):
        w = A @ Q[i] - bprev * prev
        a = float(np.vdot(Q[i], w).real)
        w = w - a * Q[i]
        for _ in range(2):
            for qj in Q:
                w = w - np.vdot(qj, w) * qj
        b = float(np.linalg.norm(w))
        al.append(a)
        be.append(b)
        if i + 1 < k:
            prev, bprev = Q[i], b
            Q.append(w / b)
    return np.array(al), np.array(be), np.stack(Q, axis=1)


def storage_bound(alpha, beta, nrm, reps, rabs):
    """Bound of the error from rounding the stored Krylov vectors u_2..u_k
    (relative rounding reps, absolute rabs per vector):
    ||psi|| sum_{j<k} f_j (reps beta_j + rabs) / (1 - reps) with f_j a bound
    of int_0^1 |[exp(-itT)]_{j1}| dt.  T's Gershgorin interval has centre c0
    and half-width R.  R <= 40: f_j = (1.01 int_0^1 |[exp(-itT)]_{j1}|^2 dt)^(1/2)
    (Cauchy-Schwarz), the integral by 48-node Gauss-Legendre quadrature of the
    eigendecomposition (numpy eigh); R <= 70: f_j = [exp(|T - c0 I|)]_{j1}
    (path sums; scipy expm); both capped at 1, and 1 beyond."""
    import scipy.linalg
    al = np.asarray(alpha, dtype=float)
    be = np.asarray(beta, dtype=float)
    k = len(al)
    off = np.r_[be[:k - 1], 0.0]
    rad = np.abs(off) + np.abs(np.r_[0.0, be[:k - 1]])
    lo, hi = np.min(al - rad), np.max(al + rad)
    c0, R = 0.5 * (lo + hi), 0.5 * (hi - lo)
    if R <= 40:
        T = np.diag(al - c0) + np.diag(be[:k - 1], 1) + np.diag(be[:k - 1], -1)
        lam, V = np.linalg.eigh(T)
        x, wq = np.polynomial.legendre.leggauss(48)
        integral = np.zeros(k)
        for tq, w in zip(0.5 * (x + 1.0), 0.5 * wq):
            integral += w * np.abs(V @ (np.exp(-1j * tq * lam) * V[0, :])) ** 2
        f = np.minimum(1.0, np.sqrt(1.01 * integral))
    elif R <= 70:
        X = np.diag(np.abs(al - c0)) + np.diag(np.abs(be[:k - 1]), 1) + np.diag(np.abs(be[:k - 1]), -1)
        f = np.minimum(1.0, scipy.linalg.expm(X)[:, 0])
    else:
        f = np.ones(k)
    tot = sum(f[j - 1] * (reps * be[j - 1] + rabs) / (1.0 - reps) for j in range(1, k))
    return nrm * tot


def round_to_bits(z, bits):
    """Round the real and imaginary parts of z to `bits` significand bits
    (round to nearest), emulating a narrower storage format."""
    def rnd(x):
        m, e = np.frexp(x)
        scale = 2.0 ** bits
        return np.ldexp(np.round(m * scale) / scale, e)
    return rnd(z.real) + 1j * rnd(z.imag)


def match_converged(a_vals, a_bds, b_vals, b_bds, tol, robust=0.25):
    """Compare two sets of converged Ritz values (each within its bound of an
    eigenvalue of H).  Every value of either set whose bound is <= robust*tol
    must have a partner in the other set within 2 (b_a + b_b) + 1e-8; a value
    with a larger bound (it converged near the end, or only just) may be
    missing on the other side, but if a partner lies within tol it must meet
    the same closeness.  Returns the number of matched pairs; raises
    AssertionError with the offending value otherwise."""
    a_vals, a_bds = np.asarray(a_vals), np.asarray(a_bds)
    b_vals, b_bds = np.asarray(b_vals), np.asarray(b_bds)
    matched = 0
    for (xv, xb, yv, yb, side) in ((a_vals, a_bds, b_vals, b_bds, "first"), (b_vals, b_bds, a_vals, a_bds, "second")):
        for v, bd in zip(xv, xb):
            d = np.abs(yv - v) if len(yv) else np.array([np.inf])
            i = int(np.argmin(d))
            close = len(yv) > 0 and d[i] <= 2.0 * (bd + yb[i]) + 1e-8
            if bd <= robust * tol:
                assert close, (side, float(v), float(bd), "no partner")
            elif len(yv) and d[i] <= tol:
                assert close, (side, float(v), float(bd), float(yv[i]), "partner too far")
            if side == "first" and close:
                matched += 1
    return matched
