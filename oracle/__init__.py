"""CPU FP64 oracle for the Lanczos Dirac propagator -- TEST INFRASTRUCTURE.

Thin ctypes wrapper over ``dirac_oracle.c`` (plain C, double precision,
literal Fig. 1 of Beerwerth & Bauke, arXiv:1407.7370).  Only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import this module;
the GPU library never does.  It shares no code with the GPU library.

Functions take a plain ``dict`` describing the physical problem (the keys of
``ORC_KEYS``) and numpy complex128 arrays of shape ``(2, ny, nx)``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dirac_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("x_min", ctypes.c_double), ("x_max", ctypes.c_double),
        ("y_min", ctypes.c_double), ("y_max", ctypes.c_double),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("mass", ctypes.c_double), ("c", ctypes.c_double), ("charge", ctypes.c_double),
        ("bz", ctypes.c_double),
        ("pot_kind", ctypes.c_int32), ("pot_z", ctypes.c_double), ("pot_a", ctypes.c_double),
        ("v_table", ctypes.c_void_p),
        ("pulse_kind", ctypes.c_int32),
        ("pulse_e", ctypes.c_double * 2), ("a0", ctypes.c_double), ("omega", ctypes.c_double),
        ("t_pulse", ctypes.c_double),
        ("n_coef", ctypes.c_int32), ("coef", ctypes.c_void_p),
        ("chirality", ctypes.c_int32),
    ]


class _HParams(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("scale", ctypes.c_double), ("mass", ctypes.c_double),
                ("c", ctypes.c_double), ("charge", ctypes.c_double), ("bz", ctypes.c_double),
                ("pot_kind", ctypes.c_int32), ("pot_z", ctypes.c_double), ("pot_a", ctypes.c_double),
                ("chirality", ctypes.c_int32)]


def _hparams(hprob: dict) -> _HParams:
    p = _HParams()
    p.n = int(hprob["n"])
    p.scale = float(hprob["scale"])
    for k, d in (("mass", 1.0), ("c", 137.036), ("charge", -1.0), ("bz", 0.0), ("pot_z", 0.0), ("pot_a", 0.0)):
        setattr(p, k, float(hprob.get(k, d)))
    p.pot_kind = int(hprob.get("pot_kind", 0))
    p.chirality = int(hprob.get("chirality", 0))
    return p


class _Stat(ctypes.Structure):
    _fields_ = [("k_eff", ctypes.c_int32), ("err_est", ctypes.c_double),
                ("cum_bound", ctypes.c_double), ("norm2", ctypes.c_double)]


ORC_KEYS = ("nx", "ny", "x_min", "x_max", "y_min", "y_max", "bc_x", "bc_y", "mass", "c",
            "charge", "bz", "pot_kind", "pot_z", "pot_a", "v_table", "pulse_kind", "pulse_e",
            "a0", "omega", "t_pulse", "coef", "chirality")

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Params)
        D = ctypes.POINTER(ctypes.c_double)
        lib.orc_apply_h.argtypes = [P, D, D, D]
        lib.orc_pulse.argtypes = [P, ctypes.c_double, D]
        lib.orc_field_average.argtypes = [P, ctypes.c_double, ctypes.c_double, D]
        lib.orc_lanczos.argtypes = [P, D, ctypes.c_double, D, ctypes.c_int, ctypes.c_int, D, D, D]
        lib.orc_lanczos.restype = ctypes.c_int
        lib.orc_lanczos_plain.argtypes = [P, D, ctypes.c_double, D, ctypes.c_int, D, D]
        lib.orc_lanczos_plain.restype = ctypes.c_int
        lib.orc_tridiag_eig.argtypes = [ctypes.c_int, D, D, D, D]
        lib.orc_expm_e1.argtypes = [ctypes.c_int, D, D, ctypes.c_double, D]
        lib.orc_propagate.argtypes = [P, D, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_int, ctypes.POINTER(_Stat)]
        lib.orc_propagate.restype = ctypes.c_int
        lib.orc_eigen.argtypes = [P, D, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int, D, D,
                                  ctypes.POINTER(ctypes.c_int)]
        lib.orc_eigen.restype = ctypes.c_int
        lib.orc_eigen_vectors.argtypes = [P, D, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_int, D, D,
                                          ctypes.POINTER(ctypes.c_int), D]
        lib.orc_eigen_vectors.restype = ctypes.c_int
        lib.orc_pauli.argtypes = [ctypes.c_int, D]
        HP = ctypes.POINTER(_HParams)
        lib.orc_hermite_nodes.argtypes = [ctypes.c_int, D, D]
        lib.orc_hermite_dmat.argtypes = [ctypes.c_int, D, D, D]
        lib.orc_hermite_operator.argtypes = [HP, D, D]
        lib.orc_apply_h_hermite.argtypes = [HP, D, D]
        lib.orc_lanczos_plain_hermite.argtypes = [HP, D, ctypes.c_int, D, D]
        lib.orc_lanczos_plain_hermite.restype = ctypes.c_int
        lib.orc_expectations.argtypes = [P, D, D]
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class _Problem:
    """Keeps the ctypes struct and the arrays it points to alive together."""

    def __init__(self, prob: dict):
        self.p = _Params()
        self.keep = []
        for k in ("nx", "ny", "bc_x", "bc_y", "pot_kind", "pulse_kind", "chirality"):
            setattr(self.p, k, int(prob.get(k, 0)))
        defaults = {"mass": 1.0, "c": 137.036, "charge": -1.0}
        for k in ("x_min", "x_max", "y_min", "y_max", "mass", "c", "charge", "bz", "pot_z",
                  "pot_a", "a0", "omega", "t_pulse"):
            setattr(self.p, k, float(prob.get(k, defaults.get(k, 0.0))))
        e = prob.get("pulse_e", (0.0, 0.0))
        self.p.pulse_e[0], self.p.pulse_e[1] = float(e[0]), float(e[1])
        vt = prob.get("v_table")
        if vt is not None:
            vt = np.ascontiguousarray(vt, dtype=np.float64)
            assert vt.shape == (self.p.ny, self.p.nx)
            self.keep.append(vt)
            self.p.v_table = vt.ctypes.data
        coef = prob.get("coef")
        if coef is not None and len(coef) > 0:
            coef = np.ascontiguousarray(coef, dtype=np.float64)
            self.keep.append(coef)
            self.p.coef = coef.ctypes.data
            self.p.n_coef = len(coef)

    @property
    def ref(self):
        return ctypes.byref(self.p)


def _check_psi(prob, psi):
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    assert psi.shape == (2, int(prob["ny"]), int(prob["nx"])), psi.shape
    return psi


def apply_h(prob: dict, psi: np.ndarray, a_hom=(0.0, 0.0)) -> np.ndarray:
    """H psi with homogeneous extra vector potential ``a_hom`` (Sec. 3 Hamiltonian)."""
    lib = _load()
    pb = _Problem(prob)
    psi = _check_psi(prob, psi)
    out = np.empty_like(psi)
    a = np.array(a_hom, dtype=np.float64)
    lib.orc_apply_h(pb.ref, _dp(a), _dp(psi.view(np.float64)), _dp(out.view(np.float64)))
    return out


def pulse(prob: dict, t: float) -> np.ndarray:
    lib = _load()
    pb = _Problem(prob)
    a = np.zeros(2)
    lib.orc_pulse(pb.ref, float(t), _dp(a))
    return a


def field_average(prob: dict, t0: float, dt: float) -> np.ndarray:
    lib = _load()
    pb = _Problem(prob)
    a = np.zeros(2)
    lib.orc_field_average(pb.ref, float(t0), float(dt), _dp(a))
    return a


def lanczos(prob: dict, psi: np.ndarray, k: int, dt: float = 1.0, a_hom=(0.0, 0.0),
            reorth: bool = False):
    """Fig. 1 on A = dt*H.  Returns (k_eff, Q[k_eff], alpha[k_eff], beta[k_eff])."""
    lib = _load()
    pb = _Problem(prob)
    psi = _check_psi(prob, psi)
    Q = np.zeros((k,) + psi.shape, dtype=np.complex128)
    al = np.zeros(k)
    be = np.zeros(k)
    a = np.array(a_hom, dtype=np.float64)
    keff = lib.orc_lanczos(pb.ref, _dp(a), float(dt), _dp(psi.view(np.float64)), int(k),
                           int(bool(reorth)), _dp(Q.view(np.float64)), _dp(al), _dp(be))
    return keff, Q[:keff], al[:keff], be[:keff]


def lanczos_plain(prob: dict, psi: np.ndarray, k: int, dt: float = 1.0, a_hom=(0.0, 0.0)):
    """The recurrence of ``lanczos`` (no reorthogonalisation) with three stored
    vectors: returns (k_eff, alpha[k_eff], beta[k_eff]) only."""
    lib = _load()
    pb = _Problem(prob)
    psi = _check_psi(prob, psi)
    al = np.zeros(k)
    be = np.zeros(k)
    a = np.array(a_hom, dtype=np.float64)
    keff = lib.orc_lanczos_plain(pb.ref, _dp(a), float(dt), _dp(psi.view(np.float64)), int(k), _dp(al),
                                 _dp(be))
    return keff, al[:keff], be[:keff]


def ritz_clusters(alpha, beta, e_lo: float, e_hi: float, tol: float, max_out: int = 64):
    """Ritz values of T_k (diagonal alpha, off-diagonal beta[:-1]) in
    [e_lo, e_hi] with the bound of Sec. 2 eq. error_est, |beta_k| times the
    last eigenvector components, taken over clusters of neighbours closer than
    tol (a converged value and its copies after the loss of orthogonality form
    one cluster).  Clusters with bound <= tol are returned ascending as their
    mean: (values, bounds).  The eigenpairs of T come from LAPACK's tridiagonal
    solver (scipy eigh_tridiagonal), restricted to the window."""
    from scipy.linalg import eigh_tridiagonal

    al = np.asarray(alpha, dtype=np.float64)
    be = np.asarray(beta, dtype=np.float64)
    k = len(al)
    if k == 0:
        return np.zeros(0), np.zeros(0)
    if k == 1:
        lam, last = al.copy(), np.ones(1)
        keep = (lam >= e_lo) & (lam <= e_hi)
        lam, last = lam[keep], last[keep]
    else:
        lam, vec = eigh_tridiagonal(al, be[:k - 1], select="v", select_range=(e_lo, e_hi))
        last = vec[k - 1, :] if len(lam) else np.zeros(0)
    order = np.argsort(lam, kind="stable")
    lam, last = lam[order], last[order]
    vals, bnds = [], []
    a = 0
    while a < len(lam):
        b = a + 1
        while b < len(lam) and lam[b] - lam[b - 1] <= tol:
            b += 1
        bound = abs(be[k - 1]) * math.sqrt(float(np.sum(last[a:b] ** 2)))
        if bound <= tol and len(vals) < max_out:
            vals.append(float(np.mean(lam[a:b])))
            bnds.append(bound)
        a = b
    return np.array(vals), np.array(bnds)


def converged_union(alpha, beta, e_lo: float, e_hi: float, tol: float, check_every: int = 64,
                    max_out: int = 64, return_first: bool = False):
    """Converged Ritz clusters accumulated over the leading blocks T_j,
    j = check_every, 2 check_every, ..., and j = k (all of T).  Once
    orthogonality is lost a converged Ritz value acquires copies whose
    eigenvectors of T mix with its own, so its bound |beta_j t_j| can grow
    again while the value stays put; a value whose bound was <= tol at some j
    lies within that bound of an eigenvalue of H all the same (Paige's
    analysis of the finite-precision recurrence).  Values closer than tol are
    one eigenvalue; each keeps the value and bound of its smallest bound.
    Returns (values, bounds), ascending (at most max_out, the lowest), and
    with return_first also the first j at which each value converged."""
    k = len(alpha)
    marks = list(range(check_every, k, check_every)) + [k]
    found = []  # [value, bound, first j]
    for j in marks:
        ev, bd = ritz_clusters(alpha[:j], beta[:j], e_lo, e_hi, tol, max_out=1 << 30)
        for e, b in zip(ev, bd):
            near = [f for f in found if abs(f[0] - e) <= tol]
            if not near:
                found.append([e, b, j])
            elif b < near[0][1]:
                near[0][0], near[0][1] = e, b
    found.sort()
    found = found[:max_out]
    out = (np.array([f[0] for f in found]), np.array([f[1] for f in found]))
    if return_first:
        out += (np.array([f[2] for f in found], dtype=np.int64),)
    return out


def eigen_plain(prob: dict, psi0: np.ndarray, k: int, e_lo: float, e_hi: float, tol: float,
                max_out: int = 64, check_every: int = 64):
    """Eigenvalue mode without reorthogonalisation at any grid size: k
    iterations of the three-vector recurrence on H (fields at t = 0), then the
    converged Ritz clusters of the leading blocks of T accumulated over the
    checkpoints (``converged_union``).  Returns (values, bounds, k_eff)."""
    keff, al, be = lanczos_plain(prob, psi0, k)
    ev, bd = converged_union(al, be, e_lo, e_hi, tol, check_every, max_out)
    return ev, bd, keff


def tridiag_eig(alpha, beta):
    lib = _load()
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    k = len(al)
    be = np.zeros(max(k, 1))
    be[:len(beta)] = beta
    ev = np.zeros(k)
    V = np.zeros((k, k))
    lib.orc_tridiag_eig(k, _dp(al), _dp(be), _dp(ev), _dp(V))
    return ev, V


def expm_e1(alpha, beta, nrm: float = 1.0) -> np.ndarray:
    lib = _load()
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    k = len(al)
    be = np.zeros(max(k, 1))
    be[:len(beta)] = beta
    out = np.zeros(k, dtype=np.complex128)
    lib.orc_expm_e1(k, _dp(al), _dp(be), float(nrm), _dp(out.view(np.float64)))
    return out


def propagate(prob: dict, psi: np.ndarray, t0: float, dt: float, n_steps: int, m: int):
    """n_steps Lanczos short-time steps.  Returns (psi_new, stats dict of arrays)."""
    lib = _load()
    pb = _Problem(prob)
    psi = _check_psi(prob, psi).copy()
    st = (_Stat * max(n_steps, 1))()
    lib.orc_propagate(pb.ref, _dp(psi.view(np.float64)), float(t0), float(dt), int(n_steps),
                      int(m), st)
    stats = {
        "k_eff": np.array([s.k_eff for s in st[:n_steps]], dtype=np.int32),
        "err_est": np.array([s.err_est for s in st[:n_steps]]),
        "cum_bound": np.array([s.cum_bound for s in st[:n_steps]]),
        "norm2": np.array([s.norm2 for s in st[:n_steps]]),
    }
    return psi, stats


def eigen(prob: dict, psi0: np.ndarray, k: int, e_lo: float, e_hi: float, tol: float,
          reorth: bool = False, max_out: int = 64):
    """Ritz values of H in [e_lo, e_hi] converged to ``tol`` after k Lanczos steps."""
    lib = _load()
    pb = _Problem(prob)
    psi0 = _check_psi(prob, psi0)
    ev = np.zeros(max_out)
    bd = np.zeros(max_out)
    nf = ctypes.c_int(0)
    keff = lib.orc_eigen(pb.ref, _dp(psi0.view(np.float64)), int(k), int(bool(reorth)),
                         float(e_lo), float(e_hi), float(tol), int(max_out), _dp(ev), _dp(bd),
                         ctypes.byref(nf))
    return ev[:nf.value].copy(), bd[:nf.value].copy(), keff


def eigen_vectors(prob: dict, psi0: np.ndarray, k: int, e_lo: float, e_hi: float, tol: float,
                  max_out: int = 16):
    """Ritz values, bounds and Ritz vectors (full reorthogonalisation).

    Vector i has shape (2, ny, nx) and the sign that makes <psi0, y_i> real
    and positive (Sec. 2 eq. eigenvec_approx)."""
    lib = _load()
    pb = _Problem(prob)
    psi0 = _check_psi(prob, psi0)
    ev = np.zeros(max_out)
    bd = np.zeros(max_out)
    vecs = np.zeros((max_out,) + psi0.shape, dtype=np.complex128)
    nf = ctypes.c_int(0)
    keff = lib.orc_eigen_vectors(pb.ref, _dp(psi0.view(np.float64)), int(k), float(e_lo), float(e_hi),
                                 float(tol), int(max_out), _dp(ev), _dp(bd), ctypes.byref(nf),
                                 _dp(vecs.view(np.float64)))
    return ev[:nf.value].copy(), bd[:nf.value].copy(), vecs[:nf.value].copy(), keff


def pauli(which: int) -> np.ndarray:
    lib = _load()
    out = np.zeros(8)
    lib.orc_pauli(int(which), _dp(out))
    return out.view(np.complex128).reshape(2, 2)


def expectations(prob: dict, psi: np.ndarray) -> np.ndarray:
    """[<psi|psi>, <x>, <y>, <p_x>, <p_y>] (normalised expectations)."""
    lib = _load()
    pb = _Problem(prob)
    psi = _check_psi(prob, psi)
    out = np.zeros(5)
    lib.orc_expectations(pb.ref, _dp(psi.view(np.float64)), _dp(out))
    return out


LOSS_X, LOSS_Y, LOSS_PX, LOSS_PY = 1, 2, 4, 8


def loss_value(prob: dict, psi: np.ndarray, loss_kind: int) -> float:
    """Sum of the expectations selected by the loss_kind bit flags."""
    e = expectations(prob, psi)
    return float(sum(e[1 + b] for b in range(4) if loss_kind & (1 << b)))


# ---------------------------------------------------------------------------
# Gradient of a final observable with respect to the Fourier laser
# coefficients (the adjoint mode's target).  Two independent definitions:
#   fd_gradient          -- central differences of the oracle's own Lanczos
#                           forward map (the derivative of what is computed);
#   dense_exact_gradient -- tiny grids only: exact propagators
#                           exp(-i dt H(Abar_n)) and their Frechet derivatives
#                           by the block-triangular exponential
#                           expm([[X, E], [0, X]]) = [[e^X, L(X, E)], [0, e^X]],
#                           propagated forward (tangent mode).
# Both take the loss as the sum of the final expectations selected by
# loss_kind (expectations() above), the step-averaged field of Sec. 3 (first
# Magnus term) from field_average().
# ---------------------------------------------------------------------------
def final_loss(prob: dict, psi0: np.ndarray, t0: float, dt: float, n_steps: int, m: int,
               loss_kind: int) -> float:
    """Loss of the state after n_steps oracle steps."""
    psi, _ = propagate(prob, psi0, t0, dt, n_steps, m)
    return loss_value(prob, psi, loss_kind)


def fd_gradient(prob: dict, psi0: np.ndarray, t0: float, dt: float, n_steps: int, m: int,
                loss_kind: int, h: float = 1e-3, idx=None, richardson: bool = True) -> np.ndarray:
    """Central-difference gradient over prob["coef"] (entries ``idx``, default
    all); with ``richardson`` the steps h and h/2 are combined to cancel the
    O(h^2) term."""
    coef = np.asarray(prob["coef"], dtype=np.float64)
    idx = range(len(coef)) if idx is None else idx
    out = np.zeros(len(coef))

    def central(j, step):
        cp = coef.copy()
        cp[j] += step
        lp = final_loss(dict(prob, coef=cp), psi0, t0, dt, n_steps, m, loss_kind)
        cp[j] -= 2 * step
        lm = final_loss(dict(prob, coef=cp), psi0, t0, dt, n_steps, m, loss_kind)
        return (lp - lm) / (2 * step)

    for j in idx:
        d1 = central(j, h)
        out[j] = (4.0 * central(j, h / 2) - d1) / 3.0 if richardson else d1
    return out


def dense_matrix(prob: dict, a_hom=(0.0, 0.0)) -> np.ndarray:
    """H (static fields plus a homogeneous vector potential) as a dense matrix
    in the flattened (2, ny, nx) basis, one column per unit vector."""
    shape = (2, int(prob["ny"]), int(prob["nx"]))
    d = int(np.prod(shape))
    H = np.zeros((d, d), dtype=np.complex128)
    e = np.zeros(d, dtype=np.complex128)
    for col in range(d):
        e[:] = 0.0
        e[col] = 1.0
        H[:, col] = apply_h(prob, e.reshape(shape), a_hom).reshape(-1)
    return H


def _loss_quadratic(prob: dict, v: np.ndarray, loss_kind: int) -> float:
    """<v|O|v> for the selected observables (unnormalised)."""
    e = expectations(prob, v)
    return float(e[0] * sum(e[1 + b] for b in range(4) if loss_kind & (1 << b)))


def dense_exact_gradient(prob: dict, psi0: np.ndarray, t0: float, dt: float, n_steps: int,
                         loss_kind: int):
    """(loss, gradient) of the exact (dense exp) propagation, tiny grids only."""
    from scipy.linalg import expm

    shape = (2, int(prob["ny"]), int(prob["nx"]))
    d = int(np.prod(shape))
    assert d <= 512, "dense_exact_gradient is for tiny grids"
    coef = np.asarray(prob["coef"], dtype=np.float64)
    nc = len(coef)
    static = dict(prob, pulse_kind=0)
    H0 = dense_matrix(static)
    Hx = dense_matrix(static, (1.0, 0.0)) - H0
    Hy = dense_matrix(static, (0.0, 1.0)) - H0
    # step weights w[n, j, axis]: the field average is linear in the coefficients
    w = np.zeros((n_steps, nc, 2))
    for j in range(nc):
        unit = np.zeros(nc)
        unit[j] = 1.0
        pj = dict(prob, coef=unit)
        for n in range(n_steps):
            w[n, j] = field_average(pj, t0 + n * dt, dt)
    psi = _check_psi(prob, psi0).reshape(-1).copy()
    tang = np.zeros((nc, d), dtype=np.complex128)
    Z = np.zeros((d, d), dtype=np.complex128)
    for n in range(n_steps):
        a = field_average(prob, t0 + n * dt, dt)
        X = -1j * dt * (H0 + a[0] * Hx + a[1] * Hy)
        frechet = []
        for E in (-1j * dt * Hx, -1j * dt * Hy):
            B = expm(np.block([[X, E], [Z, X]]))
            frechet.append(B[:d, d:] @ psi)
        U = B[:d, :d]
        tang = tang @ U.T + np.outer(w[n, :, 0], frechet[0]) + np.outer(w[n, :, 1], frechet[1])
        psi = U @ psi
    v = psi.reshape(shape)
    nrm = float(np.vdot(psi, psi).real)
    loss = _loss_quadratic(prob, v, loss_kind) / nrm
    grad = np.zeros(nc)
    for j in range(nc):
        t = tang[j]
        s = np.sqrt(nrm / max(float(np.vdot(t, t).real), 1e-300))
        tv = (s * t).reshape(shape)
        # Re<psi|O|t> by polarisation of the quadratic form
        re_o = (_loss_quadratic(prob, v + tv, loss_kind) - _loss_quadratic(prob, v - tv, loss_kind)) / (4 * s)
        re_n = float(np.vdot(psi, t).real)
        grad[j] = 2.0 * (re_o - loss * re_n) / nrm
    return loss, grad


# ---------------------------------------------------------------------------
# Hermite pseudospectral discretisation (Sec. 5).  A Hermite problem is a dict
# with keys n (collocation points per axis), scale (x = scale * xi), mass, c,
# charge, bz, pot_kind, pot_z, pot_a, chirality; spinors are complex128
# arrays (2, n, n) of the variables sqrt(lambda_i lambda_j) psi(x_i, y_j).
# ---------------------------------------------------------------------------
def hermite_nodes(n: int):
    """Roots xi of the n-th Hermite polynomial (ascending) and the
    Christoffel numbers lambda of the Hermite functions (unit scale)."""
    lib = _load()
    xi = np.zeros(n)
    lam = np.zeros(n)
    lib.orc_hermite_nodes(int(n), _dp(xi), _dp(lam))
    return xi, lam


def hermite_dmat(n: int) -> np.ndarray:
    """The antisymmetric derivative matrix D~ of the collocation variables
    (unit scale), built from the Hermite functions."""
    lib = _load()
    xi, lam = hermite_nodes(n)
    D = np.zeros((n, n))
    lib.orc_hermite_dmat(int(n), _dp(xi), _dp(lam), _dp(D))
    return D


def hermite_operator(hprob: dict):
    """(scaled nodes x, D~ / scale) of a Hermite problem."""
    lib = _load()
    p = _hparams(hprob)
    n = p.n
    x = np.zeros(n)
    D = np.zeros((n, n))
    lib.orc_hermite_operator(ctypes.byref(p), _dp(x), _dp(D))
    return x, D


def apply_h_hermite(hprob: dict, phi: np.ndarray) -> np.ndarray:
    lib = _load()
    p = _hparams(hprob)
    phi = np.ascontiguousarray(phi, dtype=np.complex128)
    assert phi.shape == (2, p.n, p.n)
    out = np.empty_like(phi)
    lib.orc_apply_h_hermite(ctypes.byref(p), _dp(phi.view(np.float64)), _dp(out.view(np.float64)))
    return out


def lanczos_plain_hermite(hprob: dict, phi: np.ndarray, k: int):
    """Three-vector Lanczos on the Hermite H: (k_eff, alpha, beta)."""
    lib = _load()
    p = _hparams(hprob)
    phi = np.ascontiguousarray(phi, dtype=np.complex128)
    assert phi.shape == (2, p.n, p.n)
    al = np.zeros(k)
    be = np.zeros(k)
    keff = lib.orc_lanczos_plain_hermite(ctypes.byref(p), _dp(phi.view(np.float64)), int(k), _dp(al), _dp(be))
    return keff, al[:keff], be[:keff]


def eigen_hermite(hprob: dict, phi0: np.ndarray, k: int, e_lo: float, e_hi: float, tol: float,
                  max_out: int = 64, check_every: int = 64):
    """Eigenvalue mode on the Hermite H: converged Ritz clusters accumulated
    over the checkpoints (converged_union).  Returns (values, bounds, k_eff)."""
    keff, al, be = lanczos_plain_hermite(hprob, phi0, k)
    ev, bd = converged_union(al, be, e_lo, e_hi, tol, check_every, max_out)
    return ev, bd, keff
