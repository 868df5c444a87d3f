"""Seeded synthetic inputs: problem descriptions and initial wave packets.

This module is shared by the GPU path, the oracle tests and the benchmark.  It
holds none of the propagator's arithmetic (no Hamiltonian action, no Lanczos,
no exponential): only the physical problem parameters of the workloads and the
initial states.

Initial state (Sec. 7 of Beerwerth & Bauke, arXiv:1407.7370: a Gaussian
superposition of positive-energy free-particle states): a Gaussian
exp(-|r-r0|^2/(4 sigma^2)) exp(i p0.r) (1, 0)^T is projected mode by mode onto
the positive-energy eigenspace of the free lattice Hamiltonian of the periodic
grid, P+(k) = (1 + H0(k)/E(k))/2 with lattice momentum sin(k h)/h, and
normalised to h_x h_y sum |psi|^2 = 1.  Momenta are drawn uniformly in a disk,
p0 = p_max sqrt(u) (cos 2 pi v, sin 2 pi v), from numpy's default_rng(seed).
"""
from __future__ import annotations

import math

import numpy as np

C_LIGHT = 137.036  # speed of light in atomic units (configuration value)

# ----------------------------------------------------------------------------
# Workloads.  A problem is a plain dict understood by both the GPU binding and
# the oracle wrapper.  Keys: nx, ny, x_min, x_max, y_min, y_max, bc_x, bc_y
# (0 Dirichlet, 1 periodic), mass, c, charge, bz, pot_kind (0 none,
# 1 -Z/sqrt(r^2+a^2), 2 the soft-core form of the paper), pot_z, pot_a,
# pulse_kind (0 none, 1 A0 sin(wt) sin^2(pi t/T) e, 2 Fourier series times
# sin^2), pulse_e, a0, omega, t_pulse, coef.
# ----------------------------------------------------------------------------


def _base(n, lo, hi, bc):
    return dict(nx=n, ny=n, x_min=lo, x_max=hi, y_min=lo, y_max=hi, bc_x=bc, bc_y=bc,
                mass=1.0, c=C_LIGHT, charge=-1.0, bz=0.0, pot_kind=0, pot_z=0.0, pot_a=0.0,
                pulse_kind=0, pulse_e=(0.0, 0.0), a0=0.0, omega=0.0, t_pulse=1.0, coef=None)


def free_packet_64(seed: int = 0):
    """64x64 periodic grid over [-20,20)^2, free electron, m=10, dt=1e-3, 100 steps."""
    prob = _base(64, -20.0, 20.0, 1)
    return dict(name="free_64x64_periodic_fp64", problem=prob, m=10, dt=1e-3, steps=100,
                sigma=2.0, p_max=50.0, center=(0.0, 0.0), seed=seed, precision="fp64")


def landau_softcore_1024(seed: int = 0):
    """1024x1024 Dirichlet grid over [-40,40)^2, B_z=0.5 plus -1/sqrt(r^2+1), m=20."""
    prob = _base(1024, -40.0, 40.0, 0)
    prob.update(bz=0.5, pot_kind=1, pot_z=1.0, pot_a=1.0)
    return dict(name="landau_softcore_1024x1024_fp64", problem=prob, m=20, dt=5e-4, steps=1000,
                sigma=3.0, p_max=0.0, center=(0.0, 0.0), seed=seed, precision="fp64",
                eigen=dict(k_max=2000, e_lo_rel=-2.0, e_hi_rel=5.0, tol=1e-8, n_wanted=8))


def laser_4096(seed: int = 0, precision: str = "mixed"):
    """4096x4096 Dirichlet grid over [-40,40)^2, A(t) = 50 sin(t) sin^2(pi t/T) y-hat,
    T = 500 dt = 0.1, m=16, dt=2e-4, 500 steps."""
    prob = _base(4096, -40.0, 40.0, 0)
    prob.update(pulse_kind=1, pulse_e=(0.0, 1.0), a0=50.0, omega=1.0, t_pulse=0.1)
    return dict(name="laser_4096x4096_" + precision, problem=prob, m=16, dt=2e-4, steps=500,
                sigma=3.0, p_max=50.0, center=(0.0, 0.0), seed=seed, precision=precision)


def fourier_pulse_512(seed: int = 0):
    """512x512 Dirichlet grid over [-20,20)^2, A(t) = sin^2(pi t/T) sum_k Fourier terms,
    T = 2.0, 16 coefficients uniform in [-20,20], m=12, dt=1e-3, 2000 steps."""
    rng = np.random.default_rng(1000 + seed)
    coef = rng.uniform(-20.0, 20.0, size=16)
    prob = _base(512, -20.0, 20.0, 0)
    prob.update(pulse_kind=2, t_pulse=2.0, coef=coef)
    return dict(name="fourier_pulse_512x512_fp64", problem=prob, m=12, dt=1e-3, steps=2000,
                sigma=2.0, p_max=50.0, center=(0.0, 0.0), seed=seed, precision="fp64",
                ckpt_every=50)


def paper_packet_8192(seed: int = 0):
    """The paper's Sec. 7 benchmark shape: 8192^2, k=10, dt=1e-7, mean p=(100,0),
    momentum width 400 (box unstated in the paper: [-0.02,0.02)^2, periodic)."""
    prob = _base(8192, -0.02, 0.02, 1)
    return dict(name="paper_packet_8192x8192_fp64", problem=prob, m=10, dt=1e-7, steps=10,
                sigma=1.0 / (2.0 * 400.0), p_fixed=(100.0, 0.0), center=(0.0, 0.0), seed=seed,
                precision="fp64")


def packet_batch(seed: int = 0, n_packets: int = 256, sizes=(128, 192, 256, 384, 512), h: float = 0.078125):
    """A batch of independent packets of different sizes and fields: grid
    n_b x n_b with n_b drawn from `sizes`, fixed spacing h (box n_b*h, centred),
    Dirichlet, uniform B_z ~ U[0, 2], no potential, packet centre uniform in
    [-n_b h/4, n_b h/4]^2, |p0| <= 5 uniform in the disk, sigma = 2; mixed,
    m = 12, dt = 1e-3, 200 steps.  Returns a list of workload dicts."""
    rng = np.random.default_rng(5000 + seed)
    out = []
    for b in range(n_packets):
        n = int(rng.choice(sizes))
        half = 0.5 * n * h
        prob = _base(n, -half, half, 0)
        prob["bz"] = float(rng.uniform(0.0, 2.0))
        q = 0.25 * n * h
        center = (float(rng.uniform(-q, q)), float(rng.uniform(-q, q)))
        out.append(dict(name=f"batch_{n}x{n}", problem=prob, m=12, dt=1e-3, steps=200, sigma=2.0, p_max=5.0,
                        center=center, seed=int(rng.integers(0, 2 ** 31)), precision="mixed"))
    return out


def with_grid(cfg: dict, n: int):
    """Same workload on an n x n grid over the same box (reduced-size parity cases)."""
    cfg = dict(cfg)
    prob = dict(cfg["problem"])
    prob["nx"] = prob["ny"] = int(n)
    cfg["problem"] = prob
    return cfg


# ----------------------------------------------------------------------------
# Initial states
# ----------------------------------------------------------------------------


def draw_momentum(seed: int, p_max: float):
    rng = np.random.default_rng(seed)
    u, v = rng.random(2)
    r = p_max * math.sqrt(u)
    return (r * math.cos(2 * math.pi * v), r * math.sin(2 * math.pi * v))


def grid_axes(prob: dict):
    hx = (prob["x_max"] - prob["x_min"]) / prob["nx"]
    hy = (prob["y_max"] - prob["y_min"]) / prob["ny"]
    x = prob["x_min"] + hx * np.arange(prob["nx"])
    y = prob["y_min"] + hy * np.arange(prob["ny"])
    return x, y, hx, hy


def positive_energy_projection(psi: np.ndarray, prob: dict) -> np.ndarray:
    """Project each DFT mode of a (2, ny, nx) spinor onto the positive-energy
    eigenspace of the free periodic lattice Hamiltonian of the problem's
    chirality (alpha2 = chi sigma2, chi = -1 when prob["chirality"] < 0)."""
    _, _, hx, hy = grid_axes(prob)
    nx, ny = prob["nx"], prob["ny"]
    c, m = prob["c"], prob["mass"]
    chi = -1.0 if prob.get("chirality", 0) < 0 else 1.0
    kx = np.sin(2 * np.pi * np.fft.fftfreq(nx)) / hx  # sin(k h)/h with k h = 2 pi f
    ky = chi * np.sin(2 * np.pi * np.fft.fftfreq(ny)) / hy
    KX, KY = np.meshgrid(kx, ky)
    mc2 = m * c * c
    E = np.sqrt(mc2 * mc2 + c * c * (KX * KX + KY * KY))
    f0 = np.fft.fft2(psi[0])
    f1 = np.fft.fft2(psi[1])
    # H0 = [[mc2, c(kx - i chi ky)], [c(kx + i chi ky), -mc2]] (chi folded into KY)
    g0 = 0.5 * (f0 + (mc2 * f0 + c * (KX - 1j * KY) * f1) / E)
    g1 = 0.5 * (f1 + (c * (KX + 1j * KY) * f0 - mc2 * f1) / E)
    out = np.empty_like(psi)
    out[0] = np.fft.ifft2(g0)
    out[1] = np.fft.ifft2(g1)
    return out


def gaussian_packet(prob: dict, sigma: float, p0, center=(0.0, 0.0), project: bool = True):
    """Normalised Gaussian spinor packet (2, ny, nx) complex128."""
    x, y, hx, hy = grid_axes(prob)
    X, Y = np.meshgrid(x, y)
    dx, dy = X - center[0], Y - center[1]
    env = np.exp(-(dx * dx + dy * dy) / (4.0 * sigma * sigma))
    phase = np.exp(1j * (p0[0] * X + p0[1] * Y))
    psi = np.zeros((2, prob["ny"], prob["nx"]), dtype=np.complex128)
    psi[0] = env * phase
    if project:
        psi = positive_energy_projection(psi, prob)
    nrm = math.sqrt(hx * hy * float(np.sum(np.abs(psi) ** 2)))
    return psi / nrm


def initial_state(cfg: dict) -> np.ndarray:
    """The seeded initial packet of a workload."""
    prob = cfg["problem"]
    if "p_fixed" in cfg:
        p0 = cfg["p_fixed"]
    else:
        p0 = draw_momentum(cfg.get("seed", 0), cfg.get("p_max", 0.0))
    return gaussian_packet(prob, cfg["sigma"], p0, cfg.get("center", (0.0, 0.0)))


def random_spinor(prob: dict, seed: int) -> np.ndarray:
    """Unstructured complex normal spinor (for algebraic checks)."""
    rng = np.random.default_rng(seed)
    shape = (2, prob["ny"], prob["nx"])
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ----------------------------------------------------------------------------
# Hermite pseudospectral problems (Sec. 5 of the paper).  A Hermite problem is
# a dict: n (collocation points per axis), scale (x = scale * xi, xi the roots
# of the n-th Hermite polynomial), mass, c, charge, bz, pot_kind, pot_z, pot_a,
# chirality.  Spinors are complex128 arrays (2, n, n) of the collocation
# variables sqrt(w_i w_j) psi(x_i, y_j) (w: the scaled quadrature weights of
# the Hermite functions), so that sum |phi|^2 is the L^2 norm.
# ----------------------------------------------------------------------------


def softcore_hermite(Z: float, n: int = 64, kappa: float = 1.8, chirality: int = 0):
    """The paper's soft-core problem (eq. soft_core_pot, -(3/2) Z / sqrt(r^2 +
    3/Z^2)) on n x n Hermite collocation points with length scale kappa / Z
    (the scale is not stated in the paper; kappa = 1.8 lies on the plateau
    where the ground states of its soft-core table converge)."""
    return dict(n=int(n), scale=kappa / Z, mass=1.0, c=C_LIGHT, charge=-1.0, bz=0.0, pot_kind=2,
                pot_z=float(Z), pot_a=0.0, chirality=int(chirality))


def hermite_packet(hprob: dict, width: float, center=(0.0, 0.0)) -> np.ndarray:
    """Normalised Gaussian start vector exp(-|r - r0|^2 / (2 width^2)) (1, 0)^T
    in the collocation variables (nodes and weights from numpy's Gauss-Hermite
    rule; an off-centre r0 couples to every angular momentum)."""
    from numpy.polynomial.hermite import hermgauss
    n, s = int(hprob["n"]), float(hprob["scale"])
    xi, w = hermgauss(n)
    x = s * xi
    sw = np.sqrt(s * w * np.exp(xi * xi))
    gx = np.exp(-((x - center[0]) ** 2) / (2 * width * width)) * sw
    gy = np.exp(-((x - center[1]) ** 2) / (2 * width * width)) * sw
    phi = np.zeros((2, n, n), dtype=np.complex128)
    phi[0] = np.outer(gy, gx)
    return phi / np.linalg.norm(phi)
