"""Pins of the oracle's Hermite pseudospectral discretisation (Sec. 5): the
collocation points and weights against numpy's Gauss-Hermite rule, the
derivative matrix against exact derivatives and the closed form of its
entries, Hermiticity, the free two-dimensional Dirac spectrum, the Lanczos
relation, and the paper's printed soft-core energies (tables
tab:soft_core_groundstates and tab:soft_core_eigenstates_Z_50)."""
import math
import os

import numpy as np
import pytest
from numpy.polynomial.hermite import hermgauss

from paper_1407_7370_amd import packets

C = 137.036
MC2 = C * C
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def hprob(n, scale=1.0, **kw):
    p = dict(n=n, scale=scale, mass=1.0, c=C, charge=-1.0, bz=0.0, pot_kind=0, pot_z=0.0, pot_a=0.0, chirality=0)
    p.update(kw)
    return p


def dense(orc, hp):
    n = hp["n"]
    d = 2 * n * n
    H = np.zeros((d, d), dtype=np.complex128)
    e = np.zeros(d, dtype=np.complex128)
    for k in range(d):
        e[:] = 0.0
        e[k] = 1.0
        H[:, k] = orc.apply_h_hermite(hp, e.reshape(2, n, n)).ravel()
    return H


@pytest.mark.parametrize("n", [8, 33, 64])
def test_nodes_and_weights_vs_gauss_hermite(orc, n):
    xi, lam = orc.hermite_nodes(n)
    x2, w2 = hermgauss(n)
    assert np.max(np.abs(xi - x2)) <= 1e-13 * max(1.0, np.abs(x2).max())
    assert np.max(np.abs(lam / (w2 * np.exp(x2 * x2)) - 1.0)) <= 1e-11


@pytest.mark.parametrize("n", [10, 64])
def test_dmat_exact_on_gaussian_times_polynomial(orc, n):
    """f = exp(-x^2/2) P(x) with deg P <= n - 2 lies in the span with its
    derivative exp(-x^2/2) (P' - x P): D~ maps the collocation values of f to
    those of f' exactly (to rounding), and D~ is antisymmetric with the
    textbook entries (-1)^(i+j) / (xi_i - xi_j) up to one overall sign."""
    xi, lam = orc.hermite_nodes(n)
    D = orc.hermite_dmat(n)
    assert np.max(np.abs(D + D.T)) <= 1e-12 * np.abs(D).max()
    rng = np.random.default_rng(n)
    coef = rng.standard_normal(n - 1) / np.arange(1, n) ** 2   # degree n - 2
    P = np.polynomial.Polynomial(coef)
    f = np.exp(-xi * xi / 2) * P(xi)
    fd = np.exp(-xi * xi / 2) * (P.deriv()(xi) - xi * P(xi))
    sq = np.sqrt(lam)
    assert np.max(np.abs(D @ (sq * f) - sq * fd)) <= 1e-11 * np.max(np.abs(sq * fd))
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    with np.errstate(divide="ignore"):
        F = np.where(i != j, (-1.0) ** (i + j) / (xi[:, None] - xi[None, :]), 0.0)
    assert min(np.max(np.abs(D - F)), np.max(np.abs(D + F))) <= 1e-12 * np.abs(F).max()


@pytest.mark.parametrize("chirality", [1, -1])
def test_hermiticity_with_fields(orc, chirality):
    hp = hprob(10, 0.7, bz=0.9, pot_kind=1, pot_z=1.3, pot_a=0.6, chirality=chirality)
    rng = np.random.default_rng(4)
    u = rng.standard_normal((2, 10, 10)) + 1j * rng.standard_normal((2, 10, 10))
    v = rng.standard_normal((2, 10, 10)) + 1j * rng.standard_normal((2, 10, 10))
    lhs = np.vdot(u.ravel(), orc.apply_h_hermite(hp, v).ravel())
    rhs = np.vdot(orc.apply_h_hermite(hp, u).ravel(), v.ravel())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("chirality", [1, -1])
def test_free_dirac_spectrum(orc, chirality):
    """V = 0, B = 0: p_x and p_y commute and anticommute with the Dirac
    matrices, so the spectrum is +-sqrt(m^2 c^4 + c^2 (k_a^2 + k_b^2)) with
    i k the eigenvalues of D~ / scale (numpy's dense eigensolvers)."""
    n, s = 8, 0.05
    hp = hprob(n, s, chirality=chirality)
    ev = np.linalg.eigvalsh(dense(orc, hp))
    k = np.linalg.eigvals(orc.hermite_dmat(n) / s).imag
    K = np.add.outer(k * k, k * k).ravel()
    e = np.sqrt(MC2 * MC2 + C * C * K)
    ref = np.sort(np.r_[e, -e])
    assert np.max(np.abs(np.sort(ev) - ref)) <= 1e-11 * MC2


def test_lanczos_relation_hermite(orc):
    """The three-vector recurrence on the Hermite H: T from alpha, beta is the
    projection of the dense H onto a Krylov basis built here (numpy, full
    reorthogonalisation) -- same alpha and beta to rounding."""
    import harness as hz
    hp = hprob(8, 0.4, bz=0.5, pot_kind=2, pot_z=2.0)
    psi = packets.hermite_packet(hp, 0.5, (0.2, -0.1))
    keff, al, be = orc.lanczos_plain_hermite(hp, psi, 12)
    al2, be2, _ = hz.lanczos_dense(dense(orc, hp), psi, 12)
    assert keff == 12
    assert np.allclose(al, al2, rtol=0, atol=1e-9 * MC2)
    assert np.allclose(be, be2, rtol=1e-7)


def _table2():
    rows = {}
    with open(os.path.join(GOLDEN, "softcore_ground_states.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                z, lanczos, _, _ = line.split()
                rows[float(z)] = lanczos
    return rows


def _last_digit(text):
    """One unit in the last printed digit of a number as printed."""
    return 10.0 ** -(len(text.split(".")[1]))


@pytest.mark.slow
@pytest.mark.parametrize("Z", [1.0, 2.0, 3.0, 5.0, 10.0, 50.0])
def test_softcore_ground_state_table(orc, Z):
    """Table tab:soft_core_groundstates (64 x 64 Hermite functions, 1000
    Lanczos iterations): the ground state E - m c^2 to within 1.5 units of the
    last printed digit (scale 1.8 / Z, the plateau where the ground state has
    converged; the scale is not given in the paper)."""
    printed = _table2()[Z]
    hp = packets.softcore_hermite(Z)
    psi = packets.hermite_packet(hp, 1.0 / Z, (0.4 / Z, 0.25 / Z))
    ev, bd, _ = orc.eigen_hermite(hp, psi, 1000, MC2 - 0.6 * Z * Z, MC2 - 0.4 * Z * Z, 1e-9 * Z * Z)
    assert len(ev) >= 1
    e = ev[0] - MC2
    print(f"Z={Z}: E - mc^2 = {e:.10f} (paper {printed})", flush=True)
    assert abs(e - float(printed)) <= 1.5 * _last_digit(printed)
    assert e < -0.5 * Z * Z  # below the nonrelativistic value: the relativistic shift


@pytest.mark.slow
def test_softcore_z50_states_table(orc):
    """Table tab:soft_core_eigenstates_Z_50 (1000 iterations): states 1-3 to
    within 1.5 units of the last printed digit; states 4-6, which the paper
    describes as subject to boundary effects (its Lanczos and Fourier columns
    differ by up to 9e-3 there), within 5e-3."""
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "softcore_z50_states.txt"))
            if ln.strip() and not ln.startswith("#")]
    Z = 50.0
    hp = packets.softcore_hermite(Z)
    psi = packets.hermite_packet(hp, 1.0 / Z, (0.4 / Z, 0.25 / Z))
    ev, bd, _ = orc.eigen_hermite(hp, psi, 1000, MC2 - 0.6 * Z * Z, MC2 - 0.14 * Z * Z, 1e-5)
    e = ev - MC2
    print("Z=50 states:", np.round(e, 6).tolist(), flush=True)
    assert len(e) >= 6
    for k in range(6):
        printed = rows[k][1]
        tol = 1.5 * _last_digit(printed) if k < 3 else 5e-3
        assert abs(e[k] - float(printed)) <= tol, (k + 1, e[k], printed)
