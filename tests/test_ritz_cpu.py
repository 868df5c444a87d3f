"""The host half of the eigen modes on the CPU (dirac_lanczos_ritz: Ritz
values of T in a window by bisection, last eigenvector components by
inverse iteration, Sec. 2 eq. error_est), pinned by closed forms, by a matrix
with pairs of nearly equal eigenvalues, and against the oracle's converged
union on Lanczos recurrences of the workloads."""
import numpy as np
import pytest

import oracle as orc
from paper_1407_7370_amd import binding, packets


def _laplacian(k):
    d = np.full(k, 2.0)
    e = np.full(k, -1.0)
    j = np.arange(1, k + 1)
    lam = 2.0 - 2.0 * np.cos(j * np.pi / (k + 1))
    last = np.sqrt(2.0 / (k + 1)) * np.sin(k * j * np.pi / (k + 1))
    return d, e, lam, last


def test_closed_form_laplacian():
    """tridiag(-1, 2, -1): eigenvalues 2 - 2 cos(j pi/(k+1)), eigenvector
    components sqrt(2/(k+1)) sin(i j pi/(k+1)); with beta_k = 1e-9 every value
    in the window converges with bound 1e-9 |last component|."""
    k = 300
    d, e, lam, last = _laplacian(k)
    e[-1] = 1e-9
    lo, hi = 0.5, 1.5
    sel = (lam >= lo) & (lam <= hi)
    ev, bd = binding.ritz(d, e, lo, hi, 1e-8, check_every=0, n_wanted=k)
    assert len(ev) == sel.sum()
    np.testing.assert_allclose(ev, lam[sel], rtol=0, atol=4e-15)
    np.testing.assert_allclose(bd, 1e-9 * np.abs(last[sel]), rtol=1e-9, atol=1e-24)


def test_window_edges_and_single():
    """The window is (e_lo, e_hi] (as LAPACK's selection by value, which the
    oracle uses); k = 1 is its diagonal."""
    d = np.array([1.0, 3.0])
    e = np.array([0.0, 1e-12])  # decoupled: eigenvalues 1 and 3, last components 0 and 1
    ev, bd = binding.ritz(d, e, 0.5, 3.0, 1e-6, check_every=0)
    np.testing.assert_allclose(ev, [1.0, 3.0], rtol=4e-16)
    np.testing.assert_allclose(bd, [0.0, 1e-12], atol=1e-28)
    ev, bd = binding.ritz(d, e, 1.0, 3.0, 1e-6, check_every=0)
    np.testing.assert_allclose(ev, [3.0], rtol=4e-16)
    ev, bd = binding.ritz(np.array([2.5]), np.array([1e-9]), 2.0, 3.0, 1e-6, check_every=0)
    np.testing.assert_array_equal(ev, [2.5])  # k = 1: the diagonal itself
    np.testing.assert_allclose(bd, [1e-9])
    ev, bd = binding.ritz(d, e, 1.5, 2.5, 1e-6, check_every=0)
    assert len(ev) == 0


def test_near_equal_pairs_wilkinson():
    """Wilkinson's W+_{2m+1} (diagonal |m - i|, off-diagonal 1) has pairs of
    eigenvalues that agree to rounding at its top end.  A tol-cluster of such a
    pair reports the pair's mean and beta_k times the weight of e_k on the
    pair's invariant subspace: vectors of one pair must come out orthogonal.
    Reference: LAPACK's dense symmetric solver (numpy.linalg.eigh)."""
    m = 20
    k = 2 * m + 1
    d = np.abs(m - np.arange(k)).astype(float)
    e = np.ones(k)
    beta_k = 1e-7
    e[-1] = beta_k
    T = np.diag(d) + np.diag(e[:-1], 1) + np.diag(e[:-1], -1)
    w, V = np.linalg.eigh(T)
    tol = 1e-6
    lo, hi = 5.0, 30.0
    groups, cur = [], []
    for i in np.where((w >= lo) & (w <= hi))[0]:
        if cur and w[i] - w[cur[-1]] > tol:
            groups.append(cur)
            cur = []
        cur.append(i)
    groups.append(cur)
    assert any(len(g) == 2 for g in groups)  # the matrix has its close pairs in the window
    ref_v = np.array([w[g].mean() for g in groups])
    ref_b = np.array([beta_k * np.sqrt(np.sum(V[k - 1, g] ** 2)) for g in groups])
    ev, bd = binding.ritz(d, e, lo, hi, tol, check_every=0, n_wanted=k)
    assert len(ev) == len(groups)
    np.testing.assert_allclose(ev, ref_v, rtol=0, atol=1e-13)
    # last components carry an absolute error of order eps ||T|| / gap
    np.testing.assert_allclose(bd, ref_b, rtol=1e-6, atol=beta_k * 1e-14)


def _cmp_union(al, be, lo, hi, tol, n_wanted=64):
    ev, bd = binding.ritz(al, be, lo, hi, tol, check_every=64, n_wanted=n_wanted)
    ov, ob = orc.converged_union(al, be, lo, hi, tol, 64, n_wanted)
    assert len(ev) == len(ov)
    np.testing.assert_allclose(ev, ov, rtol=0, atol=1e-12 * max(1.0, np.max(np.abs(ov))))
    # bounds far below rounding level (|beta| eps ||T||) carry no digits
    floor = 1e-11 * np.max(np.abs(al))
    big = ob > floor
    np.testing.assert_allclose(bd[big], ob[big], rtol=1e-4)
    assert np.all(bd[~big] <= 10 * floor)
    return ev


def test_union_vs_oracle_fd_landau():
    """The plain recurrence of a 96 x 96 B + soft-core grid (the 1024^2
    workload's physics on a coarse grid) run past the loss of orthogonality:
    the union over checkpoints equals the oracle's."""
    cfg = packets.with_grid(packets.landau_softcore_1024(), 96)
    prob = cfg["problem"]
    mc2 = prob["mass"] * prob["c"] ** 2
    keff, al, be = orc.lanczos_plain(prob, packets.initial_state(cfg), 700)
    assert keff == 700
    ev = _cmp_union(al, be, mc2 - 2.0, mc2 + 5.0, 1e-6)
    assert len(ev) >= 3


@pytest.mark.parametrize("z", [1.0, 50.0])
def test_union_vs_oracle_hermite(z):
    """The Hermite pseudospectral recurrence (n = 32) of the soft-core
    ground-state problem, 600 iterations."""
    hp = packets.softcore_hermite(z, n=32)
    phi = packets.hermite_packet(hp, 1.0 / z, (0.4 / z, 0.25 / z))
    keff, al, be = orc.lanczos_plain_hermite(hp, phi, 600)
    mc2 = 137.036 ** 2
    ev = _cmp_union(al, be, mc2 - 0.6 * z * z, mc2 - 0.35 * z * z, 2.5e-6)
    assert len(ev) >= 1


def test_rejections():
    al = np.ones(4)
    be = np.ones(4)
    for kw in (dict(e_lo=1.0, e_hi=0.0), dict(tol=-1.0), dict(check_every=-1), dict(n_wanted=0)):
        args = dict(e_lo=0.0, e_hi=1.0, tol=1e-6, check_every=64, n_wanted=4)
        args.update(kw)
        with pytest.raises(binding.DlError):
            binding.ritz(al, be, args["e_lo"], args["e_hi"], args["tol"], args["check_every"], args["n_wanted"])
    with pytest.raises(binding.DlError):
        binding.ritz(al[:0], be[:0], 0.0, 1.0, 1e-6)
