"""GPU parity of the eigen mode with full reorthogonalisation (Sec. 2) and of
the Ritz vectors (Sec. 2 eq. eigenvec_approx), through the C ABI.

Ritz values: against dense eigenvalues (k = dim) and the oracle's values with
full reorthogonalisation.  Ritz vectors: element by element against the
oracle's (same sign convention, <psi0, y> > 0), and by the residual identity
||H y - theta y|| = |beta_k t_k| with H assembled independently, at any size.
Every case prints its name before touching the GPU.
"""
import time

import numpy as np
import pytest

import harness as hz
from paper_1407_7370_amd import packets

pytestmark = pytest.mark.gpu

C = 137.036


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def Prop(torch_cuda):
    from paper_1407_7370_amd.binding import Propagator
    return Propagator


def say(msg):
    print(f"[gpu case] {msg}", flush=True)


def prob_of(nx, ny, bc=0, lo=-4.0, hi=4.0, **kw):
    p = dict(nx=nx, ny=ny, x_min=lo, x_max=hi, y_min=lo * 0.8, y_max=hi * 1.1, bc_x=bc, bc_y=bc,
             mass=1.0, c=C, charge=-1.0, bz=1.0, pot_kind=1, pot_z=1.3, pot_a=0.7, pulse_kind=0,
             pulse_e=(0.0, 0.0), a0=0.0, omega=0.0, t_pulse=1.0, coef=None)
    p.update(kw)
    return p


def residual_check(prob, ev, bd, Y, floor):
    H = hz.dense_h(prob)
    M = Y.reshape(len(ev), -1)
    for th, b, y in zip(ev, bd, M):
        r = np.linalg.norm(H @ y - th * y)
        assert abs(r - b) <= 1e-6 * b + floor, (th, r, b)


def test_reorth_values_small_dense(torch_cuda, Prop, orc):
    """k = dim = 128: every Ritz value is an eigenvalue of the dense H."""
    torch = torch_cuda
    prob = prob_of(8, 8)
    w = np.linalg.eigvalsh(hz.dense_h(prob).toarray())
    psi0 = packets.random_spinor(prob, 2)
    say("eigen reorth 8x8 K=128 (all eigenvalues)")
    prop = Prop(prob, 1, "fp64", k_eigen=128, reorth=True)
    ev, bd = prop.eigen(torch.from_numpy(psi0).cuda(), 128, -1e9, 1e9, 1e-6, n_wanted=256, reorth=True)
    prop.close()
    assert len(ev) == 128
    assert np.allclose(ev, w, atol=1e-8 * np.abs(w).max())
    rev, _, _ = orc.eigen(prob, psi0, 128, -1e9, 1e9, 1e-6, reorth=True, max_out=256)
    assert np.allclose(ev, rev, atol=1e-9 * np.abs(w).max())


def test_ritz_vectors_small_vs_oracle(torch_cuda, Prop, orc):
    torch = torch_cuda
    prob = prob_of(8, 8)
    psi0 = packets.random_spinor(prob, 2)
    say("ritz vectors 8x8 K=128")
    prop = Prop(prob, 1, "fp64", k_eigen=128, reorth=True)
    ev, bd, Y = prop.eigen_vectors(torch.from_numpy(psi0).cuda(), 128, -1e9, 1e9, 1e-6, n_wanted=128)
    prop.close()
    Y = Y.cpu().numpy()
    rev, rbd, RY, keff = orc.eigen_vectors(prob, psi0, 128, -1e9, 1e9, 1e-6, max_out=128)
    assert keff == 128 and len(ev) == len(rev) == 128
    assert np.allclose(ev, rev, atol=1e-9 * np.abs(rev).max())
    err = np.abs(Y - RY).reshape(128, -1).max(axis=1)
    print("ritz 8x8: max |y_gpu - y_oracle| =", float(err.max()), flush=True)
    assert np.all(err <= 1e-8)


@pytest.mark.parametrize("nx,ny,bc", [(37, 29, 0), (40, 33, 1)])
def test_ritz_vectors_ragged_vs_oracle(torch_cuda, Prop, orc, nx, ny, bc):
    """Ragged grids (several projection tiles and a partial one): values,
    vectors and the residual identity."""
    torch = torch_cuda
    prob = prob_of(nx, ny, bc, c=5.0, bz=0.7)
    psi0 = packets.random_spinor(prob, 5)
    say(f"ritz vectors {nx}x{ny} bc={bc} K=140")
    prop = Prop(prob, 1, "fp64", k_eigen=140, reorth=True)
    ev, bd, Y = prop.eigen_vectors(torch.from_numpy(psi0).cuda(), 140, -1e9, 1e9, 1e-4, n_wanted=64)
    prop.close()
    Y = Y.cpu().numpy()
    rev, rbd, RY, keff = orc.eigen_vectors(prob, psi0, 140, -1e9, 1e9, 1e-4, max_out=64)
    print(f"ritz {nx}x{ny}: {len(ev)} values, bounds {bd.min():.1e}..{bd.max():.1e}", flush=True)
    assert keff == 140 and len(ev) == len(rev) and len(ev) >= 5
    assert np.allclose(ev, rev, rtol=0, atol=1e-9 * np.abs(rev).max())
    assert np.allclose(bd, rbd, rtol=1e-4, atol=1e-12)
    err = np.abs(Y - RY).reshape(len(ev), -1).max(axis=1)
    print("  max |y_gpu - y_oracle| =", float(err.max()), flush=True)
    assert np.all(err <= 1e-8)
    residual_check(prob, ev, bd, Y, 1e-12)
    M = Y.reshape(len(ev), -1)
    assert np.allclose(M.conj() @ M.T, np.eye(len(ev)), atol=1e-10)


def test_reorth_edge_cases(torch_cuda, Prop, orc):
    from paper_1407_7370_amd import binding
    torch = torch_cuda
    prob = prob_of(16, 12)
    say("eigen reorth edge cases 16x12")
    prop = Prop(prob, 1, "fp64", k_eigen=40, reorth=True)
    # zero start vector: nothing to report
    z = torch.zeros((2, 12, 16), dtype=torch.complex128, device="cuda")
    ev, bd = prop.eigen(z, 40, -1e9, 1e9, 1e-6, reorth=True)
    assert len(ev) == 0
    ev, bd, Y = prop.eigen_vectors(z, 40, -1e9, 1e9, 1e-6)
    assert len(ev) == 0
    # k_max = 1: the Rayleigh quotient, bound beta_1 = ||H q - alpha q||
    psi0 = packets.random_spinor(prob, 7)
    ev, bd, Y = prop.eigen_vectors(torch.from_numpy(psi0).cuda(), 1, -1e9, 1e9, 1e9)
    q = psi0.reshape(-1) / np.linalg.norm(psi0)
    Hq = hz.dense_h(prob) @ q
    ray = np.vdot(q, Hq).real
    assert len(ev) == 1 and abs(ev[0] - ray) <= 1e-12 * abs(ray)
    assert abs(bd[0] - np.linalg.norm(Hq - ray * q)) <= 1e-10 * bd[0]
    assert np.allclose(Y[0].cpu().numpy().reshape(-1), q, atol=1e-14)
    # bitwise reproducible
    psi = torch.from_numpy(psi0).cuda()
    a = prop.eigen_vectors(psi, 40, -1e9, 1e9, 1e-3)
    b = prop.eigen_vectors(psi, 40, -1e9, 1e9, 1e-3)
    assert np.array_equal(a[0], b[0]) and torch.equal(a[2], b[2])
    # non-finite start vector
    bad = psi0.copy()
    bad[0, 3, 3] = np.nan
    with pytest.raises(binding.DlError) as ei:
        prop.eigen(torch.from_numpy(bad).cuda(), 40, -1e9, 1e9, 1e-6, reorth=True)
    assert ei.value.status == binding.DL_ERR_NONFINITE
    # more iterations than the workspace holds
    with pytest.raises(binding.DlError) as ei:
        prop.eigen_vectors(psi, 41, -1e9, 1e9, 1e-6)
    assert ei.value.status == binding.DL_ERR_WORKSPACE
    prop.close()
    # a plain eigen workspace does not hold the stored basis
    plain = Prop(prob, 1, "fp64", k_eigen=40)
    with pytest.raises(binding.DlError) as ei:
        plain.eigen(psi, 40, -1e9, 1e9, 1e-6, reorth=True)
    assert ei.value.status == binding.DL_ERR_WORKSPACE
    plain.close()


def test_reorth_exact_eigenvector(torch_cuda, Prop):
    """A uniform upper spinor on a periodic field-free grid is an exact
    eigenvector (value m c^2): breakdown after one iteration."""
    torch = torch_cuda
    prob = prob_of(8, 8, 1, bz=0.0, pot_kind=0)
    say("eigen reorth exact eigenvector 8x8 periodic")
    const = np.zeros((2, 8, 8), dtype=np.complex128)
    const[0] = 1.0
    prop = Prop(prob, 1, "fp64", k_eigen=20, reorth=True)
    ev, bd, Y = prop.eigen_vectors(torch.from_numpy(const).cuda(), 20, -1e9, 1e9, 1e-6)
    prop.close()
    assert len(ev) == 1 and abs(ev[0] - C * C) <= 1e-10 * C * C
    assert bd[0] <= 1e-9
    assert np.allclose(Y[0].cpu().numpy(), const / 8.0, atol=1e-15)


def test_reorth_vs_plain_softcore_256(torch_cuda, Prop, orc):
    """B + soft core on 256^2 (the 1024^2 eigen workload's physics): values
    converged with full reorthogonalisation are values of the plain run."""
    torch = torch_cuda
    mc2 = C * C
    cfg = packets.with_grid(packets.landau_softcore_1024(), 256)
    prob = cfg["problem"]
    psi0 = packets.initial_state(cfg)
    lo, hi, tol = mc2 - 2.0, mc2 + 5.0, 1e-6
    say("eigen reorth vs plain 256x256 K=800/600")
    pr = Prop(prob, 1, "fp64", k_eigen=800, reorth=True)
    ev, bd, Y = pr.eigen_vectors(torch.from_numpy(psi0).cuda(), 800, lo, hi, tol, n_wanted=16)
    pr.close()
    pp = Prop(prob, 1, "fp64", k_eigen=600)
    pev, pbd = pp.eigen(torch.from_numpy(psi0).cuda(), 600, lo, hi, tol)
    pp.close()
    print("reorth:", np.round(ev - mc2, 9).tolist(), "plain:", np.round(pev - mc2, 9).tolist(), flush=True)
    assert len(ev) >= 2
    common = [e for e in ev if np.min(np.abs(pev - e)) <= 1e-7]
    assert len(common) >= min(len(ev), len(pev)) - 1
    residual_check(prob, ev, bd, Y.cpu().numpy(), 1e-9)


def test_reorth_full_grid_properties(torch_cuda, Prop, orc):
    """1024^2 B + soft-core workload, K = 500 with full reorthogonalisation:
    orthonormal Ritz vectors, sign convention, the residual identity with the
    oracle's H, and the sustained bandwidth of the reorthogonalisation."""
    torch = torch_cuda
    mc2 = C * C
    cfg = packets.landau_softcore_1024()
    prob = cfg["problem"]
    psi0 = packets.initial_state(cfg)
    K = 500
    lo, hi, tol = mc2 - 2.0, mc2 + 5.0, 1e-6
    say(f"eigen reorth 1024x1024 K={K}")
    prop = Prop(prob, 1, "fp64", k_eigen=K, reorth=True)
    psi = torch.from_numpy(psi0).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev, bd, Y = prop.eigen_vectors(psi, K, lo, hi, tol, n_wanted=8)
    t1 = time.perf_counter()
    prop.close()
    n = psi0.size
    # algorithmic bytes: per iteration i two passes of (read i vectors + z for
    # the projection, read i vectors + read/write z for the update)
    byt = sum(2 * (2 * i + 3) * 16 * n for i in range(1, K + 1))
    print(f"reorth 1024^2 K={K}: {t1 - t0:.2f} s, {byt / (t1 - t0) / 1e9:.0f} GB/s of CGS2 traffic; "
          f"values (E - mc^2): {np.round(ev - mc2, 8).tolist()}", flush=True)
    assert 1 <= len(ev) <= 8
    assert np.all(bd <= tol) and np.all(np.diff(ev) > tol)
    M = Y.reshape(len(ev), -1)
    G = (M.conj() @ M.T).cpu().numpy()
    assert np.allclose(G, np.eye(len(ev)), atol=1e-10)
    ov = (M.conj() @ psi.reshape(-1)).cpu().numpy()
    assert np.all(ov.real > 0) and np.all(np.abs(ov.imag) <= 1e-9 * ov.real)
    Yh = Y.cpu().numpy()
    for th, b, y in zip(ev, bd, Yh):
        r = np.linalg.norm((orc.apply_h(prob, y) - th * y).reshape(-1))
        assert abs(r - b) <= 1e-6 * b + 1e-9, (th, r, b)


def test_eigen_early_stop(torch_cuda, Prop):
    """The recurrence stops at the first check (every 64 iterations) where
    n_wanted clusters have converged: asking for fewer values returns values
    of the longer run, sooner."""
    torch = torch_cuda
    mc2 = C * C
    cfg = packets.landau_softcore_1024()
    prob = cfg["problem"]
    psi = torch.from_numpy(packets.initial_state(cfg)).cuda()
    lo, hi, tol = mc2 - 2.0, mc2 + 5.0, 1e-6
    say("eigen early stop 1024x1024 K<=2000, n_wanted 2 vs 8")
    prop = Prop(prob, 1, "fp64", k_eigen=2000)
    times, res = {}, {}
    for nw in (8, 2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res[nw] = prop.eigen(psi, 2000, lo, hi, tol, n_wanted=nw)
        times[nw] = time.perf_counter() - t0
    prop.close()
    print(f"n_wanted 8: {times[8]:.2f} s {np.round(res[8][0] - mc2, 8).tolist()}; n_wanted 2: {times[2]:.2f} s "
          f"{np.round(res[2][0] - mc2, 8).tolist()}", flush=True)
    ev2, bd2 = res[2]
    assert len(ev2) == 2 and np.all(bd2 <= tol)
    for e in ev2:
        assert np.min(np.abs(res[8][0] - e)) <= 1e-7
