"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

FP64 results must match the oracle to 1e-10 relative L2 (the bound stated for
the FP64 propagator); single-operator applications to 1e-13.  Every case
prints its name before touching the GPU.
"""
import math
import os

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


def gpu_run(torch, Prop, prob, m, prec, psi0, t0, dt, n, **kw):
    prop = Prop(prob, m, prec, **kw)
    psi = torch.from_numpy(np.ascontiguousarray(psi0)).to("cuda")
    st = prop.step(psi, t0, dt, n)
    out = psi.cpu().numpy()
    prop.close()
    return out, st


def box(nx, ny, bc, lo=-6.0, hi=6.0, **kw):
    p = dict(nx=nx, ny=ny, x_min=lo, x_max=hi, y_min=lo * 0.9, y_max=hi * 1.2, bc_x=bc, bc_y=bc,
             mass=1.0, c=C, charge=-1.0, bz=0.0, pot_kind=0, pot_z=0.0, pot_a=0.0, pulse_kind=0,
             pulse_e=(0.0, 0.0), a0=0.0, omega=0.0, t_pulse=1.0, coef=None)
    p.update(kw)
    return p


# ---------------------------------------------------------------------------
# Single application of H
# ---------------------------------------------------------------------------
APPLY_CASES = {
    "free_64_periodic": (box(64, 64, 1), 0.0),
    "ragged_131x77_dirichlet_b_soft": (box(131, 77, 0, bz=0.8, pot_kind=1, pot_z=1.0, pot_a=1.0), 0.0),
    "ragged_61x5_periodic_b": (box(61, 5, 1, bz=-1.3), 0.0),
    "tiny_3x3_dirichlet": (box(3, 3, 0, bz=0.4), 0.0),
    "tiny_4x3_periodic": (box(4, 3, 1, pot_kind=2, pot_z=2.0), 0.0),
    "x_periodic_y_dirichlet_200x130": (dict(box(200, 130, 0, bz=0.3), bc_x=1), 0.0),
    "laser_t": (dict(box(96, 70, 0), pulse_kind=1, pulse_e=(0.6, 0.8), a0=50.0, omega=1.0,
                     t_pulse=0.1), 0.037),
    "fourier_t": (dict(box(70, 96, 0), pulse_kind=2, t_pulse=2.0,
                       coef=np.random.default_rng(3).uniform(-20, 20, 16)), 0.71),
    "one_strip_boundary_124x200": (box(124, 200, 0, bz=0.5), 0.0),
    "chirality_minus_b_laser": (dict(box(96, 70, 0, bz=0.6, pot_kind=1, pot_z=1.0, pot_a=1.0), pulse_kind=1,
                                     pulse_e=(0.6, 0.8), a0=50.0, omega=1.0, t_pulse=0.1, chirality=-1), 0.037),
    "chirality_minus_periodic": (dict(box(64, 48, 1, bz=-0.9), chirality=-1), 0.0),
}


@pytest.mark.parametrize("case", sorted(APPLY_CASES))
def test_apply_vs_oracle(torch_cuda, Prop, orc, case):
    prob, t = APPLY_CASES[case]
    say(f"apply {case} {prob['nx']}x{prob['ny']}")
    torch = torch_cuda
    psi = packets.random_spinor(prob, 5)
    prop = Prop(prob, 4, "fp64")
    y = prop.apply(torch.from_numpy(psi).cuda(), t).cpu().numpy()
    prop.close()
    ref = orc.apply_h(prob, psi, orc.pulse(prob, t))
    assert np.max(np.abs(y - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_apply_potential_table(torch_cuda, Prop, orc):
    prob = box(90, 66, 0, bz=0.2)
    say("apply potential table 90x66")
    vt = np.random.default_rng(1).standard_normal((66, 90))
    psi = packets.random_spinor(prob, 6)
    prop = Prop(prob, 4, "fp64", v_table=vt)
    y = prop.apply(torch_cuda.from_numpy(psi).cuda(), 0.0).cpu().numpy()
    prop.close()
    ref = orc.apply_h(dict(prob, v_table=vt), psi)
    assert np.max(np.abs(y - ref)) <= 1e-13 * np.max(np.abs(ref))


# ---------------------------------------------------------------------------
# Time steps, FP64
# ---------------------------------------------------------------------------
def test_free_packet_64_full(torch_cuda, Prop, orc):
    cfg = packets.free_packet_64(seed=0)
    say("free packet 64x64 periodic m=10 100 steps fp64")
    prob = cfg["problem"]
    psi0 = packets.initial_state(cfg)
    got, st = gpu_run(torch_cuda, Prop, prob, cfg["m"], "fp64", psi0, 0.0, cfg["dt"], cfg["steps"])
    ref, rst = orc.propagate(prob, psi0, 0.0, cfg["dt"], cfg["steps"], cfg["m"])
    assert hz.rel_l2(got, ref) <= 1e-10
    assert np.array_equal(st["k_eff"], rst["k_eff"])
    assert np.allclose(st["norm2"], rst["norm2"], rtol=1e-12)
    # also the exact lattice solution
    assert hz.rel_l2(got, hz.free_propagate_fft(prob, psi0, cfg["steps"] * cfg["dt"])) <= 1e-10


@pytest.mark.parametrize("n", [96, 160])
def test_landau_softcore_reduced(torch_cuda, Prop, orc, n):
    cfg = packets.landau_softcore_1024()
    cfg = packets.with_grid(cfg, n)
    prob = dict(cfg["problem"], ny=n - 27)  # ragged, non-square
    say(f"B + soft-core Dirichlet {prob['nx']}x{prob['ny']} m=20 40 steps fp64")
    psi0 = packets.gaussian_packet(prob, cfg["sigma"], (0.0, 0.0))
    got, st = gpu_run(torch_cuda, Prop, prob, cfg["m"], "fp64", psi0, 0.0, cfg["dt"], 40)
    ref, rst = orc.propagate(prob, psi0, 0.0, cfg["dt"], 40, cfg["m"])
    assert hz.rel_l2(got, ref) <= 1e-10
    assert np.array_equal(st["k_eff"], rst["k_eff"])


def test_landau_softcore_full_grid(torch_cuda, Prop, orc):
    cfg = packets.landau_softcore_1024()
    say("B + soft-core Dirichlet 1024x1024 m=20 3 steps fp64 (full grid)")
    prob = cfg["problem"]
    psi0 = packets.initial_state(cfg)
    got, st = gpu_run(torch_cuda, Prop, prob, cfg["m"], "fp64", psi0, 0.0, cfg["dt"], 3)
    ref, _ = orc.propagate(prob, psi0, 0.0, cfg["dt"], 3, cfg["m"])
    assert hz.rel_l2(got, ref) <= 1e-10


@pytest.mark.parametrize("n", [128, 250])
def test_laser_reduced_fp64(torch_cuda, Prop, orc, n):
    cfg = packets.with_grid(packets.laser_4096(precision="fp64"), n)
    prob = dict(cfg["problem"], t_pulse=40 * cfg["dt"])
    say(f"laser pulse Dirichlet {n}x{n} m=16 40 steps fp64")
    psi0 = packets.initial_state(cfg)
    got, _ = gpu_run(torch_cuda, Prop, prob, cfg["m"], "fp64", psi0, 0.0, cfg["dt"], 40)
    ref, _ = orc.propagate(prob, psi0, 0.0, cfg["dt"], 40, cfg["m"])
    assert hz.rel_l2(got, ref) <= 1e-10


def test_fourier_pulse_reduced_fp64(torch_cuda, Prop, orc):
    cfg = packets.with_grid(packets.fourier_pulse_512(), 100)
    prob = dict(cfg["problem"], t_pulse=0.06)
    say("Fourier pulse Dirichlet 100x100 m=12 80 steps fp64")
    psi0 = packets.initial_state(cfg)
    got, _ = gpu_run(torch_cuda, Prop, prob, cfg["m"], "fp64", psi0, 0.0, cfg["dt"], 80)
    ref, _ = orc.propagate(prob, psi0, 0.0, cfg["dt"], 80, cfg["m"])
    assert hz.rel_l2(got, ref) <= 1e-10


@pytest.mark.parametrize("m", [1, 2, 3, 5])
def test_small_krylov_dims(torch_cuda, Prop, orc, m):
    prob = box(70, 45, 0, bz=0.7, pot_kind=1, pot_z=1.0, pot_a=1.0)
    say(f"small Krylov m={m} 70x45")
    psi0 = packets.gaussian_packet(prob, 1.5, (2.0, -1.0))
    got, st = gpu_run(torch_cuda, Prop, prob, m, "fp64", psi0, 0.0, 2e-4, 5)
    ref, rst = orc.propagate(prob, psi0, 0.0, 2e-4, 5, m)
    assert hz.rel_l2(got, ref) <= 1e-10
    assert np.allclose(st["err_est"], rst["err_est"], rtol=1e-6, atol=1e-300)


@pytest.mark.parametrize("dt,prec,tol", [(1e-3, "fp64", 1e-10), (1e-2, "fp64", 1e-10), (1e-2, "mixed", 1e-6)])
def test_max_krylov_dim(torch_cuda, Prop, orc, dt, prec, tol):
    """The largest Krylov dimension, m = 64 (the small exponential then uses
    all 64 lanes of its wave): the Chebyshev expansion (dt = 1e-3, R = 20) and
    the QR eigendecomposition (dt = 1e-2, R = 205), three steps against the
    oracle."""
    prob = box(48, 40, 0, bz=0.7, pot_kind=1, pot_z=1.0, pot_a=1.0)
    psi0 = packets.gaussian_packet(prob, 0.8, (3.0, -2.0))
    say(f"max Krylov m=64 dt={dt} {prec} 48x40")
    got, st = gpu_run(torch_cuda, Prop, prob, 64, prec, psi0, 0.0, dt, 3)
    ref, rst = orc.propagate(prob, psi0, 0.0, dt, 3, 64)
    err = hz.rel_l2(got, ref)
    if prec == "mixed":
        tol = mixed_tolerance(st, psi0, rst)
    print(f"m=64 dt={dt} {prec}: rel-L2 {err:.3e} (tolerance {tol:.3e})", flush=True)
    assert err <= tol
    assert np.all(st["k_eff"] == 64) and np.all(rst["k_eff"] == 64)
    assert np.allclose(st["norm2"], rst["norm2"], rtol=tol, atol=0.0)


@pytest.mark.parametrize("dt", [1e-5, 1e-3, 3e-3, 1e-2, 3e-2])
def test_small_exponential_ranges(torch_cuda, Prop, orc, dt):
    """The half-width R of the spectrum of the shifted T grows with dt
    (R = 0.2 .. 600 here, m = 16): the Chebyshev expansion (R up to ~190) and
    the QR eigendecomposition (beyond) both match the oracle's Jacobi
    eigendecomposition."""
    prob = box(48, 40, 0, bz=0.7, pot_kind=1, pot_z=1.0, pot_a=1.0)
    psi0 = packets.gaussian_packet(prob, 0.8, (3.0, -2.0))
    keff, _, al, be = orc.lanczos(prob, psi0, 16, dt=dt)
    d, e = al - al[0], be[:keff - 1]
    rad = np.abs(np.r_[e, 0.0]) + np.abs(np.r_[0.0, e])
    R = 0.5 * (np.max(d + rad) - np.min(d - rad))
    say(f"small exponential dt={dt} (R = {R:.1f}) 48x40 m=16")
    got, st = gpu_run(torch_cuda, Prop, prob, 16, "fp64", psi0, 0.0, dt, 3)
    ref, rst = orc.propagate(prob, psi0, 0.0, dt, 3, 16)
    assert hz.rel_l2(got, ref) <= 1e-10
    # |c_k| from a dense eigendecomposition carries an absolute rounding error
    # of a few eps (1 + ||T'||) ||psi||, so the estimate beta_k ||psi|| |c_k| is
    # compared above that floor (the oracle's value is that noise when the true
    # one is far smaller: |c_k| = 3e-50 at dt = 1e-5, checked in 60-digit
    # arithmetic, which the expansion resolves)
    floor = 20 * np.finfo(float).eps * (1.0 + R) * be[keff - 1] * np.linalg.norm(psi0)
    assert np.allclose(st["err_est"], rst["err_est"], rtol=1e-6, atol=floor)


def test_backward_returns(torch_cuda, Prop, orc):
    cfg = packets.with_grid(packets.laser_4096(precision="fp64"), 120)
    prob = dict(cfg["problem"], t_pulse=0.01, a0=300.0)
    say("time reversal 120x120 laser 50+50 steps")
    torch = torch_cuda
    psi0 = packets.initial_state(cfg)
    prop = Prop(prob, 16, "fp64")
    psi = torch.from_numpy(psi0).cuda()
    prop.step(psi, 0.0, 2e-4, 50)
    mid = psi.cpu().numpy()
    prop.step(psi, 50 * 2e-4, -2e-4, 50)
    back = psi.cpu().numpy()
    prop.close()
    assert hz.rel_l2(mid, psi0) > 1e-3
    assert hz.rel_l2(back, psi0) <= 1e-11


# ---------------------------------------------------------------------------
# Determinism and resume
# ---------------------------------------------------------------------------
def test_bitwise_repeat_and_resume(torch_cuda, Prop):
    cfg = packets.with_grid(packets.landau_softcore_1024(), 200)
    prob = cfg["problem"]
    say("determinism 200x200 B+soft-core 20 steps: repeat and 7+13 resume")
    torch = torch_cuda
    psi0 = packets.initial_state(cfg)
    outs = []
    for split in (None, None, 7):
        prop = Prop(prob, 20, "fp64")
        psi = torch.from_numpy(psi0).cuda()
        if split is None:
            prop.step(psi, 0.0, 5e-4, 20)
        else:
            prop.step(psi, 0.0, 5e-4, split)
            prop.step(psi, split * 5e-4, 5e-4, 20 - split)
        outs.append(psi.cpu().numpy())
        prop.close()
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], outs[2])


# ---------------------------------------------------------------------------
# Degenerate cases
# ---------------------------------------------------------------------------
def test_breakdown_plane_wave_and_zero(torch_cuda, Prop, orc):
    torch = torch_cuda
    prob = box(8, 8, 1, lo=-0.04, hi=0.04)
    prob["y_min"], prob["y_max"] = -0.04, 0.04
    x, y, hx, hy = hz.axes(prob)
    X, Y = np.meshgrid(x, y)
    psi0 = np.stack([np.exp(1j * 2 * math.pi * 2 / 0.08 * X), np.zeros_like(X, dtype=complex)])
    say("breakdown: periodic plane wave 8x8 (k_eff 2)")
    got, st = gpu_run(torch, Prop, prob, 10, "fp64", psi0, 0.0, 1e-3, 3)
    ref, rst = orc.propagate(prob, psi0, 0.0, 1e-3, 3, 10)
    assert np.all(st["k_eff"] == 2) and np.all(rst["k_eff"] == 2)
    assert hz.rel_l2(got, ref) <= 1e-12
    say("zero state 8x8")
    z, st = gpu_run(torch, Prop, prob, 10, "fp64", np.zeros_like(psi0), 0.0, 1e-3, 3)
    assert np.all(z == 0) and np.all(st["k_eff"] == 0) and np.all(st["norm2"] == 0)
    say("uniform upper spinor 8x8 periodic: exact eigenvector, k_eff 1")
    const = np.stack([np.ones_like(X, dtype=complex), np.zeros_like(X, dtype=complex)])
    got, st = gpu_run(torch, Prop, prob, 6, "fp64", const, 0.0, 1e-3, 2)
    assert np.all(st["k_eff"] == 1)
    assert np.allclose(got, const * np.exp(-2j * 1e-3 * C * C), atol=1e-12)


def test_nonfinite_input(torch_cuda, Prop):
    from paper_1407_7370_amd import binding
    torch = torch_cuda
    prob = box(40, 40, 0)
    say("non-finite input 40x40")
    psi0 = packets.gaussian_packet(prob, 1.0, (0.0, 0.0))
    psi0[1, 20, 20] = np.nan
    prop = Prop(prob, 8, "fp64")
    psi = torch.from_numpy(psi0).cuda()
    with pytest.raises(binding.DlError) as ei:
        prop.step(psi, 0.0, 1e-3, 4)
    assert ei.value.status == binding.DL_ERR_NONFINITE
    # nothing completed: psi still holds the input
    back = psi.cpu().numpy()
    assert np.array_equal(np.isnan(back), np.isnan(psi0))
    assert np.array_equal(back[~np.isnan(back)], psi0[~np.isnan(psi0)])
    prop.close()


def test_invalid_calls(torch_cuda, Prop):
    from paper_1407_7370_amd import binding
    torch = torch_cuda
    prob = box(16, 16, 0)
    say("invalid calls 16x16")
    prop = Prop(prob, 4, "fp64")
    psi = torch.zeros((2, 16, 16), dtype=torch.complex128, device="cuda")
    for dt in (0.0, float("nan")):
        with pytest.raises(binding.DlError) as ei:
            prop.step(psi, 0.0, dt, 1)
        assert ei.value.status == binding.DL_ERR_INVALID
    with pytest.raises(binding.DlError) as ei:
        prop.step(psi, 0.0, 1e-3, -1)
    assert ei.value.status == binding.DL_ERR_INVALID
    with pytest.raises(binding.DlError) as ei:
        prop.eigen(psi, 10, -1.0, 1.0, 1e-6, reorth=True)
    assert ei.value.status in (binding.DL_ERR_UNSUPPORTED, binding.DL_ERR_WORKSPACE)
    import ctypes
    loss = ctypes.c_double(0)
    grad = (ctypes.c_double * 16)()
    # loss_kind 0 selects no observable; a missing adjoint workspace is also rejected
    st = binding.dirac_lanczos_adjoint(prop.ctx, psi.data_ptr(), 0.0, 1e-3, 10, 5, 0, 0, 0,
                                       ctypes.byref(loss), grad)
    assert st == binding.DL_ERR_INVALID
    st = binding.dirac_lanczos_adjoint(prop.ctx, psi.data_ptr(), 0.0, 1e-3, 10, 5, 1, 0, 0,
                                       ctypes.byref(loss), grad)
    assert st in (binding.DL_ERR_UNSUPPORTED, binding.DL_ERR_WORKSPACE)
    prop.close()


# ---------------------------------------------------------------------------
# Mixed precision
# ---------------------------------------------------------------------------
def mixed_tolerance(st, psi0, rst=None):
    """Relative distance allowed between a mixed-precision run and the FP64
    oracle: the summed a-priori storage bounds of the steps (round_bound) plus
    both runs' Krylov estimates, relative to ||psi_0||, plus the FP64 parity
    tolerance 1e-10 for the arithmetic both share."""
    nrm = np.linalg.norm(psi0)
    kry = st["cum_bound"][-1] + (rst["cum_bound"][-1] if rst is not None else 0.0)
    return (st["cum_round_bound"][-1] + kry) / nrm + 1e-10


def test_mixed_vs_fp64_reduced(torch_cuda, Prop, orc):
    cfg = packets.with_grid(packets.laser_4096(), 256)
    prob = dict(cfg["problem"], t_pulse=100 * cfg["dt"])
    say("mixed vs fp64 laser 256x256 m=16 100 steps")
    psi0 = packets.initial_state(cfg)
    mx, smx = gpu_run(torch_cuda, Prop, prob, 16, "mixed", psi0, 0.0, cfg["dt"], 100)
    ref, rst = orc.propagate(prob, psi0, 0.0, cfg["dt"], 100, 16)
    err = hz.rel_l2(mx, ref)
    tol = mixed_tolerance(smx, psi0, rst)
    print(f"mixed rel-L2 vs oracle after 100 steps: {err:.3e} (bound {tol:.3e})", flush=True)
    assert err <= tol and tol <= 1e-6
    assert np.all(smx["k_eff"] == 16)
    assert np.all(smx["round_bound"] > 0)
    # the device's bound of step 1 is the formula on the step's tridiagonal T
    # (here the oracle's T, which differs from the mixed run's by rounding)
    _, _, al, be = orc.lanczos(prob, psi0, 16, dt=cfg["dt"], a_hom=tuple(orc.field_average(prob, 0.0, cfg["dt"])))
    expect = hz.storage_bound(al, be, np.linalg.norm(psi0), 2.0 ** -24,
                              2.0 ** -126 * math.sqrt(4 * prob["nx"] * prob["ny"]))
    # (the later beta_j of the mixed run differ from the oracle's by the amplified
    # storage rounding, so the two bounds agree to a few per mille, not to rounding)
    assert abs(smx["round_bound"][0] - expect) <= 2e-2 * expect, (smx["round_bound"][0], expect)
    _, sfp = gpu_run(torch_cuda, Prop, prob, 16, "fp64", psi0, 0.0, cfg["dt"], 3)
    assert np.all(sfp["round_bound"] == 0.0)


@pytest.mark.parametrize("m,dt_scale", [(24, 1.0), (40, 1.0), (24, 4.0)])
def test_storage_bound_wide_krylov(torch_cuda, Prop, orc, m, dt_scale):
    """The storage bound of one mixed step at Krylov dimensions whose vector
    spans 32 and 64 lanes (the quadrature's node sums over two lane groups or
    one), and over a longer step (a wider Gershgorin interval, more nodes and
    terms), against the formula on the oracle's tridiagonal T (Sec. 4 with the
    perturbed Lanczos relation of the stored vectors)."""
    cfg = packets.with_grid(packets.laser_4096(), 256)
    dt = cfg["dt"] * dt_scale
    prob = dict(cfg["problem"], t_pulse=100 * cfg["dt"])
    say(f"storage bound 256x256 m={m} dt={dt}")
    psi0 = packets.initial_state(cfg)
    _, st = gpu_run(torch_cuda, Prop, prob, m, "mixed", psi0, 0.0, dt, 1)
    assert st["k_eff"][0] == m
    keff, _, al, be = orc.lanczos(prob, psi0, m, dt=dt, a_hom=tuple(orc.field_average(prob, 0.0, dt)))
    assert keff == m
    rad = np.abs(np.r_[be[:m - 1], 0.0]) + np.abs(np.r_[0.0, be[:m - 1]])
    half_width = 0.5 * (np.max(al + rad) - np.min(al - rad))
    expect = hz.storage_bound(al, be, np.linalg.norm(psi0), 2.0 ** -24,
                              2.0 ** -126 * math.sqrt(4 * prob["nx"] * prob["ny"]))
    print(f"R = {half_width:.2f}: device {st['round_bound'][0]:.6e}, formula {expect:.6e}", flush=True)
    assert half_width <= 40.0  # the quadrature branch
    assert abs(st["round_bound"][0] - expect) <= 2e-2 * expect, (st["round_bound"][0], expect)


def test_wide_recombination_ragged(torch_cuda, Prop, orc):
    """A mixed-precision grid above the size where the recombination switches
    to 16 sites per thread (one wide tile per compute unit: 1,048,576 sites
    on 256 CUs), with a partial last tile: two steps against the oracle."""
    cfg = packets.with_grid(packets.laser_4096(), 1100)
    prob = dict(cfg["problem"], ny=997, t_pulse=50 * cfg["dt"])
    assert prob["nx"] * prob["ny"] > 256 * 256 * 16 and (prob["nx"] * prob["ny"]) % 4096 != 0
    say("wide recombination 1100x997 mixed m=16 2 steps")
    psi0 = packets.initial_state(dict(cfg, problem=prob))
    got, st = gpu_run(torch_cuda, Prop, prob, 16, "mixed", psi0, 0.0, cfg["dt"], 2)
    ref, rst = orc.propagate(prob, psi0, 0.0, cfg["dt"], 2, 16)
    err = hz.rel_l2(got, ref)
    tol = mixed_tolerance(st, psi0, rst)
    print(f"1100x997 mixed: rel-L2 {err:.3e} (bound {tol:.3e})", flush=True)
    assert err <= tol
    np.testing.assert_allclose(st["norm2"], rst["norm2"], rtol=2 * tol)


# ---------------------------------------------------------------------------
# Eigenvalue mode
# ---------------------------------------------------------------------------
def test_eigen_landau_vs_oracle(torch_cuda, Prop, orc):
    torch = torch_cuda
    mc2 = C * C
    prob = dict(nx=64, ny=64, x_min=-5.0, x_max=5.0, y_min=-5.0, y_max=5.0, bc_x=0, bc_y=0,
                mass=1.0, c=C, charge=-1.0, bz=2.0, pot_kind=0, pot_z=0.0, pot_a=0.0,
                pulse_kind=0, pulse_e=(0.0, 0.0), a0=0.0, omega=0.0, t_pulse=1.0, coef=None)
    say("eigen Landau 64x64 K=200")
    psi0 = packets.gaussian_packet(prob, 0.9, (0.0, 0.0))
    prop = Prop(prob, 1, "fp64", k_eigen=200)
    ev, bd = prop.eigen(torch.from_numpy(psi0).cuda(), 200, mc2 - 0.5, mc2 + 9.0, 1e-5)
    prop.close()
    rev, rbd, _ = orc.eigen_plain(prob, psi0, 200, mc2 - 0.5, mc2 + 9.0, 1e-5)
    assert len(ev) >= 1 and len(ev) == len(rev)
    assert np.allclose(ev, rev, atol=1e-8)
    # first Landau level of this lattice (h = 10/64) within its O(h^2) error
    lvl = hz.landau_levels(prob, 1)[0]
    assert abs(ev[0] - lvl) < 0.01 * (lvl - mc2)


def test_eigen_landau_softcore_vs_oracle(torch_cuda, Prop, orc):
    """B = 0.5 plus soft-core potential (the 1024^2 workload's physics) on a
    256^2 grid over the same box: the converged Ritz values of the GPU's plain
    recurrence and of the oracle's (both accumulated over the checkpoints
    k = 64, 128, ...) are the same eigenvalues, every one of them."""
    torch = torch_cuda
    mc2 = C * C
    cfg = packets.with_grid(packets.landau_softcore_1024(), 256)
    prob = cfg["problem"]
    say("eigen B+soft-core 256x256 K=600")
    psi0 = packets.initial_state(cfg)
    lo, hi, tol = mc2 - 2.0, mc2 + 5.0, 1e-6
    prop = Prop(prob, 1, "fp64", k_eigen=600)
    ev, bd = prop.eigen(torch.from_numpy(psi0).cuda(), 600, lo, hi, tol)
    prop.close()
    rev, rbd, _ = orc.eigen_plain(prob, psi0, 600, lo, hi, tol)
    print("eigen 256^2 gpu:", np.round(ev - mc2, 9).tolist(), "oracle:", np.round(rev - mc2, 9).tolist(),
          flush=True)
    assert len(rev) >= 2
    assert hz.match_converged(ev, bd, rev, rbd, tol) == len(ev) == len(rev)
    assert np.all(bd <= tol) and np.all(np.diff(ev) > tol)


def _golden_eigen_1024():
    path = os.path.join(os.path.dirname(__file__), "golden", "eigen_landau_softcore_1024.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    return (np.array([float(r[0]) for r in rows]), np.array([float(r[1]) for r in rows]),
            np.array([int(r[2]) for r in rows]))


def test_eigen_full_grid_vs_oracle(torch_cuda, Prop):
    """The full 1024^2 eigen workload (plain Lanczos, K = 2000, window
    E - mc^2 in [-2, 5], tol 1e-6) against the oracle's converged values for
    the same start vector (tests/golden/eigen_landau_softcore_1024.txt, written
    by make_eigen_landau1024.py from the oracle alone, K = 4000, with the
    iteration at which each value first converged).  Which values converge
    near the end of a run depends on the rounding history, so: every GPU value
    with a bound below tol/4 is an oracle value; every oracle value converged
    by k = 1500 is a GPU value; and the eight values of a run that stops once
    eight have converged (the benchmark's call) are oracle values."""
    torch = torch_cuda
    mc2 = C * C
    cfg = packets.landau_softcore_1024()
    prob = cfg["problem"]
    say("eigen B+soft-core 1024x1024 K=2000 vs oracle")
    psi0 = packets.initial_state(cfg)
    lo, hi, tol = mc2 - 2.0, mc2 + 5.0, 1e-6
    gold, gbd, gfirst = _golden_eigen_1024()
    prop = Prop(prob, 1, "fp64", k_eigen=2000)
    x = torch.from_numpy(psi0).cuda()
    ev, bd = prop.eigen(x, 2000, lo, hi, tol, n_wanted=64)
    ev8, bd8 = prop.eigen(x, 2000, lo, hi, tol, n_wanted=8)
    prop.close()
    print("eigen 1024^2 (E - mc^2) gpu:", np.round(ev - mc2, 9).tolist(), flush=True)
    print("               oracle K=4000:", np.round(gold, 9).tolist(), flush=True)
    print("            gpu, stop at 8:", np.round(ev8 - mc2, 9).tolist(), flush=True)

    def partner(v, b, vals, bds):
        i = int(np.argmin(np.abs(vals - v)))
        return abs(vals[i] - v) <= 2.0 * (b + bds[i]) + 1e-8

    for v, b in zip(ev - mc2, bd):
        if b <= 0.25 * tol:
            assert partner(v, b, gold, gbd), ("gpu value not in the oracle set", v, b)
    early = gfirst <= 1500
    assert early.sum() >= 8
    for v, b in zip(gold[early], gbd[early]):
        assert partner(v, b, ev - mc2, bd), ("oracle value converged by k = 1500 missing", v, b)
    assert len(ev8) == 8
    for v, b in zip(ev8 - mc2, bd8):
        assert partner(v, b, gold, gbd), ("stop-at-8 value not in the oracle set", v, b)
    assert np.all(bd <= tol) and np.all(np.diff(ev) > tol)
    assert np.all(ev >= lo) and np.all(ev <= hi)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_chirality_minus_propagation(torch_cuda, Prop, orc, prec):
    """alpha2 = -sigma2 with a magnetic field, a soft core and a y-polarised
    laser: every sigma2 term (y derivative, A_y of both fields) changes sign."""
    prob = dict(box(130, 77, 0, bz=0.8, pot_kind=1, pot_z=1.0, pot_a=1.0), pulse_kind=1, pulse_e=(0.3, 0.95),
                a0=40.0, omega=1.0, t_pulse=0.02, chirality=-1)
    psi0 = packets.gaussian_packet(prob, 0.8, packets.draw_momentum(4, 3.0), project=True)
    say(f"chirality -1 propagation {prec}")
    out, st = gpu_run(torch_cuda, Prop, prob, 12, prec, psi0, 0.0, 1e-3, 20)
    ref, rst = orc.propagate(prob, psi0, 0.0, 1e-3, 20, 12)
    err = hz.rel_l2(out, ref)
    assert err <= (1e-10 if prec == "fp64" else mixed_tolerance(st, psi0, rst)), err
    plus, _ = orc.propagate(dict(prob, chirality=1), psi0, 0.0, 1e-3, 20, 12)
    assert hz.rel_l2(plus, ref) > 1e-3  # the chirality matters for this state
