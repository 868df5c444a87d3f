"""Adaptive Krylov dimension (dirac_lanczos_step_ktol) through the C ABI.

Each step's result must be the oracle's step of the dimension the GPU chose
(replayed step by step, FP64 <= 1e-10); the chosen dimensions must stay in
[k_min, m] and keep the per-step estimate near the tolerance.
"""
import numpy as np
import pytest

import harness as hz
from paper_1407_7370_amd import packets

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def say(msg):
    print(f"[gpu case] {msg}", flush=True)


def laser(n):
    cfg = packets.with_grid(packets.laser_4096(), n)
    return cfg, dict(cfg["problem"], t_pulse=200 * cfg["dt"])


@pytest.mark.parametrize("ktol", [1e-8, 1e-12])
def test_ktol_replayed_by_oracle(torch_cuda, orc, ktol):
    from paper_1407_7370_amd.binding import Propagator
    torch = torch_cuda
    cfg, prob = laser(192)
    dt, m, n = cfg["dt"], 16, 60
    psi0 = packets.initial_state(cfg)
    say(f"adaptive k laser 192x192 ktol={ktol} {n} steps")
    prop = Propagator(prob, m, "fp64")
    psi = torch.from_numpy(psi0).cuda()
    st = prop.step(psi, 0.0, dt, n, ktol=ktol, k_min=3)
    # a plain call afterwards is back to the fixed dimension
    chk = torch.from_numpy(psi0).cuda()
    st2 = prop.step(chk, 0.0, dt, 2)
    prop.close()
    k = st["k_eff"]
    print(f"ktol={ktol}: k per step {k.tolist()}", flush=True)
    print(f"  estimates max {st['err_est'].max():.2e}, after the first step max "
          f"{st['err_est'][1:].max():.2e}", flush=True)
    assert k[0] == m and np.all(k >= 3) and np.all(k <= m)
    assert k[1:].mean() < m
    assert np.all(st2["k_eff"] == m)
    # the estimate stays within the tolerance except where k had to grow
    over = np.nonzero(st["err_est"] > ktol)[0]
    assert len(over) <= max(2, n // 10), over
    for i in over:
        if i + 1 < n:
            assert k[i + 1] > k[i] or k[i + 1] == m
    # replay: the oracle's step of the chosen dimension, step by step
    ref = psi0.copy()
    for i in range(n):
        ref, _ = orc.propagate(prob, ref, i * dt, dt, 1, int(k[i]))
    assert hz.rel_l2(psi.cpu().numpy(), ref) <= 1e-10


def test_ktol_limits(torch_cuda):
    from paper_1407_7370_amd import binding
    from paper_1407_7370_amd.binding import Propagator
    torch = torch_cuda
    cfg, prob = laser(96)
    dt = cfg["dt"]
    psi0 = packets.initial_state(cfg)
    say("adaptive k limits 96x96")
    prop = Propagator(prob, 12, "mixed")
    # a tolerance no step can meet keeps the full dimension
    a = torch.from_numpy(psi0).cuda()
    st = prop.step(a, 0.0, dt, 8, ktol=1e-300, k_min=2)
    assert np.all(st["k_eff"] == 12)
    # a loose one drops to k_min
    b = torch.from_numpy(psi0).cuda()
    st = prop.step(b, 0.0, dt, 8, ktol=1e3, k_min=2)
    assert st["k_eff"][0] == 12 and np.all(st["k_eff"][1:] == 2)
    for bad_tol, bad_k in ((0.0, 2), (float("nan"), 2), (1e-8, 0), (1e-8, 13)):
        with pytest.raises(binding.DlError) as ei:
            binding.load_library()
            st = prop.lib.dirac_lanczos_step_ktol(prop.ctx, a.data_ptr(), 0.0, dt, 2, bad_tol, bad_k, None)
            binding._check(prop.lib, prop.ctx, st)
        assert ei.value.status == binding.DL_ERR_INVALID
    prop.close()


def test_ktol_full_grid_mixed(torch_cuda):
    """The 4096^2 laser workload (mixed): with a per-step bound of 1e-12 the
    dimension drops well below 16 and the state stays within the summed
    estimates of the fixed-dimension result."""
    from paper_1407_7370_amd.binding import Propagator
    import time
    torch = torch_cuda
    cfg = packets.laser_4096(precision="mixed")
    prob, dt = cfg["problem"], cfg["dt"]
    psi0 = torch.from_numpy(packets.initial_state(cfg)).cuda()
    n = 100
    say(f"adaptive k laser 4096x4096 mixed {n} steps")
    prop = Propagator(prob, 16, "mixed", tuning_cache=True)
    fixed = psi0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prop.step(fixed, 0.0, dt, n, want_stats=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ad = psi0.clone()
    st = prop.step(ad, 0.0, dt, n, ktol=1e-12, k_min=4)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    prop.close()
    k = st["k_eff"]
    diff = float(torch.linalg.vector_norm(ad - fixed) / torch.linalg.vector_norm(fixed))
    print(f"4096^2: fixed m=16 {1e3 * (t1 - t0) / n:.3f} ms/step, adaptive {1e3 * (t2 - t1) / n:.3f} ms/step, "
          f"mean k {k.mean():.2f} (min {k.min()}), rel-L2 vs fixed {diff:.2e}, sum of estimates "
          f"{st['err_est'].sum():.2e}", flush=True)
    assert k[1:].max() < 16
    # the mixed-precision rounding of both runs (~1e-10) dominates the Krylov error
    assert diff <= 1e-8
