"""Asynchronous steps (stats == NULL): the call only enqueues work on the
caller's stream; dirac_lanczos_wait synchronises and reports.  Results are
bit for bit those of the synchronous call (the same kernels in the same
order); a device-side failure is reported by wait or by the next synchronous
call."""
import numpy as np
import pytest

from paper_1407_7370_amd import packets

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu case] {msg}", flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def test_async_step_returns_with_work_pending_4096(torch_cuda):
    from paper_1407_7370_amd.binding import Propagator
    torch = torch_cuda
    cfg = packets.laser_4096(precision="mixed")
    psi0 = packets.initial_state(cfg)
    n = 20
    say(f"async step laser 4096x4096 mixed {n} steps")
    prop = Propagator(cfg["problem"], cfg["m"], "mixed", tuning_cache=True)
    ref = torch.from_numpy(psi0).to("cuda")
    st_sync = prop.step(ref, 0.0, cfg["dt"], n)
    psi = torch.from_numpy(psi0).to("cuda")
    torch.cuda.synchronize()
    prop.step_async(psi, 0.0, cfg["dt"], n)
    ev = torch.cuda.Event()
    ev.record(torch.cuda.current_stream())
    pending = not ev.query()
    st = prop.wait(want_stats=True)
    assert ev.query()
    print(f"work pending after the asynchronous call returned: {pending}", flush=True)
    assert pending, "the asynchronous call waited for the stream"
    assert torch.equal(psi, ref)
    for key in ("k_eff", "err_est", "cum_bound", "norm2", "round_bound"):
        assert np.array_equal(st[key], st_sync[key]), key
    prop.close()


@pytest.mark.parametrize("split", [(7, 13), (1, 1, 1), (5,)])
def test_async_chained_calls_equal_sync(torch_cuda, split):
    """Several asynchronous calls in a row (odd and even step counts, the
    state ends in psi each time) equal one synchronous call bit for bit."""
    from paper_1407_7370_amd.binding import Propagator
    torch = torch_cuda
    cfg = packets.with_grid(packets.landau_softcore_1024(), 200)
    prob = cfg["problem"]
    psi0 = packets.initial_state(cfg)
    total = sum(split)
    say(f"async chained {split} 200x200 fp64")
    prop = Propagator(prob, 12, "fp64")
    ref = torch.from_numpy(psi0).cuda()
    prop.step(ref, 0.0, 5e-4, total)
    psi = torch.from_numpy(psi0).cuda()
    t = 0.0
    for k in split:
        prop.step_async(psi, t, 5e-4, k)
        t += k * 5e-4
    prop.wait()
    assert torch.equal(psi, ref)
    # lowmem and adaptive-k variants take the same asynchronous path
    for kw in (dict(lowmem=True), dict(ktol=1e-12, k_min=4)):
        a = torch.from_numpy(psi0).cuda()
        b = torch.from_numpy(psi0).cuda()
        prop.step(a, 0.0, 5e-4, 3, **kw)
        prop.step_async(b, 0.0, 5e-4, 3, **kw)
        prop.wait()
        assert torch.equal(a, b), kw
    prop.close()


def test_async_failure_reported(torch_cuda):
    from paper_1407_7370_amd import binding
    from paper_1407_7370_amd.binding import Propagator
    torch = torch_cuda
    prob = dict(nx=40, ny=40, x_min=-6.0, x_max=6.0, y_min=-5.4, y_max=7.2, bc_x=0, bc_y=0, mass=1.0, c=137.036,
                charge=-1.0, bz=0.0, pot_kind=0, pot_z=0.0, pot_a=0.0, pulse_kind=0, pulse_e=(0.0, 0.0), a0=0.0,
                omega=0.0, t_pulse=1.0, coef=None)
    say("async non-finite input 40x40")
    good = packets.gaussian_packet(prob, 1.0, (0.0, 0.0))
    bad = good.copy()
    bad[1, 20, 20] = np.nan
    prop = Propagator(prob, 8, "fp64")
    psi = torch.from_numpy(bad).cuda()
    prop.step_async(psi, 0.0, 1e-3, 3)
    with pytest.raises(binding.DlError) as ei:
        prop.wait()
    assert ei.value.status == binding.DL_ERR_NONFINITE
    back = psi.cpu().numpy()
    assert np.array_equal(np.isnan(back), np.isnan(bad))
    # a failure not collected by wait is reported by the next synchronous call,
    # and the context works again afterwards
    prop.step_async(psi, 0.0, 1e-3, 2)
    with pytest.raises(binding.DlError) as ei:
        prop.step(torch.from_numpy(good).cuda(), 0.0, 1e-3, 2)
    assert ei.value.status == binding.DL_ERR_NONFINITE
    ok = torch.from_numpy(good).cuda()
    st = prop.step(ok, 0.0, 1e-3, 2)
    assert np.all(st["k_eff"] == 8)
    prop.close()
