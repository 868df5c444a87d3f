"""The library's event timing (dirac_lanczos_timing) behind the bench's
roofline: launches counted per kernel class (iterations 4..m timed as one
block of m - 3 launches), and timing leaves the result bit for bit unchanged."""
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


@pytest.mark.parametrize("m", [3, 4, 9])
def test_timing_counts_and_neutrality(torch_cuda, m):
    from paper_1407_7370_amd.binding import Propagator
    torch = torch_cuda
    cfg = packets.with_grid(packets.laser_4096(precision="mixed"), 96)
    psi0 = torch.from_numpy(packets.initial_state(cfg)).to("cuda")
    steps = 3
    say(f"event timing 96x96 mixed m={m} {steps} steps")
    prop = Propagator(cfg["problem"], m, "mixed")
    plain = psi0.clone()
    prop.step(plain, 0.0, cfg["dt"], steps, want_stats=False)
    timed = psi0.clone()
    prop.timing(True)
    prop.step(timed, 0.0, cfg["dt"], steps, want_stats=False)
    t = prop.timing(False)
    prop.close()
    assert torch.equal(plain, timed)
    expect = {"first": steps, "recur_basis": steps * max(m - 3, 0), "recur_psi": steps * (min(m, 3) - 1),
              "tridiag": steps, "recombine": steps}
    for cls, n in expect.items():
        launches, ms = t[cls]
        assert launches == n, (cls, launches, n)
        assert (ms > 0.0) == (n > 0), (cls, ms)
