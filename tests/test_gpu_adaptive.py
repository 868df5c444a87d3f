"""Adaptive time steps on the GPU (the error estimate of each step steering
dt: the Krylov estimate plus the bound of the step-averaged field's
deviation): the accepted step sequence replayed by the oracle, the true error
of static and time-dependent problems against the cumulative estimate, and the
failure paths."""
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


def box(nx, ny, bc, **kw):
    p = dict(nx=nx, ny=ny, x_min=-8.0, x_max=8.0, y_min=-6.0, y_max=6.0, bc_x=bc, bc_y=bc, mass=1.0, c=C,
             charge=-1.0, bz=0.0, pot_kind=0, pot_z=0.0, pot_a=0.0, pulse_kind=0, pulse_e=(0.0, 0.0), a0=0.0,
             omega=0.0, t_pulse=1.0, coef=None)
    p.update(kw)
    return p


def test_adaptive_replay_vs_oracle(torch_cuda, Prop, orc):
    """A laser pulse through the run: the GPU's accepted steps, replayed one by
    one by the oracle at the same times and sizes, give the same state."""
    prob = box(96, 72, 0, bz=0.4, pulse_kind=1, pulse_e=(0.6, 0.8), a0=40.0, omega=1.0, t_pulse=0.03)
    psi0 = packets.gaussian_packet(prob, 0.9, packets.draw_momentum(3, 4.0), project=True)
    say("adaptive replay 96x72")
    prop = Prop(prob, 10, "fp64")
    psi = torch_cuda.from_numpy(psi0).to("cuda")
    tol = 1e-2 * float(np.linalg.norm(psi0))
    st, dts = prop.step_adaptive(psi, 0.0, 0.03, 1e-4, tol, 1e-7, 5e-3)
    prop.close()
    assert st["t_reached"] == 0.03 and st["accepted"] == len(dts) > 1
    assert abs(dts.sum() - 0.03) <= 1e-14
    assert st["cum_bound"] <= tol and st["cum_magnus"] > 0.0
    ref = psi0
    t = 0.0
    for h in dts:
        ref, _ = orc.propagate(prob, ref, t, h, 1, 10)
        t += h
    assert hz.rel_l2(psi.cpu().numpy(), ref) <= 1e-10


def test_adaptive_laser_error_within_estimate(torch_cuda, Prop):
    """A fast laser field: the distance of the adaptive result to a fine
    fixed-step reference (1e-6 steps, whose own field bound is ~1e-2 of the
    adaptive one) stays within the cumulative estimate, whose field part --
    the bound c |q| ||psi|| int |a - a_bar| of the step-averaged field --
    dominates; the Krylov estimates alone would not cover the distance."""
    prob = box(96, 72, 0, bz=0.4, pulse_kind=1, pulse_e=(0.0, 1.0), a0=50.0, omega=1.0, t_pulse=0.02)
    psi0 = packets.gaussian_packet(prob, 0.9, packets.draw_momentum(5, 4.0), project=True)
    say("adaptive laser vs fine reference 96x72")
    nrm = float(np.linalg.norm(psi0))
    prop = Prop(prob, 16, "fp64")
    psi = torch_cuda.from_numpy(psi0).to("cuda")
    tol = 1e-2 * nrm
    st, dts = prop.step_adaptive(psi, 0.0, 0.02, 2e-4, tol, 1e-8, 5e-3)
    ref = torch_cuda.from_numpy(psi0).to("cuda")
    n_ref = 20000
    prop.step(ref, 0.0, 0.02 / n_ref, n_ref, want_stats=False)
    prop.close()
    err = float(np.linalg.norm(psi.cpu().numpy() - ref.cpu().numpy()))
    print(f"adaptive laser: {st['accepted']} steps ({st['rejected']} rejected, h {dts.min():.2e}..{dts.max():.2e}), "
          f"distance {err:.3e}, estimate {st['cum_bound']:.3e} (field part {st['cum_magnus']:.3e})", flush=True)
    assert st["cum_bound"] <= tol
    assert err <= st["cum_bound"], (err, st)
    assert err >= 1e-2 * st["cum_bound"]  # the bound is within two orders of the error
    assert st["cum_magnus"] > 10 * (st["cum_bound"] - st["cum_magnus"])
    assert err > st["cum_bound"] - st["cum_magnus"]


def test_adaptive_static_error_within_bound(torch_cuda, Prop):
    """No time dependence (the Magnus step is exact): the distance to a
    fine-step reference stays within the cumulative error bound."""
    prob = box(80, 64, 0, bz=0.8, pot_kind=1, pot_z=1.0, pot_a=1.0)
    psi0 = packets.gaussian_packet(prob, 0.8, (2.0, -1.0), project=True)
    say("adaptive static bound 80x64")
    prop = Prop(prob, 8, "fp64")
    psi = torch_cuda.from_numpy(psi0).to("cuda")
    tol = 1e-6 * float(np.linalg.norm(psi0))
    st, dts = prop.step_adaptive(psi, 0.0, 0.02, 1e-4, tol, 1e-8, 1e-2)
    ref = torch_cuda.from_numpy(psi0).to("cuda")
    prop2 = Prop(prob, 16, "fp64")
    prop2.step(ref, 0.0, 0.02 / 400, 400, want_stats=False)
    prop.close()
    prop2.close()
    err = float(np.linalg.norm(psi.cpu().numpy() - ref.cpu().numpy()))
    assert st["cum_bound"] <= tol
    assert err <= max(st["cum_bound"], 1e-12 * float(np.linalg.norm(psi0))), (err, st)
    assert st["rejected"] >= 0 and len(dts) == st["accepted"]


def test_adaptive_failure_keeps_state(torch_cuda, Prop):
    from paper_1407_7370_amd.binding import DlError, DL_ERR_INVALID
    prob = box(64, 48, 1)
    psi0 = packets.gaussian_packet(prob, 0.8, (3.0, 0.0), project=True)
    say("adaptive failure paths")
    prop = Prop(prob, 6, "fp64")
    psi = torch_cuda.from_numpy(psi0).to("cuda")
    with pytest.raises(DlError) as e:
        prop.step_adaptive(psi, 0.0, 0.1, 1e-2, 1e-300, 1e-3, 1e-2)
    assert e.value.status == DL_ERR_INVALID
    assert np.array_equal(psi.cpu().numpy(), psi0)  # no step accepted: untouched
    with pytest.raises(DlError) as e:
        prop.step_adaptive(psi, 0.1, 0.0, 1e-3, 1e-6, 1e-6, 1e-2)
    assert e.value.status == DL_ERR_INVALID
    prop.close()
