"""GPU adjoint (gradient of a final observable w.r.t. the Fourier laser
coefficients) through the C ABI, against the oracle.

Gradients must match the oracle's central differences of its own Lanczos
forward map to 1e-6 (max error relative to the largest component); the loss
must match the oracle's loss to 1e-10.  Every case prints its name before
touching the GPU.
"""
import numpy as np
import pytest

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


def fourier_box(nx, ny, bc, lo, hi, n_coef, t_pulse, seed, **kw):
    p = dict(nx=nx, ny=ny, x_min=lo, x_max=hi, y_min=lo, y_max=hi, bc_x=bc, bc_y=bc, mass=1.0, c=C,
             charge=-1.0, bz=0.0, pot_kind=0, pot_z=0.0, pot_a=0.0, pulse_kind=2, pulse_e=(0.0, 0.0),
             a0=0.0, omega=0.0, t_pulse=t_pulse,
             coef=np.random.default_rng(seed).uniform(-20, 20, n_coef))
    p.update(kw)
    return p


def packet(prob, seed, sigma, p_max):
    cfg = {"problem": prob, "sigma": sigma, "p_max": p_max, "center": (0.0, 0.0), "seed": seed}
    return packets.initial_state(cfg)


def gpu_adjoint(torch, Prop, prob, m, psi0, t0, dt, n, ckpt, loss_kind):
    prop = Prop(prob, m, "fp64")
    psi = torch.from_numpy(np.ascontiguousarray(psi0)).to("cuda")
    loss, grad = prop.adjoint(psi, t0, dt, n, ckpt, loss_kind)
    same_input = bool(torch.equal(psi.cpu(), torch.from_numpy(np.ascontiguousarray(psi0))))
    prop.close()
    return loss, grad, same_input


def rel_max(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# grid 88x40 Dirichlet with a field and a soft-core potential: several sweep
# tiles and a ragged last strip; 24 steps, checkpoints every 5 (ragged last
# segment)
SMALL = dict(nx=88, ny=40, bc=0, lo=-10.0, hi=10.0, n_coef=8, t_pulse=0.024, seed=11)


def small_case(**over):
    kw = dict(SMALL)
    kw.update(over)
    prob = fourier_box(kw.pop("nx"), kw.pop("ny"), kw.pop("bc"), kw.pop("lo"), kw.pop("hi"),
                       kw.pop("n_coef"), kw.pop("t_pulse"), kw.pop("seed"), **kw)
    return prob


@pytest.mark.parametrize("loss_kind", [1, 9, 6])
def test_adjoint_vs_oracle_fd(torch_cuda, Prop, orc, loss_kind):
    prob = small_case(bz=0.4, pot_kind=1, pot_z=1.0, pot_a=1.0)
    psi0 = packet(prob, 2, 1.5, 3.0)
    dt, n, m = 1e-3, 24, 12
    say(f"adjoint vs oracle FD 88x40 loss {loss_kind}")
    loss, grad, same = gpu_adjoint(torch_cuda, Prop, prob, m, psi0, 0.0, dt, n, 5, loss_kind)
    assert same, "psi0 must not be modified"
    lo = orc.final_loss(prob, psi0, 0.0, dt, n, m, loss_kind)
    assert abs(loss - lo) <= 1e-10 * max(1.0, abs(lo))
    gf = orc.fd_gradient(prob, psi0, 0.0, dt, n, m, loss_kind, h=0.5)
    assert rel_max(grad, gf) <= 1e-6, (grad, gf)


def test_adjoint_chirality_minus_vs_oracle_fd(torch_cuda, Prop, orc):
    prob = small_case(bz=0.4, chirality=-1)
    psi0 = packet(prob, 12, 1.5, 3.0)
    say("adjoint chirality -1 vs oracle FD 88x40")
    loss, grad, _ = gpu_adjoint(torch_cuda, Prop, prob, 12, psi0, 0.0, 1e-3, 24, 5, 10)
    assert abs(loss - orc.final_loss(prob, psi0, 0.0, 1e-3, 24, 12, 10)) <= 1e-10 * max(1.0, abs(loss))
    gf = orc.fd_gradient(prob, psi0, 0.0, 1e-3, 24, 12, 10, h=0.5)
    assert rel_max(grad, gf) <= 1e-6, (grad, gf)


def test_adjoint_checkpoint_interval_is_bitwise_neutral(torch_cuda, Prop):
    prob = small_case()
    psi0 = packet(prob, 3, 1.5, 3.0)
    say("adjoint checkpoint intervals 1, 5, 24 (88x40)")
    res = [gpu_adjoint(torch_cuda, Prop, prob, 12, psi0, 0.0, 1e-3, 24, ck, 9) for ck in (1, 5, 24, 100)]
    for loss, grad, _ in res[1:]:
        assert loss == res[0][0]
        assert np.array_equal(grad, res[0][1])


def test_adjoint_dense_exact_tiny(torch_cuda, Prop, orc):
    """6x6 grid: the exact (dense exponential) gradient of the oracle."""
    prob = fourier_box(6, 6, 0, -3.0, 3.0, 8, 2e-3, 3, bz=0.3, pot_kind=1, pot_z=1.0, pot_a=1.0)
    rng = np.random.default_rng(3)
    rng.uniform(-20, 20, 8)
    psi0 = rng.standard_normal((2, 6, 6)) + 1j * rng.standard_normal((2, 6, 6))
    say("adjoint vs dense exact gradient 6x6")
    loss, grad, _ = gpu_adjoint(torch_cuda, Prop, prob, 12, psi0, 0.0, 1e-4, 20, 7, 9)
    le, ge = orc.dense_exact_gradient(prob, psi0, 0.0, 1e-4, 20, 9)
    assert abs(loss - le) <= 1e-10 * abs(le)
    assert rel_max(grad, ge) <= 1e-6, (grad, ge)


def test_adjoint_free_momentum_gradient_vanishes(torch_cuda, Prop):
    """Periodic grid, no static field or potential: H commutes with the
    lattice momentum, so <p_x>, <p_y> do not depend on the laser."""
    prob = small_case(bc=1)
    psi0 = packet(prob, 4, 1.5, 3.0)
    say("adjoint free momentum 88x40 periodic")
    _, gx, _ = gpu_adjoint(torch_cuda, Prop, prob, 12, psi0, 0.0, 1e-3, 24, 6, 1)
    _, gp, _ = gpu_adjoint(torch_cuda, Prop, prob, 12, psi0, 0.0, 1e-3, 24, 6, 12)
    assert np.max(np.abs(gp)) <= 1e-8 * np.max(np.abs(gx))


def test_adjoint_autograd_function(torch_cuda, Prop):
    torch = torch_cuda
    from paper_1407_7370_amd.autograd import final_observable
    prob = small_case()
    psi0 = packet(prob, 5, 1.5, 3.0)
    say("adjoint autograd.Function 88x40")
    coef = torch.tensor(prob["coef"], dtype=torch.float64, requires_grad=True)
    psi = torch.from_numpy(psi0).to("cuda")
    loss = final_observable(coef, prob, psi, 0.0, 1e-3, 24, 12, ckpt_every=5, loss_kind=9)
    (2.0 * loss).backward()
    l2, g2, _ = gpu_adjoint(torch, Prop, prob, 12, psi0, 0.0, 1e-3, 24, 5, 9)
    assert float(loss.detach()) == l2
    assert np.array_equal(coef.grad.numpy(), 2.0 * g2)


def test_adjoint_rejections(torch_cuda, Prop):
    from paper_1407_7370_amd.binding import DlError, DL_ERR_UNSUPPORTED, DL_ERR_INVALID
    torch = torch_cuda
    prob = small_case()
    psi = torch.from_numpy(packet(prob, 6, 1.5, 3.0)).to("cuda")
    say("adjoint rejections")
    for m, prec, status in ((12, "mixed", DL_ERR_UNSUPPORTED), (20, "fp64", DL_ERR_UNSUPPORTED)):
        prop = Prop(prob, m, prec)
        with pytest.raises(DlError) as e:
            prop.adjoint(psi, 0.0, 1e-3, 4, 2, 9)
        assert e.value.status == status
        prop.close()
    prop = Prop(prob, 12, "fp64")
    for args in ((0.0, 1e-3, 4, 2, 0), (0.0, 1e-3, 4, 2, 16), (0.0, -1e-3, 4, 2, 1)):
        with pytest.raises(DlError) as e:
            prop.adjoint(psi, *args)
        assert e.value.status == DL_ERR_INVALID
    prop.close()
    laser = dict(prob, pulse_kind=1, pulse_e=(0.0, 1.0), a0=50.0, omega=1.0, t_pulse=0.1, coef=None)
    prop = Prop(laser, 12, "fp64")
    with pytest.raises(DlError) as e:
        prop.adjoint(psi, 0.0, 1e-3, 4, 2, 9)
    assert e.value.status == DL_ERR_UNSUPPORTED
    prop.close()


def test_adjoint_fourier_512_full(torch_cuda, Prop, orc):
    """The 512^2, 2000-step Fourier-pulse workload (checkpoints every 50):
    every gradient component against central differences of the GPU forward
    map, whose loss is evaluated by the oracle on the final state."""
    torch = torch_cuda
    cfg = packets.fourier_pulse_512(seed=0)
    prob, m, dt, n = cfg["problem"], cfg["m"], cfg["dt"], cfg["steps"]
    psi0 = packets.initial_state(cfg)
    say(f"adjoint fourier 512^2 {n} steps")
    loss, grad, _ = gpu_adjoint(torch, Prop, prob, m, psi0, 0.0, dt, n, cfg["ckpt_every"], 9)
    assert np.all(np.isfinite(grad))

    def loss_at(coef):
        p = dict(prob, coef=coef)
        prop = Prop(p, m, "fp64")
        psi = torch.from_numpy(psi0).to("cuda")
        prop.step(psi, 0.0, dt, n, want_stats=False)
        out = orc.loss_value(p, psi.cpu().numpy(), 9)
        prop.close()
        return out

    c0 = np.asarray(prob["coef"], dtype=np.float64)
    assert abs(loss - loss_at(c0)) <= 1e-10 * max(1.0, abs(loss))
    for j in range(len(c0)):
        # over 2000 steps the loss is far from quadratic at h ~ 0.5; central
        # differences enter their O(h^2) regime below h ~ 0.1
        h = 0.0625

        def central(step):
            cp, cm = c0.copy(), c0.copy()
            cp[j] += step
            cm[j] -= step
            return (loss_at(cp) - loss_at(cm)) / (2 * step)

        fd = (4.0 * central(h / 2) - central(h)) / 3.0
        say(f"  coef {j}: adjoint {grad[j]:.10e} fd {fd:.10e}")
        assert abs(grad[j] - fd) <= 1e-6 * np.max(np.abs(grad))
