#!/usr/bin/env python3
"""Benchmark: Lanczos short-time propagator of the 2D Dirac equation on one MI355X.

Workload (the metric's configuration): 4096 x 4096 Dirichlet grid over
[-40, 40)^2, laser vector potential A(t) = 50 sin(t) sin^2(pi t/T) y-hat with
T = 500 dt = 0.1, Krylov dimension m = 16, dt = 2e-4, seeded positive-energy
Gaussian packet (sigma = 3).  A "step" is one full short-time step
psi <- exp(-i dt H) psi: m Lanczos sweeps, the tridiagonal exponential and the
recombination.  The mixed form (complex64 Krylov vectors, FP64 arithmetic,
state and reductions) is the headline value; the FP64 form runs the same
steps from the same state and the relative L2 difference of the two final
states is reported.

  python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints ONE JSON line.  site-matvecs/s = nx * ny * m * K / wall time of the K
timed steps (inputs resident in HBM, torch.cuda.synchronize on both sides).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "site-matvecs/s and % HBM peak, mixed vs FP64 propagator at ≤1e-6 err"
# sources of the sweep kernels: the HBM traffic counters are valid for these only
KERNEL_SRCS = [os.path.join(ROOT, "paper_1407_7370_amd", "csrc", f)
               for f in ("kernels.hip", "sweeps.h", "device_reduce.h", "dl_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_recur_laser4096.json")


def cpu_model():
    """The host CPU's model name (Linux), for the CPU baseline."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_digest():
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def load_traffic(precision):
    """HBM bytes per launch of the dominant kernel from committed rocprofv3
    counter runs, valid only while the kernel sources are unchanged."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernels_sha256") != kernel_digest():
        return None
    v = rec.get(precision, {}).get("bytes_per_launch")
    return float(v) if v else None


def run_precision(torch, Propagator, cfg, psi0_dev, precision, steps, warmup, copy_mib):
    """Warm up, then two timed regions of `steps` steps from the same state:
    a clean one (the reported rate) and one with per-launch HIP events recorded
    by the library on its stream (kernel durations for the roofline)."""
    prop_args = (cfg["problem"], cfg["m"], precision)
    dt = cfg["dt"]
    prop = Propagator(*prop_args, tuning_cache=True)
    psi = psi0_dev.clone()
    if warmup > 0:
        prop.step(psi, 0.0, dt, warmup, want_stats=False)
    if copy_mib:
        # kernels of known traffic that calibrate the HBM byte counters: a fill
        # (writes copy_mib MiB) and a negation (reads and writes copy_mib MiB)
        a = torch.empty(copy_mib << 17, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.neg(a, out=b)
        torch.cuda.synchronize()
        del a, b
    psi.copy_(psi0_dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = prop.step(psi, 0.0, dt, steps, want_stats=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # instrumented region (same work, same state)
    psi2 = psi0_dev.clone()
    prop.timing(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prop.step(psi2, 0.0, dt, steps, want_stats=False)
    torch.cuda.synchronize()
    wall_ev = time.perf_counter() - t1
    timing = prop.timing(False)
    prop.close()
    same = bool(torch.equal(psi, psi2))
    del psi2
    return psi, stats, wall, timing, wall_ev, same


def run_mixed_accuracy(torch, Propagator, cfg, psi0_dev):
    """The workload's full length (cfg["steps"] = 500 steps) in mixed precision
    and in FP64 from the same state: the relative L2 distance of the final
    states beside the a-priori bound the mixed run reports (the summed
    per-step storage bounds plus both runs' Krylov estimates, relative to
    ||psi_0||).  Runs whatever --steps is."""
    n = cfg["steps"]
    out = {}
    psis = {}
    for prec in ("mixed", "fp64"):
        prop = Propagator(cfg["problem"], cfg["m"], prec, tuning_cache=True)
        psi = psi0_dev.clone()
        st = prop.step(psi, 0.0, cfg["dt"], n)
        prop.close()
        psis[prec] = psi
        out[prec] = st
    nrm0 = float(torch.linalg.vector_norm(psi0_dev))
    err = float(torch.linalg.vector_norm(psis["mixed"] - psis["fp64"]) / torch.linalg.vector_norm(psis["fp64"]))
    storage = float(out["mixed"]["cum_round_bound"][-1]) / nrm0
    krylov = float(out["mixed"]["cum_bound"][-1] + out["fp64"]["cum_bound"][-1]) / nrm0
    del psis
    log(f"mixed vs fp64 over {n} steps: rel-L2 {err:.3e}, bound {storage + krylov:.3e}")
    return {"steps": n, "rel_l2": err, "bound": storage + krylov, "storage_bound": storage,
            "krylov_estimates": krylov, "within_bound": err <= storage + krylov + 1e-10}


def run_lowmem(torch, Propagator, cfg, psi0_dev, steps):
    """The memory-saving step (second Lanczos run, three rolling Krylov
    vectors) on the same workload and precision as the headline, against the
    stored-basis step over the same steps."""
    from paper_1407_7370_amd.binding import dirac_lanczos_workspace_bytes, DL_MODE_LOWMEM, DL_MODE_STEP
    prob, m, dt = cfg["problem"], cfg["m"], cfg["dt"]
    sites = prob["nx"] * prob["ny"]
    prop = Propagator(prob, m, "mixed", tuning_cache=True)
    ws_low = dirac_lanczos_workspace_bytes(prop.params, DL_MODE_LOWMEM, 0)
    ws_full = dirac_lanczos_workspace_bytes(prop.params, DL_MODE_STEP, 0)
    ref = psi0_dev.clone()
    prop.step(ref, 0.0, dt, steps, want_stats=False)
    psi = psi0_dev.clone()
    prop.step(psi, 0.0, dt, 1, want_stats=False, lowmem=True)
    psi.copy_(psi0_dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prop.step(psi, 0.0, dt, steps, want_stats=False, lowmem=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prop.close()
    err = float(torch.linalg.vector_norm(psi - ref) / torch.linalg.vector_norm(ref))
    log(f"lowmem: {wall * 1e3 / steps:.3f} ms/step, workspace {ws_low / 2**30:.2f} GiB vs "
        f"{ws_full / 2**30:.2f} GiB stored basis, rel-L2 vs stored basis {err:.1e}")
    return {"what": "second Lanczos run instead of the stored basis (mixed, same workload)", "steps": steps,
            "ms_per_step": wall * 1e3 / steps, "value": sites * m * steps / wall, "unit": "site-matvecs/s",
            "workspace_bytes": ws_low, "stored_basis_workspace_bytes": ws_full,
            "rel_l2_vs_stored_basis": err}


def run_adaptive_dt(torch, Propagator, cfg, psi0_dev, n_fixed=50):
    """Adaptive time steps on the grid and packet of the workload in FP64 over
    the interval of n_fixed steps of the fixed dt, with step sizes chosen from
    each step's error estimate, against a reference over the same interval.
    Field off: the step is exact up to the Lanczos error; estimate
    1e-10 ||psi||, reference n_fixed fixed steps.  Laser on: the estimate also
    bounds the replacement of the field by its step average (first Magnus
    term); estimate 1e-3 ||psi||, reference 8 n_fixed fixed steps (its own
    field bound is 8x smaller than that of the fixed dt).  Both report the
    distance to the reference beside the cumulative estimate, and the time
    against n_fixed fixed steps."""
    m, dt = cfg["m"], cfg["dt"]
    t_end = n_fixed * dt
    nrm = float(torch.linalg.vector_norm(psi0_dev))
    out = {"what": f"adaptive step sizes over t in [0, {t_end:g}] (FP64, m={m}) against {n_fixed} fixed steps "
                   f"of {dt:g}; the distance to a reference beside the cumulative estimate"}
    cases = (("field_off", dict(cfg["problem"], pulse_kind=0), 1e-10, n_fixed),
             ("laser", cfg["problem"], 1e-3, 8 * n_fixed))
    for name, prob, rel_tol, n_ref in cases:
        tol = rel_tol * nrm
        sites = prob["nx"] * prob["ny"]
        prop = Propagator(prob, m, "fp64", tuning_cache=True)
        fixed = psi0_dev.clone()
        prop.step(fixed, 0.0, dt, 2, want_stats=False)
        fixed.copy_(psi0_dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prop.step(fixed, 0.0, dt, n_fixed, want_stats=False)
        torch.cuda.synchronize()
        wall_fixed = time.perf_counter() - t0
        if n_ref == n_fixed:
            ref = fixed
        else:
            ref = psi0_dev.clone()
            prop.step(ref, 0.0, t_end / n_ref, n_ref, want_stats=False)
        psi = psi0_dev.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, dts = prop.step_adaptive(psi, 0.0, t_end, dt, tol, 1e-3 * dt, 100 * dt)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prop.close()
        dist = float(torch.linalg.vector_norm(psi - ref))
        dist_fixed = float(torch.linalg.vector_norm(psi - fixed))
        log(f"adaptive dt ({name}): {st['accepted']} accepted, {st['rejected']} rejected, {wall * 1e3:.1f} ms vs "
            f"{wall_fixed * 1e3:.1f} ms for {n_fixed} fixed steps, |psi - psi_ref| {dist:.1e} (estimate "
            f"{st['cum_bound']:.1e}, field part {st['cum_magnus']:.1e})")
        out[name] = {"tol_rel": rel_tol, "accepted": st["accepted"], "rejected": st["rejected"], "seconds": wall,
                     "fixed_seconds": wall_fixed, "speedup_vs_fixed": wall_fixed / wall,
                     "dt_min": float(dts.min()), "dt_max": float(dts.max()), "cum_bound": st["cum_bound"],
                     "cum_magnus": st["cum_magnus"], "reference_steps": n_ref, "dist_to_reference": dist,
                     "within_estimate": dist <= st["cum_bound"], "dist_to_fixed": dist_fixed,
                     "matvecs_per_s": float(sites * m * (st["accepted"] + st["rejected"]) / wall)}
        del psi, ref, fixed
    return out


def run_chirality(torch, Propagator, cfg, psi0_dev, steps=50):
    """The workload with the other 2D representation (alpha2 = -sigma2,
    chirality -1), mixed: the same kernels with the sign of every sigma2 term
    flipped, so the rate must match chirality +1."""
    prob, m, dt = dict(cfg["problem"], chirality=-1), cfg["m"], cfg["dt"]
    sites = prob["nx"] * prob["ny"]
    prop = Propagator(prob, m, "mixed", tuning_cache=True)
    psi = psi0_dev.clone()
    prop.step(psi, 0.0, dt, 2, want_stats=False)
    psi.copy_(psi0_dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = prop.step(psi, 0.0, dt, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prop.close()
    n0 = float(torch.linalg.vector_norm(psi0_dev)) ** 2
    log(f"chirality -1: {wall * 1e3 / steps:.3f} ms/step")
    return {"what": "chirality -1 (alpha2 = -sigma2), mixed, same workload", "steps": steps,
            "ms_per_step": wall * 1e3 / steps, "value": sites * m * steps / wall, "unit": "site-matvecs/s",
            "norm_drift": abs(float(st["norm2"][-1]) / n0 - 1.0)}


def run_paper_shape(torch, Propagator, packets, steps=10):
    """The paper's own benchmark shape (Sec. 7): 8192^2 periodic grid, FP64,
    k = 10, dt = 1e-7, a free packet of mean momentum (100, 0); the paper
    quotes about two minutes per step for it on one CPU core."""
    cfg = packets.paper_packet_8192(seed=0)
    prob, m, dt = cfg["problem"], cfg["m"], cfg["dt"]
    sites = prob["nx"] * prob["ny"]
    psi0 = torch.from_numpy(packets.initial_state(cfg)).to("cuda")
    prop = Propagator(prob, m, "fp64", tuning_cache=True)
    psi = psi0.clone()
    prop.step(psi, 0.0, dt, 1, want_stats=False)
    psi.copy_(psi0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = prop.step(psi, 0.0, dt, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prop.close()
    n0 = float(torch.linalg.vector_norm(psi0)) ** 2
    del psi, psi0
    ms = wall * 1e3 / steps
    log(f"paper shape 8192^2 FP64 k={m}: {ms:.2f} ms/step")
    return {"workload": cfg["name"] + f" (k={m}, dt={dt:g}, {steps} steps)", "ms_per_step": ms,
            "value": sites * m * steps / wall, "unit": "site-matvecs/s",
            # algorithmic bytes of an FP64 step: (4 m - 2) complex128 vectors per site
            "hbm_frac_step": round(sites * 32 * (4 * m - 2) * steps / wall / 1e9 / HBM_PEAK_GBS, 4),
            "norm_drift": abs(float(st["norm2"][-1]) / n0 - 1.0),
            "paper_seconds_per_step": 120.0, "ratio_vs_paper_one_core": 120.0 / (ms / 1e3)}


def run_ktol(torch, Propagator, cfg, psi0_dev, steps, ktol=1e-12, k_min=4):
    """Adaptive Krylov dimension on the same workload (mixed): the per-step
    estimate bounded by ktol, k in [k_min, 16], against the fixed m = 16."""
    prob, m, dt = cfg["problem"], cfg["m"], cfg["dt"]
    sites = prob["nx"] * prob["ny"]
    prop = Propagator(prob, m, "mixed", tuning_cache=True)
    ref = psi0_dev.clone()
    prop.step(ref, 0.0, dt, steps, want_stats=False)
    psi = psi0_dev.clone()
    prop.step(psi, 0.0, dt, 2, want_stats=False, ktol=ktol, k_min=k_min)
    psi.copy_(psi0_dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = prop.step(psi, 0.0, dt, steps, ktol=ktol, k_min=k_min)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prop.close()
    err = float(torch.linalg.vector_norm(psi - ref) / torch.linalg.vector_norm(ref))
    k = st["k_eff"]
    log(f"adaptive k (tol {ktol:g} per step): {wall * 1e3 / steps:.3f} ms/step, mean k {k.mean():.2f}, "
        f"rel-L2 vs m={m} {err:.1e}")
    return {"what": f"adaptive Krylov dimension in [{k_min}, {m}], per-step estimate <= {ktol:g} (mixed)",
            "steps": steps, "ms_per_step": wall * 1e3 / steps, "mean_k": float(k.mean()), "min_k": int(k.min()),
            # algorithmic bytes of a mixed step of dimension k: (64 k + 48) per site
            "hbm_frac_step": round(float(sites * (64 * k + 48).sum()) / wall / 1e9 / HBM_PEAK_GBS, 4),
            "matvecs_per_s": float(sites * k.sum() / wall), "sum_err_est": float(st["err_est"].sum()),
            "rel_l2_vs_fixed_m": err}


def run_adjoint(torch, Propagator, packets):
    """Gradient of <x> + <p_y> after the 2000-step 512^2 Fourier-pulse workload
    with respect to its 16 laser coefficients (checkpoints every 50 steps),
    against one forward propagation of the same workload."""
    cfg = packets.fourier_pulse_512(seed=0)
    prob, m, dt, n = cfg["problem"], cfg["m"], cfg["dt"], cfg["steps"]
    psi0 = torch.from_numpy(packets.initial_state(cfg)).to("cuda")
    prop = Propagator(prob, m, "fp64", tuning_cache=True)
    psi = psi0.clone()
    prop.step(psi, 0.0, dt, 10, want_stats=False)
    psi.copy_(psi0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prop.step(psi, 0.0, dt, n, want_stats=False)
    torch.cuda.synchronize()
    fwd = time.perf_counter() - t0
    t1 = time.perf_counter()
    loss, grad = prop.adjoint(psi0, 0.0, dt, n, cfg["ckpt_every"], 9)
    torch.cuda.synchronize()
    adj = time.perf_counter() - t1
    prop.close()
    ncoef = len(grad)
    log(f"adjoint 512^2 x {n} steps: forward {fwd:.3f} s, loss + gradient ({ncoef} coefficients) {adj:.3f} s")
    return {"workload": cfg["name"] + f" ({n} steps, m={m}, checkpoints every {cfg['ckpt_every']})",
            "forward_s": fwd, "adjoint_s": adj, "adjoint_over_forward": adj / fwd, "coefficients": ncoef,
            "central_differences_s": 2 * ncoef * fwd, "speedup_vs_central_differences": 2 * ncoef * fwd / adj}


def run_eigen(torch, Propagator, packets):
    """Eigen mode on the 1024^2 B + soft-core workload: plain Lanczos up to
    2000 iterations stopping at 8 converged values in E - mc^2 in [-2, 5], and
    500 iterations with full reorthogonalisation (sustained CGS2 bandwidth)."""
    cfg = packets.landau_softcore_1024(seed=0)
    prob = cfg["problem"]
    mc2 = prob["c"] ** 2 * prob["mass"]
    psi0 = torch.from_numpy(packets.initial_state(cfg)).to("cuda")
    out = {"workload": cfg["name"], "window": "E - mc^2 in [-2, 5]", "tol": 1e-6}
    pr = Propagator(prob, 1, "fp64", k_eigen=2000)
    pr.eigen(psi0, 64, mc2 - 2.0, mc2 + 5.0, 1e-6, n_wanted=8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev, bd = pr.eigen(psi0, 2000, mc2 - 2.0, mc2 + 5.0, 1e-6, n_wanted=8)
    wall = time.perf_counter() - t0
    pr.close()
    out["plain"] = {"k_max": 2000, "n_wanted": 8, "found": len(ev), "seconds": wall,
                    "values_minus_mc2": [round(float(e - mc2), 9) for e in ev]}
    K = 500
    pr = Propagator(prob, 1, "fp64", k_eigen=K, reorth=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev, bd = pr.eigen(psi0, K, mc2 - 2.0, mc2 + 5.0, 1e-6, n_wanted=64, reorth=True)
    wall = time.perf_counter() - t0
    pr.close()
    nel = psi0.numel()
    byt = sum(2 * (2 * i + 3) * 16 * nel for i in range(1, K + 1))
    out["full_reorthogonalisation"] = {"k": K, "found": len(ev), "seconds": wall,
                                       "cgs2_bytes": byt, "cgs2_GBps": byt / wall / 1e9,
                                       "values_minus_mc2": [round(float(e - mc2), 9) for e in ev]}
    log(f"eigen 1024^2: plain {out['plain']['seconds']:.2f} s ({out['plain']['found']} values), reorth K={K} "
        f"{wall:.2f} s, {byt / wall / 1e9:.0f} GB/s")
    return out


def run_hermite(torch, packets, k=1000):
    """Hermite pseudospectral eigenvalue mode (64 x 64 collocation points,
    k Lanczos iterations per problem, one workgroup per problem in one
    launch): the six problems of the paper's ground-state table, the Z = 50
    excited-state table, and a 256-problem scan of the soft-core ground state
    over Z = 1 .. 50 (one problem per compute unit).  The matrix
    products, 16 n^3 FP64 flops per H application, run on the matrix cores."""
    from paper_1407_7370_amd import binding
    mc2 = 137.036 ** 2
    out = {"what": f"Hermite pseudospectral eigen mode, n = 64, {k} Lanczos iterations per problem"}
    flops_mv = 16 * 64 ** 3

    def run(probs, lo, hi, tol, nw):
        starts = [torch.from_numpy(packets.hermite_packet(h, 1.0 / h["pot_z"], (0.4 / h["pot_z"], 0.25 / h["pot_z"])))
                  .cuda() for h in probs]
        binding.hermite_eigen(probs[:1], starts[:1], 16, lo[:1], hi[:1], tol, nw)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = binding.hermite_eigen(probs, starts, k, lo, hi, tol, nw)
        torch.cuda.synchronize()
        return res, time.perf_counter() - t0

    zs = [1.0, 2.0, 3.0, 5.0, 10.0, 50.0]
    probs = [packets.softcore_hermite(z) for z in zs]
    res, sec = run(probs, [mc2 - 0.6 * z * z for z in zs], [mc2 - 0.4 * z * z for z in zs], 2.5e-6, 4)
    out["ground_state_table"] = {"problems": len(zs), "seconds": sec,
                                 "values_minus_mc2": {str(z): round(float(r[0][0] - mc2), 10) for z, r in zip(zs, res)},
                                 "tflops": len(zs) * k * flops_mv / sec / 1e12}
    hp = packets.softcore_hermite(50.0)
    res, sec = run([hp], [mc2 - 1500.0], [mc2 - 350.0], 1e-5, 9)
    out["z50_states"] = {"seconds": sec, "values_minus_mc2": [round(float(v - mc2), 6) for v in res[0][0]]}
    zscan = [1.0 + 49.0 * i / 255 for i in range(256)]
    scan = [packets.softcore_hermite(z) for z in zscan]
    res, sec = run(scan, [mc2 - 0.6 * z * z for z in zscan], [mc2 - 0.4 * z * z for z in zscan], 2.5e-6, 1)
    achieved = 256 * k * flops_mv / sec / 1e12
    # the same launch with a window below the spectrum: the host's Ritz step
    # finds nothing at once, so this is the device recurrence and the copies
    _, sec_dev = run(scan, [-2.0] * 256, [-1.0] * 256, 2.5e-6, 1)
    dev = 256 * k * flops_mv / sec_dev / 1e12
    out["z_scan_256"] = {"problems": 256, "Z": "1 .. 50", "seconds": sec, "tflops": achieved,
                         "frac_of_fp64_matrix_peak": achieved / 78.6,
                         "device_seconds": sec_dev, "device_tflops": dev,
                         "device_frac_of_fp64_matrix_peak": dev / 78.6,
                         "converged": int(sum(len(r[0]) > 0 for r in res)),
                         "ground_state_Z1_Z50": [round(float(res[0][0][0] - mc2), 9) if len(res[0][0]) else None,
                                                 round(float(res[-1][0][0] - mc2), 6) if len(res[-1][0]) else None]}
    log(f"hermite: table of 6 in {out['ground_state_table']['seconds'] * 1e3:.1f} ms, Z=50 in "
        f"{out['z50_states']['seconds'] * 1e3:.1f} ms, 256-problem Z scan in {sec * 1e3:.1f} ms "
        f"({achieved:.2f} TFLOP/s FP64 matrix; recurrence alone {sec_dev * 1e3:.1f} ms, {dev:.1f} TFLOP/s)")
    return out


def run_batch(torch, packets, steps):
    """The 256-packet batch (grids 128^2..512^2, B_z ~ U[0,2], mixed, m = 12):
    one batched step call vs the same packets propagated one context at a
    time (a few steps each, rate extrapolated)."""
    from paper_1407_7370_amd.binding import BatchPropagator, Propagator
    cfgs = packets.packet_batch(seed=0)
    probs = [c["problem"] for c in cfgs]
    m, dt = cfgs[0]["m"], cfgs[0]["dt"]
    sites = sum(p["nx"] * p["ny"] for p in probs)
    psi0 = [torch.from_numpy(packets.initial_state(c)).to("cuda") for c in cfgs]
    log(f"batch: {len(probs)} packets, {sites / 1e6:.1f}M sites, m={m}, {steps} steps")
    bp = BatchPropagator(probs, m, "mixed", tuning_cache=True)
    psis = [x.clone() for x in psi0]
    bp.step(psis, 0.0, dt, 2, want_stats=False)
    psis = [x.clone() for x in psi0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bp.step(psis, 0.0, dt, steps, want_stats=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    bp.close()
    # one context per packet, 2 steps each
    seq_steps = 2
    props = [Propagator(p, m, "mixed") for p in probs]
    qs = [x.clone() for x in psi0]
    props[0].step(qs[0], 0.0, dt, 1, want_stats=False)
    qs = [x.clone() for x in psi0]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for pr, q in zip(props, qs):
        pr.step(q, 0.0, dt, seq_steps, want_stats=False)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t1
    for pr in props:
        pr.close()
    rate = sites * m * steps / wall
    seq_rate = sites * m * seq_steps / seq
    log(f"batch: {wall * 1e3 / steps:.3f} ms/step ({rate:.3e} site-matvecs/s); one context per packet: "
        f"{seq * 1e3 / seq_steps:.2f} ms/step")
    return {"workload": "packet_batch_256 (grids 128^2..512^2, mixed, m=12, dt=1e-3)", "packets": len(probs),
            "sites": sites, "steps": steps, "ms_per_step": wall * 1e3 / steps, "value": rate,
            "unit": "site-matvecs/s", "per_packet_contexts": {"ms_per_step": seq * 1e3 / seq_steps,
                                                              "value": seq_rate},
            "speedup": seq_rate and rate / seq_rate,
            # algorithmic bytes of a mixed step: (64 m + 48) per site
            "hbm_frac_step": round(sites * (64 * m + 48) * steps / wall / 1e9 / HBM_PEAK_GBS, 4)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--grid", type=int, default=4096, help="grid size (default: the 4096^2 workload)")
    ap.add_argument("--precision", choices=("both", "mixed", "fp64"), default="both")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=50,
                    help="steps of the 256-packet batch measurement (0: skip)")
    ap.add_argument("--lowmem-steps", type=int, default=20,
                    help="steps of the memory-saving (second Lanczos run) measurement (0: skip)")
    ap.add_argument("--extras", default="ktol,adaptive_dt,chirality,paper_shape,adjoint,eigen,hermite",
                    help="comma-separated extra measurements: ktol, adaptive_dt, chirality, paper_shape, "
                         "adjoint, eigen, hermite (empty: none)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run a plain copy of this many MiB (counter calibration for rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the propagator has no multi-GPU path "
              "(sharding the lattice into row strips with halo exchange is not implemented).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1407_7370_amd import packets
    from paper_1407_7370_amd.binding import Propagator

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    cfg = packets.laser_4096(seed=0, precision="mixed")
    if args.grid != 4096:
        cfg = packets.with_grid(cfg, args.grid)
    prob, m, dt = cfg["problem"], cfg["m"], cfg["dt"]
    nx, ny = prob["nx"], prob["ny"]
    sites = nx * ny
    log(f"workload {nx}x{ny} m={m} dt={dt} steps={args.steps} warmup={args.warmup}")
    psi0 = packets.initial_state(cfg)
    psi0_dev = torch.from_numpy(psi0).to("cuda")

    precs = ("mixed", "fp64") if args.precision == "both" else (args.precision,)
    res = {}
    for prec in precs:
        log(f"running {prec}")
        psi, stats, wall, timing, wall_ev, same = run_precision(
            torch, Propagator, cfg, psi0_dev, prec, args.steps, args.warmup, args.copy_calib_mib)
        res[prec] = dict(psi=psi, stats=stats, wall=wall, timing=timing, wall_ev=wall_ev, same=same)
        log(f"{prec}: {wall * 1e3 / args.steps:.3f} ms/step ({wall_ev * 1e3 / args.steps:.3f} with "
            f"events; bitwise repeat {same}), timing {timing}")

    # mixed vs FP64 difference of the final states
    err = None
    if "mixed" in res and "fp64" in res:
        d = torch.linalg.vector_norm(res["mixed"]["psi"] - res["fp64"]["psi"])
        err = float(d / torch.linalg.vector_norm(res["fp64"]["psi"]))
        log(f"rel-L2(mixed - fp64) after {args.steps} steps = {err:.3e}")

    head = "mixed" if "mixed" in res else "fp64"
    r = res[head]
    site_mv = sites * m * args.steps
    value = site_mv / r["wall"]
    bps = {"mixed": 16, "fp64": 32}  # bytes per site per Krylov vector
    state_b = 32

    def step_bytes(prec):
        # algorithmic bytes of one step: 4m-2 vector transfers (state vectors complex128)
        b = bps[prec]
        if prec == "fp64":
            return sites * b * (4 * m - 2)
        # first sweep 32, sweep 2: 32+16, sweep 3: 16+32+16, sweeps 4..m: 48, recombination 32+(m-1)16+32
        return sites * (state_b + (state_b + b) + (b + state_b + b) + 3 * b * (m - 3)
                        + state_b + (m - 1) * b + state_b)

    def roofline(prec):
        n, ms = r_t = res[prec]["timing"]["recur_basis"]
        if n == 0:
            return None
        avg_s = ms / n / 1e3
        bytes_launch = 3 * bps[prec] * sites  # read u_{p-1}, u_{p-2}; write u_p
        achieved = bytes_launch / avg_s / 1e9
        traffic = load_traffic(prec)
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_recur (Lanczos sweep, iterations 4..m)",
                "bytes_per_launch": bytes_launch, "avg_launch_us": round(avg_s * 1e6, 2),
                "launches": n}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "site-matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["wall"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "storage": "complex64 Krylov vectors, complex128 state" if head == "mixed" else "complex128",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "grid": f"{nx}x{ny}", "krylov_dim": m, "dt": dt,
                   "precision": head, "boundary": "dirichlet", "box": "[-40,40)^2",
                   "field": "A(t)=50 sin(t) sin^2(pi t/0.1) y", "seed": cfg["seed"]},
        "hbm_frac_step": round(step_bytes(head) * args.steps / r["wall"] / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": roofline(head),
    }
    if "fp64" in res and head != "fp64":
        f = res["fp64"]
        out["fp64"] = {"value": site_mv / f["wall"], "ms_per_step": f["wall"] * 1e3 / args.steps,
                       "hbm_frac_step": round(step_bytes("fp64") * args.steps / f["wall"] / 1e9
                                              / HBM_PEAK_GBS, 4),
                       "roofline": roofline("fp64")}
        out["mixed_over_fp64_speedup"] = round(f["wall"] / r["wall"], 3)
    out["err_mixed_vs_fp64"] = err
    if "mixed" in res and "fp64" in res and args.grid == 4096:
        out["mixed_vs_fp64_full_run"] = run_mixed_accuracy(torch, Propagator, cfg, psi0_dev)
    st = r["stats"]
    out["stats"] = {"k_eff_min": int(st["k_eff"].min()), "cum_err_bound": float(st["cum_bound"][-1]),
                    "norm_drift": float(abs(st["norm2"][-1] / float(np.sum(np.abs(psi0) ** 2)) - 1.0))}
    out["kernel_ms"] = {k: (v[0], round(v[1], 3)) for k, v in r["timing"].items()}
    out["events_region_ms_per_step"] = r["wall_ev"] * 1e3 / args.steps
    out["bitwise_repeat"] = all(v["same"] for v in res.values())
    out["paper_context"] = {"value": 5.6e6, "unit": "site-matvecs/s",
                            "what": "derived from ~2 min per step, 8192^2 grid, k=10, one process on a "
                                    "dual Xeon-E5 cluster node (Sec. 7); context, not the target"}

    if args.lowmem_steps > 0 and "mixed" in res:
        out["lowmem"] = run_lowmem(torch, Propagator, cfg, psi0_dev, args.lowmem_steps)

    if args.batch_steps > 0:
        out["batch_packets"] = run_batch(torch, packets, args.batch_steps)

    extras = {e for e in args.extras.split(",") if e}
    if "ktol" in extras and "mixed" in res:
        out["adaptive_k"] = run_ktol(torch, Propagator, cfg, psi0_dev, 100)
    if "adaptive_dt" in extras:
        out["adaptive_dt"] = run_adaptive_dt(torch, Propagator, cfg, psi0_dev)
    if "chirality" in extras and "mixed" in res:
        out["chirality_minus"] = run_chirality(torch, Propagator, cfg, psi0_dev)
    if "paper_shape" in extras:
        out["paper_shape"] = run_paper_shape(torch, Propagator, packets)
    if "adjoint" in extras:
        out["adjoint"] = run_adjoint(torch, Propagator, packets)
    if "eigen" in extras:
        out["eigen"] = run_eigen(torch, Propagator, packets)
    if "hermite" in extras:
        out["hermite"] = run_hermite(torch, packets)

    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        log("timing the CPU oracle on one step of the same workload")
        t0 = time.perf_counter()
        oracle.propagate(prob, psi0, 0.0, dt, 1, m)
        cw = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": sites * m / cw, "unit": "site-matvecs/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"one time step (m={m}) of the {nx}x{ny} laser workload, "
                                         f"single-threaded C oracle, {cw:.1f} s",
                               "cpu": cpu_model()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
