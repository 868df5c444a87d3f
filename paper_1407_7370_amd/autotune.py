"""Launch-shape autotuner.

Times candidate launch shapes of the Lanczos sweeps on the device and caches
the fastest per workload class in a JSON file:
  - single grids: the cap on waves per compute unit of the sweeps
    (`dirac_lanczos_set_launch`), keyed by (device, nx, ny, precision, m,
    periodic y, site terms);
  - batches: the rows per chunk of the batched sweeps
    (`dirac_lanczos_batch_set_launch`), keyed by (device, precision, m,
    periodic y, the histogram of packet grid sizes).
Every shape computes the same result to rounding (the reductions are folded
over other partial sums); the cache only changes speed.

  python -m paper_1407_7370_amd.autotune --workload laser_4096 --precision mixed
  python -m paper_1407_7370_amd.autotune --workload fourier_pulse_512 --precision fp64
  python -m paper_1407_7370_amd.autotune --workload packet_batch
"""
from __future__ import annotations

import argparse
import collections
import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuning_cache.json")
SINGLE_CANDIDATES = (4, 6, 8, 12, 16)
BATCH_CANDIDATES = (32, 64, 128, 256, 0)


def _site_terms(p: dict) -> bool:
    return bool(p.get("pot_kind", 0)) or p.get("v_table") is not None or float(p.get("bz", 0.0)) != 0.0


def key_single(problem: dict, m: int, precision: str, arch: str) -> str:
    return (f"single/{arch}/{int(problem['nx'])}x{int(problem['ny'])}/{precision}/m{int(m)}"
            f"/py{int(problem.get('bc_y', 0))}/site{int(_site_terms(problem))}")


def key_batch(problems, m: int, precision: str, arch: str) -> str:
    hist = collections.Counter((int(p["nx"]), int(p["ny"])) for p in problems)
    sizes = ",".join(f"{nx}x{ny}:{c}" for (nx, ny), c in sorted(hist.items()))
    site = int(any(_site_terms(p) for p in problems))
    return f"batch/{arch}/{precision}/m{int(m)}/py{int(problems[0].get('bc_y', 0))}/site{site}/{sizes}"


def load(cache: str = DEFAULT_CACHE) -> dict:
    try:
        with open(cache) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def store(key: str, entry: dict, cache: str = DEFAULT_CACHE) -> None:
    data = load(cache)
    data[key] = entry
    tmp = cache + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, cache)


def lookup(key: str, cache: str = DEFAULT_CACHE):
    """The cached shape for `key`, or None."""
    e = load(cache).get(key)
    return None if e is None else int(e["best"])


def device_arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _time_steps(step, steps: int) -> float:
    import torch
    step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step(steps)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def tune_single(problem: dict, psi0, m: int, precision: str, dt: float, steps: int = 4,
                candidates=SINGLE_CANDIDATES, cache: str = DEFAULT_CACHE) -> dict:
    """Time each sweep cap on `steps` steps of the problem; store and return the result."""
    import torch
    from .binding import Propagator
    prop = Propagator(problem, m, precision)
    times = {}
    for c in candidates:
        used = prop.set_launch(c)
        psi = psi0.clone()

        def step(n):
            prop.step(psi, 0.0, dt, n, want_stats=False)

        times[str(c)] = {"waves_per_cu": used, "ms_per_step": _time_steps(step, steps) * 1e3}
    prop.close()
    best = min(candidates, key=lambda c: times[str(c)]["ms_per_step"])
    entry = {"best": best, "times": times, "steps": steps}
    store(key_single(problem, m, precision, device_arch()), entry, cache)
    torch.cuda.synchronize()
    return entry


def tune_batch(problems, psi0, m: int, precision: str, dt: float, steps: int = 4,
               candidates=BATCH_CANDIDATES, cache: str = DEFAULT_CACHE) -> dict:
    """Time each rows-per-chunk choice of the batched sweeps; store and return the result."""
    from .binding import BatchPropagator
    bp = BatchPropagator(problems, m, precision)
    times = {}
    for c in candidates:
        used = bp.set_launch(c)
        psis = [x.clone() for x in psi0]

        def step(n):
            bp.step(psis, 0.0, dt, n, want_stats=False)

        times[str(c)] = {"rows_per_chunk": used, "ms_per_step": _time_steps(step, steps) * 1e3}
    bp.close()
    best = min(candidates, key=lambda c: times[str(c)]["ms_per_step"])
    entry = {"best": best, "times": times, "steps": steps}
    store(key_batch(problems, m, precision, device_arch()), entry, cache)
    return entry


def main():
    import torch
    from . import packets
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", choices=("laser_4096", "fourier_pulse_512", "packet_batch"), default="laser_4096")
    ap.add_argument("--precision", choices=("mixed", "fp64"), default="mixed")
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--cache", default=DEFAULT_CACHE)
    ap.add_argument("--candidates", default="",
                    help="comma-separated shapes to time (waves per CU, or rows per chunk for batches)")
    args = ap.parse_args()
    cand = tuple(int(c) for c in args.candidates.split(",") if c)
    if args.workload in ("laser_4096", "fourier_pulse_512"):
        if args.workload == "laser_4096":
            cfg = packets.laser_4096(seed=0, precision=args.precision)
        else:
            cfg = packets.fourier_pulse_512(seed=0)
        psi0 = torch.from_numpy(packets.initial_state(cfg)).to("cuda")
        e = tune_single(cfg["problem"], psi0, cfg["m"], args.precision, cfg["dt"], args.steps,
                        candidates=cand or SINGLE_CANDIDATES, cache=args.cache)
    else:
        cfgs = packets.packet_batch(seed=0)
        psi0 = [torch.from_numpy(packets.initial_state(c)).to("cuda") for c in cfgs]
        e = tune_batch([c["problem"] for c in cfgs], psi0, cfgs[0]["m"], args.precision, cfgs[0]["dt"],
                       args.steps, candidates=cand or BATCH_CANDIDATES, cache=args.cache)
    print(json.dumps(e))


if __name__ == "__main__":
    main()
