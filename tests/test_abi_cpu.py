"""CPU checks of the C ABI: the library loads, exports every declared symbol,
its ctypes mirror matches the C struct layout, and host-side validation
rejects bad arguments before any device work."""
import ctypes
import os
import re
import subprocess

import numpy as np

import pytest

from paper_1407_7370_amd import binding, packets

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dirac_lanczos.h")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dirac_lanczos_\w+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = binding.load_library()
    names = header_functions()
    assert set(names) == set(binding.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    for n in names:
        assert n in exported, n
        getattr(lib, n)


def test_params_layout_matches_c(tmp_path):
    """Every struct of the header has the binding's size and field offsets."""
    structs = [("dl_params", binding.DlParams), ("dl_step_stat", binding.DlStepStat),
               ("dl_adapt_stat", binding.DlAdaptStat), ("dl_timing", binding.DlTiming)]
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "dirac_lanczos.h"', "int main(){"]
    for cname, cls in structs:
        src.append(f'printf("%zu\\n", sizeof({cname}));')
        for f in cls._fields_:
            src.append(f'printf("%zu\\n", offsetof({cname}, {f[0]}));')
    src.append("return 0;}")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), str(c), "-o", str(exe)])
    vals = iter(int(v) for v in subprocess.check_output([str(exe)], text=True).split())
    for cname, cls in structs:
        assert next(vals) == ctypes.sizeof(cls), cname
        for f in cls._fields_:
            assert next(vals) == getattr(cls, f[0]).offset, (cname, f[0])


def _params(cfg, m, prec):
    return binding.make_params(cfg["problem"], m, prec)[0]


def test_workspace_bytes_plan():
    cfg = packets.laser_4096()
    n = 2 * 4096 * 4096
    pm = _params(cfg, 16, binding.DL_PREC_MIXED)
    pf = _params(cfg, 16, binding.DL_PREC_FP64)
    bm = binding.dirac_lanczos_workspace_bytes(pm)
    bf = binding.dirac_lanczos_workspace_bytes(pf)
    # second state buffer (complex128) + 15 Krylov vectors + < 4 MiB of scalars/tables
    assert n * 16 + 15 * n * 8 <= bm <= n * 16 + 15 * n * 8 + (4 << 20)
    assert n * 16 + 15 * n * 16 <= bf <= n * 16 + 15 * n * 16 + (4 << 20)
    # eigen mode: at least three complex128 vectors
    small = packets.with_grid(cfg, 64)
    p1 = _params(small, 1, binding.DL_PREC_FP64)
    assert binding.dirac_lanczos_workspace_bytes(p1, binding.DL_MODE_EIGEN, 100) >= 3 * 2 * 64 * 64 * 16
    assert binding.dirac_lanczos_workspace_bytes(p1, binding.DL_MODE_EIGEN, 0) == 0
    # full reorthogonalisation: z plus k stored complex128 vectors, growing with k
    nv = 2 * 64 * 64 * 16
    r100 = binding.dirac_lanczos_workspace_bytes(p1, binding.DL_MODE_EIGEN_REORTH, 100)
    r200 = binding.dirac_lanczos_workspace_bytes(p1, binding.DL_MODE_EIGEN_REORTH, 200)
    assert 101 * nv <= r100 <= 101 * (nv + 8192) + (8 << 20)
    assert r200 - r100 >= 100 * nv
    assert binding.dirac_lanczos_workspace_bytes(p1, binding.DL_MODE_EIGEN_REORTH, 0) == 0
    assert binding.dirac_lanczos_workspace_bytes(p1, 4, 10) == 0


@pytest.mark.parametrize("bad", [
    dict(nx=2), dict(ny=1), dict(x_max=-50.0), dict(bc_x=2), dict(c=0.0), dict(mass=-1.0),
    dict(pot_kind=3), dict(pot_kind=1, pot_a=0.0), dict(pot_kind=2, pot_z=0.0), dict(pulse_kind=5),
    dict(pulse_kind=1, t_pulse=0.0), dict(pulse_kind=2, coef=[1.0, 2.0, 3.0]),
    dict(bz=float("nan")),
])
def test_invalid_params_rejected(bad):
    cfg = packets.with_grid(packets.laser_4096(), 64)
    prob = dict(cfg["problem"], **bad)
    p, _ = binding.make_params(prob, 16, binding.DL_PREC_FP64)
    assert binding.dirac_lanczos_workspace_bytes(p) == 0
    with pytest.raises(binding.DlError) as ei:
        binding.dirac_lanczos_init(p, 256, 1 << 40, 0)
    assert ei.value.status == binding.DL_ERR_INVALID


@pytest.mark.parametrize("m,prec", [(0, 0), (65, 0), (16, 2)])
def test_invalid_krylov_or_precision(m, prec):
    cfg = packets.with_grid(packets.laser_4096(), 64)
    p, _ = binding.make_params(cfg["problem"], m, prec)
    assert binding.dirac_lanczos_workspace_bytes(p) == 0
    with pytest.raises(binding.DlError) as ei:
        binding.dirac_lanczos_init(p, 256, 1 << 40, 0)
    assert ei.value.status == binding.DL_ERR_INVALID


def test_workspace_errors():
    cfg = packets.with_grid(packets.laser_4096(), 64)
    p, _ = binding.make_params(cfg["problem"], 16, binding.DL_PREC_FP64)
    # init needs the smaller (second-run) layout; the stored basis needs more
    need = binding.dirac_lanczos_workspace_bytes(p, binding.DL_MODE_LOWMEM)
    assert 0 < need < binding.dirac_lanczos_workspace_bytes(p)
    for ptr, size in ((0, need), (256 + 8, need), (256, need - 1)):
        with pytest.raises(binding.DlError) as ei:
            binding.dirac_lanczos_init(p, ptr, size, 0)
        assert ei.value.status == binding.DL_ERR_WORKSPACE


def test_autotune_cache_roundtrip(tmp_path):
    """Cache keys separate workload classes; entries survive a store/load."""
    from paper_1407_7370_amd import autotune
    a = dict(nx=64, ny=48, bc_y=0, bz=0.0, pot_kind=0)
    b = dict(a, bz=0.5)
    ka = autotune.key_single(a, 12, "mixed", "gfx950")
    kb = autotune.key_single(b, 12, "mixed", "gfx950")
    assert ka != kb and "64x48" in ka and "site1" in kb
    kbat = autotune.key_batch([a, a, dict(a, nx=32)], 12, "mixed", "gfx950")
    assert "64x48:2" in kbat and "32x48:1" in kbat
    cache = str(tmp_path / "tune.json")
    assert autotune.lookup(ka, cache) is None
    autotune.store(ka, {"best": 6, "times": {}}, cache)
    autotune.store(kbat, {"best": 64, "times": {}}, cache)
    assert autotune.lookup(ka, cache) == 6
    assert autotune.lookup(kbat, cache) == 64
    assert autotune.lookup(kb, cache) is None


def test_missing_library_raises(monkeypatch, tmp_path):
    """No CPU fallback: without the built HIP library the binding refuses to load."""
    from paper_1407_7370_amd import binding
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "libdirac_lanczos.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        binding.load_library()


def test_hermite_nodes_host():
    """The library's collocation points and weights (a host computation:
    Golub-Welsch with Newton polish, Christoffel-Darboux weights) against
    numpy's Gauss-Hermite rule."""
    from numpy.polynomial.hermite import hermgauss
    for n, s in ((16, 0.5), (64, 0.036)):
        x, w = binding.hermite_nodes(n, s)
        xi, wg = hermgauss(n)
        assert np.max(np.abs(x / s - xi)) <= 1e-13 * np.abs(xi).max()
        assert np.max(np.abs(w / (s * wg * np.exp(xi * xi)) - 1.0)) <= 1e-11


def test_hermite_rejections_host():
    """Invalid Hermite problems are rejected before any device work."""
    p = binding.make_hermite_params(dict(n=20, scale=1.0))
    assert binding.load_library().dirac_lanczos_hermite_workspace_bytes(ctypes.byref(p), 1, 10) == 0
    p = binding.make_hermite_params(dict(n=32, scale=-1.0))
    assert binding.load_library().dirac_lanczos_hermite_workspace_bytes(ctypes.byref(p), 1, 10) == 0
    p = binding.make_hermite_params(dict(n=32, scale=0.1))
    assert binding.load_library().dirac_lanczos_hermite_workspace_bytes(ctypes.byref(p), 1, 10) > 0
