"""ctypes binding of libdirac_lanczos.so (include/dirac_lanczos.h).

Argument marshalling only: every step of the propagator runs in the HIP
library.  Device memory and streams come from PyTorch (the caller's tensors,
a uint8 workspace tensor, torch's current stream).  There is no CPU fallback:
if the shared library or a gfx950 device is missing, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdirac_lanczos.so")

DL_OK, DL_ERR_INVALID, DL_ERR_DEVICE, DL_ERR_NONFINITE, DL_ERR_WORKSPACE, DL_ERR_UNSUPPORTED = range(6)
DL_PREC_FP64, DL_PREC_MIXED = 0, 1
DL_MODE_STEP, DL_MODE_EIGEN, DL_MODE_LOWMEM, DL_MODE_EIGEN_REORTH = 0, 1, 2, 3
STATUS_NAMES = {0: "DL_OK", 1: "DL_ERR_INVALID", 2: "DL_ERR_DEVICE", 3: "DL_ERR_NONFINITE",
                4: "DL_ERR_WORKSPACE", 5: "DL_ERR_UNSUPPORTED"}

# every symbol declared in include/dirac_lanczos.h
EXPORTS = ("dirac_lanczos_workspace_bytes", "dirac_lanczos_init", "dirac_lanczos_apply",
           "dirac_lanczos_step", "dirac_lanczos_eigen", "dirac_lanczos_adjoint_workspace_bytes",
           "dirac_lanczos_adjoint", "dirac_lanczos_timing", "dirac_lanczos_destroy",
           "dirac_lanczos_last_error", "dirac_lanczos_batch_workspace_bytes", "dirac_lanczos_batch_init",
           "dirac_lanczos_batch_step", "dirac_lanczos_batch_destroy", "dirac_lanczos_batch_last_error",
           "dirac_lanczos_set_launch", "dirac_lanczos_batch_set_launch", "dirac_lanczos_step_adaptive",
           "dirac_lanczos_step_lowmem", "dirac_lanczos_eigen_vectors", "dirac_lanczos_step_ktol",
           "dirac_lanczos_wait", "dirac_lanczos_step_noalloc", "dirac_lanczos_hermite_nodes",
           "dirac_lanczos_hermite_workspace_bytes", "dirac_lanczos_hermite_apply", "dirac_lanczos_hermite_eigen",
           "dirac_lanczos_hermite_last_error", "dirac_lanczos_ritz")
DL_LOSS_X, DL_LOSS_Y, DL_LOSS_PX, DL_LOSS_PY = 1, 2, 4, 8


class DlParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("x_min", ctypes.c_double), ("x_max", ctypes.c_double),
        ("y_min", ctypes.c_double), ("y_max", ctypes.c_double),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("mass", ctypes.c_double), ("c", ctypes.c_double), ("charge", ctypes.c_double),
        ("krylov_dim", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("bz", ctypes.c_double),
        ("pot_kind", ctypes.c_int32), ("pot_z", ctypes.c_double), ("pot_a", ctypes.c_double),
        ("v_table", ctypes.c_void_p),
        ("pulse_kind", ctypes.c_int32),
        ("pulse_e", ctypes.c_double * 2), ("a0", ctypes.c_double), ("omega", ctypes.c_double),
        ("t_pulse", ctypes.c_double),
        ("n_coef", ctypes.c_int32), ("coef", ctypes.c_void_p),
        ("chirality", ctypes.c_int32),
    ]


class DlStepStat(ctypes.Structure):
    _fields_ = [("k_eff", ctypes.c_int32), ("err_est", ctypes.c_double),
                ("cum_bound", ctypes.c_double), ("norm2", ctypes.c_double),
                ("round_bound", ctypes.c_double)]


def stats_dict(stats) -> dict:
    """Numpy arrays of a sequence of DlStepStat (cum_round_bound: the running
    sum of round_bound)."""
    rb = np.array([s.round_bound for s in stats])
    return {"k_eff": np.array([s.k_eff for s in stats], dtype=np.int32),
            "err_est": np.array([s.err_est for s in stats]),
            "cum_bound": np.array([s.cum_bound for s in stats]),
            "norm2": np.array([s.norm2 for s in stats]),
            "round_bound": rb,
            "cum_round_bound": np.cumsum(rb)}


class DlHermiteParams(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("scale", ctypes.c_double), ("mass", ctypes.c_double),
                ("c", ctypes.c_double), ("charge", ctypes.c_double), ("bz", ctypes.c_double),
                ("pot_kind", ctypes.c_int32), ("pot_z", ctypes.c_double), ("pot_a", ctypes.c_double),
                ("chirality", ctypes.c_int32)]


def make_hermite_params(hprob: dict) -> DlHermiteParams:
    """dl_hermite_params from a Hermite problem dict (keys as in packets.py)."""
    p = DlHermiteParams()
    p.n = int(hprob["n"])
    p.scale = float(hprob["scale"])
    for k, d in (("mass", 1.0), ("c", 137.036), ("charge", -1.0), ("bz", 0.0), ("pot_z", 0.0), ("pot_a", 0.0)):
        setattr(p, k, float(hprob.get(k, d)))
    p.pot_kind = int(hprob.get("pot_kind", 0))
    p.chirality = int(hprob.get("chirality", 0))
    return p


class DlAdaptStat(ctypes.Structure):
    _fields_ = [("accepted", ctypes.c_int32), ("rejected", ctypes.c_int32), ("t_reached", ctypes.c_double),
                ("dt_next", ctypes.c_double), ("cum_bound", ctypes.c_double), ("norm2", ctypes.c_double),
                ("cum_magnus", ctypes.c_double)]


class DlTiming(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 5), ("total_ms", ctypes.c_double * 5)]


TIMING_CLASSES = ("first", "recur_basis", "recur_psi", "tridiag", "recombine")


class DlError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library():
    """Load the HIP library (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads torch's HIP runtime first)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1407_7370_amd.build`"
                           " (there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(DlParams)
    vp, D = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    lib.dirac_lanczos_workspace_bytes.argtypes = [P, ctypes.c_int32, ctypes.c_int32]
    lib.dirac_lanczos_workspace_bytes.restype = ctypes.c_size_t
    lib.dirac_lanczos_init.argtypes = [P, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.dirac_lanczos_init.restype = ctypes.c_int
    lib.dirac_lanczos_apply.argtypes = [vp, vp, vp, ctypes.c_double]
    lib.dirac_lanczos_apply.restype = ctypes.c_int
    lib.dirac_lanczos_step.argtypes = [vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                       ctypes.POINTER(DlStepStat)]
    lib.dirac_lanczos_step.restype = ctypes.c_int
    lib.dirac_lanczos_step_lowmem.argtypes = lib.dirac_lanczos_step.argtypes
    lib.dirac_lanczos_step_lowmem.restype = ctypes.c_int
    lib.dirac_lanczos_step_ktol.argtypes = [vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                            ctypes.c_double, ctypes.c_int32, ctypes.POINTER(DlStepStat)]
    lib.dirac_lanczos_step_ktol.restype = ctypes.c_int
    lib.dirac_lanczos_wait.argtypes = [vp, ctypes.POINTER(DlStepStat), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.dirac_lanczos_wait.restype = ctypes.c_int
    lib.dirac_lanczos_step_noalloc.argtypes = [P, vp, ctypes.c_double, ctypes.c_double, ctypes.c_int32, vp,
                                               ctypes.POINTER(DlStepStat)]
    lib.dirac_lanczos_step_noalloc.restype = ctypes.c_int
    HP = ctypes.POINTER(DlHermiteParams)
    lib.dirac_lanczos_ritz.argtypes = [D, D, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int32, ctypes.c_int32, D, D, ctypes.POINTER(ctypes.c_int32)]
    lib.dirac_lanczos_ritz.restype = ctypes.c_int
    lib.dirac_lanczos_hermite_nodes.argtypes = [ctypes.c_int32, ctypes.c_double, D, D]
    lib.dirac_lanczos_hermite_nodes.restype = ctypes.c_int
    lib.dirac_lanczos_hermite_workspace_bytes.argtypes = [HP, ctypes.c_int32, ctypes.c_int32]
    lib.dirac_lanczos_hermite_workspace_bytes.restype = ctypes.c_size_t
    lib.dirac_lanczos_hermite_apply.argtypes = [HP, vp, vp, vp, ctypes.c_size_t, vp]
    lib.dirac_lanczos_hermite_apply.restype = ctypes.c_int
    lib.dirac_lanczos_hermite_eigen.argtypes = [HP, ctypes.c_int32, ctypes.POINTER(vp), ctypes.c_int32, D, D,
                                                ctypes.c_double, ctypes.c_int32, vp, ctypes.c_size_t, vp, D, D,
                                                ctypes.POINTER(ctypes.c_int32)]
    lib.dirac_lanczos_hermite_eigen.restype = ctypes.c_int
    lib.dirac_lanczos_hermite_last_error.argtypes = []
    lib.dirac_lanczos_hermite_last_error.restype = ctypes.c_char_p
    lib.dirac_lanczos_eigen.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_int32, D, D,
                                        ctypes.POINTER(ctypes.c_int32)]
    lib.dirac_lanczos_eigen.restype = ctypes.c_int
    lib.dirac_lanczos_eigen_vectors.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                                ctypes.c_double, ctypes.c_int32, D, D,
                                                ctypes.POINTER(ctypes.c_int32), vp]
    lib.dirac_lanczos_eigen_vectors.restype = ctypes.c_int
    lib.dirac_lanczos_adjoint_workspace_bytes.argtypes = [P, ctypes.c_int32, ctypes.c_int32]
    lib.dirac_lanczos_adjoint_workspace_bytes.restype = ctypes.c_size_t
    lib.dirac_lanczos_adjoint.argtypes = [vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_size_t, D, D]
    lib.dirac_lanczos_adjoint.restype = ctypes.c_int
    lib.dirac_lanczos_timing.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(DlTiming)]
    lib.dirac_lanczos_timing.restype = ctypes.c_int
    lib.dirac_lanczos_destroy.argtypes = [vp]
    lib.dirac_lanczos_destroy.restype = ctypes.c_int
    lib.dirac_lanczos_last_error.argtypes = [vp]
    lib.dirac_lanczos_last_error.restype = ctypes.c_char_p
    lib.dirac_lanczos_batch_workspace_bytes.argtypes = [P, ctypes.c_int32]
    lib.dirac_lanczos_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.dirac_lanczos_batch_init.argtypes = [P, ctypes.c_int32, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.dirac_lanczos_batch_init.restype = ctypes.c_int
    lib.dirac_lanczos_batch_step.argtypes = [vp, ctypes.POINTER(vp), ctypes.c_double, ctypes.c_double,
                                             ctypes.c_int32, ctypes.POINTER(DlStepStat)]
    lib.dirac_lanczos_batch_step.restype = ctypes.c_int
    lib.dirac_lanczos_batch_destroy.argtypes = [vp]
    lib.dirac_lanczos_batch_destroy.restype = ctypes.c_int
    lib.dirac_lanczos_batch_last_error.argtypes = [vp]
    lib.dirac_lanczos_batch_last_error.restype = ctypes.c_char_p
    I = ctypes.POINTER(ctypes.c_int32)
    lib.dirac_lanczos_set_launch.argtypes = [vp, ctypes.c_int32, I]
    lib.dirac_lanczos_set_launch.restype = ctypes.c_int
    lib.dirac_lanczos_batch_set_launch.argtypes = [vp, ctypes.c_int32, I]
    lib.dirac_lanczos_batch_set_launch.restype = ctypes.c_int
    lib.dirac_lanczos_step_adaptive.argtypes = [vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                                D, ctypes.POINTER(DlAdaptStat)]
    lib.dirac_lanczos_step_adaptive.restype = ctypes.c_int
    _lib = lib
    return lib


def make_params(problem: dict, krylov_dim: int, precision: int = DL_PREC_FP64, v_table_ptr: int = 0):
    """dl_params from a problem dict (keys as in packets.py).  Returns (struct, keepalive)."""
    p = DlParams()
    keep = []
    for k in ("nx", "ny", "bc_x", "bc_y", "pot_kind", "pulse_kind"):
        setattr(p, k, int(problem.get(k, 0)))
    defaults = {"mass": 1.0, "c": 137.036, "charge": -1.0}
    for k in ("x_min", "x_max", "y_min", "y_max", "mass", "c", "charge", "bz", "pot_z", "pot_a",
              "a0", "omega", "t_pulse"):
        setattr(p, k, float(problem.get(k, defaults.get(k, 0.0))))
    e = problem.get("pulse_e", (0.0, 0.0))
    p.pulse_e[0], p.pulse_e[1] = float(e[0]), float(e[1])
    p.krylov_dim = int(krylov_dim)
    p.precision = int(precision)
    p.chirality = int(problem.get("chirality", 0))
    p.v_table = int(v_table_ptr) if v_table_ptr else None
    coef = problem.get("coef")
    if coef is not None and len(coef) > 0:
        arr = np.ascontiguousarray(coef, dtype=np.float64)
        keep.append(arr)
        p.coef = arr.ctypes.data
        p.n_coef = len(arr)
    return p, keep


def _err(lib, ctx):
    msg = lib.dirac_lanczos_last_error(ctx)
    return msg.decode() if msg else ""


def _check(lib, ctx, status):
    if status != DL_OK:
        raise DlError(status, _err(lib, ctx))


# ---------------------------------------------------------------------------
# Functions with the C names (raw pointers in, status codes out)
# ---------------------------------------------------------------------------
def dirac_lanczos_workspace_bytes(params: DlParams, mode: int = DL_MODE_STEP, k_eigen: int = 0) -> int:
    return int(load_library().dirac_lanczos_workspace_bytes(ctypes.byref(params), mode, k_eigen))


def dirac_lanczos_init(params: DlParams, workspace_ptr: int, ws_bytes: int, stream_ptr: int):
    lib = load_library()
    ctx = ctypes.c_void_p()
    st = lib.dirac_lanczos_init(ctypes.byref(params), ctypes.c_void_p(workspace_ptr), ws_bytes,
                                ctypes.c_void_p(stream_ptr), ctypes.byref(ctx))
    if st != DL_OK:
        raise DlError(st, _err(lib, None))
    return ctx


def dirac_lanczos_apply(ctx, x_ptr: int, y_ptr: int, t: float) -> int:
    return load_library().dirac_lanczos_apply(ctx, ctypes.c_void_p(x_ptr), ctypes.c_void_p(y_ptr), t)


def dirac_lanczos_step(ctx, psi_ptr: int, t0: float, dt: float, n_steps: int, stats=None) -> int:
    return load_library().dirac_lanczos_step(ctx, ctypes.c_void_p(psi_ptr), t0, dt, n_steps, stats)


def dirac_lanczos_step_noalloc(params: DlParams, psi_ptr: int, t0: float, dt: float, n_steps: int,
                               stream_ptr: int, stats=None) -> int:
    return load_library().dirac_lanczos_step_noalloc(ctypes.byref(params), ctypes.c_void_p(psi_ptr), t0, dt,
                                                     n_steps, ctypes.c_void_p(stream_ptr), stats)


def dirac_lanczos_wait(ctx, stats=None, n_stats: int = 0, steps_done=None) -> int:
    return load_library().dirac_lanczos_wait(ctx, stats, n_stats, steps_done)


def dirac_lanczos_eigen(ctx, psi_ptr: int, k_max: int, reorth: int, e_lo: float, e_hi: float,
                        tol: float, n_wanted: int, evals, bounds, n_found) -> int:
    return load_library().dirac_lanczos_eigen(ctx, ctypes.c_void_p(psi_ptr), k_max, reorth, e_lo, e_hi,
                                              tol, n_wanted, evals, bounds, n_found)


def dirac_lanczos_eigen_vectors(ctx, psi_ptr: int, k_max: int, e_lo: float, e_hi: float, tol: float,
                                n_wanted: int, evals, bounds, n_found, vecs_ptr: int) -> int:
    return load_library().dirac_lanczos_eigen_vectors(ctx, ctypes.c_void_p(psi_ptr), k_max, e_lo, e_hi, tol,
                                                      n_wanted, evals, bounds, n_found,
                                                      ctypes.c_void_p(vecs_ptr))


def dirac_lanczos_adjoint_workspace_bytes(params: DlParams, n_steps: int, ckpt_every: int) -> int:
    return int(load_library().dirac_lanczos_adjoint_workspace_bytes(ctypes.byref(params), n_steps,
                                                                     ckpt_every))


def dirac_lanczos_adjoint(ctx, psi_ptr: int, t0: float, dt: float, n_steps: int, ckpt_every: int,
                          loss_kind: int, adj_ptr: int, adj_bytes: int, loss, grad) -> int:
    return load_library().dirac_lanczos_adjoint(ctx, ctypes.c_void_p(psi_ptr), t0, dt, n_steps,
                                                ckpt_every, loss_kind, ctypes.c_void_p(adj_ptr),
                                                adj_bytes, loss, grad)


def dirac_lanczos_timing(ctx, enable: int, out=None) -> int:
    return load_library().dirac_lanczos_timing(ctx, enable, out)


def dirac_lanczos_destroy(ctx) -> int:
    return load_library().dirac_lanczos_destroy(ctx)


def dirac_lanczos_last_error(ctx) -> str:
    return _err(load_library(), ctx)


def dirac_lanczos_batch_workspace_bytes(params_array, n_packets: int) -> int:
    return int(load_library().dirac_lanczos_batch_workspace_bytes(params_array, n_packets))


def dirac_lanczos_batch_init(params_array, n_packets: int, workspace_ptr: int, ws_bytes: int, stream_ptr: int):
    lib = load_library()
    b = ctypes.c_void_p()
    st = lib.dirac_lanczos_batch_init(params_array, n_packets, ctypes.c_void_p(workspace_ptr), ws_bytes,
                                      ctypes.c_void_p(stream_ptr), ctypes.byref(b))
    if st != DL_OK:
        msg = lib.dirac_lanczos_batch_last_error(None)
        raise DlError(st, msg.decode() if msg else "")
    return b


def dirac_lanczos_batch_step(batch, psi_ptrs, t0: float, dt: float, n_steps: int, stats=None) -> int:
    arr = (ctypes.c_void_p * len(psi_ptrs))(*[ctypes.c_void_p(p) for p in psi_ptrs])
    return load_library().dirac_lanczos_batch_step(batch, arr, t0, dt, n_steps, stats)


def dirac_lanczos_batch_destroy(batch) -> int:
    return load_library().dirac_lanczos_batch_destroy(batch)


def dirac_lanczos_batch_last_error(batch) -> str:
    msg = load_library().dirac_lanczos_batch_last_error(batch)
    return msg.decode() if msg else ""


# ---------------------------------------------------------------------------
# Convenience wrapper over torch tensors
# ---------------------------------------------------------------------------
class Propagator:
    """Owns a context and its torch-allocated workspace on the current device.

    psi tensors are complex128 of shape (2, ny, nx), contiguous, on the GPU.
    """

    def __init__(self, problem: dict, krylov_dim: int, precision: str = "fp64", k_eigen: int = 0,
                 stream=None, v_table=None, tuning_cache=None, lowmem: bool = False, reorth: bool = False):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.problem = dict(problem)
        self.prec = DL_PREC_MIXED if precision == "mixed" else DL_PREC_FP64
        self.v_table = None
        vptr = 0
        if v_table is not None:
            self.v_table = torch.as_tensor(v_table, dtype=torch.float64, device="cuda").contiguous()
            vptr = self.v_table.data_ptr()
        self.params, self._keep = make_params(problem, krylov_dim, self.prec, vptr)
        if k_eigen > 0:
            mode = DL_MODE_EIGEN_REORTH if reorth else DL_MODE_EIGEN
        else:
            mode = DL_MODE_LOWMEM if lowmem else DL_MODE_STEP
        nbytes = dirac_lanczos_workspace_bytes(self.params, mode, k_eigen)
        if nbytes == 0:
            raise DlError(DL_ERR_INVALID, "invalid parameters (workspace_bytes returned 0)")
        self.ws_bytes = nbytes
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        self.ws_ptr = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.ctx = dirac_lanczos_init(self.params, self.ws_ptr, nbytes, self.stream.cuda_stream)
        self.shape = (2, int(problem["ny"]), int(problem["nx"]))
        if tuning_cache:
            # launch shape from the autotuner's cache (True: the package's cache file)
            from . import autotune
            path = autotune.DEFAULT_CACHE if tuning_cache is True else tuning_cache
            best = autotune.lookup(autotune.key_single(problem, krylov_dim, precision, autotune.device_arch()),
                                   path)
            if best is not None:
                self.set_launch(best)

    def _check_psi(self, psi):
        t = self.torch
        if not (isinstance(psi, t.Tensor) and psi.is_cuda and psi.dtype == t.complex128
                and tuple(psi.shape) == self.shape and psi.is_contiguous()):
            raise ValueError(f"psi must be a contiguous complex128 CUDA tensor of shape {self.shape}")

    def apply(self, x, t: float = 0.0):
        self._check_psi(x)
        y = self.torch.empty_like(x)
        _check(self.lib, self.ctx, dirac_lanczos_apply(self.ctx, x.data_ptr(), y.data_ptr(), t))
        return y

    def _call_step(self, psi, t0, dt, n_steps, stats, lowmem, ktol, k_min):
        if ktol > 0.0:
            return self.lib.dirac_lanczos_step_ktol(self.ctx, ctypes.c_void_p(psi.data_ptr()), t0, dt, n_steps,
                                                    ktol, int(k_min), stats)
        fn = self.lib.dirac_lanczos_step_lowmem if lowmem else self.lib.dirac_lanczos_step
        return fn(self.ctx, ctypes.c_void_p(psi.data_ptr()), t0, dt, n_steps, stats)

    def step(self, psi, t0: float, dt: float, n_steps: int, want_stats: bool = True, lowmem: bool = False,
             ktol: float = 0.0, k_min: int = 1):
        """In-place propagation of psi by n_steps steps (lowmem: the second-run
        variant; ktol > 0: adaptive Krylov dimension in [k_min, m] with the
        per-step estimate bounded by ktol).  Returns a dict of numpy stats
        (want_stats), or None after waiting for the work (no statistics)."""
        self._check_psi(psi)
        if not want_stats:
            self.step_async(psi, t0, dt, n_steps, lowmem=lowmem, ktol=ktol, k_min=k_min)
            self.wait()
            return None
        stats = (DlStepStat * max(n_steps, 1))()
        st = self._call_step(psi, t0, dt, n_steps, stats, lowmem, ktol, k_min)
        out = stats_dict(stats[:n_steps])
        _check(self.lib, self.ctx, st)
        return out

    def step_async(self, psi, t0: float, dt: float, n_steps: int, lowmem: bool = False, ktol: float = 0.0,
                   k_min: int = 1):
        """Enqueue n_steps in-place steps of psi on the context's stream and
        return at once (the C call with stats = NULL); wait() reports them."""
        self._check_psi(psi)
        self._last_async = n_steps
        _check(self.lib, self.ctx, self._call_step(psi, t0, dt, n_steps, None, lowmem, ktol, k_min))

    def wait(self, want_stats: bool = False):
        """Wait for the asynchronous steps; raise DlError on a device-side
        failure.  With want_stats, the statistics of the last call's steps
        (up to 2048) as step() returns them."""
        n = min(int(getattr(self, "_last_async", 0)), 2048) if want_stats else 0
        stats = (DlStepStat * max(n, 1))()
        done = ctypes.c_int32(0)
        st = dirac_lanczos_wait(self.ctx, stats if n else None, n, ctypes.byref(done))
        _check(self.lib, self.ctx, st)
        return stats_dict(stats[:n]) if want_stats else None

    def step_adaptive(self, psi, t0: float, t_end: float, dt_init: float, tol: float, dt_min: float,
                      dt_max: float, max_steps: int = 100000):
        """In-place propagation from t0 to t_end with adaptive step sizes
        (cumulative error estimate <= tol: the Krylov estimates plus the bound
        of the field's deviation from its step average).  Returns (stats
        dict, accepted step sizes)."""
        self._check_psi(psi)
        out = DlAdaptStat()
        dts = (ctypes.c_double * max_steps)()
        st = self.lib.dirac_lanczos_step_adaptive(self.ctx, ctypes.c_void_p(psi.data_ptr()), t0, t_end, dt_init,
                                                  tol, dt_min, dt_max, max_steps, dts, ctypes.byref(out))
        stats = {"accepted": out.accepted, "rejected": out.rejected, "t_reached": out.t_reached,
                 "dt_next": out.dt_next, "cum_bound": out.cum_bound, "norm2": out.norm2,
                 "cum_magnus": out.cum_magnus}
        _check(self.lib, self.ctx, st)
        return stats, np.array(dts[:out.accepted])

    def eigen(self, psi0, k_max: int, e_lo: float, e_hi: float, tol: float, n_wanted: int = 64,
              reorth: bool = False):
        self._check_psi(psi0)
        ev = (ctypes.c_double * n_wanted)()
        bd = (ctypes.c_double * n_wanted)()
        nf = ctypes.c_int32(0)
        st = dirac_lanczos_eigen(self.ctx, psi0.data_ptr(), k_max, int(bool(reorth)), e_lo, e_hi, tol,
                                 n_wanted, ev, bd, ctypes.byref(nf))
        _check(self.lib, self.ctx, st)
        return np.array(ev[:nf.value]), np.array(bd[:nf.value])

    def eigen_vectors(self, psi0, k_max: int, e_lo: float, e_hi: float, tol: float, n_wanted: int = 16):
        """Ritz values, bounds and Ritz vectors (full reorthogonalisation; the
        context needs k_eigen >= k_max and reorth=True).  Vectors: complex128
        tensor (n_found, 2, ny, nx), <psi0, y> real and positive."""
        self._check_psi(psi0)
        ev = (ctypes.c_double * n_wanted)()
        bd = (ctypes.c_double * n_wanted)()
        nf = ctypes.c_int32(0)
        vecs = self.torch.zeros((n_wanted,) + self.shape, dtype=self.torch.complex128, device="cuda")
        st = dirac_lanczos_eigen_vectors(self.ctx, psi0.data_ptr(), k_max, e_lo, e_hi, tol, n_wanted, ev, bd,
                                         ctypes.byref(nf), vecs.data_ptr())
        _check(self.lib, self.ctx, st)
        k = nf.value
        return np.array(ev[:k]), np.array(bd[:k]), vecs[:k]

    def adjoint(self, psi0, t0: float, dt: float, n_steps: int, ckpt_every: int, loss_kind: int):
        """Loss (sum of the final expectations selected by loss_kind) and its
        gradient with respect to the Fourier laser coefficients (numpy array in
        the order of problem["coef"]).  psi0 is not modified."""
        self._check_psi(psi0)
        nbytes = dirac_lanczos_adjoint_workspace_bytes(self.params, n_steps, ckpt_every)
        if nbytes == 0:
            raise DlError(DL_ERR_INVALID, "invalid adjoint arguments (adjoint_workspace_bytes returned 0)")
        ws = self.torch.empty(nbytes + 256, dtype=self.torch.uint8, device="cuda")
        ptr = (ws.data_ptr() + 255) & ~255
        ncoef = max(int(self.params.n_coef), 1)
        loss = ctypes.c_double(0.0)
        grad = (ctypes.c_double * ncoef)()
        st = dirac_lanczos_adjoint(self.ctx, psi0.data_ptr(), t0, dt, n_steps, ckpt_every, loss_kind,
                                   ptr, nbytes, ctypes.byref(loss), grad)
        _check(self.lib, self.ctx, st)
        del ws
        return float(loss.value), np.array(grad[:int(self.params.n_coef)])

    def set_launch(self, sweep_waves_per_cu: int) -> int:
        """Sweep launch shape (0: default); returns the waves per CU in use."""
        w = ctypes.c_int32(0)
        _check(self.lib, self.ctx, self.lib.dirac_lanczos_set_launch(self.ctx, int(sweep_waves_per_cu),
                                                                     ctypes.byref(w)))
        return int(w.value)

    def timing(self, enable: bool):
        """Start (True) or stop (False) event timing; returns the accumulated
        {class: (launches, total_ms)} collected so far."""
        t = DlTiming()
        _check(self.lib, self.ctx, dirac_lanczos_timing(self.ctx, int(bool(enable)), ctypes.byref(t)))
        return {name: (int(t.launches[i]), float(t.total_ms[i])) for i, name in enumerate(TIMING_CLASSES)}

    def close(self):
        if getattr(self, "ctx", None):
            dirac_lanczos_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPropagator:
    """A batch of independent packets (one dict per packet, keys as in
    packets.py) sharing krylov_dim, precision and bc_y; psi tensors are
    complex128 of shape (2, ny_i, nx_i), contiguous, on the GPU."""

    def __init__(self, problems, krylov_dim: int, precision: str = "fp64", stream=None, tuning_cache=None):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.prec = DL_PREC_MIXED if precision == "mixed" else DL_PREC_FP64
        self.n = len(problems)
        arr = (DlParams * self.n)()
        self._keep = []
        for i, prob in enumerate(problems):
            p, keep = make_params(prob, krylov_dim, self.prec)
            arr[i] = p
            self._keep.append(keep)
        self.params = arr
        nbytes = dirac_lanczos_batch_workspace_bytes(arr, self.n)
        if nbytes == 0:
            raise DlError(DL_ERR_INVALID, "invalid batch parameters (batch_workspace_bytes returned 0)")
        self.ws_bytes = nbytes
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        self.ws_ptr = (self.workspace.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.batch = dirac_lanczos_batch_init(arr, self.n, self.ws_ptr, nbytes, self.stream.cuda_stream)
        self.shapes = [(2, int(p["ny"]), int(p["nx"])) for p in problems]
        if tuning_cache:
            from . import autotune
            path = autotune.DEFAULT_CACHE if tuning_cache is True else tuning_cache
            best = autotune.lookup(autotune.key_batch(problems, krylov_dim, precision, autotune.device_arch()), path)
            if best is not None:
                self.set_launch(best)

    def step(self, psis, t0: float, dt: float, n_steps: int, want_stats: bool = True):
        """In-place propagation of every packet.  Returns per-packet stats dicts."""
        t = self.torch
        if len(psis) != self.n:
            raise ValueError(f"expected {self.n} states")
        for psi, shp in zip(psis, self.shapes):
            if not (isinstance(psi, t.Tensor) and psi.is_cuda and psi.dtype == t.complex128
                    and tuple(psi.shape) == shp and psi.is_contiguous()):
                raise ValueError(f"every psi must be a contiguous complex128 CUDA tensor of its packet's shape")
        stats = (DlStepStat * max(self.n * n_steps, 1))() if want_stats else None
        st = dirac_lanczos_batch_step(self.batch, [p.data_ptr() for p in psis], t0, dt, n_steps, stats)
        out = None
        if want_stats:
            out = []
            for i in range(self.n):
                out.append(stats_dict(stats[i * n_steps:(i + 1) * n_steps]))
        if st != DL_OK:
            raise DlError(st, dirac_lanczos_batch_last_error(self.batch))
        return out

    def set_launch(self, rows_per_chunk: int) -> int:
        """Rows per chunk of the batched sweeps (0: default); returns the value in use."""
        r = ctypes.c_int32(0)
        st = self.lib.dirac_lanczos_batch_set_launch(self.batch, int(rows_per_chunk), ctypes.byref(r))
        if st != DL_OK:
            raise DlError(st, dirac_lanczos_batch_last_error(self.batch))
        return int(r.value)

    def close(self):
        if getattr(self, "batch", None):
            dirac_lanczos_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Hermite pseudospectral problems (dl_hermite_params; spinors (2, n, n) of the
# collocation variables)
# ---------------------------------------------------------------------------
def _herm_check(st):
    if st != DL_OK:
        msg = load_library().dirac_lanczos_hermite_last_error()
        raise DlError(st, msg.decode() if msg else "")


def ritz(alpha, beta, e_lo: float, e_hi: float, tol: float, check_every: int = 64, n_wanted: int = 64):
    """Converged Ritz clusters of the tridiagonal (alpha, beta) in [e_lo, e_hi]
    (dirac_lanczos_ritz, host only): (values, bounds) numpy arrays."""
    lib = load_library()
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    be = np.ascontiguousarray(beta, dtype=np.float64)
    if al.shape != be.shape or al.ndim != 1:
        raise ValueError("alpha and beta must be 1-D arrays of one length")
    ev = np.zeros(max(int(n_wanted), 1))
    bd = np.zeros_like(ev)
    nf = ctypes.c_int32(0)
    D = ctypes.POINTER(ctypes.c_double)
    st = lib.dirac_lanczos_ritz(al.ctypes.data_as(D), be.ctypes.data_as(D), int(len(al)), float(e_lo), float(e_hi),
                                float(tol), int(check_every), int(n_wanted), ev.ctypes.data_as(D),
                                bd.ctypes.data_as(D), ctypes.byref(nf))
    if st != DL_OK:
        raise DlError(st, "invalid arguments of dirac_lanczos_ritz")
    return ev[:nf.value].copy(), bd[:nf.value].copy()


def hermite_nodes(n: int, scale: float):
    """Collocation points and weights of the library (numpy arrays)."""
    lib = load_library()
    x = np.zeros(n)
    w = np.zeros(n)
    _herm_check(lib.dirac_lanczos_hermite_nodes(int(n), float(scale), x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return x, w


def hermite_apply(hprob: dict, x, stream=None):
    """y = H x for a Hermite problem (x: complex128 CUDA tensor (2, n, n))."""
    import torch
    lib = load_library()
    p = make_hermite_params(hprob)
    nb = int(lib.dirac_lanczos_hermite_workspace_bytes(ctypes.byref(p), 1, 1))
    if nb == 0:
        raise DlError(DL_ERR_INVALID, "invalid Hermite parameters")
    ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    ptr = (ws.data_ptr() + 255) & ~255
    y = torch.empty_like(x)
    st = stream if stream is not None else torch.cuda.current_stream()
    _herm_check(lib.dirac_lanczos_hermite_apply(ctypes.byref(p), ctypes.c_void_p(x.data_ptr()),
                                                ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(ptr), nb,
                                                ctypes.c_void_p(st.cuda_stream)))
    return y


def hermite_eigen(hprobs, psi0s, k_max: int, e_lo, e_hi, tol: float, n_wanted: int = 16, stream=None):
    """Eigenvalue mode for a batch of Hermite problems (one start vector and
    window per problem).  Returns a list of (values, bounds) numpy pairs."""
    import torch
    lib = load_library()
    n = len(hprobs)
    arr = (DlHermiteParams * n)(*[make_hermite_params(h) for h in hprobs])
    nb = int(lib.dirac_lanczos_hermite_workspace_bytes(arr, n, int(k_max)))
    if nb == 0:
        raise DlError(DL_ERR_INVALID, "invalid Hermite parameters")
    ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    ptr = (ws.data_ptr() + 255) & ~255
    ptrs = (ctypes.c_void_p * n)(*[ctypes.c_void_p(p.data_ptr()) for p in psi0s])
    lo = (ctypes.c_double * n)(*[float(v) for v in e_lo])
    hi = (ctypes.c_double * n)(*[float(v) for v in e_hi])
    ev = (ctypes.c_double * (n * n_wanted))()
    bd = (ctypes.c_double * (n * n_wanted))()
    nf = (ctypes.c_int32 * n)()
    st = stream if stream is not None else torch.cuda.current_stream()
    _herm_check(lib.dirac_lanczos_hermite_eigen(arr, n, ptrs, int(k_max), lo, hi, float(tol), int(n_wanted),
                                                ctypes.c_void_p(ptr), nb, ctypes.c_void_p(st.cuda_stream), ev, bd,
                                                nf))
    return [(np.array(ev[i * n_wanted:i * n_wanted + nf[i]]), np.array(bd[i * n_wanted:i * n_wanted + nf[i]]))
            for i in range(n)]
