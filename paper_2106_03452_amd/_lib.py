"""ctypes binding of ``libpsr.so`` (argument marshalling only).

Every step of the solve runs in the HIP library; this module only checks
tensor properties, allocates device buffers through PyTorch's caching
allocator and passes raw pointers and the current HIP stream to the C ABI
declared in ``include/psr.h``. There is no CPU fallback: if the library is
missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os
import re
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
# PSR_LIBRARY overrides the library path (A/B comparisons of build variants)
LIB_PATH = os.environ.get("PSR_LIBRARY") or os.path.join(HERE, "libpsr.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "psr.h")

PSR_OK = 0
PSR_EINVAL = -1
PSR_ENOMEM = -2
PSR_EDEGENERATE = -3
PSR_EDEVICE = -4
PSR_ENOTREADY = -5
PSR_ENONFINITE = -6
PSR_ETOOBIG = -7
PSR_JOB_FORWARD = 0
PSR_JOB_BACKWARD = 2


class PSRError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


class PsrJob(ctypes.Structure):
    _fields_ = [
        ("points", ctypes.c_void_p),
        ("normals", ctypes.c_void_p),
        ("npoints", ctypes.c_int64),
        ("res", ctypes.c_int),
        ("sigma", ctypes.c_float),
        ("chi", ctypes.c_void_p),
        ("saved", ctypes.c_void_p),
        ("dchi", ctypes.c_void_p),
        ("dpoints", ctypes.c_void_p),
        ("dnormals", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("stages", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


_lib = None
_lock = threading.Lock()


def _declare(L):
    vp, i32, i64, f32, f64, sz = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_float,
                                  ctypes.c_double, ctypes.c_size_t)
    P = ctypes.POINTER
    sigs = {
        "psr_version": ([], i32),
        "psr_strerror": ([i32], ctypes.c_char_p),
        "psr_ctx_create": ([P(vp), i32], i32),
        "psr_ctx_destroy": ([vp], i32),
        "psr_ctx_set": ([vp, ctypes.c_char_p, f64], i32),
        "psr_ctx_get": ([vp, ctypes.c_char_p, P(f64)], i32),
        "psr_workspace_bytes": ([i32, i64, i32, P(sz)], i32),
        "psr_saved_bytes": ([i32, i64, P(sz)], i32),
        "psr_forward": ([vp, vp, vp, i64, i32, f32, vp, vp, vp, sz, vp], i32),
        "psr_forward_static": ([vp, vp, vp, i64, i32, f32, vp, vp], i32),
        "psr_backward": ([vp, i64, i32, f32, vp, vp, vp, vp, vp, vp, sz, vp], i32),
        "psr_ctx_prepare": ([vp, i32, f32, vp], i32),
        "psr_saved_status": ([vp, vp, P(i32)], i32),
        "psr_saved_scalars": ([vp, vp, P(f64), P(f64), P(f64), P(f64)], i32),
        "psr_run_batched": ([vp, i32, P(PsrJob), vp], i32),
        "psr_debug_spectral": ([vp, vp, i32, f32, vp, vp, sz, vp], i32),
        "psr_debug_splat": ([vp, vp, vp, i64, i32, vp, vp, vp, sz, vp], i32),
        "psr_slab_workspace_bytes": ([i32, i64, i32, P(sz)], i32),
        "psr_slab_forward": ([vp, vp, vp, i64, i32, f32, i32, vp, vp, vp, sz, vp], i32),
        "psr_slab_debug_spectral": ([vp, vp, i32, f32, i32, vp, vp, sz, vp], i32),
        "psr_mc_state_bytes": ([i32, P(sz)], i32),
        "psr_marching_cubes": ([vp, vp, i32, f32, vp, vp, vp, i64, vp, i64, vp, vp], i32),
        "psr_mc_counts": ([vp, vp, P(i64), P(i64), P(i32)], i32),
        "psr_marching_cubes_backward": ([vp, vp, i32, f32, vp, vp, vp, i64, vp, vp], i32),
        "psr_mc_case_table": ([vp, vp], i32),
        "psr_mesh_sample_workspace_bytes": ([i64, P(sz)], i32),
        "psr_mesh_sample": ([vp, vp, vp, i64, vp, i64, vp, vp, i64, vp, vp, vp, vp, vp, sz, vp], i32),
        "psr_mesh_sample_backward": ([vp, vp, i64, vp, vp, vp, i64, vp, vp], i32),
        "psr_chamfer_workspace_bytes": ([i64, i64, P(sz)], i32),
        "psr_chamfer": ([vp, vp, i64, vp, i64, vp, vp, vp, vp, vp, vp, sz, vp], i32),
        "psr_chamfer_backward": ([vp, vp, i64, vp, i64, vp, vp, vp, vp], i32),
        "psr_mesh_components_workspace_bytes": ([i64, i64, P(sz)], i32),
        "psr_mesh_components": ([vp, vp, i64, vp, i64, vp, vp, vp, sz, vp], i32),
        "psr_opt_step_workspace_bytes": ([i32, i64, i64, i64, i64, i64, P(sz)], i32),
        "psr_opt_step": ([vp, vp, vp, i64, vp, vp, vp, vp, i64, f32, f32, f32, f32, vp, i64, vp, i64, i32, f32,
                          i64, i64, vp, P(i64), vp, sz, vp], i32),
        "psr_ctx_stage_times": ([vp, P(f64), P(i64), i32], i32),
        "psr_ctx_reset_timers": ([vp], i32),
        "psr_stage_name": ([i32], ctypes.c_char_p),
        "psr_num_stages": ([], i32),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res


def lib():
    """Load ``libpsr.so`` (once). Raises ImportError if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(
                    f"{LIB_PATH} is missing: build the HIP library first "
                    "(python -m paper_2106_03452_amd.build, or __graft_entry__.build())")
            L = ctypes.CDLL(LIB_PATH)
            _declare(L)
            _lib = L
    return _lib


def header_symbols() -> list[str]:
    """Names of the functions that include/psr.h declares."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*|int64_t|void)\s+(psr_\w+)\s*\(", txt, re.M)))


def strerror(code: int) -> str:
    try:
        return lib().psr_strerror(int(code)).decode()
    except ImportError:
        return "libpsr.so not loaded"


def check(code: int, what: str) -> None:
    if code != PSR_OK:
        raise PSRError(code, what)


def workspace_bytes(res: int, npoints: int, with_backward: bool = True) -> int:
    out = ctypes.c_size_t(0)
    check(lib().psr_workspace_bytes(int(res), int(npoints), int(with_backward), ctypes.byref(out)),
          "psr_workspace_bytes")
    return int(out.value)


def saved_bytes(res: int, npoints: int) -> int:
    out = ctypes.c_size_t(0)
    check(lib().psr_saved_bytes(int(res), int(npoints), ctypes.byref(out)), "psr_saved_bytes")
    return int(out.value)


class Context:
    """Owns one ``psr_ctx`` (twiddle tables and options) on one HIP device."""

    def __init__(self, device: int = 0):
        self.device = int(device)
        h = ctypes.c_void_p()
        check(lib().psr_ctx_create(ctypes.byref(h), self.device), "psr_ctx_create")
        self.handle = h

    def set(self, key: str, value: float) -> None:
        check(lib().psr_ctx_set(self.handle, key.encode(), float(value)), f"psr_ctx_set({key})")

    def get(self, key: str) -> float:
        v = ctypes.c_double(0.0)
        check(lib().psr_ctx_get(self.handle, key.encode(), ctypes.byref(v)), f"psr_ctx_get({key})")
        return float(v.value)

    def stage_times(self) -> dict:
        L = lib()
        n = L.psr_num_stages()
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        check(L.psr_ctx_stage_times(self.handle, ms, cnt, n), "psr_ctx_stage_times")
        return {L.psr_stage_name(i).decode(): (float(ms[i]), int(cnt[i])) for i in range(n)}

    def reset_timers(self) -> None:
        check(lib().psr_ctx_reset_timers(self.handle), "psr_ctx_reset_timers")

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib().psr_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_contexts: dict[int, Context] = {}


def context(device: int = 0) -> Context:
    """Process-wide context per device (created on first use)."""
    with _lock:
        c = _contexts.get(int(device))
    if c is None:
        c = Context(device)
        with _lock:
            _contexts.setdefault(int(device), c)
            c = _contexts[int(device)]
    return c
