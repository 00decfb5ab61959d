"""ctypes binding of ``libtrals.so`` (the C ABI in ``include/trals.h``).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtrals.so")

TRALS_OK, TRALS_EINVAL, TRALS_ENOMEM, TRALS_ESINGULAR, TRALS_EHIP, TRALS_ESTATE = 0, -1, -2, -3, -4, -5
TRALS_ERANGE = -6
TRALS_NOALLOC_SCRATCH_BYTES = 16 << 20
TRALS_PENDING = 1
TRALS_ASYNC_FIT = 1
TRALS_F64, TRALS_F32, TRALS_BF16, TRALS_BF16_CHAINS = 0, 1, 2, 3
TRALS_LEVERAGE, TRALS_UNIFORM, TRALS_EXACT = 0, 1, 2

# every symbol include/trals.h declares
EXPORTS = (
    "trals_workspace_bytes", "trals_create", "trals_sweep", "trals_step", "trals_fit_error",
    "trals_destroy", "trals_get_cores", "trals_set_cores", "trals_get_last_samples",
    "trals_update_counter", "trals_set_update_counter", "trals_strerror", "trals_profile",
    "trals_profile_read", "trals_workspace_bytes_generated", "trals_create_generated",
    "trals_sweep_async", "trals_query", "trals_set_samples", "trals_samples", "trals_tr_norm",
    "trals_sweep_until", "trals_fit_error_noalloc", "trals_fit_estimate", "trals_sweep_until_estimate",
)
KERNELS = {"draw": 0, "contract": 1, "reduce": 2, "factor": 3, "solve": 4, "table": 5}


class Desc(C.Structure):
    _fields_ = [
        ("order", C.c_int32),
        ("dims", C.POINTER(C.c_int64)),
        ("ranks", C.POINTER(C.c_int32)),
        ("samples", C.c_int64),
        ("seed", C.c_uint64),
        ("stream_id", C.c_uint64),
        ("precision", C.c_int32),
        ("init_cores", C.c_void_p),
        ("init_dtype", C.c_int32),
        ("method", C.c_int32),
        ("normalize", C.c_int32),
    ]


class Source(C.Structure):
    _fields_ = [
        ("true_cores", C.c_void_p),
        ("true_dtype", C.c_int32),
        ("true_ranks", C.POINTER(C.c_int32)),
        ("noise_rel", C.c_double),
        ("noise_seed", C.c_uint64),
        ("noise_stream", C.c_uint64),
    ]


class TralsError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


_lib = None


def load(path: str = LIB_PATH):
    """Load the library once (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_2010_08581_amd/build.py (or __graft_entry__.build())")
    lib = C.CDLL(path)
    vp, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
    sig = {
        "trals_workspace_bytes": (C.c_int, [C.POINTER(Desc), C.POINTER(C.c_size_t)]),
        "trals_create": (C.c_int, [C.POINTER(Desc), vp, i32, vp, C.c_size_t, vp, C.POINTER(vp)]),
        "trals_sweep": (C.c_int, [vp, i32]),
        "trals_step": (C.c_int, [vp, i32]),
        "trals_fit_error": (C.c_int, [vp, C.POINTER(C.c_double)]),
        "trals_destroy": (C.c_int, [vp]),
        "trals_get_cores": (C.c_int, [vp, vp, i32]),
        "trals_set_cores": (C.c_int, [vp, vp, i32]),
        "trals_get_last_samples": (C.c_int, [vp, vp, vp]),
        "trals_update_counter": (i64, [vp]),
        "trals_set_update_counter": (C.c_int, [vp, i64]),
        "trals_strerror": (C.c_char_p, [C.c_int]),
        "trals_profile": (C.c_int, [vp, i32]),
        "trals_profile_read": (C.c_int, [vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
        "trals_workspace_bytes_generated": (C.c_int, [C.POINTER(Desc), C.POINTER(Source), C.POINTER(C.c_size_t)]),
        "trals_sweep_async": (C.c_int, [vp, i32, i32]),
        "trals_query": (C.c_int, [vp, C.POINTER(C.c_double)]),
        "trals_set_samples": (C.c_int, [vp, i64]),
        "trals_samples": (i64, [vp]),
        "trals_tr_norm": (C.c_int, [vp, C.POINTER(C.c_double)]),
        "trals_sweep_until": (C.c_int, [vp, i32, C.c_double, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
        "trals_create_generated": (C.c_int, [C.POINTER(Desc), C.POINTER(Source), vp, C.c_size_t, vp, C.POINTER(vp)]),
        "trals_fit_error_noalloc": (C.c_int, [i32, C.POINTER(C.c_int64), C.POINTER(C.c_int32), vp, i32, vp, i32,
                                              vp, vp]),
        "trals_fit_estimate": (C.c_int, [vp, i64, u64, C.POINTER(C.c_double)]),
        "trals_sweep_until_estimate": (C.c_int, [vp, i32, C.c_double, i64, C.POINTER(C.c_int32),
                                                 C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().trals_strerror(int(code)).decode()


def check(code: int, what: str):
    if code != TRALS_OK:
        raise TralsError(code, what)


def make_desc(dims, ranks, samples, seed=0, stream_id=0, precision=TRALS_F32, init_ptr=None,
              init_dtype=TRALS_F64, method=TRALS_LEVERAGE, normalize=False):
    """Build a Desc plus the host arrays it points to (keep the tuple alive)."""
    N = len(dims)
    d_arr = (C.c_int64 * N)(*[int(v) for v in dims])
    r_arr = (C.c_int32 * N)(*[int(v) for v in ranks])
    desc = Desc(N, d_arr, r_arr, int(samples), int(seed), int(stream_id), int(precision),
                C.c_void_p(init_ptr) if init_ptr else None, int(init_dtype), int(method), int(bool(normalize)))
    return desc, (d_arr, r_arr)


def workspace_bytes(dims, ranks, samples, precision=TRALS_F32, method=TRALS_LEVERAGE):
    desc, keep = make_desc(dims, ranks, samples, precision=precision, method=method)
    out = C.c_size_t(0)
    check(load().trals_workspace_bytes(C.byref(desc), C.byref(out)), "trals_workspace_bytes")
    return int(out.value)


def make_source(true_ptr, true_dtype, true_ranks, noise_rel, noise_seed, noise_stream):
    """Build a Source plus the host array it points to (keep the tuple alive)."""
    r_arr = None
    if true_ranks is not None:
        r_arr = (C.c_int32 * len(true_ranks))(*[int(v) for v in true_ranks])
    src = Source(C.c_void_p(true_ptr), int(true_dtype), r_arr, float(noise_rel), int(noise_seed),
                 int(noise_stream))
    return src, (r_arr,)
