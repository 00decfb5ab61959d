"""Leverage-score-sampled tensor-ring ALS on MI355X (gfx950).

``TRALS`` wraps one handle of the C ABI (``include/trals.h``).  PyTorch
supplies the device memory (the caller-owned workspace, the data tensor,
core buffers) and the stream; every step of the method runs in the library's
HIP kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import TRALS_F32, TRALS_F64, TRALS_BF16, TRALS_BF16_CHAINS, TralsError  # noqa: F401

_PREC = {"f64": TRALS_F64, "f32": TRALS_F32, "bf16": TRALS_BF16, "bf16c": TRALS_BF16_CHAINS}
_METHOD = {"leverage": _lib.TRALS_LEVERAGE, "uniform": _lib.TRALS_UNIFORM, "exact": _lib.TRALS_EXACT}


def _torch():
    import torch
    return torch


def torch_device(d):
    return _torch().device(d)


def fit_error_noalloc(X, cores_flat, ranks, out, stream=None):
    """trals_fit_error_noalloc: enqueue ||TR(G) - X||_F / ||X||_F into ``out`` (a one-element
    float64 CUDA tensor) on ``stream`` (default: X's current stream); nothing is allocated or
    synchronised.  X: float32/float64 CUDA tensor in C order.  cores_flat: contiguous
    float32/float64 CUDA tensor holding the N cores (R[n-1], I[n], R[n]) one after the other.
    ranks: R[0..N-1]."""
    torch = _torch()
    lib = _lib.load()
    dims = tuple(int(v) for v in X.shape)
    N = len(dims)
    code = {torch.float64: TRALS_F64, torch.float32: TRALS_F32}
    d_arr = (C.c_int64 * N)(*dims)
    r_arr = (C.c_int32 * N)(*[int(r) for r in ranks])
    st = torch.cuda.current_stream(X.device) if stream is None else stream
    _lib.check(lib.trals_fit_error_noalloc(N, d_arr, r_arr, C.c_void_p(cores_flat.data_ptr()),
                                           code[cores_flat.dtype], C.c_void_p(X.data_ptr()), code[X.dtype],
                                           C.c_void_p(out.data_ptr()), C.c_void_p(st.cuda_stream)),
               "trals_fit_error_noalloc")


class TRALS:
    """One sampled TR-ALS problem held on the GPU.

    X: CUDA tensor (float32 or float64), C order.  ranks: R[0..N-1] (core n is
    R[n-1] x I[n] x R[n]).  samples: J per core update.  precision: "f64",
    "f32", "bf16" or "bf16c" (the BF16 form with its subchain products on BF16
    matrix cores as well).  init_cores: optional list of N tensors (any device) of
    shapes (R[n-1], I[n], R[n]); None draws N(0,1) entries on the GPU.
    method: "leverage" (Algorithm 2), "uniform" (Algorithm 2 with uniform
    sampling) or "exact" (Algorithm 1; samples is ignored).  normalize:
    orthonormalise each updated core along its bond to the next (QR, R moved
    into the next core); TR(G) and the sampling are unchanged.
    """

    def __init__(self, X, ranks, samples, seed=0, stream_id=0, precision="f32", init_cores=None,
                 stream=None, source=None, method="leverage", normalize=False, workspace=None):
        torch = _torch()
        self.lib = _lib.load()
        self.method = method
        self.normalize = bool(normalize)
        self._arena = workspace  # optional preallocated uint8 CUDA tensor for the workspace
        if source is not None:
            self._init_generated(source, ranks, samples, seed, stream_id, precision, init_cores, stream)
            return
        if not X.is_cuda:
            raise ValueError("X must be a CUDA tensor")
        X = X.contiguous()
        self.dims = tuple(int(v) for v in X.shape)
        self.ranks = tuple(int(v) for v in ranks)
        self.N = len(self.dims)
        self.J = int(samples)
        self.precision = precision
        self.device = X.device
        self.stream = torch.cuda.current_stream(X.device) if stream is None else stream
        xdt = {torch.float64: TRALS_F64, torch.float32: TRALS_F32}[X.dtype]
        init_ptr, init_dt, init_buf = None, TRALS_F64, None
        if init_cores is not None:
            init_buf = torch.cat([torch.as_tensor(np.asarray(c) if not isinstance(c, torch.Tensor) else c)
                                  .to(device=X.device, dtype=torch.float64).reshape(-1) for c in init_cores])
            init_ptr = init_buf.data_ptr()
        desc, self._keep = _lib.make_desc(self.dims, self.ranks, self.J, seed, stream_id, _PREC[precision],
                                          init_ptr, init_dt, _METHOD[method], self.normalize)
        nbytes = C.c_size_t(0)
        _lib.check(self.lib.trals_workspace_bytes(C.byref(desc), C.byref(nbytes)), "trals_workspace_bytes")
        self.workspace = self._take_workspace(int(nbytes.value), X.device)
        h = C.c_void_p(0)
        _lib.check(self.lib.trals_create(C.byref(desc), C.c_void_p(X.data_ptr()), xdt,
                                         C.c_void_p(self.workspace.data_ptr()), nbytes,
                                         C.c_void_p(self.stream.cuda_stream), C.byref(h)), "trals_create")
        self.h = h
        self.core_shapes = [(self.ranks[(n - 1) % self.N], self.dims[n], self.ranks[n]) for n in range(self.N)]

    @classmethod
    def generated(cls, true_cores, ranks, samples, noise_rel=0.0, noise_seed=0, noise_stream=0,
                  seed=0, stream_id=0, precision="f32", init_cores=None, stream=None, device=None,
                  method="leverage", normalize=False, workspace=None):
        """Handle whose data is TR(true_cores) + noise, generated fiber by fiber on the GPU
        (never materialised).  true_cores: list of N arrays/tensors (R[n-1], I[n], R[n])."""
        src = dict(true_cores=true_cores, noise_rel=noise_rel, noise_seed=noise_seed,
                   noise_stream=noise_stream, device=device)
        return cls(None, ranks, samples, seed=seed, stream_id=stream_id, precision=precision,
                   init_cores=init_cores, stream=stream, source=src, method=method, normalize=normalize,
                   workspace=workspace)

    def _init_generated(self, source, ranks, samples, seed, stream_id, precision, init_cores, stream):
        torch = _torch()
        tc = source["true_cores"]
        dev = source.get("device") or (tc[0].device if isinstance(tc[0], torch.Tensor) and tc[0].is_cuda
                                        else torch.device("cuda", torch.cuda.current_device()))
        self.dims = tuple(int(c.shape[1]) for c in tc)
        self.ranks = tuple(int(v) for v in ranks)
        self.N = len(self.dims)
        self.J = int(samples)
        self.precision = precision
        self.device = dev
        self.stream = torch.cuda.current_stream(dev) if stream is None else stream
        true_ranks = [int(c.shape[2]) for c in tc]
        init_ptr, init_buf = None, None
        if init_cores is not None:
            init_buf = torch.cat([torch.as_tensor(np.asarray(c) if not isinstance(c, torch.Tensor) else c)
                                  .to(device=dev, dtype=torch.float64).reshape(-1) for c in init_cores])
            init_ptr = init_buf.data_ptr()
        desc, keep = _lib.make_desc(self.dims, self.ranks, self.J, seed, stream_id, _PREC[precision],
                                    init_ptr, TRALS_F64, _METHOD[self.method], self.normalize)
        sizing, keep2 = _lib.make_source(None, TRALS_F64, true_ranks, source["noise_rel"], source["noise_seed"],
                                         source["noise_stream"])
        nbytes = C.c_size_t(0)
        _lib.check(self.lib.trals_workspace_bytes_generated(C.byref(desc), C.byref(sizing), C.byref(nbytes)),
                   "trals_workspace_bytes_generated")
        self.workspace_bytes = int(nbytes.value)
        # true cores (FP64, concatenated): behind the workspace in the arena when it has room
        n_true = sum(int(np.prod(c.shape)) for c in tc)
        off = (self.workspace_bytes + 255) // 256 * 256
        a = self._arena
        if a is not None and a.device == torch_device(dev) and a.numel() >= off + 8 * n_true:
            self.workspace = a[:self.workspace_bytes]
            self._true_buf = a[off:off + 8 * n_true].view(torch.float64)
            if all(not isinstance(c, torch.Tensor) for c in tc):
                flat = np.concatenate([np.asarray(c, dtype=np.float64).reshape(-1) for c in tc])
                self._true_buf.copy_(torch.from_numpy(flat))
            else:
                self._true_buf.copy_(torch.cat([torch.as_tensor(c).to(device=dev, dtype=torch.float64).reshape(-1)
                                                for c in tc]))
        else:
            self.workspace = self._take_workspace(self.workspace_bytes, dev)
            if all(not isinstance(c, torch.Tensor) for c in tc):
                flat = np.concatenate([np.asarray(c, dtype=np.float64).reshape(-1) for c in tc])
                self._true_buf = torch.from_numpy(flat).to(device=dev)
            else:
                self._true_buf = torch.cat([torch.as_tensor(np.asarray(c) if not isinstance(c, torch.Tensor) else c)
                                            .to(device=dev, dtype=torch.float64).reshape(-1) for c in tc])
        src, keep3 = _lib.make_source(self._true_buf.data_ptr(), TRALS_F64, true_ranks, source["noise_rel"],
                                      source["noise_seed"], source["noise_stream"])
        self._keep = (keep, keep2, keep3, init_buf)
        h = C.c_void_p(0)
        _lib.check(self.lib.trals_create_generated(C.byref(desc), C.byref(src), C.c_void_p(self.workspace.data_ptr()),
                                                   nbytes, C.c_void_p(self.stream.cuda_stream), C.byref(h)),
                   "trals_create_generated")
        self.h = h
        self.core_shapes = [(self.ranks[(n - 1) % self.N], self.dims[n], self.ranks[n]) for n in range(self.N)]

    def _take_workspace(self, nbytes, device):
        a = self._arena
        if a is not None and a.numel() >= nbytes and a.device == torch_device(device):
            return a[:nbytes]
        return _torch().empty(nbytes, dtype=_torch().uint8, device=device)

    # -- driving the iteration --
    def sweep(self, n=1):
        _lib.check(self.lib.trals_sweep(self.h, int(n)), "trals_sweep")

    def sweep_async(self, n=1, fit=False):
        """Enqueue n sweeps on the handle's stream without waiting (see query); fit=True also
        enqueues the relative error, available from async_fit once query() is True."""
        flags = _lib.TRALS_ASYNC_FIT if fit else 0
        _lib.check(self.lib.trals_sweep_async(self.h, int(n), flags), "trals_sweep_async")
        self.async_fit = None

    def query(self) -> bool:
        """True once the enqueued work has finished (raises if a solve failed)."""
        out = C.c_double(0.0)
        rc = self.lib.trals_query(self.h, C.byref(out))
        if rc == _lib.TRALS_PENDING:
            return False
        _lib.check(rc, "trals_query")
        self.async_fit = float(out.value)
        return True

    def step(self, n=1):
        _lib.check(self.lib.trals_step(self.h, int(n)), "trals_step")

    def set_samples(self, J):
        """Sample count of the following updates (at most the J given at creation)."""
        _lib.check(self.lib.trals_set_samples(self.h, int(J)), "trals_set_samples")
        self.J = int(J)

    def tr_norm(self) -> float:
        """||TR(G)||_F of the current cores (transfer matrices on the GPU)."""
        out = C.c_double(0.0)
        _lib.check(self.lib.trals_tr_norm(self.h, C.byref(out)), "trals_tr_norm")
        return float(out.value)

    def sweep_until(self, max_sweeps, rel_tol):
        """Sweeps until the relative change of ||TR(G)||_F falls below rel_tol; returns
        (sweeps run, last relative change)."""
        done, change = C.c_int32(0), C.c_double(0.0)
        _lib.check(self.lib.trals_sweep_until(self.h, int(max_sweeps), float(rel_tol), C.byref(done),
                                              C.byref(change)), "trals_sweep_until")
        return int(done.value), float(change.value)

    def fit_estimate(self, samples, tag=0) -> float:
        """Relative error estimated from `samples` uniformly drawn entries of X (Section 3.1)."""
        out = C.c_double(0.0)
        _lib.check(self.lib.trals_fit_estimate(self.h, int(samples), int(tag), C.byref(out)), "trals_fit_estimate")
        return float(out.value)

    def sweep_until_estimate(self, max_sweeps, rel_tol, samples):
        """Sweeps until the relative change of the sampled error estimate falls below rel_tol;
        returns (sweeps run, last estimate, last relative change)."""
        done, est, change = C.c_int32(0), C.c_double(0.0), C.c_double(0.0)
        _lib.check(self.lib.trals_sweep_until_estimate(self.h, int(max_sweeps), float(rel_tol), int(samples),
                                                       C.byref(done), C.byref(est), C.byref(change)),
                   "trals_sweep_until_estimate")
        return int(done.value), float(est.value), float(change.value)

    def fit_error(self) -> float:
        out = C.c_double(0.0)
        _lib.check(self.lib.trals_fit_error(self.h, C.byref(out)), "trals_fit_error")
        return float(out.value)

    @property
    def update_counter(self) -> int:
        return int(self.lib.trals_update_counter(self.h))

    @update_counter.setter
    def update_counter(self, v):
        _lib.check(self.lib.trals_set_update_counter(self.h, int(v)), "trals_set_update_counter")

    # -- state --
    def get_cores(self, dtype=None):
        torch = _torch()
        dtype = dtype or torch.float64
        total = sum(a * b * c for a, b, c in self.core_shapes)
        buf = torch.empty(total, dtype=dtype, device=self.device)
        code = TRALS_F64 if dtype == torch.float64 else TRALS_F32
        _lib.check(self.lib.trals_get_cores(self.h, C.c_void_p(buf.data_ptr()), code), "trals_get_cores")
        out, off = [], 0
        for s in self.core_shapes:
            cnt = s[0] * s[1] * s[2]
            out.append(buf[off:off + cnt].reshape(s))
            off += cnt
        return out

    def set_cores(self, cores):
        torch = _torch()
        buf = torch.cat([torch.as_tensor(c).to(device=self.device, dtype=torch.float64).reshape(-1) for c in cores])
        _lib.check(self.lib.trals_set_cores(self.h, C.c_void_p(buf.data_ptr()), TRALS_F64), "trals_set_cores")

    def last_samples(self):
        idx = np.empty((self.J, self.N - 1), dtype=np.int32)
        w = np.empty(self.J, dtype=np.float64)
        _lib.check(self.lib.trals_get_last_samples(self.h, idx.ctypes.data_as(C.c_void_p),
                                                   w.ctypes.data_as(C.c_void_p)), "trals_get_last_samples")
        return idx, w

    def profile(self, enable=True):
        """Time every kernel group with HIP events on the handle's stream."""
        _lib.check(self.lib.trals_profile(self.h, int(bool(enable))), "trals_profile")

    def profile_read(self, kernel):
        """(total ms, launches) of a kernel group since profiling was enabled."""
        ms, cnt = C.c_double(0.0), C.c_int64(0)
        _lib.check(self.lib.trals_profile_read(self.h, _lib.KERNELS[kernel], C.byref(ms), C.byref(cnt)),
                   "trals_profile_read")
        return float(ms.value), int(cnt.value)

    def close(self):
        if getattr(self, "h", None):
            self.lib.trals_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
