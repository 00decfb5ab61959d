"""Seeded synthetic inputs for sampled tensor-ring ALS experiments.

This module only *makes data*: random tensor-ring (TR) cores, dense tensors
assembled from them, noise, a video-shaped tensor of moving Gaussian blobs and
a stream of serving requests.  It holds none of the decomposition method's
arithmetic (no leverage scores, sampling, subchain sketches or least-squares
solves) and it imports neither the oracle nor the GPU package, so both can use
it without sharing any code with each other.

Conventions shared by every generator:

* A tensor is a C-order array ``X[i_0, ..., i_{N-1}]`` (last index fastest).
* Core ``n`` has shape ``(R[n-1], I[n], R[n])`` with the cyclic convention
  ``R[-1] = R[N-1]`` (the ring closure of the TR format, eq. (1) of the
  paper, Section 2.1).
* All randomness comes from ``numpy.random.default_rng`` seeded with a
  ``(seed, tag)`` pair so that the true cores, the noise and the ALS
  initialisation are independent streams of one seed.

Workload recipes (the sizes, distributions and noise models of the paper's
synthetic experiments, Section 4.1.1, and of the stand-ins for its image/video
datasets, Section 4.1.3):

* ``ring_tensor``: cores with iid N(0,1) entries contracted into a dense tensor.
* ``add_noise_abs``: iid Gaussian noise of a fixed standard deviation.
* ``add_noise_rel``: Gaussian noise scaled to a given fraction of ``||X||_F``.
* ``video_tensor``: H x W x C x T frames of K smooth Gaussian blobs moving on
  straight lines, plus uniform noise, clipped to [0, 1].
* ``serving_requests``: Poisson arrivals of small decomposition requests.
* ``oscillatory_tensor``: a highly oscillatory function sampled at 4^10 points and
  reshaped to a 10-way 4 x ... x 4 tensor (Section 4.1.2).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng_for",
    "core_shapes",
    "random_cores",
    "ring_tensor",
    "add_noise_abs",
    "add_noise_rel",
    "video_tensor",
    "serving_requests",
    "serving_true_cores",
    "OSC_FUNCTIONS",
    "oscillatory_tensor",
    "CONFIGS",
    "make_config",
]

# Stream tags for default_rng((seed, tag)).
TAG_TRUE_CORES = 1
TAG_NOISE = 2
TAG_INIT = 3
TAG_VIDEO = 4
TAG_SERVE = 5


def rng_for(seed: int, tag: int) -> np.random.Generator:
    """Independent generator for one (seed, purpose) pair."""
    return np.random.default_rng([int(seed), int(tag)])


def core_shapes(dims, ranks):
    """Shapes ``(R[n-1], I[n], R[n])`` of the N cores of a TR format."""
    N = len(dims)
    if len(ranks) != N:
        raise ValueError("need one rank per mode")
    return [(int(ranks[(n - 1) % N]), int(dims[n]), int(ranks[n])) for n in range(N)]


def random_cores(dims, ranks, rng: np.random.Generator, dtype=np.float64):
    """Cores with iid standard normal entries (the paper's initialisation and
    synthetic-data model, Sections 3 and 4.1.1)."""
    return [rng.standard_normal(s).astype(dtype) for s in core_shapes(dims, ranks)]


def ring_tensor(cores, dtype=np.float64):
    """Dense tensor whose entries are the ring contraction of ``cores``.

    Used only to *build* synthetic inputs.  The contraction walks the ring
    left to right, keeping an array ``W[a, i_0, ..., i_k, c]`` (first and last
    bond index), and closes the ring with one matrix product at the end.
    """
    N = len(cores)
    W = np.asarray(cores[0], dtype=np.float64)  # (R_{-1}, I_0, R_0)
    for n in range(1, N - 1):
        G = np.asarray(cores[n], dtype=np.float64)
        a, *mid, b = W.shape
        W = (W.reshape(-1, b) @ G.reshape(b, -1)).reshape(a, *mid, G.shape[1], G.shape[2])
    G = np.asarray(cores[N - 1], dtype=np.float64)  # (R_{N-2}, I_{N-1}, R_{-1})
    a = W.shape[0]
    b = W.shape[-1]
    mid = W.shape[1:-1]
    # X[mid, i] = sum_{a, b} W[a, mid, b] * G[b, i, a]
    Wm = np.moveaxis(W, 0, -1).reshape(-1, b * a)  # rows: mid, cols: (b, a)
    Gm = np.transpose(G, (0, 2, 1)).reshape(b * a, -1)  # rows: (b, a), cols: i
    X = (Wm @ Gm).reshape(*mid, G.shape[1])
    return X.astype(dtype, copy=False)


def add_noise_abs(X, sigma: float, rng: np.random.Generator):
    """X + iid N(0, sigma^2) noise (in the dtype of X)."""
    E = rng.standard_normal(X.shape)
    return (X + sigma * E).astype(X.dtype, copy=False)


def add_noise_rel(X, frac: float, rng: np.random.Generator):
    """X + E with E Gaussian and ``||E||_F = frac * ||X||_F`` exactly (in FP64)."""
    E = rng.standard_normal(X.shape)
    xn = float(np.linalg.norm(X.astype(np.float64, copy=False).ravel()))
    en = float(np.linalg.norm(E.ravel()))
    return (X.astype(np.float64, copy=False) + (frac * xn / en) * E).astype(X.dtype, copy=False)


def video_tensor(H=240, W=320, C=3, T=2000, K=16, seed=0, noise=0.02, dtype=np.float32,
                 t_chunk=250):
    """Video-shaped H x W x C x T tensor with pixel values in [0, 1].

    K Gaussian blobs; blob k has width sigma_k ~ U[6, 24] px, per-channel
    amplitude ~ U[0.2, 1], a start point uniform in the frame and a constant
    velocity ~ U[-0.1, 0.1] px/frame per axis.  Frames are the blob sum plus
    U(-noise, noise), clipped to [0, 1].  Mode order (H, W, C, T) follows the
    paper's colour-image-sequence tensor (Section 4.1.3).
    """
    rng = rng_for(seed, TAG_VIDEO)
    sig = rng.uniform(6.0, 24.0, K)
    amp = rng.uniform(0.2, 1.0, (K, C))
    y0 = rng.uniform(0.0, H, K)
    x0 = rng.uniform(0.0, W, K)
    vy = rng.uniform(-0.1, 0.1, K)
    vx = rng.uniform(-0.1, 0.1, K)
    X = np.empty((H, W, C, T), dtype=dtype)
    hh = np.arange(H, dtype=np.float64)
    ww = np.arange(W, dtype=np.float64)
    nrng = rng_for(seed, TAG_NOISE)
    for t0 in range(0, T, t_chunk):
        t = np.arange(t0, min(T, t0 + t_chunk), dtype=np.float64)
        cy = y0[:, None] + vy[:, None] * t[None, :]  # (K, t)
        cx = x0[:, None] + vx[:, None] * t[None, :]
        gy = np.exp(-((hh[None, None, :] - cy[:, :, None]) ** 2) / (2 * sig[:, None, None] ** 2))
        gx = np.exp(-((ww[None, None, :] - cx[:, :, None]) ** 2) / (2 * sig[:, None, None] ** 2))
        # frame[t, h, w, c] = sum_k gy[k, t, h] * gx[k, t, w] * amp[k, c]
        gxa = gx[:, :, :, None] * amp[:, None, None, :]  # (K, t, W, C)
        # per frame: (H x K) @ (K x W*C), batched over the frames of the chunk
        fr = np.matmul(np.transpose(gy, (1, 2, 0)), np.transpose(gxa.reshape(K, len(t), W * C), (1, 0, 2)))
        fr = fr.astype(np.float32).reshape(len(t), H, W, C)
        fr += nrng.uniform(-noise, noise, fr.shape).astype(np.float32)
        np.clip(fr, 0.0, 1.0, out=fr)
        X[:, :, :, t0:t0 + len(t)] = np.transpose(fr, (1, 2, 3, 0)).astype(dtype)
    return X


def serving_requests(n_requests: int, rate: float = 200.0, seed: int = 0,
                     orders=(3, 4, 5), dim_range=(32, 256), rank_range=(3, 12),
                     samples: int = 2048, sweeps: int = 5):
    """Poisson stream of decomposition requests (arrival times in seconds).

    Each request gets an order N uniform in ``orders``, mode sizes iid
    uniform integers in ``dim_range`` and bond ranks iid uniform integers in
    ``rank_range``; its tensor is drawn later from ``seed`` and the request
    id, so a request can be regenerated on its own.
    """
    rng = rng_for(seed, TAG_SERVE)
    gaps = rng.exponential(1.0 / rate, n_requests)
    t = np.cumsum(gaps)
    reqs = []
    for r in range(n_requests):
        N = int(rng.choice(orders))
        dims = [int(v) for v in rng.integers(dim_range[0], dim_range[1] + 1, N)]
        ranks = [int(v) for v in rng.integers(rank_range[0], rank_range[1] + 1, N)]
        reqs.append(dict(id=r, arrival=float(t[r]), dims=dims, ranks=ranks,
                         samples=int(samples), sweeps=int(sweeps), seed=int(seed)))
    return reqs


# Highly oscillatory functions (Section 4.1.2) and the intervals they are sampled on.  The
# paper gives the functions but not the grid; each is evaluated at 4^10 points
# x_k = a + (k + 1) (b - a) / 4^10, k = 0 .. 4^10 - 1 (the left end excluded: two of the
# functions are singular at 0), on an interval over which it oscillates many times.
OSC_FUNCTIONS = {
    "linear_growth": ((0.0, 1.0), lambda x: (x + 1.0) * np.sin(100.0 * (x + 1.0) ** 2)),
    "airy": ((0.0, 100.0), lambda x: x ** -0.25 * np.sin(2.0 * x ** 1.5 / 3.0)),
    "chirp": ((0.0, 10.0), lambda x: np.sin(4.0 / x) * np.cos(x ** 2)),
}


def oscillatory_tensor(name, levels=10, dtype=np.float64):
    """The function sampled at 4^levels points, reshaped to a levels-way 4 x ... x 4 tensor in
    C order (x's index k = sum_j i_j 4^(levels-1-j): the first mode is the coarsest scale)."""
    (a, b), f = OSC_FUNCTIONS[name]
    n = 4 ** levels
    x = a + (np.arange(n, dtype=np.float64) + 1.0) * ((b - a) / n)
    return f(x).reshape((4,) * levels).astype(dtype)


def serving_true_cores(req, dtype=np.float64):
    """True cores of one serving request: iid N(0,1), drawn from the request's
    seed and id alone (so the request can be rebuilt without the others)."""
    rng = np.random.default_rng([int(req["seed"]), TAG_SERVE, int(req["id"])])
    return random_cores(req["dims"], req["ranks"], rng, dtype)


# Workloads: sizes and noise of the paper's synthetic experiments
# (Section 4.1.1) and stand-ins for its dataset experiments (Section 4.1.3).
CONFIGS = {
    "c1": dict(name="fp64-60^3-R3", dims=(60, 60, 60), ranks=(3, 3, 3), samples=2000, sweeps=10,
               noise=("abs", 1e-3), precision="f64", seed=0),
    "c2": dict(name="fp32-500^3-R10", dims=(500, 500, 500), ranks=(10, 10, 10), samples=8192,
               sweeps=20, noise=("rel", 1e-2), precision="f32", seed=0),
    "c3": dict(name="fp32-40^5-R5", dims=(40,) * 5, ranks=(5,) * 5, samples=4096, sweeps=10,
               noise=("rel", 1e-2), precision="f32", seed=0),
    "c4": dict(name="video-240x320x3x2000-R20", dims=(240, 320, 3, 2000), ranks=(20,) * 4,
               samples=16384, sweeps=10, noise=("video", 2e-2), precision="f32", seed=0),
}


def make_config(cfg, dims=None, dtype=np.float32, seed=None, ranks=None):
    """Build ``(X, true_cores, init_cores)`` for a workload recipe.

    ``dims`` (and ``ranks``) may replace the recipe's mode sizes (and ranks)
    with the same noise model and seed, for small parity cases.
    ``true_cores`` is None for the video recipe.
    """
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    dims = tuple(cfg["dims"] if dims is None else dims)
    ranks = tuple(cfg["ranks"] if ranks is None else ranks)
    seed = cfg["seed"] if seed is None else seed
    kind, level = cfg["noise"]
    if kind == "video":
        X = video_tensor(*dims, seed=seed, noise=level, dtype=dtype)
        true = None
    else:
        true = random_cores(dims, ranks, rng_for(seed, TAG_TRUE_CORES))
        X = ring_tensor(true, dtype=np.float64)
        nrng = rng_for(seed, TAG_NOISE)
        X = add_noise_abs(X, level, nrng) if kind == "abs" else add_noise_rel(X, level, nrng)
        X = X.astype(dtype, copy=False)
    init = random_cores(dims, ranks, rng_for(seed, TAG_INIT), dtype=np.float64)
    return X, true, init
