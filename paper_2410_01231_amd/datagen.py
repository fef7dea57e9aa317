"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws data; it holds none of the method's arithmetic, so both
the HIP path and the oracle may be fed from it.  The paper's datasets (Table
"Data statistics": Sift1M, Gist1M, Deep1M, ...) are not available; these
generators stand in for them:

* ``uniform_int``  i.i.d. integers in [0, 255] stored as float32 (tiny case).
* ``int_grid``     i.i.d. integers in [lo, hi] stored as float32 (small ranges
                   give many equal distances and exact right angles; negative
                   ranges give signed data).
* ``sift_like``    mixture of Gaussian clusters with centres uniform in
                   [0, 255]^d and per-dimension sigma, rounded and clipped to
                   [0, 255] (SIFT-shaped, 128-d).
* ``gist_like``    nonnegative Gamma(2, scale 0.05) values plus one of
                   ``n_clusters`` offsets drawn uniform in [0, 0.2]^d (GIST-shaped).
* ``unit_mixture`` unit-normalised Gaussian mixture (Deep-shaped; also the
                   per-collection law of the serving mix).

Every generator takes a master seed; data and queries use separate
substreams of the same mixture so that queries follow the data's law.
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int, sub: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(sub)]))


def uniform_int(n: int, d: int, seed: int) -> np.ndarray:
    """floor(256 * U[0,1)) per coordinate, as float32."""
    return np.floor(_rng(seed, 0).random((n, d)) * 256.0).astype(np.float32)


def int_grid(n: int, d: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Integers uniform in [lo, hi] per coordinate, as float32."""
    return _rng(seed, 0).integers(lo, hi + 1, size=(n, d)).astype(np.float32)


def _mixture_labels(rng, n, n_clusters):
    return rng.integers(0, n_clusters, size=n)


def sift_like(n: int, nq: int = 0, d: int = 128, n_clusters: int = 100,
              sigma: float = 20.0, seed: int = 2, chunk: int = 1 << 18):
    """Returns (X, Q): clip(round(c_z + sigma * N(0,1)), 0, 255) as float32."""
    centres = _rng(seed, 0).random((n_clusters, d)) * 255.0

    def draw(count, sub):
        out = np.empty((count, d), np.float32)
        rng = _rng(seed, sub)
        for s in range(0, count, chunk):
            e = min(count, s + chunk)
            z = _mixture_labels(rng, e - s, n_clusters)
            x = centres[z] + sigma * rng.standard_normal((e - s, d))
            out[s:e] = np.clip(np.rint(x), 0.0, 255.0)
        return out

    return draw(n, 1), draw(nq, 2)


def gist_like(n: int, nq: int = 0, d: int = 960, n_clusters: int = 50,
              shape: float = 2.0, scale: float = 0.05, offset_hi: float = 0.2,
              seed: int = 3, chunk: int = 1 << 16):
    """Returns (X, Q): o_z + Gamma(shape, scale) per coordinate, float32."""
    offsets = _rng(seed, 0).random((n_clusters, d)) * offset_hi

    def draw(count, sub):
        out = np.empty((count, d), np.float32)
        rng = _rng(seed, sub)
        for s in range(0, count, chunk):
            e = min(count, s + chunk)
            z = _mixture_labels(rng, e - s, n_clusters)
            out[s:e] = offsets[z] + rng.gamma(shape, scale, size=(e - s, d))
        return out

    return draw(n, 1), draw(nq, 2)


def unit_mixture(n: int, nq: int = 0, d: int = 96, n_clusters: int = 1000,
                 noise: float = 1.0, seed: int = 4, chunk: int = 1 << 18):
    """Returns (X, Q): normalize(c_z + noise * N(0, I)) with c ~ N(0, I), float32."""
    centres = _rng(seed, 0).standard_normal((n_clusters, d))

    def draw(count, sub):
        out = np.empty((count, d), np.float32)
        rng = _rng(seed, sub)
        for s in range(0, count, chunk):
            e = min(count, s + chunk)
            z = _mixture_labels(rng, e - s, n_clusters)
            x = centres[z] + noise * rng.standard_normal((e - s, d))
            x /= np.linalg.norm(x, axis=1, keepdims=True)
            out[s:e] = x
        return out

    return draw(n, 1), draw(nq, 2)


def sample_ids(n: int, count: int, seed: int, sub: int = 9) -> np.ndarray:
    """count distinct ids in [0, n), sorted (evaluation subsamples)."""
    count = min(count, n)
    return np.sort(_rng(seed, sub).choice(n, size=count, replace=False)).astype(np.int32)


def entry_sample(n: int, count: int, seed: int = 21) -> np.ndarray:
    """count distinct ids in [0, n), sorted: the seeded entering points that a
    search takes beside the graph's entry point (the same set on every side)."""
    return sample_ids(n, count, seed, sub=15)


def random_candidates(n: int, C: int, seed: int, sub: int = 11) -> np.ndarray:
    """n x C candidate ids drawn uniformly from [0, n) (repeats and self allowed)."""
    return _rng(seed, sub).integers(0, n, size=(n, C)).astype(np.int32)


def uniform_open01(n: int, seed: int, sub: int = 13) -> np.ndarray:
    """n uniform draws in (0, 1] as float64 (the layer draws of an HNSW build)."""
    return 1.0 - _rng(seed, sub).random(n)
