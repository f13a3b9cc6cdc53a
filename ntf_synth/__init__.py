"""Seeded synthetic inputs for non-negative CP factorisation (NTF).

This module only draws random numbers and builds the planted data model of
Section II (a tensor that is a sum of F non-negative rank-one terms plus
i.i.d. Gaussian noise, Section VI-A).  It holds none of the factorisation
method's arithmetic, so both the FP64 oracle and the GPU path can take their
inputs from it.

Draw order for one tensor (fixed, so every consumer sees the same numbers):
  1. planted factors A0 (I x F), B0 (J x F), C0 (K x F), row-major, from
     ``numpy.random.default_rng(seed)``;
  2. the noise tensor in C storage order (i slowest, k fastest), same stream;
  3. initial factors H1 (I x F), H2 (J x F), H3 (K x F), Uniform[0,1], from
     ``default_rng(seed + 1)``.

Noise level: either an absolute variance ``sigma2`` (the form Section VI-A
uses) or an SNR in dB, in which case the standard deviation is
``||X0||_F / sqrt(IJK * 10**(snr_db/10))`` on the realised clean tensor.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

__all__ = ["PlantedTensor", "planted", "init_factors", "config_seed", "batch_shapes",
           "SparseSample", "sparse_planted", "planted_nway"]


@dataclass
class PlantedTensor:
    X: np.ndarray            # (I, J, K), C order, dtype as requested
    A0: np.ndarray           # planted factors, float64
    B0: np.ndarray
    C0: np.ndarray
    sigma: float             # noise standard deviation actually used
    clean_norm2: float       # ||X0||_F^2 of the clean tensor (float64)


def config_seed(config: int, tensor: int = 0) -> int:
    """Seed of tensor ``tensor`` of workload ``config``: 1000*config + tensor."""
    return 1000 * int(config) + int(tensor)


def _draw_factor(rng: np.random.Generator, rows: int, F: int, dist: str) -> np.ndarray:
    if dist == "uniform":
        return rng.random((rows, F))
    if dist == "exponential":
        return rng.exponential(1.0, (rows, F))
    raise ValueError(f"unknown factor distribution {dist!r}")


def _clean_slab(A0: np.ndarray, B0: np.ndarray, C0: np.ndarray, i0: int, i1: int) -> np.ndarray:
    # X0[i, j, k] = sum_f A0[i,f] B0[j,f] C0[k,f]   (the data model of Section II)
    I, F = A0.shape
    J, K = B0.shape[0], C0.shape[0]
    left = (A0[i0:i1, None, :] * B0[None, :, :]).reshape((i1 - i0) * J, F)
    return (left @ C0.T).reshape(i1 - i0, J, K)


def planted(dims: Sequence[int], F: int, seed: int, *, dist: str = "uniform",
            snr_db: Optional[float] = None, sigma2: Optional[float] = None,
            clip: bool = False, dtype=np.float32, slab_chunk: int = 64) -> PlantedTensor:
    """Planted non-negative rank-F tensor plus Gaussian noise.

    ``dims`` = (I, J, K).  Exactly one of ``snr_db`` / ``sigma2`` may be given
    (neither = noiseless).  ``clip`` applies max(0, .) to the noisy tensor.
    The tensor is built in slabs of ``slab_chunk`` mode-1 indices so large
    workloads do not need a float64 copy of the whole tensor; the noise stream
    is consumed in storage order, so the result does not depend on the chunk.
    """
    I, J, K = (int(d) for d in dims)
    if min(I, J, K) < 1 or F < 1:
        raise ValueError("dims and F must be positive")
    if snr_db is not None and sigma2 is not None:
        raise ValueError("give snr_db or sigma2, not both")
    rng = np.random.default_rng(seed)
    A0 = _draw_factor(rng, I, F, dist)
    B0 = _draw_factor(rng, J, F, dist)
    C0 = _draw_factor(rng, K, F, dist)

    # ||X0||^2 via the Gram identity would be method arithmetic; sum it directly.
    clean_norm2 = 0.0
    for i0 in range(0, I, slab_chunk):
        i1 = min(I, i0 + slab_chunk)
        s = _clean_slab(A0, B0, C0, i0, i1)
        clean_norm2 += float(np.dot(s.ravel(), s.ravel()))

    if snr_db is not None:
        sigma = math.sqrt(clean_norm2 / (I * J * K * 10.0 ** (snr_db / 10.0)))
    elif sigma2 is not None:
        sigma = math.sqrt(sigma2)
    else:
        sigma = 0.0

    X = np.empty((I, J, K), dtype=dtype)
    for i0 in range(0, I, slab_chunk):
        i1 = min(I, i0 + slab_chunk)
        s = _clean_slab(A0, B0, C0, i0, i1)
        if sigma > 0.0:
            s = s + sigma * rng.standard_normal(s.shape)
        if clip:
            np.maximum(s, 0.0, out=s)
        X[i0:i1] = s.astype(dtype)
    return PlantedTensor(X=X, A0=A0, B0=B0, C0=C0, sigma=sigma, clean_norm2=clean_norm2)


def init_factors(dims: Sequence[int], F: int, seed: int, dtype=np.float64):
    """Initial factors H1, H2, H3 ~ Uniform[0,1] from default_rng(seed + 1)."""
    rng = np.random.default_rng(seed + 1)
    return [rng.random((int(d), F)).astype(dtype) for d in dims]


def batch_shapes(n: int, seed: int, lo: int, hi: int, ranks: Sequence[int]):
    """Shapes and ranks of a batch of ``n`` tensors: each mode uniform on
    [lo, hi], rank uniform over ``ranks``; from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    dims = rng.integers(lo, hi + 1, size=(n, 3))
    Fs = rng.choice(np.asarray(list(ranks)), size=n)
    return [(tuple(int(x) for x in d), int(f)) for d, f in zip(dims, Fs)]


@dataclass
class SparseSample:
    idx: np.ndarray          # [n][3] int32 coordinates (i, j, k), distinct, in random order
    val: np.ndarray          # [n] values, dtype as requested
    dims: tuple
    A0: np.ndarray           # planted factors, float64
    B0: np.ndarray
    C0: np.ndarray
    sigma: float


def sparse_planted(dims: Sequence[int], F: int, nnz: int, seed: int, *, skew: float = 2.0,
                   noise_rel: float = 0.1, dtype=np.float32, chunk: int = 1 << 22) -> SparseSample:
    """A sparse tensor observed at about ``nnz`` positions of the planted model.

    Positions: per mode, ``floor(d * u**skew)`` with u ~ Uniform[0,1) (skew > 1
    gives the few heavy and many light slices that sparse tensors show), the
    index then relabelled by a random permutation of the mode so that heavy
    slices are scattered; repeated coordinates are dropped (the first draw is
    kept), so the result may hold slightly fewer than ``nnz`` entries, in a
    random order.  Values: the planted rank-F model (U[0,1] factors) at those
    positions plus Gaussian noise of standard deviation ``noise_rel`` times the
    RMS of the clean values.

    Draw order from ``default_rng(seed)``: A0, B0, C0 (row-major); the three
    position streams (i, then j, then k, each ``nnz`` uniforms); the three
    relabelling permutations; the noise (one normal per kept entry, in kept
    order); the output permutation.
    """
    I, J, K = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    A0 = _draw_factor(rng, I, F, "uniform")
    B0 = _draw_factor(rng, J, F, "uniform")
    C0 = _draw_factor(rng, K, F, "uniform")
    raw = [np.floor(d * rng.random(nnz) ** skew).astype(np.int64) for d in (I, J, K)]
    perm = [rng.permutation(d) for d in (I, J, K)]
    coords = [p[r] for p, r in zip(perm, raw)]
    key = (coords[0] * J + coords[1]) * K + coords[2]
    _, first = np.unique(key, return_index=True)
    first.sort()                                       # keep draw order
    idx = np.stack([c[first] for c in coords], axis=1).astype(np.int32)
    n = idx.shape[0]
    clean = np.empty(n, dtype=np.float64)
    for e0 in range(0, n, chunk):
        e1 = min(n, e0 + chunk)
        t = idx[e0:e1]
        # X0[i, j, k] = sum_f A0[i,f] B0[j,f] C0[k,f]   (the data model of Section II)
        clean[e0:e1] = np.sum(A0[t[:, 0]] * B0[t[:, 1]] * C0[t[:, 2]], axis=1)
    sigma = noise_rel * math.sqrt(float(np.mean(clean * clean))) if n else 0.0
    val = clean + sigma * rng.standard_normal(n)
    order = rng.permutation(n)
    return SparseSample(idx=np.ascontiguousarray(idx[order]), val=val[order].astype(dtype),
                        dims=(I, J, K), A0=A0, B0=B0, C0=C0, sigma=sigma)


def planted_nway(dims: Sequence[int], F: int, seed: int, *, dist: str = "uniform",
                 snr_db: Optional[float] = None, sigma2: Optional[float] = None,
                 dtype=np.float32, slab_chunk: int = 8):
    """Planted non-negative rank-F tensor of any order N >= 3 (the data model
    of Section II extended as in Appendix A) plus Gaussian noise.

    Draw order from ``default_rng(seed)``: the N factors (row-major, mode
    order), then the noise in C storage order.  Returns (X, factors, sigma).
    Noise as in ``planted``."""
    dims = tuple(int(d) for d in dims)
    if len(dims) < 3 or min(dims) < 1 or F < 1:
        raise ValueError("need N >= 3 positive dims and F >= 1")
    if snr_db is not None and sigma2 is not None:
        raise ValueError("give snr_db or sigma2, not both")
    rng = np.random.default_rng(seed)
    fac = [_draw_factor(rng, d, F, dist) for d in dims]
    # rows of the trailing modes' outer products, C order (last mode fastest)
    tail = fac[-1]
    for g in reversed(fac[1:-1]):
        tail = (g[:, None, :] * tail[None, :, :]).reshape(-1, F)
    rest = tail.shape[0]

    def slab(i0, i1):
        # X0[i, ...] = sum_f A0[i,f] (outer product of the other factors' column f)
        return fac[0][i0:i1] @ tail.T

    clean_norm2 = 0.0
    for i0 in range(0, dims[0], slab_chunk):
        sl = slab(i0, min(dims[0], i0 + slab_chunk))
        clean_norm2 += float(np.dot(sl.ravel(), sl.ravel()))
    n = int(np.prod(dims))
    if snr_db is not None:
        sigma = math.sqrt(clean_norm2 / (n * 10.0 ** (snr_db / 10.0)))
    elif sigma2 is not None:
        sigma = math.sqrt(sigma2)
    else:
        sigma = 0.0
    X = np.empty((dims[0], rest), dtype=dtype)
    for i0 in range(0, dims[0], slab_chunk):
        i1 = min(dims[0], i0 + slab_chunk)
        sl = slab(i0, i1)
        if sigma > 0.0:
            sl = sl + sigma * rng.standard_normal(sl.shape)
        X[i0:i1] = sl.astype(dtype)
    return X.reshape(dims), fac, sigma
