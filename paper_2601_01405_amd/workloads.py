"""Seeded synthetic point clouds for the Ball Mapper hot path.

This module only draws random numbers (numpy ``default_rng``/PCG64, float64
draws cast to the stored dtype with round-to-nearest-even).  It holds none of
the method's arithmetic, so both the GPU path and the CPU oracle can be fed
from it without sharing any computation.

Workloads (shapes and value laws of the paper's experiments and of the
benchmark configurations):

* ``gaussian``  i.i.d. N(0, I) cloud — the isotropic Gaussian data of Sec. 6.1
                (n = 20000, d = 50 in the paper's worked example).
* ``clusters``  mixture of k isotropic unit-variance Gaussians with centres
                uniform in a box, i.i.d. uniform labels (the clustered data of
                Sec. 6.1, at benchmark scale).
* ``torus``     2-D torus (R = 3, r = 1) sampled uniformly in surface area,
                lifted to d dimensions by a Haar-random orthogonal map, plus
                N(0, sigma^2) noise, stored as float16.
* ``batched``   many Gaussian mixtures of uneven n and d with an eps sweep each.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def gaussian(n: int, d: int, seed: int = 0, dtype=np.float64) -> np.ndarray:
    x = np.random.default_rng(seed).standard_normal((n, d))
    return np.ascontiguousarray(x.astype(dtype))


def clusters(n: int, d: int, k: int = 10, box: float = 20.0, std: float = 1.0,
             seed: int = 0, dtype=np.float32) -> np.ndarray:
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-box, box, (k, d))
    labels = rng.integers(0, k, n)
    x = centres[labels] + std * rng.standard_normal((n, d))
    return np.ascontiguousarray(x.astype(dtype))


def torus(n: int, d: int = 64, R: float = 3.0, r: float = 1.0, noise: float = 0.01,
          seed: int = 0, dtype=np.float16) -> np.ndarray:
    """Uniform-in-area torus sample: theta is drawn by rejection with acceptance
    probability (R + r cos theta) / (R + r), phi uniformly."""
    rng = np.random.default_rng(seed)
    thetas = []
    have = 0
    while have < n:
        m = 2 * (n - have)
        th = rng.uniform(0.0, 2.0 * math.pi, m)
        u = rng.uniform(0.0, 1.0, m)
        acc = th[u < (R + r * np.cos(th)) / (R + r)]
        thetas.append(acc)
        have += acc.shape[0]
    theta = np.concatenate(thetas)[:n]
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    ring = R + r * np.cos(theta)
    p = np.stack([ring * np.cos(phi), ring * np.sin(phi), r * np.sin(theta)], axis=1)
    q, rm = np.linalg.qr(rng.standard_normal((d, d)))
    q = q * np.sign(np.diag(rm))[None, :]
    x = p @ q[:, :3].T + noise * rng.standard_normal((n, d))
    return np.ascontiguousarray(x.astype(dtype))


@dataclass
class BatchedProblem:
    points: np.ndarray
    eps: list = field(default_factory=list)


def batched(count: int = 256, n_lo: int = 1000, n_hi: int = 200000,
            dims=(8, 32, 96), eps=tuple(0.5 * (i + 1) for i in range(8)),
            seed: int = 0, n_scale: float = 1.0) -> list[BatchedProblem]:
    """Gaussian mixtures with n log-uniform in [n_lo, n_hi], d drawn from `dims`,
    1..20 clusters (centres uniform in [-20, 20]^d, unit std) and an eps sweep.
    `n_scale` < 1 shrinks every n (same draws otherwise) for small test runs."""
    ss = np.random.SeedSequence(seed).spawn(count + 1)
    meta = np.random.default_rng(ss[0])
    out = []
    for b in range(count):
        nb = int(math.floor(math.exp(meta.uniform(math.log(n_lo), math.log(n_hi)))))
        db = int(meta.choice(np.asarray(dims)))
        kb = int(meta.integers(1, 21))
        nb = max(1, int(nb * n_scale))
        rng = np.random.default_rng(ss[b + 1])
        centres = rng.uniform(-20.0, 20.0, (kb, db))
        labels = rng.integers(0, kb, nb)
        x = (centres[labels] + rng.standard_normal((nb, db))).astype(np.float32)
        out.append(BatchedProblem(np.ascontiguousarray(x), list(eps)))
    return out


# ---- named workloads ---------------------------------------------------------

def paper_gaussian() -> np.ndarray:
    """The isotropic Gaussian of the Sec. 6.3 worked example: n = 20000, d = 50."""
    return gaussian(20000, 50, seed=0, dtype=np.float64)


def small_3d(n: int = 2000) -> np.ndarray:
    """n x 3 float64 N(0, I), seed 0."""
    return gaussian(n, 3, seed=0, dtype=np.float64)


def clusters_16d(n: int = 200000) -> np.ndarray:
    """10 unit-std clusters in [-20, 20]^16, float32, seed 0."""
    return clusters(n, 16, k=10, box=20.0, std=1.0, seed=0, dtype=np.float32)


def gaussian_128d(n: int = 1000000) -> np.ndarray:
    """N(0, I) in 128-D, float32, seed 0."""
    return gaussian(n, 128, seed=0, dtype=np.float32)


def torus_64d(n: int = 2000000) -> np.ndarray:
    """Noisy torus lifted to 64-D, float16, seed 0."""
    return torus(n, 64, seed=0, dtype=np.float16)


WORKLOADS = {
    "gauss3d_n2000_f64": dict(make=small_3d, eps=[0.5]),
    "clusters16d_n200k_f32": dict(make=clusters_16d, eps=[1.0, 2.0]),
    "gauss128d_n1m_f32": dict(make=gaussian_128d, eps=[13.0, 14.5]),
    "torus64d_n2m_f16": dict(make=torus_64d, eps=[0.1, 0.3]),
}
