"""Seeded synthetic point sets shaped like the paper's workloads.

This module only draws numbers: it holds none of the hull method's arithmetic,
so both the GPU path's tests and the CPU oracle's tests can take their inputs
from here without sharing any computation.

Every generator returns a C-contiguous ``float32`` array of shape ``[n, 2]``
holding integer values in ``[0, 2**23)`` (the domain the library accepts).
The paper's first dataset group is random points in a square produced with
Qhull's ``rbox`` (Section 3, dataset description); the uniform-square
generator stands in for it.  The paper's second group (projected 3D scan
meshes) is not reproduced.

Rounding is ``rint`` (half to even) in float64 followed by a clamp to
``[0, M]`` with ``M = 2**23 - 1``.
"""
from __future__ import annotations

import numpy as np

COORD_BITS = 23
M = (1 << COORD_BITS) - 1          # largest coordinate value
CENTER = 1 << 22                   # centre of the disk / circle / Gaussian
RADIUS = 1 << 22                   # radius of the inscribed disk and circle
SIGMA = 1 << 20                    # Gaussian standard deviation

DISTRIBUTIONS = ("square", "disk", "gaussian", "adversarial")


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _to_f32(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    out = np.empty((x.shape[0], 2), dtype=np.float32)
    out[:, 0] = x
    out[:, 1] = y
    return out


def _round_clamp(v: np.ndarray) -> np.ndarray:
    return np.clip(np.rint(v), 0, M)


def uniform_square(n: int, rng: np.random.Generator) -> np.ndarray:
    """Integer points drawn uniformly from ``[0, 2**23)**2``."""
    xy = rng.integers(0, M + 1, size=(n, 2), dtype=np.int64)
    return np.ascontiguousarray(xy.astype(np.float32))


def uniform_disk(n: int, rng: np.random.Generator) -> np.ndarray:
    """Integer points uniform in the inscribed disk, by rejection sampling.

    Candidates are drawn from the whole square and kept when
    ``(X - 2**22)**2 + (Y - 2**22)**2 <= 2**44``.
    """
    out = np.empty((n, 2), dtype=np.float32)
    got = 0
    r2 = RADIUS * RADIUS
    while got < n:
        want = n - got
        batch = int(want * 1.30) + 64
        xy = rng.integers(0, M + 1, size=(batch, 2), dtype=np.int64)
        dx = xy[:, 0] - CENTER
        dy = xy[:, 1] - CENTER
        ok = xy[(dx * dx + dy * dy) <= r2]
        take = min(want, ok.shape[0])
        out[got:got + take] = ok[:take]
        got += take
    return out


def gaussian(n: int, rng: np.random.Generator) -> np.ndarray:
    """Independent Gaussian coordinates, sigma 2**20 around 2**22, clamped."""
    v = CENTER + SIGMA * rng.standard_normal(size=(n, 2))
    return np.ascontiguousarray(_round_clamp(v).astype(np.float32))


def circle(n: int, rng: np.random.Generator) -> np.ndarray:
    """Points on the integer-rounded circle of radius 2**22 (duplicates kept)."""
    th = rng.uniform(0.0, 2.0 * np.pi, size=n)
    x = _round_clamp(CENTER + RADIUS * np.cos(th))
    y = _round_clamp(CENTER + RADIUS * np.sin(th))
    return _to_f32(x, y)


def adversarial(n: int, rng: np.random.Generator) -> np.ndarray:
    """10% on the circle and 90% uniform in the disk, shuffled."""
    nc = n // 10
    pts = np.concatenate([circle(nc, rng), uniform_disk(n - nc, rng)])
    perm = rng.permutation(n)
    return np.ascontiguousarray(pts[perm])


_GEN = {
    "square": uniform_square,
    "disk": uniform_disk,
    "gaussian": gaussian,
    "adversarial": adversarial,
}


def generate(dist: str, n: int, seed: int) -> np.ndarray:
    """One point set of ``n`` points from distribution ``dist``."""
    if dist not in _GEN:
        raise ValueError(f"unknown distribution {dist!r}")
    return _GEN[dist](int(n), rng_for(seed))


# Named workloads, with the seeds the tests and the benchmark use.
WORKLOADS = {
    "square_100k": ("square", 100_000, 1),
    "square_20m": ("square", 20_000_000, 2),
    "disk_20m": ("disk", 20_000_000, 3),
    "gaussian_20m": ("gaussian", 20_000_000, 4),
    "adversarial_20m": ("adversarial", 20_000_000, 5),
    "adversarial_100m": ("adversarial", 100_000_000, 6),
}


def workload(name: str) -> np.ndarray:
    dist, n, seed = WORKLOADS[name]
    return generate(dist, n, seed)


def batched_sets(num_sets: int, lo: int, hi: int, seed: int):
    """Sizes log-uniform in ``[lo, hi]``, each set one of square/disk/gaussian.

    Returns ``(points [N,2] f32, offsets int64[num_sets+1], dists list)``.
    """
    root = np.random.SeedSequence(seed)
    children = root.spawn(num_sets + 1)
    meta = np.random.Generator(np.random.PCG64(children[0]))
    sizes = np.floor(np.exp(meta.uniform(np.log(lo), np.log(hi), size=num_sets))).astype(np.int64)
    kinds = meta.integers(0, 3, size=num_sets)
    names = ("square", "disk", "gaussian")
    parts, dists = [], []
    for s in range(num_sets):
        g = np.random.Generator(np.random.PCG64(children[s + 1]))
        d = names[int(kinds[s])]
        parts.append(_GEN[d](int(sizes[s]), g))
        dists.append(d)
    offsets = np.zeros(num_sets + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    pts = np.ascontiguousarray(np.concatenate(parts) if parts else np.zeros((0, 2), np.float32))
    return pts, offsets, dists


def tie_free(dist: str, n: int, seed: int) -> np.ndarray:
    """``dist`` (square, disk or gaussian) with every x and every y distinct:
    points that repeat an earlier point's x or y are dropped and more are
    drawn (inputs for SPA experiments that must avoid key ties)."""
    rng = rng_for(seed)
    have = np.zeros((0, 2), np.float32)
    draw = 2 * n + 64
    while have.shape[0] < n:
        cand = np.concatenate([have, _GEN[dist](draw, rng)])
        _, ix = np.unique(cand[:, 0], return_index=True)
        cand = cand[np.sort(ix)]
        _, iy = np.unique(cand[:, 1], return_index=True)
        have = cand[np.sort(iy)]
        draw *= 2
    return np.ascontiguousarray(have[:n])


def small_lattice(n: int, k: int, rng: np.random.Generator) -> np.ndarray:
    """Points with coordinates in ``[0, k)``: heavy duplicates and collinearity."""
    xy = rng.integers(0, k, size=(n, 2), dtype=np.int64)
    return np.ascontiguousarray(xy.astype(np.float32))
