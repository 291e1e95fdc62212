"""Seeded synthetic inputs for the non-metric Vicsek step.

This module holds only input recipes (positions, headings, system sizes,
request streams).  It contains none of the method's arithmetic, and it is the
one piece of code that both the GPU path (benchmarks) and the tests of the
brute-force reference draw inputs from.

The paper (arXiv:2103.10239) measures nothing, so every workload is synthetic:

- ``uniform``: N points uniform on the integer grid [0, L)^2 and headings
  uniform in [-pi, pi) (a disordered Vicsek start, Sec. III).
- ``clustered``: N points drawn from isotropic Gaussian clusters with
  periodic wrap -- density inhomogeneity, the situation in which Sec. III
  notes that k-nearest-neighbour relations stop being reciprocal.
- ``lattice``: a square lattice (every distance tie the index rule must break).
- ``batched_sizes``: system sizes log-uniform in [lo, hi] for the
  many-systems form.
- ``request_stream``: a Poisson stream of jobs for the served form.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

BOX = 1 << 20          # side of the periodic box in integer units
SEED_POS = 1           # positions
SEED_THETA = 2         # headings
SEED_CLUSTER = 3       # cluster centres and memberships
SEED_SIZES = 4         # batched system sizes
SEED_STREAM = 5        # served request stream
NOISE_SEED = 0         # Philox key of the alignment noise


def uniform(n: int, box: int = BOX, seed_pos: int = SEED_POS, seed_theta: int = SEED_THETA):
    """x, y int32 uniform in [0, box); theta fp32 uniform in [-pi, pi)."""
    rng = np.random.default_rng(seed_pos)
    x = rng.integers(0, box, size=n, dtype=np.int64).astype(np.int32)
    y = rng.integers(0, box, size=n, dtype=np.int64).astype(np.int32)
    theta = headings(n, seed_theta)
    return x, y, theta


def headings(n: int, seed: int = SEED_THETA) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-np.pi, np.pi, size=n).astype(np.float32)


def clustered(n: int, box: int = BOX, n_clusters: int = 256, sigma_frac: float = 0.01,
              seed: int = SEED_CLUSTER, seed_theta: int = SEED_THETA):
    """Points from ``n_clusters`` isotropic Gaussians of width sigma_frac*box.

    Centres are uniform in the box, memberships uniform over clusters, and
    each coordinate is floor(centre + sigma * normal) wrapped into [0, box).
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, box, size=(n_clusters, 2))
    member = rng.integers(0, n_clusters, size=n)
    sigma = sigma_frac * box
    pts = centres[member] + sigma * rng.standard_normal(size=(n, 2))
    pts = np.floor(pts).astype(np.int64) % box
    x = pts[:, 0].astype(np.int32)
    y = pts[:, 1].astype(np.int32)
    return x, y, headings(n, seed_theta)


def lattice(m: int, box: int = BOX):
    """m x m square lattice with spacing box // m; particle index = row * m + col."""
    a = box // m
    idx = np.arange(m * m, dtype=np.int64)
    x = ((idx % m) * a).astype(np.int32)
    y = ((idx // m) * a).astype(np.int32)
    return x, y, a


def rc2_for_mean(n: int, mean: float, box: int = BOX) -> int:
    """Integer r_c^2 with on average ``mean`` other particles inside (uniform density)."""
    return int(round(mean * box * box / (math.pi * (n - 1))))


def batched_sizes(nsys: int, lo: int = 256, hi: int = 65536, seed: int = SEED_SIZES) -> np.ndarray:
    """System sizes round(exp(U[ln lo, ln hi]))."""
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=nsys))).astype(np.int64)


@dataclass
class Request:
    arrival_s: float
    n: int
    k: int
    nsteps: int
    clustered: bool
    seed: int


def request_stream(rate_hz: float, duration_s: float, n_lo: int = 1024, n_hi: int = 1 << 20,
                   ks=(7, 12), max_steps: int = 100, seed: int = SEED_STREAM):
    """Poisson arrivals of (N log-uniform, k, nsteps uniform in [1, max_steps], half clustered)."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        out.append(Request(arrival_s=t, n=n, k=int(rng.choice(ks)),
                           nsteps=int(rng.integers(1, max_steps + 1)),
                           clustered=bool(rng.integers(0, 2)), seed=int(rng.integers(0, 2**31))))
    return out
