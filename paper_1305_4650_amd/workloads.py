"""Seeded synthetic inputs for the butterfly apply.

This module holds point sets, boxes and random right-hand sides only -- none of
the method's arithmetic -- so that the GPU path, the tests and the benchmark
all draw identical inputs.

The paper measures on synthetic quasi-uniform points with analytic phases
(Sec. 3: a hyperbolic Radon transform and a 3-D generalized-Radon analogue,
and the Fourier kernel named in the same section); no dataset is involved.

Conventions
-----------
* points are float64 arrays of shape (n, d) in grid order, dimension 0 fastest;
* right-hand sides are complex128 arrays of shape (nrhs, n), entries iid
  N(0,1) + i N(0,1), all real parts drawn before all imaginary parts;
* seeds: ``numpy.random.default_rng([13054650, config_id, stream_id])`` with
  stream 0 = jitter, 1 = g, 2 = noise, 3 = subsets / sampling.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

PHASE_IDS = {"fourier": 0, "hypradon2": 1, "genradon3": 2, "separable": 3, "genradon3pi": 4}
SEED_BASE = 13054650


def rng(config_id: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE, int(config_id), int(stream)])


def grid_index(N: int, d: int) -> np.ndarray:
    """Integer multi-indices (n, d) of an N^d grid, dimension 0 fastest."""
    i = np.arange(N ** d, dtype=np.int64)
    return np.ascontiguousarray(np.stack([(i // N ** j) % N for j in range(d)], axis=1))


def grid_points(N: int, lo, hi, offset=0.0, jitter: np.ndarray | None = None) -> np.ndarray:
    """Points lo + (k + offset + jitter) * (hi - lo) / N on the N^d grid."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    d = lo.size
    k = grid_index(N, d).astype(np.float64)
    u = k + offset
    if jitter is not None:
        u = u + jitter
    return np.ascontiguousarray(lo + u * ((hi - lo) / N))


def random_rhs(gen: np.random.Generator, nrhs: int, n: int) -> np.ndarray:
    re = gen.standard_normal((nrhs, n))
    im = gen.standard_normal((nrhs, n))
    return np.ascontiguousarray(re + 1j * im)


@dataclass
class Workload:
    name: str
    d: int
    N: int
    q: int
    phase: str
    src_lo: np.ndarray
    src_hi: np.ndarray
    tgt_lo: np.ndarray
    tgt_hi: np.ndarray
    y: np.ndarray          # sources (n_src, d)
    x: np.ndarray          # targets (n_tgt, d)
    g: np.ndarray          # (nrhs, n_src) complex128
    config_id: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def nrhs(self) -> int:
        return self.g.shape[0]

    @property
    def phase_id(self) -> int:
        return PHASE_IDS[self.phase]

    @property
    def src_box(self):
        return (self.src_lo, self.src_hi)

    @property
    def tgt_box(self):
        return (self.tgt_lo, self.tgt_hi)


def fourier_grid(N: int, d: int = 2, q: int = 5, nrhs: int = 1, config_id: int = 1,
                 name: str | None = None) -> Workload:
    """Fourier kernel on uniform grids: y = j/N in [0,1)^d, x = k in [0,N)^d
    (the uniform-grid Fourier geometry; the direct sum is then an
    unnormalised inverse DFT)."""
    y = grid_points(N, np.zeros(d), np.ones(d))
    x = grid_points(N, np.zeros(d), np.full(d, float(N)))
    g = random_rhs(rng(config_id, 1), nrhs, N ** d)
    return Workload(name or f"fourier{d}d_N{N}_q{q}", d, N, q, "fourier",
                    np.zeros(d), np.ones(d), np.zeros(d), np.full(d, float(N)),
                    y, x, g, config_id)


def hypradon2(N: int, q: int = 5, nrhs: int = 1, config_id: int = 2,
              name: str | None = None) -> Workload:
    """Hyperbolic-Radon geometry: sources jittered on [1,2) x [0,1), targets
    x = k/N on [0,1)^2, tau = N x0 sqrt(y0^2 + x1^2 y1^2)."""
    d = 2
    slo, shi = np.array([1.0, 0.0]), np.array([2.0, 1.0])
    tlo, thi = np.zeros(2), np.ones(2)
    jit = rng(config_id, 0).random((N ** d, d))
    y = grid_points(N, slo, shi, jitter=jit)
    x = grid_points(N, tlo, thi)
    g = random_rhs(rng(config_id, 1), nrhs, N ** d)
    return Workload(name or f"hypradon2_N{N}_q{q}", d, N, q, "hypradon2",
                    slo, shi, tlo, thi, y, x, g, config_id)


def genradon3(N: int, q: int = 4, nrhs: int = 1, config_id: int = 3,
              name: str | None = None) -> Workload:
    """3-D generalized-Radon geometry: sources jittered on [0,1)^3, targets
    x = k/N on [0,1)^3."""
    d = 3
    lo, hi = np.zeros(3), np.ones(3)
    jit = rng(config_id, 0).random((N ** d, d))
    y = grid_points(N, lo, hi, jitter=jit)
    x = grid_points(N, lo, hi)
    g = random_rhs(rng(config_id, 1), nrhs, N ** d)
    return Workload(name or f"genradon3_N{N}_q{q}", d, N, q, "genradon3",
                    lo, hi, lo.copy(), hi.copy(), y, x, g, config_id)


def genradon3pi(N: int, q: int = 5, nrhs: int = 1, config_id: int = 6,
                name: str | None = None) -> Workload:
    """The generalized-Radon analogue exactly as the paper prints it (no N in
    the phase): targets x = k/N on [0,1)^3, sources p jittered on the
    frequency box [-N/2, N/2)^3."""
    d = 3
    tlo, thi = np.zeros(3), np.ones(3)
    slo, shi = np.full(3, -N / 2.0), np.full(3, N / 2.0)
    jit = rng(config_id, 0).random((N ** d, d))
    y = grid_points(N, slo, shi, jitter=jit)
    x = grid_points(N, tlo, thi)
    g = random_rhs(rng(config_id, 1), nrhs, N ** d)
    return Workload(name or f"genradon3pi_N{N}_q{q}", d, N, q, "genradon3pi",
                    slo, shi, tlo, thi, y, x, g, config_id)


def hypradon2_curve(N: int, q: int = 5, nrhs: int = 1, config_id: int = 7, per_leaf_row: int = 4,
                    curve_targets: bool = False, name: str | None = None) -> Workload:
    """Sparse points: the hyperbolic-Radon geometry with per_leaf_row * N
    sources on the curve y = (1 + u, 0.5 + 0.4 sin 2 pi u), u uniform on
    [0, 1) (so O(N) of the N^2 source leaves hold points), targets x = k/N on
    the full grid.  curve_targets puts the curve on the target side instead
    (x = (u, 0.5 + 0.4 sin 2 pi u)) with grid sources, the sparse input of an
    adjoint apply."""
    d = 2
    slo, shi = np.array([1.0, 0.0]), np.array([2.0, 1.0])
    tlo, thi = np.zeros(2), np.ones(2)
    u = np.sort(rng(config_id, 0).random(per_leaf_row * N))
    curve = np.stack([u, 0.5 + 0.4 * np.sin(2 * np.pi * u)], axis=1)
    if curve_targets:
        y = grid_points(N, slo, shi, jitter=rng(config_id, 3).random((N ** d, d)))
        x = np.ascontiguousarray(curve)
    else:
        y = np.ascontiguousarray(curve + np.array([1.0, 0.0]))
        x = grid_points(N, tlo, thi)
    g = random_rhs(rng(config_id, 1), nrhs, y.shape[0])
    kind = "tgtcurve" if curve_targets else "srccurve"
    return Workload(name or f"hypradon2_{kind}_N{N}_q{q}", d, N, q, "hypradon2",
                    slo, shi, tlo, thi, y, x, g, config_id)


def separable(N: int, d: int = 2, q: int = 3, nrhs: int = 1, config_id: int = 9) -> Workload:
    """Separable test phase tau = N (|x|^2 + sum y^3) on jittered unit grids."""
    lo, hi = np.zeros(d), np.ones(d)
    jit = rng(config_id, 0).random((N ** d, d))
    y = grid_points(N, lo, hi, jitter=jit)
    x = grid_points(N, lo, hi, jitter=rng(config_id, 3).random((N ** d, d)))
    g = random_rhs(rng(config_id, 1), nrhs, N ** d)
    return Workload(f"separable{d}d_N{N}_q{q}", d, N, q, "separable",
                    lo, hi, lo.copy(), hi.copy(), y, x, g, config_id)


# The five named workloads (sizes as stated for the method's benchmark set).
def C1(nrhs: int = 1) -> Workload:
    return fourier_grid(64, d=2, q=5, nrhs=nrhs, config_id=1, name="C1_fourier2d_N64_q5")


def C2(nrhs: int = 1) -> Workload:
    return hypradon2(1024, q=5, nrhs=nrhs, config_id=2, name="C2_hypradon2_N1024_q5")


def C3(nrhs: int = 1) -> Workload:
    return genradon3(64, q=4, nrhs=nrhs, config_id=3, name="C3_genradon3_N64_q4")


def C4(nrhs: int = 64) -> Workload:
    return fourier_grid(2048, d=2, q=6, nrhs=nrhs, config_id=4, name="C4_fourier2d_N2048_q6")


def C5_sizes(n_instances: int = 48) -> np.ndarray:
    """Sizes N_i of the uneven batch, drawn uniformly from {128, 256, 512, 1024}."""
    return rng(5, 3).choice(np.array([128, 256, 512, 1024]), size=n_instances)


def C5_instance(i: int, N: int, nrhs: int = 8) -> Workload:
    return hypradon2(int(N), q=5, nrhs=nrhs, config_id=500 + i, name=f"C5_{i}_hypradon2_N{N}")


def sample_indices(n: int, k: int, config_id: int) -> np.ndarray:
    """k distinct sorted indices in [0, n) (stream 3)."""
    k = min(k, n)
    return np.sort(rng(config_id, 3).choice(n, size=k, replace=False))
