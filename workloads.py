"""Seeded synthetic inputs for the H^2 evaluation workloads.

This module only draws random numbers and describes the workload shapes.  It
holds none of the method's arithmetic (no tree, no kernel function, no
compression, no evaluation), so that both the CPU oracle (test
infrastructure) and the GPU library can be fed from it without sharing code.

The paper's experiments use UCI machine-learning point sets and scientific
point sets (Table 1 of the paper), which are not available here.  Every
workload below is a synthetic stand-in with the same dimensionality class:
low-d uniform points (like the d=2..3 scientific sets) and high-d points
(d=8 Gaussian mixtures, d=28 i.i.d. normal like the d=28 UCI sets).

Recipe (numpy ``default_rng``; draws happen in exactly this order):
  * uniform cube:  X = rng.uniform(0, 1, (N, d))
  * mixture:       centres = rng.uniform(-4, 4, (C, d));
                   labels = rng.integers(0, C, N);
                   X = centres[labels] + rng.standard_normal((N, d))
  * normal:        X = rng.standard_normal((N, d))
  * W:             rng = default_rng(w_seed); W = rng.standard_normal((N, Q))
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

KERNEL_GAUSSIAN = 0  # exp(-r^2 / (2 h^2))
KERNEL_LAPLACE = 1   # exp(-r / h)

ADM_DISTANCE = 0     # far iff tau * dist > diam(a) + diam(b)
ADM_HSS = 1          # every off-diagonal block is far (weak admissibility)
ADM_BUDGET = 2       # near = each leaf's budget share of nearest leaves (H^2-b); the rest far

PART_MEDIAN = 0      # cut at the median of the widest coordinate
PART_TWO_MEANS = 1   # cut at the median along the direction between two means


@dataclasses.dataclass(frozen=True)
class Workload:
    """One compressed-matrix workload: points, kernel, compression knobs, W."""
    name: str
    N: int
    d: int
    points: str            # "uniform" | "mixture" | "normal"
    point_seed: int
    kernel: int
    h: float
    m: int                 # leaf size
    tol: float             # block (ID) tolerance
    rmax: int              # maximum rank
    adm: int               # ADM_DISTANCE | ADM_HSS
    tau: float             # admissibility parameter (distance mode)
    Q: int                 # columns of W
    w_seed: int = 1
    n_comp: int = 16       # mixture components
    sample_rows: int = 4096  # row-sample cap for the ID (exact rows below it)
    sample_seed: int = 7
    part: int = PART_MEDIAN  # tree partitioner
    budget: float = 0.0      # ADM_BUDGET: near leaves per leaf = floor(budget * #leaves)

    def key(self) -> str:
        return hashlib.sha256(repr(dataclasses.astuple(self)).encode()).hexdigest()[:16]


# Small correctness case: 4096 points uniform in the unit cube, d=3.
C1 = Workload("c1_n4096_d3_uniform", N=4096, d=3, points="uniform", point_seed=0,
              kernel=KERNEL_GAUSSIAN, h=0.5, m=64, tol=1e-5, rmax=64,
              adm=ADM_DISTANCE, tau=2.0, Q=16)

# Headline case: 65536 points, d=8, 16-component Gaussian mixture, Q=256.
C2 = Workload("c2_n65536_d8_mixture", N=65536, d=8, points="mixture", point_seed=0,
              kernel=KERNEL_GAUSSIAN, h=1.0, m=128, tol=1e-5, rmax=128,
              adm=ADM_DISTANCE, tau=2.0, Q=256)

# The headline points under the paper's high-d structure (Section 3.1: two-means
# tree for d > 3; Section 4.1: budget 0.03, "H^2-b").
C2B = Workload("c2b_n65536_d8_mixture_two_means_budget", N=65536, d=8, points="mixture", point_seed=0,
               kernel=KERNEL_GAUSSIAN, h=1.0, m=128, tol=1e-5, rmax=128,
               adm=ADM_BUDGET, tau=2.0, Q=256, part=PART_TWO_MEANS, budget=0.03)

# Mixed-precision case: 262144 points, d=28 i.i.d. normal, Laplace, HSS.
C4 = Workload("c4_n262144_d28_normal", N=262144, d=28, points="normal", point_seed=0,
              kernel=KERNEL_LAPLACE, h=4.0, m=256, tol=1e-4, rmax=256,
              adm=ADM_HSS, tau=2.0, Q=1024)


def batched_workloads(count: int = 64, base_seed: int = 1000) -> list[Workload]:
    """Many uneven matrices for the batched form: N in [2048, 32768],
    d in {3 uniform, 8 mixture}, h in [0.3, 1.5], m in [64, 128], Q in [8, 512]."""
    out = []
    for b in range(count):
        rng = np.random.default_rng(base_seed + b)
        N = int(rng.integers(2048, 32769))
        low_d = bool(rng.integers(0, 2))
        h = float(rng.uniform(0.3, 1.5))
        m = int(rng.integers(64, 129))
        Q = int(rng.integers(8, 513))
        out.append(Workload(f"b{b}", N=N, d=3 if low_d else 8,
                            points="uniform" if low_d else "mixture",
                            point_seed=base_seed + b, kernel=KERNEL_GAUSSIAN, h=h, m=m,
                            tol=1e-6, rmax=m, adm=ADM_DISTANCE, tau=2.0, Q=Q,
                            w_seed=base_seed + b + 100000))
    return out


def serving_workloads() -> list[Workload]:
    """Eight resident matrices for the serving form: N from 16384 to 524288,
    d in {3, 8, 28}, distance admissibility (H^2) for d <= 8 and HSS for d = 28
    (where distance admissibility degenerates), tol 1e-5."""
    def g(name, N, d, points, h, m, adm, kernel=KERNEL_GAUSSIAN, seed=0):
        return Workload(name, N=N, d=d, points=points, point_seed=2000 + seed, kernel=kernel, h=h,
                        m=m, tol=1e-5, rmax=m, adm=adm, tau=2.0, Q=256, w_seed=3000 + seed)
    return [
        g("s1_n16384_d3_h2", 16384, 3, "uniform", 0.5, 64, ADM_DISTANCE, seed=1),
        g("s2_n32768_d8_h2", 32768, 8, "mixture", 1.0, 128, ADM_DISTANCE, seed=2),
        g("s3_n65536_d28_hss", 65536, 28, "normal", 4.0, 128, ADM_HSS, KERNEL_LAPLACE, seed=3),
        g("s4_n65536_d3_h2", 65536, 3, "uniform", 0.5, 128, ADM_DISTANCE, seed=4),
        g("s5_n131072_d3_h2", 131072, 3, "uniform", 0.5, 128, ADM_DISTANCE, seed=5),
        g("s6_n131072_d28_hss", 131072, 28, "normal", 4.0, 128, ADM_HSS, KERNEL_LAPLACE, seed=6),
        g("s7_n262144_d3_h2", 262144, 3, "uniform", 0.5, 128, ADM_DISTANCE, seed=7),
        g("s8_n524288_d3_h2", 524288, 3, "uniform", 0.5, 128, ADM_DISTANCE, seed=8),
    ]


def small(name: str, N: int, d: int = 3, points: str = "uniform", m: int = 32,
          Q: int = 8, adm: int = ADM_DISTANCE, kernel: int = KERNEL_GAUSSIAN,
          h: float = 0.5, tol: float = 1e-6, rmax: int = 64, tau: float = 2.0,
          seed: int = 3, sample_rows: int = 4096, part: int = PART_MEDIAN,
          budget: float = 0.0) -> Workload:
    """A small workload for unit tests and edge cases."""
    return Workload(name, N=N, d=d, points=points, point_seed=seed, kernel=kernel, h=h,
                    m=m, tol=tol, rmax=rmax, adm=adm, tau=tau, Q=Q, w_seed=seed + 1,
                    sample_rows=sample_rows, part=part, budget=budget)


def gen_points(w: Workload) -> np.ndarray:
    """N x d float64 points, C-contiguous, seeded."""
    rng = np.random.default_rng(w.point_seed)
    if w.points == "uniform":
        X = rng.uniform(0.0, 1.0, (w.N, w.d))
    elif w.points == "mixture":
        centres = rng.uniform(-4.0, 4.0, (w.n_comp, w.d))
        labels = rng.integers(0, w.n_comp, w.N)
        X = centres[labels] + rng.standard_normal((w.N, w.d))
    elif w.points == "normal":
        X = rng.standard_normal((w.N, w.d))
    else:
        raise ValueError(f"unknown point distribution {w.points!r}")
    return np.ascontiguousarray(X, dtype=np.float64)


def gen_w(w: Workload, Q: int | None = None, seed: int | None = None) -> np.ndarray:
    """N x Q float64 standard-normal right-hand side, C-contiguous, seeded."""
    rng = np.random.default_rng(w.w_seed if seed is None else seed)
    return np.ascontiguousarray(rng.standard_normal((w.N, w.Q if Q is None else Q)))


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
