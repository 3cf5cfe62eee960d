"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

This module holds only inputs: lattice shapes, couplings, step counts, seeds,
random states and request streams.  It contains none of the method's
arithmetic (no schedule, no evolution, no observable) and imports neither the
GPU library nor the oracle, so both sides can draw the same inputs from it.

The shapes follow the paper's workloads (Sec. 2.1 and 2.6): the 3x3 2+1D
torus (18 links) and the 2x2x2 3+1D torus (24 links), plus the 2x2 torus (8
links) and the 4x4 torus (32 links) at the two ends of the size range.  The
paper uses no dataset; every input here is synthetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED = 20191008


@dataclass(frozen=True)
class Workload:
    name: str
    d: int
    L: tuple
    n_steps: int
    T: float
    order: int                 # 1 = first order (eq. (a)), 2 = symmetric (eq. (s))
    lambdas: tuple             # h_x / h_p values, h_p = 1
    dtype: str                 # "c64" or "c128"
    forms: tuple = ("fused",)
    extra: dict = field(default_factory=dict)

    @property
    def n_links(self) -> int:
        v = 1
        for x in self.L:
            v *= x
        return self.d * v


# the five configurations: 2x2 (8 links), 3x3 lambda scan (18), 2x2x2 (24),
# serving mix, 4x4 (32).  dt = 0.05 wherever the total time is not fixed.
CONFIG1 = Workload("2x2 first-order, T=50, 1000 steps", 2, (2, 2), 1000, 50.0, 1,
                   (1.0,), "c128")
CONFIG2 = Workload("3x3 symmetric lambda scan, T=100, 2000 steps", 2, (3, 3), 2000, 100.0, 2,
                   tuple(0.1 + 0.095 * i for i in range(21)), "c64")
CONFIG3 = Workload("2x2x2 symmetric, T=100, 2000 steps", 3, (2, 2, 2), 2000, 100.0, 2,
                   (0.2, 0.5, 1.0, 2.0), "c64", forms=("fused", "circuit"))
CONFIG5 = Workload("4x4 symmetric, T=50, 1000 steps", 2, (4, 4), 1000, 50.0, 2,
                   (0.5, 1.0, 1.5), "c64")

SERVING_MIX = (  # (probability, d, L)
    (0.6, 2, (3, 3)),
    (0.3, 3, (2, 2, 2)),
    (0.1, 2, (2, 2)),
)

# rectangular tori for the bandwidth sweep: 24, 28, 30 and 32 links
SWEEP_LATTICES = ((2, (3, 4)), (3, (2, 2, 2)), (2, (2, 7)), (2, (3, 5)), (2, (4, 4)))


def rng(seed: int = SEED, stream: int = 0) -> np.random.Generator:
    return np.random.default_rng([seed, stream])


def random_state(n_qubits: int, seed: int = SEED, stream: int = 0,
                 dtype=np.complex128) -> np.ndarray:
    """A normalised complex Gaussian state of 2^n amplitudes (Haar-like)."""
    g = rng(seed, stream)
    dim = 1 << n_qubits
    psi = g.standard_normal(dim) + 1j * g.standard_normal(dim)
    psi /= np.sqrt(np.vdot(psi, psi).real)
    return psi.astype(dtype)


def random_couplings(n: int, seed: int = SEED, stream: int = 1, lo=0.0, hi=2.0) -> np.ndarray:
    return rng(seed, stream).uniform(lo, hi, size=n)


@dataclass
class Request:
    arrival_s: float
    d: int
    L: tuple
    lam: float
    n_steps: int
    order: int


def serving_stream(n_requests: int, rate_per_s: float, seed: int = SEED,
                   steps_lo: int = 500, steps_hi: int = 4000) -> list:
    """Poisson arrivals of adiabatic runs: 60% 3x3, 30% 2x2x2, 10% 2x2 (by count).

    lambda ~ U[0, 2], steps ~ U{steps_lo..steps_hi}, order 1 or 2 with equal
    probability.  Every request uses dt = 0.05 (T = 0.05 * steps).
    """
    g = rng(seed, 7)
    gaps = g.exponential(1.0 / rate_per_s, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    probs = np.array([m[0] for m in SERVING_MIX])
    kinds = g.choice(len(SERVING_MIX), size=n_requests, p=probs / probs.sum())
    lams = g.uniform(0.0, 2.0, size=n_requests)
    steps = g.integers(steps_lo, steps_hi + 1, size=n_requests)
    orders = g.integers(1, 3, size=n_requests)
    out = []
    for i in range(n_requests):
        _, d, L = SERVING_MIX[kinds[i]]
        out.append(Request(float(t[i]), d, L, float(lams[i]), int(steps[i]), int(orders[i])))
    return out
