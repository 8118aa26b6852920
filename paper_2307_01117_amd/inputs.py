"""Seeded synthetic inputs for the heat-stencil workloads.

This module holds no arithmetic of the method: it only draws initial states
and problem parameters.  The tests feed the same arrays to the GPU library and
to the CPU oracle, and the benchmark uses it to build its workloads.

Random streams are NumPy's PCG64 (``numpy.random.default_rng``): a seed ``s``
gives ``default_rng(s)``, per-ring and per-request streams are seeded with a
list ``[workload_id, index]``.

Workloads (sizes follow the paper's benchmark of 1,000,000 nodes x 1,000 steps,
Section 5, scaled up to fill one MI355X):

* ``uniform_ring``  -- the plain FP64 ring: Uniform[0,1) cells;
* ``sine_mode``     -- u0[i] = sin(2*pi*m*i/N), a single Fourier mode;
* ``perturbed_ring``-- 1 + 1e-3*Uniform[-1,1): a large mean with small
  perturbations (stresses cancellation in reduced precision);
* ``ramp``          -- the paper's own initial condition u(0, x_i) = x_i;
* ``batch_specs``   -- 4,096 independent rings with uneven sizes and step counts;
* ``serving_trace`` -- Poisson arrivals of heat-solve requests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Named single-ring workloads: (N, nparts, r, nt, generator name, seed)
WORKLOADS = {
    # 10 partitions x 100,000 cells, r = 0.5 (k=0.5, dt=1, dx=1), 100 steps
    "ring_1e6": dict(N=1_000_000, nparts=10, r=0.5, nt=100, init="uniform", seed=0),
    # 100 partitions x 1,000,000 cells, r = 0.5, 1,000 steps
    "ring_1e8": dict(N=100_000_000, nparts=100, r=0.5, nt=1000, init="uniform", seed=1),
    # same ring, r = 0.25, perturbed state, for the FP32 / compensated FP32 forms
    "ring_1e8_perturbed": dict(N=100_000_000, nparts=100, r=0.25, nt=1000,
                               init="perturbed", seed=2),
    # a mid-size ring: 10 partitions x 1,000,000 cells, 1,000 steps
    "ring_1e7": dict(N=10_000_000, nparts=10, r=0.5, nt=1000, init="uniform", seed=0),
    # the paper's own run: 1,000,000 nodes, 1,000 steps, initial condition
    # u(0, x_i) = x_i (h = 1); r = 0.5 (the paper does not state alpha, dt, h)
    "paper_ramp_1e6": dict(N=1_000_000, nparts=40, r=0.5, nt=1000, init="ramp", seed=0),
}


def uniform_ring(N: int, seed) -> np.ndarray:
    """Uniform[0,1) binary64 cells."""
    return np.random.default_rng(seed).random(int(N))


def perturbed_ring(N: int, seed, amp: float = 1e-3) -> np.ndarray:
    """1 + amp*Uniform[-1,1)."""
    x = np.random.default_rng(seed).random(int(N))
    return 1.0 + amp * (2.0 * x - 1.0)


def sine_mode(N: int, m: int = 3) -> np.ndarray:
    """A single Fourier mode sin(2*pi*m*i/N)."""
    i = np.arange(int(N), dtype=np.float64)
    return np.sin(2.0 * np.pi * m * i / N)


def ramp(N: int, h: float = 1.0) -> np.ndarray:
    """The paper's initial condition u(0, x_i) = x_i = i*h."""
    return np.arange(int(N), dtype=np.float64) * h


def make_initial(init: str, N: int, seed=0) -> np.ndarray:
    if init == "uniform":
        return uniform_ring(N, seed)
    if init == "perturbed":
        return perturbed_ring(N, seed)
    if init == "sine":
        return sine_mode(N)
    if init == "ramp":
        return ramp(N)
    raise ValueError(f"unknown initial state {init!r}")


def small_integer_ring(N: int, seed, lo: int = -8, hi: int = 8) -> np.ndarray:
    """Integers in [lo, hi] stored as binary64 (exact-arithmetic test cases)."""
    return np.random.default_rng(seed).integers(lo, hi + 1, int(N)).astype(np.float64)


# ---------------------------------------------------------------- batching

@dataclass
class RingSpec:
    N: int
    nparts: int
    nt: int
    r: float
    seed: tuple


def batch_specs(count: int = 4096, seed: int = 4, logn_lo: float = 3.0, logn_hi: float = 6.0,
                nt_lo: int = 100, nt_hi: int = 10_000, cells_per_part: int = 1000):
    """Uneven independent rings: N log-uniform in [10^lo, 10^hi], nt uniform in
    [nt_lo, nt_hi], r uniform in (0.1, 0.5], partitions of ``cells_per_part``
    cells.  u0 of ring j comes from ``ring_initial(spec)``."""
    rng = np.random.default_rng(seed)
    logn = rng.uniform(logn_lo, logn_hi, count)
    Ns = np.floor(10.0 ** logn).astype(np.int64)
    nts = rng.integers(nt_lo, nt_hi + 1, count)
    rs = 0.5 - 0.4 * rng.random(count)
    out = []
    for j in range(count):
        N = int(Ns[j])
        out.append(RingSpec(N=N, nparts=max(1, math.ceil(N / cells_per_part)), nt=int(nts[j]),
                            r=float(rs[j]), seed=(seed, j)))
    return out


def ring_initial(spec: RingSpec) -> np.ndarray:
    return np.random.default_rng(list(spec.seed)).random(spec.N)


# ---------------------------------------------------------------- serving

@dataclass
class Request:
    t_arrival: float
    N: int
    nt: int
    r: float
    precision: int      # 0 = FP64, 2 = compensated FP32
    offset: int         # start of u0 inside the shared pool
    key: tuple


def serving_trace(rate: float, duration: float, seed: int = 5, logn_lo: float = 3.0,
                  logn_hi: float = 7.0, nt_lo: int = 100, nt_hi: int = 5000,
                  pool_size: int = 1 << 24):
    """Poisson arrivals at ``rate`` req/s over ``duration`` s.  Each request
    draws N log-uniform, nt uniform, r in (0.1, 0.5], FP64 or compensated FP32
    with probability 1/2, and a start offset into a shared Uniform[0,1) pool
    (u0[i] = pool[(offset + i) mod pool_size], see ``request_initial``)."""
    rng = np.random.default_rng([seed, int(rate)])
    reqs = []
    t = 0.0
    k = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        N = int(math.floor(10.0 ** rng.uniform(logn_lo, logn_hi)))
        nt = int(rng.integers(nt_lo, nt_hi + 1))
        r = float(0.5 - 0.4 * rng.random())
        prec = 0 if rng.random() < 0.5 else 2
        off = int(rng.integers(0, pool_size))
        reqs.append(Request(t, N, nt, r, prec, off, (seed, int(rate), k)))
        k += 1
    return reqs


def serving_pool(pool_size: int = 1 << 24, seed: int = 5) -> np.ndarray:
    return np.random.default_rng([seed, 0]).random(pool_size)


def request_initial(pool: np.ndarray, req: Request) -> np.ndarray:
    idx = (req.offset + np.arange(req.N, dtype=np.int64)) % pool.size
    return pool[idx]
