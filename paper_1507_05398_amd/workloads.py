"""Seeded synthetic workloads (instance lists only; no part of the method).

The paper's workloads are whole spaces F_2^n, fixed by (n, d, ordering), so
the only inputs to generate are which instances to build and when they
arrive.  Both the GPU path and the CPU oracle consume these lists.
"""
import numpy as np

ORDER_NAMES = ["lex", "gray", "grlex", "grevlex"]


def batched_instances(seed: int = 1507, count: int = 256, n_lo: int = 12, n_hi: int = 24,
                      d_lo: int = 3, d_hi: int = 8):
    """`count` instances with n ~ U{n_lo..n_hi}, d ~ U{d_lo..d_hi}, ordering
    uniform over the four (numpy PCG64 generator with the given seed)."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    ds = rng.integers(d_lo, d_hi + 1, size=count)
    os_ = rng.integers(0, 4, size=count)
    return [(int(n), int(d), ORDER_NAMES[int(o)]) for n, d, o in zip(ns, ds, os_)]


def served_jobs(seed: int = 1507, count: int = 10000, rate: float = 1000.0, n_lo: int = 10,
                n_hi: int = 26, d_lo: int = 3, d_hi: int = 10):
    """Poisson arrivals at `rate` jobs/s: list of (arrival_s, n, d, ordering).
    n is skewed toward small lengths, P(n) proportional to 2^(-(n - n_lo)/2);
    d ~ U{d_lo..d_hi}; ordering uniform."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    support = np.arange(n_lo, n_hi + 1)
    w = 2.0 ** (-(support - n_lo) / 2.0)
    ns = rng.choice(support, size=count, p=w / w.sum())
    ds = rng.integers(d_lo, d_hi + 1, size=count)
    os_ = rng.integers(0, 4, size=count)
    return [(float(t), int(n), int(d), ORDER_NAMES[int(o)]) for t, n, d, o in zip(arrivals, ns, ds, os_)]
