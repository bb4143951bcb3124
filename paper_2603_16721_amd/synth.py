"""Seeded synthetic mutation matrices standing in for the paper's TCGA cohorts.

The paper measures on TCGA somatic-mutation cohorts (Sec. IV-B) that are
controlled-access; these generators produce matrices of the same shape and
structure instead: genes x samples 0/1 matrices, very sparse (the paper's
median cohort is ~95.6% zeros, Fig. 3), heavy-tailed per-gene mutation rates,
a separate normal cohort, and planted co-mutated h-gene combinations.

This module holds only input generation and bit packing.  It contains none of
the method's arithmetic (no intersections, counts, scores or search), so both
the oracle-side tests and the GPU path may use it.

Bit layout used everywhere: sample ``s`` of a gene row lives in 64-bit word
``s >> 6`` at bit ``s & 63`` (LSB first); bits past the sample count are 0.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Seeds: instance ``c`` of the five workloads uses BASE_SEED + c, batched
# instance i uses BASE_SEED + 400 + i, the served stream uses BASE_SEED + 500
# for its arrivals and BASE_SEED + 501 + j for request j.
BASE_SEED = 16721000

ZIPF_CAP = 0.30
LOGNORMAL_MEDIAN = 5e-4
LOGNORMAL_SIGMA = math.log(100.0) / 2.3263  # p99 at 100x the median (5%)
LOGNORMAL_CAP = 0.40
NORMAL_RATE_FACTOR = 0.3


@dataclasses.dataclass
class Instance:
    """One cohort: unpacked 0/1 matrices plus the generation recipe."""

    name: str
    h: int
    tumor: np.ndarray          # bool [G, n_tumor]
    normal: np.ndarray         # bool [G, n_normal]
    planted: list              # list of (genes tuple, samples array)
    alpha_p: int = 1
    alpha_q: int = 10
    target_covered: int = 0    # <= 0 means all tumour samples
    seed: int = 0
    rates: np.ndarray | None = None

    @property
    def G(self) -> int:
        return self.tumor.shape[0]

    @property
    def n_tumor(self) -> int:
        return self.tumor.shape[1]

    @property
    def n_normal(self) -> int:
        return self.normal.shape[1]

    def packed(self):
        return pack_rows(self.tumor), pack_rows(self.normal)


def words_for(n_samples: int) -> int:
    return max(1, (n_samples + 63) // 64)


def pack_rows(bits: np.ndarray) -> np.ndarray:
    """bool [G, n] -> uint64 [G, ceil(n/64)] with the LSB-first layout."""
    bits = np.asarray(bits, dtype=bool)
    G, n = bits.shape
    W = words_for(n)
    padded = np.zeros((G, W * 64), dtype=bool)
    padded[:, :n] = bits
    by = np.packbits(padded, axis=1, bitorder="little")  # [G, W*8] uint8
    return np.ascontiguousarray(by).view("<u8").reshape(G, W).astype(np.uint64)


def unpack_rows(words: np.ndarray, n: int) -> np.ndarray:
    """uint64 [G, W] -> bool [G, n] (inverse of pack_rows)."""
    words = np.ascontiguousarray(np.asarray(words, dtype=np.uint64))
    G, W = words.shape
    by = words.astype("<u8").view(np.uint8).reshape(G, W * 8)
    return np.unpackbits(by, axis=1, bitorder="little")[:, :n].astype(bool)


def zipf_rates(G: int, s: float, mean: float, cap: float = ZIPF_CAP) -> np.ndarray:
    """r_k = min(c * k^-s, cap) for k = 1..G with c chosen so mean(r) == mean."""
    k = np.arange(1, G + 1, dtype=np.float64)
    base = k ** (-s)

    def mean_for(c):
        return float(np.minimum(c * base, cap).mean())

    lo, hi = 0.0, 1.0
    while mean_for(hi) < mean:
        hi *= 2.0
        if hi > 1e12:
            raise ValueError("mean density unreachable under the cap")
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mean_for(mid) < mean:
            lo = mid
        else:
            hi = mid
    return np.minimum(hi * base, cap)


def lognormal_rates(G: int, rng: np.random.Generator) -> np.ndarray:
    r = np.exp(rng.normal(math.log(LOGNORMAL_MEDIAN), LOGNORMAL_SIGMA, size=G))
    return np.minimum(r, LOGNORMAL_CAP)


def make_instance(name, rng, G, n_tumor, n_normal, h, rates_sorted, n_planted,
                  planted_sizes, target_covered=0, seed=0, alpha=(1, 10),
                  normal_factor=NORMAL_RATE_FACTOR) -> Instance:
    """Draw one cohort.

    rates_sorted are assigned to genes through a seeded permutation so that
    caller gene order is not density order.  Tumour bits are Bernoulli(r_g),
    normal bits Bernoulli(normal_factor * r_g).  Each planted combination takes
    h distinct genes from those at or below the median rate (disjoint across
    combinations) and sets them in a disjoint set of tumour samples (disjoint
    while enough unused samples remain).
    """
    perm = rng.permutation(G)
    rates = np.asarray(rates_sorted, dtype=np.float64)[perm]
    tumor = rng.random((G, n_tumor)) < rates[:, None]
    normal = rng.random((G, n_normal)) < (normal_factor * rates)[:, None]
    planted = []
    eligible = np.flatnonzero(rates <= np.median(rates))
    used_genes = np.zeros(G, dtype=bool)
    free_samples = np.ones(n_tumor, dtype=bool)
    for k in range(n_planted):
        cand = eligible[~used_genes[eligible]]
        if cand.size < h:
            break
        genes = np.sort(rng.choice(cand, size=h, replace=False))
        used_genes[genes] = True
        m = int(planted_sizes[k])
        pool = np.flatnonzero(free_samples)
        if pool.size < m:
            pool = np.arange(n_tumor)
        m = min(m, pool.size)
        samples = np.sort(rng.choice(pool, size=m, replace=False))
        free_samples[samples] = False
        tumor[np.ix_(genes, samples)] = True
        planted.append((tuple(int(g) for g in genes), samples))
    return Instance(name=name, h=h, tumor=tumor, normal=normal, planted=planted,
                    alpha_p=alpha[0], alpha_q=alpha[1],
                    target_covered=target_covered, seed=seed, rates=rates)


# ---------------------------------------------------------------- workloads
def workload_small_h2() -> Instance:
    """h=2, G=500, 200 tumour / 100 normal, Zipf(1.2) at 1% mean, 3 planted pairs x 20."""
    seed = BASE_SEED + 1
    rng = np.random.Generator(np.random.PCG64(seed))
    rates = zipf_rates(500, 1.2, 0.01)
    return make_instance("h2_G500", rng, 500, 200, 100, 2, rates, 3, [20, 20, 20],
                         target_covered=0, seed=seed)


def workload_h3_g5000() -> Instance:
    """h=3, G=5000, 1000/400, Zipf(1.1) at 0.5%, 8 planted triples x U{15..60}, stop at 95%."""
    seed = BASE_SEED + 2
    rng = np.random.Generator(np.random.PCG64(seed))
    rates = zipf_rates(5000, 1.1, 0.005)
    sizes = rng.integers(15, 61, size=8)
    return make_instance("h3_G5000", rng, 5000, 1000, 400, 3, rates, 8, sizes,
                         target_covered=int(math.ceil(0.95 * 1000)), seed=seed)


def workload_h4_g20000() -> Instance:
    """h=4, G=20000, 1000/500, log-normal rates (median 0.05%, p99 5%, max 40%),
    10 planted quadruples x U{10..40}."""
    seed = BASE_SEED + 3
    rng = np.random.Generator(np.random.PCG64(seed))
    rates = lognormal_rates(20000, rng)
    sizes = rng.integers(10, 41, size=10)
    return make_instance("h4_G20000", rng, 20000, 1000, 500, 4, rates, 10, sizes,
                         target_covered=0, seed=seed)


def batched_instance(i: int) -> Instance:
    """Instance i (0..31) of the batched workload: G~U{2000..20000},
    Nt~U{50..1200}, Nn~U{50..500}, h~U{3,4}, Zipf(1.1) at U[0.3%,1%] mean,
    U{2..6} planted combos x U{10..40} samples (capped at Nt/(2*count))."""
    seed = BASE_SEED + 400 + i
    rng = np.random.Generator(np.random.PCG64(seed))
    G = int(rng.integers(2000, 20001))
    nt = int(rng.integers(50, 1201))
    nn = int(rng.integers(50, 501))
    h = int(rng.integers(3, 5))
    mean = float(rng.uniform(0.003, 0.01))
    count = int(rng.integers(2, 7))
    sizes = np.minimum(rng.integers(10, 41, size=count), nt // (2 * count))
    rates = zipf_rates(G, 1.1, mean)
    return make_instance(f"batch{i}", rng, G, nt, nn, h, rates, count, sizes, seed=seed)


def served_arrivals(n: int = 2000, mean_gap_s: float = 0.05) -> np.ndarray:
    """Poisson arrival times (seconds from stream start) for the served workload."""
    rng = np.random.Generator(np.random.PCG64(BASE_SEED + 500))
    return np.cumsum(rng.exponential(mean_gap_s, size=n))


def served_request(j: int) -> Instance:
    """Request j of the served workload: h in {2,3,4} w.p. 0.3/0.5/0.2,
    G~U{1000..20000}, Nt~U{100..1000}, Nn~U{50..500}, Zipf(1.1) at 0.5% mean,
    U{2..6} planted combos x U{10..40} samples (capped at Nt/(2*count))."""
    seed = BASE_SEED + 501 + j
    rng = np.random.Generator(np.random.PCG64(seed))
    h = int(rng.choice([2, 3, 4], p=[0.3, 0.5, 0.2]))
    G = int(rng.integers(1000, 20001))
    nt = int(rng.integers(100, 1001))
    nn = int(rng.integers(50, 501))
    count = int(rng.integers(2, 7))
    sizes = np.minimum(rng.integers(10, 41, size=count), nt // (2 * count))
    rates = zipf_rates(G, 1.1, 0.005)
    return make_instance(f"req{j}", rng, G, nt, nn, h, rates, count, sizes, seed=seed)


def random_tiny(seed: int, G: int, n_tumor: int, n_normal: int, density: float,
                h: int, alpha=(1, 10)) -> Instance:
    """Small uniform-density instance for brute-force comparisons."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rates = np.full(G, density)
    return make_instance(f"tiny{seed}", rng, G, n_tumor, n_normal, h, rates, 0, [],
                         seed=seed, alpha=alpha)


WORKLOADS = {
    "h2_G500": workload_small_h2,
    "h3_G5000": workload_h3_g5000,
    "h4_G20000": workload_h4_g20000,
}
