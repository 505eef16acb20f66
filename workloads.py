"""Seeded synthetic inputs for the PivCo-Huffman hot path.

This module only draws bytes; it holds none of the codec's arithmetic.  The
CPU oracle, the GPU library, the tests and the benchmark all consume the same
bytes produced here, so generator details cannot break parity.

Workloads (sizes in bytes, MiB = 2**20):
  geo1m    1 MiB, one block, p(s) ~ 0.8**s over 256 symbols
  zipf256m 256 MiB in 64 KiB blocks, Zipf(1.1) over 256 ranks mapped to
           symbol ids by a seeded permutation; one tree per block, no ANS
  skew256m 256 MiB in 128 KiB blocks, p(0) = 0.9 and the remaining 0.1
           spread ~ 0.7**s over symbols 1..255; selective rANS on nodes whose
           one-bit fraction is below 0.1 or above 0.9
  mix4096  4096 independent blocks, sizes log-uniform in [4 KiB, 4 MiB]; each
           block draws its family (1/3 each): truncated geometric r~U[0.5,0.95],
           Zipf s~U[0.8,1.5] with permuted ids, uniform over k~U{2..256}
           symbols 0..k-1; selective rANS
  serve    requests with sizes log-uniform in [16 KiB, 64 MiB], same family mix,
           each coded as a stream of blocks of at most 1 MiB
A ``scale`` divisor shrinks the totals for tests while keeping block sizes
(and therefore tree shapes and per-block statistics) unchanged.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

KiB = 1 << 10
MiB = 1 << 20

_CHUNK = 1 << 24  # symbols drawn per step, bounds temporary memory


def draw(rng: np.random.Generator, p: np.ndarray, n: int) -> np.ndarray:
    """n i.i.d. symbols from the distribution p over 256 ids: inverse CDF on
    32-bit integers (symbol = number of CDF edges <= u).  A 65536-entry table
    answers every u whose upper 16 bits select a bucket without an edge inside;
    the few remaining values use a binary search, so the result equals the
    plain search exactly."""
    p = np.asarray(p, dtype=np.float64)
    p = p / p.sum()
    cdf = np.minimum(np.floor(np.cumsum(p) * 2.0 ** 32), 2.0 ** 32).astype(np.uint64)
    cdf[-1] = 1 << 32
    edges = cdf[:-1]
    lo = np.arange(1 << 16, dtype=np.uint64) << np.uint64(16)
    base = np.searchsorted(edges, lo, side="right")
    top = np.searchsorted(edges, lo + np.uint64(0xFFFF), side="right")
    table = base.astype(np.uint8)
    pure = base == top
    out = np.empty(n, dtype=np.uint8)
    for s in range(0, n, _CHUNK):
        k = min(_CHUNK, n - s)
        u = rng.integers(0, 1 << 32, size=k, dtype=np.uint64)
        hi = (u >> np.uint64(16)).astype(np.int64)
        sym = table[hi]
        mixed = np.flatnonzero(~pure[hi])
        if mixed.size:
            sym[mixed] = np.searchsorted(edges, u[mixed], side="right").astype(np.uint8)
        out[s:s + k] = sym
    return out


def geometric_p(r: float, k: int = 256) -> np.ndarray:
    p = np.zeros(256)
    p[:k] = r ** np.arange(k)
    return p


def zipf_p(s: float, rng: np.random.Generator | None, k: int = 256) -> np.ndarray:
    ranks = np.arange(1, k + 1, dtype=np.float64)
    q = ranks ** (-s)
    p = np.zeros(256)
    if rng is None:
        p[:k] = q
    else:
        perm = rng.permutation(256)[:k]
        p[perm] = q
    return p


def skew_p() -> np.ndarray:
    t = 0.7 ** np.arange(1, 256)
    p = np.zeros(256)
    p[0] = 0.9
    p[1:] = 0.1 * t / t.sum()
    return p


def family_p(rng: np.random.Generator) -> tuple[str, np.ndarray]:
    """One block's distribution for the mixed workloads."""
    fam = int(rng.integers(0, 3))
    if fam == 0:
        r = float(rng.uniform(0.5, 0.95))
        return f"geometric(r={r:.3f})", geometric_p(r)
    if fam == 1:
        s = float(rng.uniform(0.8, 1.5))
        return f"zipf(s={s:.3f})", zipf_p(s, rng)
    k = int(rng.integers(2, 257))
    p = np.zeros(256)
    p[:k] = 1.0
    return f"uniform(k={k})", p


def log_uniform_size(rng: np.random.Generator, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


@dataclass
class Workload:
    name: str
    block_size: int                      # symbols per block of each job
    ans_mode: int                        # 0 none, 1 selective rule
    jobs: list = field(default_factory=list)  # list of uint8 arrays
    labels: list = field(default_factory=list)

    @property
    def total(self) -> int:
        return int(sum(j.size for j in self.jobs))


def geo1m(seed: int = 1, scale: int = 1) -> Workload:
    rng = np.random.default_rng(seed)
    n = MiB // scale
    return Workload("geo1m", block_size=MiB, ans_mode=0, jobs=[draw(rng, geometric_p(0.8), n)],
                    labels=["geometric(r=0.8)"])


def zipf256m(seed: int = 1, scale: int = 1) -> Workload:
    rng = np.random.default_rng(seed)
    p = zipf_p(1.1, rng)
    n = 256 * MiB // scale
    return Workload("zipf256m", block_size=64 * KiB, ans_mode=0, jobs=[draw(rng, p, n)],
                    labels=["zipf(s=1.1)"])


def skew256m(seed: int = 1, scale: int = 1) -> Workload:
    rng = np.random.default_rng(seed)
    n = 256 * MiB // scale
    return Workload("skew256m", block_size=128 * KiB, ans_mode=1, jobs=[draw(rng, skew_p(), n)],
                    labels=["p0=0.9+0.7^s"])


def _mixed_item(child: np.random.SeedSequence, lo: int, hi: int):
    """One independently seeded item of the mixed workloads: a log-uniform
    size and a family drawn from its own stream, then its symbols."""
    rng = np.random.default_rng(child)
    size = log_uniform_size(rng, lo, hi)
    label, p = family_p(rng)
    return draw(rng, p, size), label


def _mixed_items(seed: int, n: int, lo: int, hi: int, workers: int):
    """Items 0..n-1 of the mixed workloads; every item has its own seed, so
    drawing them in worker processes gives the same bytes as drawing them in
    order here."""
    children = np.random.SeedSequence(seed).spawn(n)
    if workers <= 1 or n < 2:
        out = [_mixed_item(c, lo, hi) for c in children]
    else:
        import concurrent.futures as cf
        import multiprocessing as mp
        # fork: the caller draws inputs before it initialises a GPU
        with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
            out = list(ex.map(_mixed_item, children, [lo] * n, [hi] * n,
                              chunksize=max(1, n // (8 * workers))))
    return [x for x, _ in out], [lab for _, lab in out]


def mix4096(seed: int = 1, scale: int = 1, n_blocks: int = 4096,
            lo: int = 4 * KiB, hi: int = 4 * MiB, workers: int = 1) -> Workload:
    """``scale`` divides the block count (block sizes keep their range)."""
    nb = max(1, n_blocks // scale)
    jobs, labels = _mixed_items(seed, nb, lo, hi, workers)
    return Workload("mix4096", block_size=0, ans_mode=1, jobs=jobs, labels=labels)


def serve_requests(seed: int = 1, n_req: int = 64, lo: int = 16 * KiB, hi: int = 64 * MiB,
                   workers: int = 1):
    """Request payloads for the serving loop (block size 1 MiB each)."""
    jobs, labels = _mixed_items(seed, n_req, lo, hi, workers)
    return Workload("serve", block_size=MiB, ans_mode=1, jobs=jobs, labels=labels)


def poisson_arrivals(seed: int, rate_hz: float, n: int) -> np.ndarray:
    """Arrival times (seconds) of an open-loop Poisson process."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=n))


def proba80_like(seed: int = 1, n: int = MiB) -> np.ndarray:
    """p(s) ~ 0.2**s over 6 symbols: a synthetic with the statistics the paper
    lists for its proba80 set (top symbol near 0.80)."""
    rng = np.random.default_rng(seed)
    return draw(rng, geometric_p(0.2, 6), n)


WORKLOADS = {"geo1m": geo1m, "zipf256m": zipf256m, "skew256m": skew256m, "mix4096": mix4096}
