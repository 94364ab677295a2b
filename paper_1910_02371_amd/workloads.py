"""Seeded synthetic inputs shaped like the paper's completion workloads.

This module only *synthesizes inputs*: coordinates, observed values drawn
from a planted low-rank model, and initial factors.  It holds none of the
arithmetic of the completion method itself and imports neither the GPU
library nor the CPU oracle, so both sides of every parity check receive the
same inputs from here.

Random streams: ``numpy.random.Generator(numpy.random.Philox(key=seed))``.
Coordinates are linearized row-major, key = (i * I_1 + j) * I_2 + k, and the
COO order is the draw order (random), which keeps index construction
non-trivial.  Observed entries form a set (distinct coordinates), as the
index set Omega of Section 2.1 is a set.

Workloads (stand-ins for data that is not available here: the Netflix
ratings tensor of Section 5.6/5.7 and the sampled-function tensor of
Section 5.6):

1. ``cube``      200^3, 40,000 uniform distinct coordinates, planted rank 5
                 (U(0,1) factors) plus N(0, 0.01^2) noise, float64.
2. ``ratings``   480,189 x 17,770 x 2,182 (the Netflix shape), 100M distinct
                 coordinates, per-mode Zipf(1.1) degrees over a random label
                 permutation, integer values 1..5 from a rounded planted
                 rank-20 model, float32.
3. same tensor as 2 (bfloat16 factor storage is a property of the run).
4. ``counts``    2^18 cubed, 50M uniform distinct coordinates, Poisson counts
                 with rate exp(c * planted rank-10 model), mean 3, float32.
5. ``uniform``   2^20 cubed, 1.5B uniform coordinates in 2^26-nonzero
                 chunks (one GPU's share of a 10-billion-nonzero problem),
                 planted rank 10 plus N(0, 0.01^2) noise, float32.
"""
from dataclasses import dataclass, field
import numpy as np

SEED_DATA = 1910023710
SEED_INIT = 1910023810
SEED_FD = 1910023910


def rng_for(seed):
    return np.random.Generator(np.random.Philox(key=int(seed)))


@dataclass
class Workload:
    """COO tensor: ``idx`` is a list of N int32 arrays, ``t`` the values."""
    name: str
    dims: tuple
    idx: list
    t: np.ndarray
    planted: list = field(default=None, repr=False)
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self):
        return int(len(self.t))

    @property
    def order(self):
        return len(self.dims)


# ---------------------------------------------------------------------------
# helpers (coordinate decoding, threaded chunk work, planted-model synthesis)
# ---------------------------------------------------------------------------
def _threads():
    import os
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _pmap(fn, items):
    items = list(items)
    if len(items) <= 1:
        return [fn(x) for x in items]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(_threads()) as ex:
        return list(ex.map(fn, items))


def _decode(keys, dims):
    keys = np.asarray(keys, dtype=np.int64)
    strides = [int(np.prod([int(d) for d in dims[n + 1:]], dtype=np.int64))
               for n in range(len(dims))]

    def dec(n):
        return ((keys // strides[n]) % int(dims[n])).astype(np.int32)
    return _pmap(dec, range(len(dims)))


def _planted_values(idx, P, chunk=1 << 20):
    """Synthesize observed values from the planted factors P (rows gathered
    at each coordinate, multiplied across modes, summed over the planted
    rank).  Input synthesis only."""
    m = len(idx[0])
    out = np.empty(m, dtype=np.float64)

    def work(b):
        e = min(m, b + chunk)
        acc = P[0][idx[0][b:e]].astype(np.float64)
        for n in range(1, len(P)):
            acc *= P[n][idx[n][b:e]]
        out[b:e] = acc.sum(axis=1)
    _pmap(work, range(0, m, chunk))
    return out


def _first_distinct(keys):
    """Mask of the first occurrence of every key (draw order kept); keys are
    split into hash buckets that are deduplicated in parallel."""
    import pandas as pd
    keys = np.asarray(keys, dtype=np.int64)
    if keys.size < (1 << 22):
        return ~pd.Series(keys).duplicated().values
    nb = 16
    bucket = (keys ^ (keys >> 17)) & (nb - 1)
    keep = np.empty(keys.size, dtype=bool)

    def work(b):
        pos = np.flatnonzero(bucket == b)
        keep[pos] = ~pd.Series(keys[pos]).duplicated().values
    _pmap(work, range(nb))
    return keep


# ---------------------------------------------------------------------------
# generic generators
# ---------------------------------------------------------------------------
def uniform_coords(rng, dims, m):
    """m distinct uniform coordinates, in draw order."""
    total = int(np.prod([int(d) for d in dims], dtype=object))
    if m > total:
        raise ValueError("more nonzeros than entries")
    if total <= (1 << 26):
        keys = rng.choice(total, size=m, replace=False)
    else:
        keys = np.empty(0, dtype=np.int64)
        while len(keys) < m:
            draw = rng.integers(0, total, size=max(1024, int((m - len(keys)) * 1.05) + 16),
                                dtype=np.int64)
            allk = np.concatenate([keys, draw])
            keys = allk[_first_distinct(allk)]
        keys = keys[:m]
    return _decode(keys, dims)


def zipf_coords(rng, dims, m, s=1.1, chunk=1 << 24):
    """m distinct coordinates whose per-mode index degrees follow a truncated
    Zipf(s) law over a random label permutation of each mode.  Draws come in
    chunks; chunk c uses its own Philox stream keyed by (a seed drawn from
    ``rng``, c), and the first m distinct keys in draw order are kept, so the
    result does not depend on the thread count."""
    dims = [int(d) for d in dims]
    perms = [rng.permutation(I).astype(np.int64) for I in dims]
    base = int(rng.integers(0, 1 << 31))
    cdfs = []
    for I in dims:
        w = np.arange(1, I + 1, dtype=np.float64) ** (-s)
        c = np.cumsum(w)
        cdfs.append(c / c[-1])

    def draw(c):
        r = rng_for((base << 32) | c)
        u = r.random((len(dims), chunk))
        key = np.zeros(chunk, dtype=np.int64)
        for n, I in enumerate(dims):
            q = np.minimum(np.searchsorted(cdfs[n], u[n], side="right"), I - 1)
            key = key * I + perms[n][q]
        return key

    parts = []
    nchunk = 0
    want = max(1, -(-int(1.25 * m) // chunk))
    while True:
        parts.extend(_pmap(draw, range(nchunk, nchunk + want)))
        nchunk += want
        allk = np.concatenate(parts) if len(parts) > 1 else parts[0]
        keep = _first_distinct(allk)
        nd = int(np.count_nonzero(keep))
        if nd >= m:
            keys = allk[keep][:m]
            break
        parts = [allk]
        want = max(1, -(-int(2.5 * (m - nd)) // chunk))
    return _decode(keys, dims), nchunk * chunk


def random_tensor(dims, m, seed, rank=3, noise=0.01, dtype=np.float64):
    """Small uniform test tensor: distinct uniform coordinates, planted
    U(0,1) rank-``rank`` values plus Gaussian noise."""
    rng = rng_for(seed)
    idx = uniform_coords(rng, dims, m)
    P = [rng.random((int(I), rank)) for I in dims]
    t = _planted_values(idx, P) + noise * rng.standard_normal(m)
    return Workload(f"random{tuple(dims)}m{m}", tuple(int(d) for d in dims),
                    idx, t.astype(dtype), P)


def init_factors(dims, R, mean_model, seed, dtype=np.float32):
    """Initial factors U(0,1) * c with c = (mean_model / (R / 8))^(1/3), so that
    the initial model mean is about ``mean_model``: the mean observed value
    for least squares, log of the mean count for the Poisson log link."""
    rng = rng_for(seed)
    c = (max(float(mean_model), 1e-3) / (R / 8.0)) ** (1.0 / 3.0)
    return [(c * rng.random((int(I), R))).astype(dtype) for I in dims]


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------
def cube(seed=SEED_DATA + 1):
    """200^3, 40,000 nonzeros, planted rank 5 + N(0, 0.01^2), float64."""
    rng = rng_for(seed)
    dims = (200, 200, 200)
    keys = rng.choice(200 ** 3, size=40000, replace=False)
    idx = _decode(keys, dims)
    P = [rng.random((200, 5)) for _ in range(3)]
    t = _planted_values(idx, P) + 0.01 * rng.standard_normal(40000)
    return Workload("cube200_m40k", dims, idx, t.astype(np.float64), P,
                    dict(R=10, lam=1e-5, loss="ls"))


RATINGS_DIMS = (480189, 17770, 2182)


def ratings(m=100_000_000, dims=RATINGS_DIMS, seed=SEED_DATA + 2, rank=20):
    """Ratings-shaped tensor: Zipf(1.1) per-mode degrees, distinct
    coordinates, values clip(rint(1.2 * planted), 1, 5) as float32."""
    rng = rng_for(seed)
    idx, drawn = zipf_coords(rng, dims, m)
    P = [rng.random((int(I), rank)) for I in dims]
    t = np.clip(np.rint(1.2 * _planted_values(idx, P)), 1, 5).astype(np.float32)
    return Workload(f"ratings{tuple(dims)}_m{m}", tuple(int(d) for d in dims),
                    idx, t, P, dict(draws=drawn, lam=1e-5, loss="ls"))


def counts(m=50_000_000, side=1 << 18, seed=SEED_DATA + 4, rank=10, mean=3.0):
    """Poisson count tensor: uniform distinct coordinates; rate
    exp(c * planted) with c set by bisection so the mean rate is ``mean``."""
    rng = rng_for(seed)
    dims = (side, side, side)
    idx = uniform_coords(rng, dims, m)
    P = [rng.random((side, rank)) for _ in range(3)]
    base = _planted_values(idx, P)
    lo, hi = 0.0, 8.0
    for _ in range(60):
        c = 0.5 * (lo + hi)
        if np.mean(np.exp(c * base)) > mean:
            hi = c
        else:
            lo = c
    c = 0.5 * (lo + hi)
    t = rng.poisson(np.exp(c * base)).astype(np.float32)
    return Workload(f"counts{side}^3_m{m}", dims, idx, t, P,
                    dict(c=c, lam=0.1, loss="poisson"))


def uniform_chunk(c, side=1 << 20, chunk=1 << 26, seed=SEED_DATA + 5, rank=10,
                  P=None):
    """Chunk ``c`` of the uniform 2^20-cubed tensor: keys uniform in
    [0, side^3), its own Philox key (seed << 32 | c).  Duplicate coordinates
    across chunks have expected count ~1e-3 over 1.5B nonzeros and are not
    removed (the library treats duplicates as independent observations)."""
    if P is None:
        P = uniform_planted(side, seed, rank)
    rng = rng_for((int(seed) << 32) | int(c))
    keys = rng.integers(0, side ** 3, size=chunk, dtype=np.int64)
    dims = (side, side, side)
    idx = _decode(keys, dims)
    t = _planted_values(idx, P) + 0.01 * rng.standard_normal(chunk)
    return idx, t.astype(np.float32)


def uniform_planted(side=1 << 20, seed=SEED_DATA + 5, rank=10):
    rng = rng_for(seed)
    return [rng.random((side, rank)) for _ in range(3)]


def uniform(m=1_500_000_000, side=1 << 20, seed=SEED_DATA + 5, rank=10, chunk=1 << 26):
    """The 2^20-cubed uniform tensor: ceil(m / chunk) chunks (each from its
    own Philox key), generated in parallel into preallocated arrays and cut
    to m nonzeros."""
    P = uniform_planted(side, seed, rank)
    nch = -(-m // chunk)
    idx = [np.empty(m, dtype=np.int32) for _ in range(3)]
    t = np.empty(m, dtype=np.float32)

    def work(c):
        ci, ct = uniform_chunk(c, side, chunk, seed, rank, P)
        b = c * chunk
        e = min(m, b + chunk)
        for n in range(3):
            idx[n][b:e] = ci[n][:e - b]
        t[b:e] = ct[:e - b]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max(1, _threads() // 2)) as ex:
        list(ex.map(work, range(nch)))
    return Workload(f"uniform{side}^3_m{m}", (side, side, side), idx, t, P,
                    dict(lam=1e-5, loss="ls"))
