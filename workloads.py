"""Seeded synthetic inputs for the discrete Frechet distance.

Shared by the tests, the benchmark and the oracle checks.  This module holds
none of the distance computation: it only draws curves, lengths and arrival
times.  Every generator takes an explicit seed, uses numpy's PCG64
``default_rng`` and draws in the fixed order written in its docstring.

Workloads (the shapes of the benchmark configurations):

* ``plain_pair``     512 x 384 points, 2-D float32 random walks, seed 1.
* ``batched``        4096 pairs, n, m uniform in [64, 2048], 2-D; q is p
                     resampled at rate m/n plus N(0, 0.1^2) noise, seed 2.
* ``large_pair``     131072 x 131072 points, 3-D float32 walks, seed 3.
* ``cross_int``      1024 queries x 1024 database curves of 256 points,
                     2-D int32 uniform in [-2^15, 2^15), seed 4.
* ``serving_db`` / ``serving_queries`` / ``poisson_arrivals``: 10,000
  database walks and query walks with log-normal lengths (median 300,
  sigma 1 in natural log, clipped to [32, 8192]), seeds 5, 6, 7.
* ``paper_walk``     the paper's random walk with steps uniform in
                     {-1, 0, +1} per coordinate (Sec. 4 experiments).
* ``symbol_pairs``   4096 pairs of int32 symbol sequences over a 4-letter
                     alphabet with the batched lengths; q is p resampled to
                     length m with 10% of its symbols redrawn, seed 8
                     (Levenshtein distance, Appendix B).

A random walk is the cumulative sum of i.i.d. N(0, 1) steps in FP64 (the
first point is the first step), rounded once to float32.
"""
import numpy as np

__all__ = [
    "walk", "paper_walk", "plain_pair", "batched", "large_pair", "cross_int",
    "lognormal_lengths", "serving_db", "serving_queries", "poisson_arrivals",
    "random_pairs", "concat", "symbol_pairs",
]


def walk(rng, n, dim, dtype=np.float32):
    """FP64 cumulative sum of N(0,1) steps, shape (n, dim), cast once."""
    steps = rng.standard_normal((n, dim))
    return np.cumsum(steps, axis=0).astype(dtype)


def paper_walk(rng, n, dim=2):
    """Steps uniform in {-1, 0, +1} per coordinate; integer-valued float32."""
    steps = rng.integers(-1, 2, size=(n, dim))
    return np.cumsum(steps, axis=0).astype(np.float32)


def concat(curves):
    """CSR layout: (coords[sum n][D], offsets int64[len+1])."""
    off = np.zeros(len(curves) + 1, dtype=np.int64)
    off[1:] = np.cumsum([c.shape[0] for c in curves])
    dim = curves[0].shape[1]
    data = np.concatenate(curves, axis=0) if curves else np.zeros((0, dim))
    return np.ascontiguousarray(data), off


def plain_pair(seed=1, n=512, m=384, dim=2):
    """Draw order: p walk (n x dim), then q walk (m x dim)."""
    rng = np.random.default_rng(seed)
    p = walk(rng, n, dim)
    q = walk(rng, m, dim)
    return p, q


def _resample(p64, m):
    """Linear interpolation of p at m equally spaced fractional indices,
    endpoints kept (rate m / n)."""
    n = p64.shape[0]
    if m == 1 or n == 1:
        return np.repeat(p64[:1], m, axis=0)
    x = np.arange(m, dtype=np.float64) * ((n - 1) / (m - 1))
    i0 = np.minimum(np.floor(x).astype(np.int64), n - 2)
    w = (x - i0)[:, None]
    return p64[i0] * (1.0 - w) + p64[i0 + 1] * w


def batched(seed=2, npairs=4096, lo=64, hi=2048, dim=2, noise=0.1):
    """Draw order: n[npairs], m[npairs] (uniform integers in [lo, hi]); then
    for each pair k: the p_k steps (n_k x dim), then the q_k noise (m_k x dim).

    Returns P (sum n x dim float32), p_off, Q (sum m x dim float32), q_off."""
    rng = np.random.default_rng(seed)
    n = rng.integers(lo, hi + 1, size=npairs)
    m = rng.integers(lo, hi + 1, size=npairs)
    ps, qs = [], []
    for k in range(npairs):
        p64 = np.cumsum(rng.standard_normal((int(n[k]), dim)), axis=0)
        q64 = _resample(p64, int(m[k])) + noise * rng.standard_normal((int(m[k]), dim))
        ps.append(p64.astype(np.float32))
        qs.append(q64.astype(np.float32))
    P, p_off = concat(ps)
    Q, q_off = concat(qs)
    return P, p_off, Q, q_off


def large_pair(seed=3, n=131072, m=131072, dim=3):
    """Draw order: p walk (n x dim), then q walk (m x dim)."""
    rng = np.random.default_rng(seed)
    p = walk(rng, n, dim)
    q = walk(rng, m, dim)
    return p, q


def cross_int(seed=4, nq=1024, ndb=1024, length=256, dim=2, lo=-(1 << 15), hi=(1 << 15)):
    """Draw order: queries (nq x length x dim), then database (ndb x length x dim),
    int32 uniform in [lo, hi).  Returns Qs, q_off, DB, db_off (CSR)."""
    rng = np.random.default_rng(seed)
    qa = rng.integers(lo, hi, size=(nq, length, dim), dtype=np.int32)
    da = rng.integers(lo, hi, size=(ndb, length, dim), dtype=np.int32)
    q_off = np.arange(nq + 1, dtype=np.int64) * length
    db_off = np.arange(ndb + 1, dtype=np.int64) * length
    return (np.ascontiguousarray(qa.reshape(-1, dim)), q_off,
            np.ascontiguousarray(da.reshape(-1, dim)), db_off)


def lognormal_lengths(rng, count, median=300.0, sigma=1.0, lo=32, hi=8192):
    """L = clip(rint(exp(ln(median) + sigma * z)), lo, hi), z ~ N(0, 1)."""
    z = rng.standard_normal(count)
    return np.clip(np.rint(np.exp(np.log(median) + sigma * z)), lo, hi).astype(np.int64)


def serving_db(seed=5, count=10000, dim=2, **kw):
    """Draw order: lengths (count), then each walk in turn.  Returns DB, db_off."""
    rng = np.random.default_rng(seed)
    lens = lognormal_lengths(rng, count, **kw)
    return concat([walk(rng, int(L), dim) for L in lens])


def serving_queries(seed=6, count=1000, dim=2, **kw):
    """Same law as the database; returns a list of (L, dim) float32 curves."""
    rng = np.random.default_rng(seed)
    lens = lognormal_lengths(rng, count, **kw)
    return [walk(rng, int(L), dim) for L in lens]


def poisson_arrivals(seed=7, count=1000, rate=1000.0):
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def short_symbol_pairs(seed=12, npairs=262144, lo=8, hi=64, alphabet=4):
    """Many short symbol sequences (one int32 coordinate per symbol).  Draw
    order: n[npairs], m[npairs] uniform in [lo, hi]; then every p symbol and
    every q symbol uniform in [0, alphabet).  Returns P, p_off, Q, q_off."""
    rng = np.random.default_rng(seed)
    n = rng.integers(lo, hi + 1, size=npairs)
    m = rng.integers(lo, hi + 1, size=npairs)
    p_off = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    q_off = np.concatenate([[0], np.cumsum(m)]).astype(np.int64)
    P = rng.integers(0, alphabet, size=(int(p_off[-1]), 1)).astype(np.int32)
    Q = rng.integers(0, alphabet, size=(int(q_off[-1]), 1)).astype(np.int32)
    return P, p_off, Q, q_off


def short_pairs(seed=11, npairs=262144, lo=8, hi=64, dim=2, long_pairs=0, long_lo=300, long_hi=1500):
    """Many short pairs.  Draw order: n[npairs], m[npairs] uniform in [lo, hi];
    with long_pairs > 0, then n and m of that many more pairs uniform in
    [long_lo, long_hi] and a permutation of all pairs; then the N(0,1) steps
    of every p point (sum n x dim) and of every q point (sum m x dim); each
    curve is the FP64 cumulative sum of its own steps, cast once.  Returns
    P, p_off, Q, q_off."""
    rng = np.random.default_rng(seed)
    n = rng.integers(lo, hi + 1, size=npairs)
    m = rng.integers(lo, hi + 1, size=npairs)
    if long_pairs > 0:
        n = np.concatenate([n, rng.integers(long_lo, long_hi + 1, size=long_pairs)])
        m = np.concatenate([m, rng.integers(long_lo, long_hi + 1, size=long_pairs)])
        perm = rng.permutation(len(n))
        n, m = n[perm], m[perm]

    def curves(lens):
        off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        steps = rng.standard_normal((int(off[-1]), dim))
        total = np.cumsum(steps, axis=0)
        before = np.concatenate([np.zeros((1, dim)), total[off[1:-1] - 1]])  # sum of earlier curves' steps
        return (total - np.repeat(before, lens, axis=0)).astype(np.float32), off

    P, p_off = curves(n)
    Q, q_off = curves(m)
    return P, p_off, Q, q_off


def random_pairs(seed, npairs, lo, hi, dim=2, kind="walk"):
    """Independent pairs with lengths uniform in [lo, hi] (tests).

    Draw order: n[npairs], m[npairs], then per pair p then q.
    kind: "walk" (N(0,1) walks), "paper" ({-1,0,1} walks) or "int" (int32
    uniform in [-2^15, 2^15))."""
    rng = np.random.default_rng(seed)
    n = rng.integers(lo, hi + 1, size=npairs)
    m = rng.integers(lo, hi + 1, size=npairs)
    ps, qs = [], []
    for k in range(npairs):
        if kind == "walk":
            ps.append(walk(rng, int(n[k]), dim))
            qs.append(walk(rng, int(m[k]), dim))
        elif kind == "paper":
            ps.append(paper_walk(rng, int(n[k]), dim))
            qs.append(paper_walk(rng, int(m[k]), dim))
        elif kind == "int":
            ps.append(rng.integers(-(1 << 15), 1 << 15, size=(int(n[k]), dim), dtype=np.int32))
            qs.append(rng.integers(-(1 << 15), 1 << 15, size=(int(m[k]), dim), dtype=np.int32))
        else:
            raise ValueError(kind)
    P, p_off = concat(ps)
    Q, q_off = concat(qs)
    return P, p_off, Q, q_off


def _wrap(lon):
    """Longitude to [-pi, pi)."""
    return (lon + np.pi) % (2.0 * np.pi) - np.pi


def geo_walk(rng, n, step, pole_margin=1e-4):
    """A random walk on the sphere as (latitude, unwrapped longitude) in FP64
    radians.  Draw order: z uniform in [-1, 1) (latitude asin z, so the start
    is uniform on the sphere), the start longitude uniform in [-pi, pi), then
    the n - 1 steps (n - 1 x 2, N(0, step^2)): latitude steps are taken as
    drawn and clipped to pole_margin from the poles, longitude steps are
    divided by the cosine of the new latitude (about `step` radians east or
    west)."""
    lat0 = np.arcsin(rng.uniform(-1.0, 1.0))
    lon0 = rng.uniform(-np.pi, np.pi)
    d = rng.standard_normal((n - 1, 2)) * step
    lim = np.pi / 2 - pole_margin
    lat = np.clip(lat0 + np.concatenate([[0.0], np.cumsum(d[:, 0])]), -lim, lim)
    lon = lon0 + np.concatenate([[0.0], np.cumsum(d[:, 1] / np.cos(lat[1:]))])
    return np.stack([lat, lon], axis=1)


def geo_pairs(seed=9, npairs=4096, lo=64, hi=2048, step=2e-3, noise=0.1):
    """Pairs of curves on the sphere, (latitude, longitude) in radians,
    float32, for the great-circle ground distance.  Draw order: n[npairs],
    m[npairs] uniform in [lo, hi]; then per pair: the geo_walk of p (n
    points), then the q noise (m x 2, N(0, (noise * step)^2)).  q is p
    resampled at m points (linear interpolation of latitude and unwrapped
    longitude, endpoints kept) plus the noise; latitudes are clipped to 1e-4
    from the poles and longitudes wrapped to [-pi, pi), so curves cross the
    antimeridian.  Returns P, p_off, Q, q_off with 2 coordinates per point."""
    rng = np.random.default_rng(seed)
    n = rng.integers(lo, hi + 1, size=npairs)
    m = rng.integers(lo, hi + 1, size=npairs)
    lim = np.pi / 2 - 1e-4
    ps, qs = [], []
    for k in range(npairs):
        p64 = geo_walk(rng, int(n[k]), step)
        q64 = _resample(p64, int(m[k])) + (noise * step) * rng.standard_normal((int(m[k]), 2))
        for c in (p64, q64):
            c[:, 0] = np.clip(c[:, 0], -lim, lim)
            c[:, 1] = _wrap(c[:, 1])
        ps.append(p64.astype(np.float32))
        qs.append(q64.astype(np.float32))
    P, p_off = concat(ps)
    Q, q_off = concat(qs)
    return P, p_off, Q, q_off


def symbol_pairs(seed=8, npairs=4096, lo=64, hi=2048, alphabet=4, redraw=0.1):
    """Draw order: n[npairs], m[npairs] uniform in [lo, hi]; then per pair:
    p (n symbols uniform in [0, alphabet)), the resampling of p to m symbols
    (index floor(j * n / m)), a redraw mask (Bernoulli(redraw), m values) and
    the redrawn symbols (m values).  Returns int32 P, p_off, Q, q_off with
    one coordinate per symbol."""
    rng = np.random.default_rng(seed)
    n = rng.integers(lo, hi + 1, size=npairs)
    m = rng.integers(lo, hi + 1, size=npairs)
    ps, qs = [], []
    for k in range(npairs):
        p = rng.integers(0, alphabet, size=int(n[k]))
        idx = (np.arange(int(m[k])) * int(n[k])) // int(m[k])
        q = p[idx].copy()
        mask = rng.random(int(m[k])) < redraw
        new = rng.integers(0, alphabet, size=int(m[k]))
        q[mask] = new[mask]
        ps.append(p.astype(np.int32).reshape(-1, 1))
        qs.append(q.astype(np.int32).reshape(-1, 1))
    P, p_off = concat(ps)
    Q, q_off = concat(qs)
    return P, p_off, Q, q_off
