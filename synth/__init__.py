"""Seeded synthetic rating matrices with the shapes of the paper's workloads.

This module only makes inputs: sparse rating patterns, planted low-rank
values, a train/test split and CSR arrays.  It holds none of the sampler's
arithmetic and is shared by the tests, the benchmark, the HIP path's
callers and the oracle's callers alike.

The paper's benchmarks (Sec. V-B: a ChEMBL IC50 subset of 483,500 compounds x
5,775 targets, and MovieLens ml-20m with 138,493 users x 27,278 movies) are not
available here; the generators below stand in for them with the same sizes and
degree skew, driven by numpy's PCG64 from an integer seed.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Ratings:
    """Train ratings as CSR (rows = users) plus held-out test triples."""

    name: str
    M: int
    N: int
    csr_ptr: np.ndarray  # int64 [M+1]
    csr_col: np.ndarray  # int32 [nnz], strictly increasing within a row
    csr_val: np.ndarray  # float32 [nnz]
    test_row: np.ndarray  # int32 [n_test]
    test_col: np.ndarray  # int32 [n_test]
    test_val: np.ndarray  # float32 [n_test]
    K: int = 0  # suggested latent dimension for this workload

    @property
    def nnz(self) -> int:
        return int(self.csr_ptr[-1])

    def coo_rows(self) -> np.ndarray:
        return np.repeat(np.arange(self.M, dtype=np.int32), np.diff(self.csr_ptr))


def _assemble(name, M, N, rows, cols, vals, test_frac, rng, K) -> Ratings:
    """Hold out floor(test_frac * nnz) random triples, sort the rest into CSR."""
    nnz = len(rows)
    n_test = int(np.floor(test_frac * nnz))
    perm = rng.permutation(nnz)
    te, tr = perm[:n_test], perm[n_test:]
    key = rows.astype(np.int64) * N + cols
    if np.all(key[1:] > key[:-1]):  # already in row-major order
        te, tr = np.sort(te), np.sort(tr)
    else:
        te = te[np.argsort(key[te], kind="stable")]
        tr = tr[np.argsort(key[tr], kind="stable")]
    ptr = np.zeros(M + 1, np.int64)
    np.cumsum(np.bincount(rows[tr], minlength=M), out=ptr[1:])
    return Ratings(name, M, N, ptr, cols[tr].astype(np.int32), vals[tr].astype(np.float32),
                   rows[te].astype(np.int32), cols[te].astype(np.int32),
                   vals[te].astype(np.float32), K)


def _planted_dots(rng, M, N, Kstar, rows, cols, chunk=1 << 21):
    """u*_row . v*_col with u*, v* ~ N(0, I / sqrt(Kstar)) (FP64)."""
    sd = Kstar ** -0.25
    Us = (rng.standard_normal((M, Kstar)) * sd).astype(np.float32)
    Vs = (rng.standard_normal((N, Kstar)) * sd).astype(np.float32)
    out = np.empty(len(rows), np.float64)
    for s in range(0, len(rows), chunk):
        e = slice(s, s + chunk)
        out[e] = np.einsum("ij,ij->i", Us[rows[e]], Vs[cols[e]], dtype=np.float64)
    return out


def _zipf_weights(n, s, q=0.0, rng=None):
    w = (np.arange(n, dtype=np.float64) + 1.0 + q) ** (-s)
    w /= w.sum()
    if rng is not None:
        w = w[rng.permutation(n)]
    return w


def _sample_cdf(rng, cdf, size):
    """size i.i.d. category draws from a cumulative distribution, in random order."""
    p = np.diff(np.concatenate([[0.0], cdf]))
    p = np.maximum(p, 0.0)
    counts = rng.multinomial(int(size), p / p.sum())
    out = np.repeat(np.arange(len(cdf), dtype=np.int64), counts)
    rng.shuffle(out)
    return out


def _not_in_sorted(sorted_keys, k):
    """Mask of k not present in the sorted array sorted_keys."""
    if len(sorted_keys) == 0:
        return np.ones(len(k), bool)
    pos = np.minimum(np.searchsorted(sorted_keys, k), len(sorted_keys) - 1)
    return sorted_keys[pos] != k


def _distinct_pairs(rng, M, N, wu, wm, nnz, max_rounds=60):
    """nnz distinct (u, m) pairs with u ~ wu and m ~ wm independently."""
    cu, cm = np.cumsum(wu), np.cumsum(wm)
    keys = np.zeros(0, np.int64)
    for _ in range(max_rounds):
        need = nnz - len(keys)
        if need <= 0:
            break
        draw = int(need * 1.15) + 16
        k = np.unique(_sample_cdf(rng, cu, draw).astype(np.int64) * N + _sample_cdf(rng, cm, draw))
        k = k[_not_in_sorted(keys, k)]
        if len(k) > need:
            k = np.sort(rng.choice(k, need, replace=False))
        keys = np.sort(np.concatenate([keys, k]))
    if len(keys) < nnz:
        raise RuntimeError("could not place %d distinct pairs" % nnz)
    return (keys // N).astype(np.int64), (keys % N).astype(np.int64)


def _per_row_distinct(rng, R, C, deg, wc, over=1.3, rounds=8):
    """For each row r, deg[r] distinct columns, favouring columns by weight wc:
    draw about over*deg[r] columns with replacement, de-duplicate, keep
    deg[r] of them at random; rows that found too few distinct columns are
    redrawn with a doubled oversampling factor, and after the last round are
    filled uniformly from their unused columns."""
    cc = np.cumsum(wc)
    deg = np.asarray(deg, np.int64)
    todo = np.nonzero(deg > 0)[0]
    out = []
    for it in range(rounds):
        if len(todo) == 0:
            break
        d = deg[todo]
        nd = np.minimum(np.ceil(d * over).astype(np.int64) + 8, 64 * C)
        r = np.repeat(todo, nd)
        key = np.unique(r * C + _sample_cdf(rng, cc, int(nd.sum())))
        rr = key // C
        cnt = np.bincount(rr, minlength=R)
        last = it == rounds - 1
        ok_row = cnt >= deg
        keep_row = ok_row[rr]
        # rows with enough distinct columns: keep deg[r] random ones
        k_ok = key[keep_row]
        pr = rng.integers(0, 1 << 31, len(k_ok), dtype=np.int64)
        k_ok = k_ok[np.argsort(((k_ok // C) << 31) | pr)]
        rows_ok = k_ok // C
        start = np.searchsorted(rows_ok, rows_ok, side="left")
        rank = np.arange(len(k_ok)) - start
        out.append(k_ok[rank < deg[rows_ok]])
        todo = todo[~ok_row[todo]]
        over *= 2.0
        if last and len(todo):
            for row in todo:
                used = key[rr == row] % C
                free = np.setdiff1d(np.arange(C), used)
                add = rng.choice(free, deg[row] - len(used), replace=False)
                out.append(np.concatenate([row * C + used, row * C + add]))
            todo = todo[:0]
    keys = np.sort(np.concatenate(out))
    return (keys // C).astype(np.int64), (keys % C).astype(np.int64)


def _fix_total(rng, deg, lo, hi, total):
    deg = np.clip(deg, lo, hi)
    diff = int(total - deg.sum())
    while diff != 0:
        idx = rng.integers(0, len(deg), abs(diff))
        step = 1 if diff > 0 else -1
        np.add.at(deg, idx, step)
        deg = np.clip(deg, lo, hi)
        diff = int(total - deg.sum())
    return deg


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
def planted(seed=1, M=1000, N=500, nnz=20000, K=10, zipf=1.2, noise=0.5, test_frac=0.1):
    """Plain planted low-rank problem: users and movies drawn independently
    with Zipf(zipf) rank weights (ids permuted), distinct pairs,
    r = u*.v* + N(0, noise^2) with u*, v* ~ N(0, I/sqrt(K)), stored as FP32.
    Defaults: 1000 x 500, 20,000 ratings, K = 10."""
    rng = np.random.default_rng(seed)
    wu = _zipf_weights(M, zipf, rng=rng)
    wm = _zipf_weights(N, zipf, rng=rng)
    rows, cols = _distinct_pairs(rng, M, N, wu, wm, nnz)
    vals = _planted_dots(rng, M, N, K, rows, cols) + noise * rng.standard_normal(len(rows))
    return _assemble("planted-%dx%d-K%d" % (M, N, K), M, N, rows, cols,
                     vals.astype(np.float32), test_frac, rng, K)


def planted_uniform(seed=11, M=1000, N=500, density=0.4, K=10, noise=0.5, test_frac=0.1):
    """Well-conditioned planted variant: uniform pattern at the given density."""
    rng = np.random.default_rng(seed)
    mask = rng.random((M, N)) < density
    rows, cols = np.nonzero(mask)
    vals = _planted_dots(rng, M, N, K, rows, cols) + noise * rng.standard_normal(len(rows))
    return _assemble("planted-uniform", M, N, rows.astype(np.int64), cols.astype(np.int64),
                     vals.astype(np.float32), test_frac, rng, K)


def movielens_like(seed=2, M=138493, N=26744, nnz=20000263, K=32, deg_lo=20, deg_hi=9254,
                   max_movie=67310, test_frac=0.1):
    """Shape of a 20M-rating recommender: per-user degrees from a power law
    truncated to [deg_lo, deg_hi] with mean nnz/M, movies by Zipf-Mandelbrot
    popularity (exponent 1, offset solved so the top movie expects max_movie
    ratings), distinct movies per user, every movie rated at least once,
    half-star ratings clip(round_half(3.5 + u*.v* + N(0, 0.5^2)), 0.5, 5)."""
    rng = np.random.default_rng(seed)
    scale = nnz / 20000263.0
    deg_hi = min(deg_hi, N)
    # truncated power-law degrees with the requested mean
    d = np.arange(deg_lo, deg_hi + 1, dtype=np.float64)
    target = nnz / M
    lo_g, hi_g = 0.5, 4.0
    for _ in range(80):
        g = 0.5 * (lo_g + hi_g)
        w = d ** (-g)
        m = (w * d).sum() / w.sum()
        lo_g, hi_g = (g, hi_g) if m > target else (lo_g, g)
    w = d ** (-g)
    deg = d[_sample_cdf(rng, np.cumsum(w / w.sum()), M)].astype(np.int64)
    deg = _fix_total(rng, deg, deg_lo, deg_hi, nnz)
    # movie popularity (r + q)^-1: q solved so that the top movie's expected
    # number of distinct raters, sum_u 1 - (1 - p0)^deg_u, is max_movie
    want = min(max_movie * scale, 0.9 * M)
    r = np.arange(N, dtype=np.float64)
    lo_q, hi_q = 1e-4, 1e6
    for _ in range(100):
        q = np.sqrt(lo_q * hi_q)
        p0 = (1.0 / (1.0 + q)) / (1.0 / (r + 1.0 + q)).sum()
        got = (1.0 - (1.0 - p0) ** deg).sum()
        lo_q, hi_q = (q, hi_q) if got > want else (lo_q, q)
    wm = _zipf_weights(N, 1.0, q, rng)
    rows, cols = _per_row_distinct(rng, M, N, deg, wm)
    # every movie rated at least once: move a rating of a heavy user
    unrated = np.setdiff1d(np.arange(N), cols)
    if len(unrated):
        heavy = np.nonzero(np.bincount(rows, minlength=M)[rows] > deg_lo)[0]
        pick = rng.choice(heavy, len(unrated), replace=False)
        keys = rows[pick] * N + unrated
        ok = ~np.isin(keys, rows * N + cols)
        cols = cols.copy()
        cols[pick[ok]] = unrated[ok]
    vals = 3.5 + _planted_dots(rng, M, N, 32, rows, cols) + 0.5 * rng.standard_normal(len(rows))
    vals = np.clip(np.round(vals * 2.0) / 2.0, 0.5, 5.0)
    return _assemble("movielens20m-shape", M, N, rows, cols, vals.astype(np.float32), test_frac,
                     rng, K)


def netflix_like(seed=3, M=480189, N=17770, nnz=100480507, K=100, max_movie=230000,
                 max_user=17000, test_frac=0.1):
    """Shape of a 100M-rating recommender: users and movies by
    Zipf-Mandelbrot(1.1) weights (offsets solved so the heaviest movie and
    user expect max_movie and max_user ratings), distinct pairs, integer
    ratings clip(round(3.6 + u*.v* + N(0, 0.8^2)), 1, 5), planted rank 100."""
    rng = np.random.default_rng(seed)

    def offset_for(n, share):
        r = np.arange(n, dtype=np.float64)
        lo_q, hi_q = 1e-3, 1e7
        for _ in range(100):
            q = np.sqrt(lo_q * hi_q)
            w = (r + 1.0 + q) ** -1.1
            p0 = w[0] / w.sum()
            lo_q, hi_q = (q, hi_q) if p0 > share else (lo_q, q)
        return q

    wm = _zipf_weights(N, 1.1, offset_for(N, max_movie / nnz), rng)
    wu = _zipf_weights(M, 1.1, offset_for(M, max_user / nnz), rng)
    rows, cols = _distinct_pairs(rng, M, N, wu, wm, nnz)
    vals = 3.6 + _planted_dots(rng, M, N, 100, rows, cols) + 0.8 * rng.standard_normal(len(rows))
    vals = np.clip(np.round(vals), 1.0, 5.0)
    return _assemble("netflix100m-shape", M, N, rows, cols, vals.astype(np.float32), test_frac,
                     rng, K)


def netflix_mini(seed=3):
    """1/16 of the rows and columns of the 100M shape (same laws, K = 100)."""
    return netflix_like(seed, M=480189 // 16, N=17770 // 16, nnz=100480507 // 256,
                        max_movie=230000 // 16, max_user=17000 // 16)


def chembl_like(seed=4, M=483500, N=5775, nnz=2000000, K=64, n_heavy=20, heavy_share=0.3,
                median=40.0, sigma=1.9, test_frac=0.1):
    """Shape of a compound x protein activity matrix: n_heavy columns hold
    heavy_share of the observations (geometric sizes), the rest log-normal
    sizes (median 40, sigma 1.9) rescaled to the remainder; rows (compounds)
    are drawn per column with Zipf(1) weights without repetition; values
    6 + 1.5 (sqrt(0.8) s / sd(s) + sqrt(0.2) eps) with s from a planted
    rank-64 model (roughly N(6, 1.5^2), like pIC50)."""
    rng = np.random.default_rng(seed)
    n_h = int(round(heavy_share * nnz))
    ratio = 0.85
    geo = ratio ** np.arange(n_heavy)
    heavy = np.minimum(np.round(geo / geo.sum() * n_h).astype(np.int64), M)
    light = rng.lognormal(np.log(median), sigma, N - n_heavy)
    light = np.maximum(1, np.round(light / light.sum() * (nnz - heavy.sum()))).astype(np.int64)
    light = np.minimum(light, M)
    deg = np.concatenate([heavy, light])
    deg = _fix_total(rng, deg, 1, M, nnz)
    deg = deg[rng.permutation(N)]
    wr = _zipf_weights(M, 1.0, rng=rng)
    cols, rows = _per_row_distinct(rng, N, M, deg, wr)
    s = _planted_dots(rng, M, N, 64, rows, cols)
    eps = rng.standard_normal(len(rows))
    vals = 6.0 + 1.5 * (np.sqrt(0.8) * s / s.std() + np.sqrt(0.2) * eps)
    return _assemble("chembl-shape", M, N, rows, cols, vals.astype(np.float32), test_frac, rng, K)


def random_small(seed, M, N, nnz, K, empty_rows=0, test_frac=0.1):
    """Small irregular problem for unit tests (uniform pattern, planted rank K,
    optional rows/columns left without ratings)."""
    rng = np.random.default_rng(seed)
    Mr, Nr = max(1, M - empty_rows), max(1, N - empty_rows)
    nnz = min(nnz, Mr * Nr)
    rows, cols = _distinct_pairs(rng, Mr, Nr, np.full(Mr, 1.0 / Mr), np.full(Nr, 1.0 / Nr), nnz)
    vals = _planted_dots(rng, M, N, K, rows, cols) + 0.5 * rng.standard_normal(len(rows))
    return _assemble("random-small", M, N, rows, cols, vals.astype(np.float32), test_frac, rng, K)


WORKLOADS = {
    "planted": planted,
    "movielens": movielens_like,
    "netflix": netflix_like,
    "netflix_mini": netflix_mini,
    "chembl": chembl_like,
}
