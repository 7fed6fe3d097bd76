"""Fold-in serving on the GPU against the FP64 oracle, batch invariance, and
the request API's error semantics.

Tolerances: predictive means within 2e-4 absolute (FP32 draws and scores
against FP64), variances within 2e-4; the returned ids must be unrated,
distinct, sorted by mean (ties by id) and agree with the oracle's top-n up to
movies whose oracle means lie within the tolerance of the n-th mean.
"""
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bp():
    import paper_1705_04159_amd as bp

    bp.lib()
    return bp


def _chain_with_samples(bp, r, K, seed, n_samples, S=16, pool=0):
    """Run a short chain and store n_samples samples.  Also returns the ring as
    the library holds it (sample i in slot i mod S; the slot index is the
    noise counter word of the fold-in draw), each entry (V, mu_U, Lambda_U)."""
    s = bp.Sampler(r, K, prec="fp32", seed=seed, foldin_S=S, foldin_pool_bytes=pool)
    s.run_sweeps(1, 3)
    ring = [None] * S
    t = 4
    for i in range(n_samples):
        s.run_sweeps(t, 1)
        t += 1
        s.store_sample()
        V = s.get_factor(bp.SIDE_V).astype(np.float64)
        mu, Lam = s.get_hyper(bp.SIDE_U)
        ring[i % S] = (V, mu, Lam)
    return s, [x for x in ring if x is not None]


def _wait(s, rid, top_n, timeout=60.0):
    t0 = time.time()
    while True:
        res = s.foldin_poll(rid, top_n)
        if res is not None:
            return res
        if time.time() - t0 > timeout:
            raise TimeoutError("fold-in request %d did not complete" % rid)
        time.sleep(0.0005)


def _check_against_oracle(orc, s, store, movie, rating, rid, res, top_n, seed):
    ids, mean, var, lat = res
    Vs = np.stack([v for v, _, _ in store])
    mus = np.stack([m for _, m, _ in store])
    Lams = np.stack([l for _, _, l in store])
    rbar = s.mean_rating
    rc = rating.astype(np.float64) - rbar
    _, om, ov = orc.foldin(2.0, movie, rc, Vs, mus, Lams, seed, rid, rbar)
    N = len(om)
    unrated = np.setdiff1d(np.arange(N), movie)
    n_take = min(top_n, len(unrated))
    assert np.all(ids[n_take:] == -1)
    ids = ids[:n_take]
    assert len(np.unique(ids)) == n_take
    assert not np.isin(ids, movie).any()
    tol = 2e-4
    assert np.allclose(mean[:n_take], om[ids], atol=tol, rtol=0)
    assert np.allclose(var[:n_take], ov[ids], atol=tol, rtol=0)
    assert np.all(np.diff(mean[:n_take]) <= 0)
    # oracle top-n (mean desc, id asc)
    order = unrated[np.lexsort((unrated, -om[unrated]))][:n_take]
    if n_take:
        kth = om[order[-1]]
        sure = order[om[order] > kth + tol]
        assert np.isin(sure, ids).all()
        assert np.all(om[ids] >= kth - tol)
    return lat


@pytest.mark.parametrize("K", [8, 32])
def test_foldin_matches_oracle(bp, orc, K):
    r = synth.random_small(21, 500, 300, 12000, min(K, 12))
    seed = 61
    s, store = _chain_with_samples(bp, r, K, seed, n_samples=4, S=4)
    assert s.foldin_samples() == 4
    rng = np.random.default_rng(K)
    reqs = []
    for n in [0, 1, 5, 37, 299, 120]:
        movie = rng.choice(r.N, n, replace=False).astype(np.int32)
        rating = rng.normal(0.0, 1.0, n).astype(np.float32)
        top_n = [100, 1, 7, 100, 1, 64][len(reqs)]
        rid = s.foldin_submit(movie, rating, top_n)
        reqs.append((movie, rating, rid, top_n))
    for movie, rating, rid, top_n in reqs:
        res = _wait(s, rid, top_n)
        lat = _check_against_oracle(orc, s, store, movie, rating, rid, res, top_n, seed)
        assert lat > 0
    s.close()


def test_foldin_ring_keeps_last_S(bp, orc):
    """More stores than slots: the ring holds the last S samples."""
    r = synth.random_small(22, 300, 200, 6000, 6)
    s, store = _chain_with_samples(bp, r, 6, 5, n_samples=5, S=3)
    assert s.foldin_samples() == 3
    movie = np.array([3, 10, 50], np.int32)
    rating = np.array([1.0, -0.5, 2.0], np.float32)
    rid = s.foldin_submit(movie, rating, 20)
    res = _wait(s, rid, 20)
    _check_against_oracle(orc, s, store, movie, rating, rid, res, 20, 5)
    s.close()


def test_foldin_prepared_submit_matches(bp):
    """The prepared form of submit (arrays converted once) queues the same
    request: identical results to the plain form on a second context."""
    r = synth.random_small(22, 300, 200, 6000, 6)
    movie = np.array([3, 10, 50, 77], np.int32)
    rating = np.array([1.0, -0.5, 2.0, 0.25], np.float32)
    out = []
    for prepared in (False, True):
        s, _ = _chain_with_samples(bp, r, 6, 5, n_samples=3, S=3)
        if prepared:
            rid = s.foldin_submit_prepared(s.foldin_prepare(movie, rating), 20)
        else:
            rid = s.foldin_submit(movie, rating, 20)
        out.append(_wait(s, rid, 20)[:3])
        s.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_foldin_alone_equals_mixed(bp):
    """121 requests (0 to 399 ratings, every size class but the largest; top-n
    between 1 and 100) run one at a time in context A -- each submitted only
    after the previous one completed -- and in one burst in context B.  Every
    request's result (ids, means, variances) is bit-identical between the two,
    A's batches held one request each, and B's scheduler packed several
    requests per batch and had several batches on the device at once."""
    r = synth.random_small(23, 800, 400, 20000, 16)
    K, seed = 32, 7
    rng = np.random.default_rng(1)
    reqs = []
    for i in range(121):
        n = 150 if i == 0 else int(rng.integers(0, 400))
        movie = rng.choice(r.N, n, replace=False).astype(np.int32)
        rating = rng.normal(3.5, 1.0, n).astype(np.float32)
        reqs.append((movie, rating, int(rng.integers(1, 101))))
    a, _ = _chain_with_samples(bp, r, K, seed, n_samples=3, S=8)
    res_a = []
    for movie, rating, top in reqs:
        rid = a.foldin_submit(movie, rating, top)
        res_a.append((rid, _wait(a, rid, top)))
    stats_a = a.foldin_stats()
    a.close()
    b, _ = _chain_with_samples(bp, r, K, seed, n_samples=3, S=8)
    rids = [b.foldin_submit(movie, rating, top) for movie, rating, top in reqs]
    res_b = [(rid, _wait(b, rid, top)) for rid, (_, _, top) in zip(rids, reqs)]
    stats_b = b.foldin_stats()
    b.close()
    print("alone: batches %d, requests %d, max per batch %d, max in flight %d" % stats_a)
    print("burst: batches %d, requests %d, max per batch %d, max in flight %d" % stats_b)
    assert stats_a[:3] == (121, 121, 1)
    assert stats_b[1] == 121 and stats_b[2] > 1 and stats_b[3] > 1
    for (ra, xa), (rb, xb) in zip(res_a, res_b):
        assert ra == rb  # the same request id, hence the same noise
        for u, v in zip(xa[:3], xb[:3]):
            assert np.array_equal(u, v)


def test_foldin_serving_size_matches_oracle(bp, orc):
    """Fold-in at the serving workload's size: N = 26,744 movies, K = 32,
    16 stored samples, requests of 1 to 5,000 ratings (the largest request
    size), top-100, against the oracle's fold-in."""
    r = synth.random_small(26, 3000, 26744, 240000, 8)
    K, seed = 32, 41
    s, store = _chain_with_samples(bp, r, K, seed, n_samples=16, S=16)
    assert s.foldin_samples() == 16
    rng = np.random.default_rng(5)
    pop = np.bincount(r.csr_col, minlength=r.N) + 1.0
    reqs = []
    for n in [1, 9, 71, 587, 2600, 5000]:
        movie = rng.choice(r.N, n, replace=False, p=pop / pop.sum()).astype(np.int32)
        rating = np.clip(rng.normal(3.5, 1.0, n), 0.5, 5.0).astype(np.float32)
        reqs.append((movie, rating, s.foldin_submit(movie, rating, 100)))
    for movie, rating, rid in reqs:
        res = _wait(s, rid, 100)
        _check_against_oracle(orc, s, store, movie, rating, rid, res, 100, seed)
    s.close()


def test_foldin_errors(bp):
    r = synth.random_small(24, 200, 100, 3000, 4)
    s = bp.Sampler(r, 4, prec="fp32", seed=2, foldin_S=2, foldin_pool_bytes=16 << 20)
    with pytest.raises(bp.BPMFError) as e:
        s.foldin_submit(np.array([1], np.int32), np.array([1.0], np.float32))
    assert e.value.code == bp.E_NOSAMPLES
    s.run_sweeps(1, 2)
    s.store_sample()
    with pytest.raises(bp.BPMFError) as e:
        s.foldin_submit(np.array([r.N], np.int32), np.array([1.0], np.float32))
    assert e.value.code == bp.E_RANGE
    with pytest.raises(bp.BPMFError) as e:
        s.foldin_submit(np.array([3, 3], np.int32), np.array([1.0, 2.0], np.float32))
    assert e.value.code == bp.E_FORMAT
    with pytest.raises(bp.BPMFError) as e:
        s.foldin_submit(np.array([3], np.int32), np.array([1.0], np.float32), top_n=0)
    assert e.value.code == bp.E_INVAL
    with pytest.raises(bp.BPMFError) as e:
        s.foldin_poll(12345)
    assert e.value.code == bp.E_NOTFOUND
    rid = s.foldin_submit(np.array([3, 4], np.int32), np.array([1.0, 2.0], np.float32), 5)
    _wait(s, rid, 5)
    with pytest.raises(bp.BPMFError) as e:  # already collected
        s.foldin_poll(rid, 5)
    assert e.value.code == bp.E_NOTFOUND
    s.close()
    # a request larger than one batch's rating capacity (pool / 32 ratings:
    # 8 B per rating, four batch slots)
    big = synth.random_small(25, 100, 3000, 3000, 4)
    t = bp.Sampler(big, 4, prec="fp32", seed=2, foldin_S=2, foldin_pool_bytes=32 * 1000)
    t.run_sweeps(1, 1)
    t.store_sample()
    assert t.foldin_capacity() == 1000
    with pytest.raises(bp.BPMFError) as e:
        t.foldin_submit(np.arange(1001, dtype=np.int32), np.ones(1001, np.float32))
    assert e.value.code == bp.E_TOOBIG
    rid = t.foldin_submit(np.arange(1000, dtype=np.int32), np.ones(1000, np.float32), 3)
    assert _wait(t, rid, 3)[0].shape == (3,)
    t.close()
