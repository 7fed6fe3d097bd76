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


def test_foldin_alone_equals_mixed(bp):
    """A request's result is identical whether it runs alone or batched with
    many others that arrive while it is on the GPU."""
    r = synth.random_small(23, 800, 400, 20000, 16)
    K, seed = 32, 7
    rng = np.random.default_rng(1)
    movie = rng.choice(r.N, 150, replace=False).astype(np.int32)
    rating = rng.normal(3.5, 1.0, 150).astype(np.float32)
    a, _ = _chain_with_samples(bp, r, K, seed, n_samples=3, S=8)
    rid_a = a.foldin_submit(movie, rating, 50)
    res_a = _wait(a, rid_a, 50)
    a.close()
    b, _ = _chain_with_samples(bp, r, K, seed, n_samples=3, S=8)
    rid_b = b.foldin_submit(movie, rating, 50)
    others = []
    for i in range(120):
        n = int(rng.integers(0, 300))
        m = rng.choice(r.N, n, replace=False).astype(np.int32)
        others.append(b.foldin_submit(m, rng.normal(3.5, 1, n).astype(np.float32), 10))
    res_b = _wait(b, rid_b, 50)
    assert rid_a == rid_b == 1
    for x, y in zip(res_a[:3], res_b[:3]):
        assert np.array_equal(x, y)
    b.foldin_drain()
    for o in others:
        assert b.foldin_poll(o, 10) is not None
    b.close()


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
    # a request larger than one batch's rating capacity (pool / 16 ratings)
    big = synth.random_small(25, 100, 3000, 3000, 4)
    t = bp.Sampler(big, 4, prec="fp32", seed=2, foldin_S=2, foldin_pool_bytes=16 * 1000)
    t.run_sweeps(1, 1)
    t.store_sample()
    assert t.foldin_capacity() == 1000
    with pytest.raises(bp.BPMFError) as e:
        t.foldin_submit(np.arange(1001, dtype=np.int32), np.ones(1001, np.float32))
    assert e.value.code == bp.E_TOOBIG
    rid = t.foldin_submit(np.arange(1000, dtype=np.int32), np.ones(1000, np.float32), 3)
    assert _wait(t, rid, 3)[0].shape == (3,)
    t.close()
