"""Degree-order relabelling (params.reorder) on the GPU.

A relabelled context holds users and movies in descending order of their
rating counts (ties by id), the reordering of R before partitioning of
Sec. IV-B, while every call keeps the caller's ids.  It must compute, bit
for bit, what an ordinary context computes on R relabelled the same way
(the permutations are rebuilt here with numpy, independently of the
library): initial factors, RMSE histories, factors, hyperparameters, chain
state, pair predictions, a restored factor and fold-in results, each read
back in the caller's ids.  The ordinary context itself is pinned to the
oracle by the parity tests.  The CSC and plan reported in caller ids are
checked against scipy's transposition of R and against the numpy order.
"""
import sys

import numpy as np
import pytest
import scipy.sparse

import synth
from relabel import relabel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bp():
    import paper_1705_04159_amd as bp

    bp.lib()
    return bp


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


CASES = [
    # (precision, K, workload, split threshold)
    ("fp32", 10, "planted", 128),
    ("fp32", 64, "planted", 0),
    ("fp32", 100, "planted", 256),
    ("bf16", 32, "planted", 128),
    ("fp64", 8, "empty", 0),
]


def _workload(name, K):
    if name == "planted":
        return synth.planted(seed=21, M=1200, N=700, nnz=30000, K=K)
    return synth.random_small(22, 400, 300, 6000, K, empty_rows=9)


@pytest.mark.parametrize("prec,K,wl,split", CASES)
def test_reorder_equals_relabelled_input(bp, prec, K, wl, split):
    r = _workload(wl, K)
    r2, ou, ov, iu, iv = relabel(r)
    _say("reorder %s K=%d %s split=%d" % (prec, K, wl, split))
    A = bp.Sampler(r, K, prec=prec, seed=77, split_threshold=split, reorder=True)
    B = bp.Sampler(r2, K, prec=prec, seed=77, split_threshold=split)
    U, V = bp.SIDE_U, bp.SIDE_V
    assert A.mean_rating == B.mean_rating
    # plan and initial factors in caller ids
    for side, ext, inv in ((U, ou, iu), (V, ov, iv)):
        pa, nsa = A.get_plan(side)
        pb, nsb = B.get_plan(side)
        assert nsa == nsb
        assert np.array_equal(pa, ext[pb])
        assert np.array_equal(A.get_factor(side), B.get_factor(side)[inv])
    # the CSC in caller ids
    ptr, row, rc = A.get_csc()
    C = scipy.sparse.csr_matrix((r.csr_val, r.csr_col, r.csr_ptr), shape=(r.M, r.N)).tocsc()
    C.sort_indices()
    assert np.array_equal(ptr, C.indptr)
    assert np.array_equal(row, C.indices)
    want = C.data.astype(np.float64) - A.mean_rating
    assert np.array_equal(rc, want if prec == "fp64" else want.astype(np.float32))
    # chains
    aa, al = A.run_sweeps(1, 4)
    ba, bl = B.run_sweeps(1, 4)
    assert np.array_equal(aa, ba) and np.array_equal(al, bl)
    for side, inv in ((U, iu), (V, iv)):
        assert np.array_equal(A.get_factor(side), B.get_factor(side)[inv])
        ma, La = A.get_hyper(side)
        mb, Lb = B.get_hyper(side)
        assert np.array_equal(ma, mb) and np.array_equal(La, Lb)
    psa, na = A.get_chain_state()
    psb, nb = B.get_chain_state()
    assert na == nb and np.array_equal(psa, psb)
    # pair predictions, both entry points
    rng = np.random.default_rng(5)
    i = rng.integers(0, r.M, 3000).astype(np.int32)
    j = rng.integers(0, r.N, 3000).astype(np.int32)
    pb = B.predict(iu[i], iv[j])
    assert np.array_equal(A.predict(i, j), pb)
    assert np.array_equal(A.predict_noalloc(i, j), pb)
    # a factor set in caller order, then more sweeps
    X = (0.3 * rng.standard_normal((r.M, K))).astype(A.dtype)
    A.set_factor(U, X)
    B.set_factor(U, X[ou])
    assert np.array_equal(A.get_factor(U), X)
    aa, al = A.run_sweeps(5, 2)
    ba, bl = B.run_sweeps(5, 2)
    assert np.array_equal(aa, ba) and np.array_equal(al, bl)
    for side, inv in ((U, iu), (V, iv)):
        assert np.array_equal(A.get_factor(side), B.get_factor(side)[inv])
    # fold-in (FP32 factors, K <= 64): the same request in both labellings
    if prec == "fp32" and K <= 64:
        A.store_sample()
        B.store_sample()
        movie = np.sort(rng.choice(r.N, 40, replace=False)).astype(np.int32)
        rating = (3 + rng.standard_normal(40)).astype(np.float32)
        top = 50
        ra = A.foldin_submit(movie, rating, top)
        rb = B.foldin_submit(iv[movie], rating, top)
        assert ra == rb  # the request id is the noise key
        A.foldin_drain()
        B.foldin_drain()
        ida, mna, vra, _ = A.foldin_poll(ra, top)
        idb, mnb, vrb, _ = B.foldin_poll(rb, top)
        assert np.array_equal(ida, np.where(idb >= 0, ov[np.maximum(idb, 0)], -1))
        assert np.array_equal(mna, mnb) and np.array_equal(vra, vrb)
        assert not np.isin(ida, movie).any()
    A.close()
    B.close()


def test_reorder_rejects_bad_ids(bp):
    """Range checks happen on the caller's ids, before any mapping: at create
    (a column out of range, a CSC that is not the transpose) and on every
    call that takes ids."""
    r = synth.planted(seed=3, M=300, N=200, nnz=4000, K=8)
    bad = synth.Ratings(**{**r.__dict__})
    bad.csr_col = r.csr_col.copy()
    bad.csr_col[0] = r.N
    with pytest.raises(bp.BPMFError) as e:
        bp.Sampler(bad, 8, reorder=True)
    assert e.value.code == bp.E_RANGE
    C = scipy.sparse.csr_matrix((r.csr_val, r.csr_col, r.csr_ptr), shape=(r.M, r.N)).tocsc()
    C.sort_indices()
    wrong = C.data.copy()
    wrong[0] += 1
    with pytest.raises(bp.BPMFError) as e:
        bp.Sampler(r, 8, csc=(C.indptr, C.indices, wrong), reorder=True)
    assert e.value.code == bp.E_FORMAT
    A = bp.Sampler(r, 8, prec="fp32", seed=1, reorder=True, csc=(C.indptr, C.indices, C.data))
    with pytest.raises(bp.BPMFError) as e:
        A.predict(np.array([0, r.M], np.int32), np.array([0, 0], np.int32))
    assert e.value.code == bp.E_RANGE
    with pytest.raises(bp.BPMFError) as e:
        A.predict_noalloc(np.array([0], np.int32), np.array([-1], np.int32))
    assert e.value.code == bp.E_RANGE
    A.store_sample()
    with pytest.raises(bp.BPMFError) as e:
        A.foldin_submit(np.array([1, r.N], np.int32), np.array([1.0, 2.0], np.float32), 5)
    assert e.value.code == bp.E_RANGE
    A.close()
