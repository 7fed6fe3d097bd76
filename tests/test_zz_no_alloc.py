"""bpmf_predict_noalloc (the prediction entry point for callers that cannot
allocate device memory) against bpmf_predict: the same predictions bit for
bit, on two calls in a row (the second smaller, so stale staging contents
from the first would show), on FP32 and FP64 contexts, with the size limit
and range checks of the C ABI, and no change in free device memory."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bp():
    import paper_1705_04159_amd as bp

    bp.lib()
    return bp


def _free_device_bytes():
    hip = ctypes.CDLL("libamdhip64.so.7")  # the library's own HIP runtime
    hip.hipMemGetInfo.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    free, total = ctypes.c_size_t(), ctypes.c_size_t()
    assert hip.hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)) == 0
    return free.value


@pytest.mark.parametrize("prec,K", [("fp32", 16), ("fp32", 100), ("fp64", 10)])
def test_predict_noalloc_matches_predict(bp, prec, K):
    r = synth.random_small(31, 3000, 1200, 40000, min(K, 12))
    s = bp.Sampler(r, K, prec=prec, seed=7)
    s.run_sweeps(1, 2)
    rng = np.random.default_rng(K)
    s.predict_noalloc(np.array([0], np.int32), np.array([0], np.int32))  # runtime warm-up
    for n in (400_000, 3_001):
        row = rng.integers(0, r.M, n).astype(np.int32)
        col = rng.integers(0, r.N, n).astype(np.int32)
        free0 = _free_device_bytes()
        got = s.predict_noalloc(row, col)
        assert _free_device_bytes() == free0  # nothing allocated
        ref = s.predict(row, col)
        assert np.array_equal(got, ref)
        assert np.isfinite(got).all()
    # the limit of the staging area and the range checks
    big = np.zeros((1 << 19) + 1, np.int32)
    with pytest.raises(bp.BPMFError) as e:
        s.predict_noalloc(big, big)
    assert e.value.code == bp.E_TOOBIG
    with pytest.raises(bp.BPMFError) as e:
        s.predict_noalloc(np.array([r.M], np.int32), np.array([0], np.int32))
    assert e.value.code == bp.E_RANGE
    # still usable, and an empty call is a no-op
    assert s.predict_noalloc(np.zeros(0, np.int32), np.zeros(0, np.int32)).shape == (0,)
    s.close()


def test_predict_noalloc_two_contexts_share_the_device_array(bp):
    """Two contexts on one GPU share the staging area; calls one after the
    other each see their own inputs."""
    r1 = synth.random_small(32, 500, 300, 6000, 8)
    r2 = synth.random_small(33, 700, 200, 6000, 8)
    a = bp.Sampler(r1, 8, prec="fp32", seed=1)
    b = bp.Sampler(r2, 8, prec="fp32", seed=2)
    ra, ca = np.arange(500, dtype=np.int32), (np.arange(500) % 300).astype(np.int32)
    rb, cb = (np.arange(300) % 700).astype(np.int32), (np.arange(300) % 200).astype(np.int32)
    ga = a.predict_noalloc(ra, ca)
    gb = b.predict_noalloc(rb, cb)
    assert np.array_equal(ga, a.predict(ra, ca))
    assert np.array_equal(gb, b.predict(rb, cb))
    a.close()
    b.close()
