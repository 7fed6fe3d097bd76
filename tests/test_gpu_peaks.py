"""GPU checks of the measurement kernels (include/bpmf_peaks.h): each returns
a rate inside what the MI355X spec sheet allows (HBM 8 TB/s; FP32 vector and
matrix 157.3, BF16 matrix 2500, FP64 matrix 78.6 TFLOP/s), and the gather
rate falls as the source leaves L2 for the Infinity Cache and then HBM."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bp():
    import paper_1705_04159_amd as bp

    return bp


def test_triad(bp):
    gbs = bp.peak_triad(1 << 30, 5)
    print("triad GB/s", gbs, flush=True)
    assert 1000.0 < gbs < 8000.0 * 1.02


@pytest.mark.parametrize("kind,lo,hi", [(0, 10.0, 157.3), (1, 30.0, 157.3), (2, 300.0, 2500.0),
                                        (3, 10.0, 78.6)])
def test_compute(bp, kind, lo, hi):
    tf = bp.peak_compute(kind, 3)
    print("kind", kind, "TFLOP/s", tf, flush=True)
    assert lo < tf < hi * 1.02


def test_gather_hierarchy(bp):
    rates = [bp.peak_gather(mb << 20, 128, 1 << 22, 3) for mb in (3, 1024)]
    print("gather GB/s (3 MiB, 1 GiB sources)", rates, flush=True)
    assert all(r > 100.0 for r in rates)
    assert rates[0] > rates[1]
