"""hm_mfma_rate: the sustained rate of the kernel apply's matrix-core
instruction, the practical ceiling its roofline fraction is read against.

Bars: positive, at most the published peak (FP64 78.6, FP32 157.3 TFLOP/s)
plus 5 %, the FP32 instruction at least as fast as the FP64 one; a bad dtype
is an argument error."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_03406_amd as m
    return m


def test_mfma_rate(hm):
    r64 = hm.mfma_rate(hm.HM_F64)
    r32 = hm.mfma_rate(hm.HM_F32)
    print("sustained 16x16x4 MFMA: FP64 %.1f, FP32 %.1f TFLOP/s" % (r64, r32))
    assert 1.0 < r64 <= 78.6 * 1.05
    assert 1.0 < r32 <= 157.3 * 1.05
    assert r32 >= r64
    with pytest.raises(hm.HMError):
        hm.mfma_rate(7)
