"""enkf_mfma_peak: the measured matrix-core throughput is positive, no higher
than the published dense peak of the type (with 5% slack for the clock), and
unsupported input types are refused."""
import pytest

pytestmark = pytest.mark.gpu

PUBLISHED = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "f16": 2500.0}


@pytest.mark.parametrize("math", ["f64", "f32", "bf16", "f16"])
def test_mfma_peak_is_plausible(math):
    import paper_1302_3876_amd as pk
    t = pk.mfma_peak(math)
    print(math, t, flush=True)
    assert 0.05 * PUBLISHED[math] < t <= 1.05 * PUBLISHED[math]


def test_mfma_peak_rejects_split_types():
    import paper_1302_3876_amd as pk
    with pytest.raises(pk.EnkfError) as e:
        pk.mfma_peak("bf16x3")
    assert e.value.code == 6
