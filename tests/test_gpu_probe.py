"""GPU test of the int32 vector-ALU probe: its rate is a plausible fraction
of the device's published vector rate (128 lanes per CU per cycle x 256 CUs
x 2.4 GHz = 7.86e13 lane-ops/s on MI355X) and never above it by more than
the clock's boost margin."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_probe_rate_is_plausible():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    import paper_2405_07989_amd as fz
    r = fz.probe_int_valu()
    peak = 128 * 256 * 2.4e9
    assert r["ms"] > 0
    assert 0.5 * peak < r["lane_ops_per_s"] < 1.05 * peak, r


def test_write_probe_rate_is_plausible():
    """The HBM write probe (16-byte stores over a fresh 1 GiB buffer) reports
    a rate between a tenth and the published 8 TB/s."""
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    import paper_2405_07989_amd as fz
    r = fz.probe_hbm_write(1 << 30)
    assert r["ms"] > 0
    assert 0.8e12 < r["bytes_per_s"] < 8.0e12, r
