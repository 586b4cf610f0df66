"""The VALU issue-rate probe runs and reports a rate of the right order: at
most the int16x2 rate derived from unit counts and clock (plus clock slack),
and not far below it."""
import pytest

pytestmark = pytest.mark.gpu


def test_valu_probe_rate():
    from paper_1909_00899_amd import valu_probe
    derived = 256 * 4 * 16 * 2.4e9 * 2
    r = valu_probe.measure(grid=2048, trips=2000)
    assert 0.3 * derived < r < 1.05 * derived, r / derived


def test_valu_probe_int32_rate():
    # one 32-bit op per lane per instruction, 16 lanes per SIMD per cycle; the
    # probe's instructions are counted exactly (written out, not compiled from
    # a foldable chain), so it cannot beat the unit-count rate beyond clock slack
    from paper_1909_00899_amd import valu_probe
    derived = 256 * 4 * 16 * 2.4e9
    r = valu_probe.measure_i32(grid=2048, trips=2000)
    assert 0.3 * derived < r < 1.05 * derived, r / derived
