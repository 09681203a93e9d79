"""The projection's reciprocal (hardware estimate + one FMA correction, full
division outside [2^-125, 2^126]) equals the IEEE quotient 1.0f / w for every
positive finite float: an exhaustive check on the device."""
import pytest

from paper_2104_07526_amd import pcr

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("lo,hi", [
    (0x00000001, 0x007FFFFF),   # subnormals (full-division path for the small ones)
    (0x00800000, 0x3F7FFFFF),   # normals below 1
    (0x3F800000, 0x7F7FFFFF),   # 1 and above, up to the largest finite float
])
def test_reciprocal_exact_for_every_float(lo, hi):
    assert pcr.check_reciprocal(lo, hi) == 0
