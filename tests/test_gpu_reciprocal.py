"""The projection's reciprocal (hardware estimate + one Newton-Raphson step,
full division outside [2^-125, 2^126]) equals the IEEE quotient 1.0f / w for
every positive finite float: an exhaustive check on the device against the
device division, and a digest of the same reciprocals compared with IEEE
quotients computed on the host (numpy float32 division), so that the check does
not rest on the device division alone."""
import numpy as np
import pytest

from paper_2104_07526_amd import pcr

pytestmark = pytest.mark.gpu

RANGES = [
    (0x00000001, 0x007FFFFF),   # subnormals (full-division path for the small ones)
    (0x00800000, 0x3F7FFFFF),   # normals below 1
    (0x3F800000, 0x7F7FFFFF),   # 1 and above, up to the largest finite float
]


def host_digest(lo, hi, chunk=1 << 25):
    """Sum (mod 2^64) and xor of the bit patterns of np.float32(1) / w."""
    total, x = np.uint64(0), np.uint32(0)
    one = np.float32(1.0)
    with np.errstate(over="ignore", divide="ignore", under="ignore"):
        for a in range(lo, hi + 1, chunk):
            b = min(hi + 1, a + chunk)
            w = np.arange(a, b, dtype=np.uint32).view(np.float32)
            q = (one / w).view(np.uint32)
            total = np.uint64((int(total) + int(q.sum(dtype=np.uint64))) % (1 << 64))
            x ^= np.bitwise_xor.reduce(q)
    return int(total), int(x)


@pytest.mark.parametrize("lo,hi", RANGES)
def test_reciprocal_exact_for_every_float(lo, hi):
    bad, s, x = pcr.check_reciprocal(lo, hi)
    assert bad == 0
    hs, hx = host_digest(lo, hi)
    assert (s, x) == (hs, hx), (hex(s), hex(hs), hex(x), hex(hx))
