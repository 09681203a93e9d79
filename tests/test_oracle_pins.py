"""The CPU oracle against its pins (closed forms, hand values, exact-arithmetic
bounds, brute-force gathers, published test vectors, invariants)."""
import pytest

import pins


def test_fp_environment(orc):
    assert orc.fp_env_ok(), "flush-to-zero or denormals-are-zero is set in this process"


@pytest.mark.parametrize("check", pins.ALL_CHECKS, ids=lambda c: c.__name__)
def test_pin(orc, check):
    check(orc)


def test_golden_scene(orc):
    pins.check_golden_scene(orc)
