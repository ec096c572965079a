"""The oracle against what the paper and the mathematics fix (not gpu)."""
import pytest

import oracle
import oracle_pins


@pytest.fixture(scope="module")
def orc():
    return oracle.get()


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(orc, pin):
    fails = pin(orc)
    assert not fails, "\n".join(fails[:20])


def test_bad_arguments(orc):
    import numpy as np
    A = np.zeros((4, 4), order="F")
    assert orc.gemm("X", "N", 2, 2, 2, 1.0, A, "d", 4, A, "d", 4, 0.0, A, "d", 4)[0] == oracle.ERR_ARG
    assert orc.gemm("N", "N", 5, 2, 2, 1.0, A, "d", 4, A, "d", 4, 0.0, A, "d", 4)[0] == oracle.ERR_ARG
    assert orc.gemm("N", "N", 2, 2, 2, 1.0, A, 9, 4, A, "d", 4, 0.0, A, "d", 4)[0] == oracle.ERR_ARG
