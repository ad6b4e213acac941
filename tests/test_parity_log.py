"""The parity recorder the GPU tests use (CPU only): parity_log.allclose
records the largest |got - ref| / (atol + rtol |ref|) and asserts as
np.testing.assert_allclose does, NaN in the same places counting as equal."""
import numpy as np
import pytest

import parity_log


def test_allclose_records_the_error_over_its_bar():
    parity_log.RECORDS.clear()
    ref = np.array([1.0, -2.0, np.nan, 0.0])
    got = ref * (1.0 + 5e-10)
    parity_log.allclose("case", got, ref, rtol=1e-9, atol=1e-12)
    (name, err, bar), = parity_log.RECORDS
    assert name == "case (error / bar)" and bar == 1.0
    assert 0.4 < err < 0.6  # 5e-10 |ref| over (1e-12 + 1e-9 |ref|), for |ref| = 1 and 2


def test_allclose_fails_beyond_the_bar_and_on_nan_mismatch():
    with pytest.raises(AssertionError):
        parity_log.allclose("over", np.array([1.0 + 1e-8]), np.array([1.0]), rtol=1e-9)
    with pytest.raises(AssertionError):
        parity_log.allclose("nan", np.array([np.nan]), np.array([1.0]), rtol=1e-9)
    parity_log.RECORDS.clear()
    parity_log.allclose("zero bar", np.array([0.0, 3.0]), np.array([0.0, 3.0]), rtol=0.0)
    assert parity_log.RECORDS[-1][1] == 0.0
