"""The comparison helpers the GPU parity tests use, checked on the CPU against planted
differences: each bound must accept rounding-sized differences and reject the mistakes it
is there to catch."""
import numpy as np
import pytest

from parity import close, close_after_adam


def test_close_accepts_rounding_and_rejects_a_wrong_element():
    rng = np.random.default_rng(0)
    y = rng.standard_normal(1000)
    close(y * (1 + 1e-7), y, rtol=1e-5, floor=1e-3)
    bad = y.copy()
    bad[17] += 1e-4            # small normwise, far beyond rounding for that element
    with pytest.raises(AssertionError, match="elements out of bound"):
        close(bad, y, rtol=1e-5, floor=1e-3)
    with pytest.raises(AssertionError, match="normwise"):
        close(y * 1.01, y, rtol=1e-5, floor=1e-3)


def test_close_after_adam():
    rng = np.random.default_rng(1)
    lr, steps = 0.1, 3
    y = rng.standard_normal(200000)
    x = y * (1 + 1e-7)
    x[:5] += 5e-3 * lr         # a few nearly cancelling gradients whose update moved
    close_after_adam(x, y, steps, lr)
    # a move beyond Adam's per-step bound
    z = x.copy()
    z[10] += 2 * lr * steps + 1e-3
    with pytest.raises(AssertionError, match="step bound"):
        close_after_adam(z, y, steps, lr)
    # too many elements off by more than rounding (a systematic error, e.g. a lost term)
    w = y.copy()
    w[: y.size // 100] += 1e-3
    with pytest.raises(AssertionError):
        close_after_adam(w, y, steps, lr)
    # a normwise difference
    with pytest.raises(AssertionError, match="normwise"):
        close_after_adam(y * 1.001, y, steps, lr)
