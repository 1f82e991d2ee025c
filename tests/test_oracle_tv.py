"""Pins of the oracle's total-variation regulariser (section 2, efficient TV loss).

The gradient is pinned by closed forms (constant field, a linear ramp in the quadratic
regime: zero inside, +-a on the two end faces; an isolated spike in the saturated regime),
by central finite differences of the oracle's own loss value, by 2-homogeneity of the
quadratic regime (sum v dL/dv = 2 L), and the sparse mode by its rule: vertices whose
incoming gradient is zero are left bitwise unchanged, the others get the dense value.
"""
import numpy as np
import pytest

import synth


def _grid(data):
    data = np.ascontiguousarray(data, np.float32)
    if data.ndim == 3:
        data = data[..., None]
    return synth.Grid(data, np.full(3, -1.0, np.float32), np.full(3, 1.0, np.float32))


@pytest.mark.parametrize("shape", [(4, 5, 3, 1), (3, 3, 3, 12), (1, 4, 2, 2)])
def test_constant_field_has_no_gradient(orc, shape):
    g = _grid(np.full(shape, 0.7, np.float32))
    L, grad = orc.tv(g, weight=0.1, delta=0.5)
    assert L == 0.0
    assert not grad.any()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_linear_ramp_closed_form(orc, axis):
    # v = a * index along one axis, |a| <= delta: interior differences cancel, each end
    # face keeps its single neighbour: dL/dv = 2 w / (N C) * (-a) at index 0, (+a) at n-1
    n, a, w = (5, 6, 4), 0.375, 3.0
    idx = np.indices(n)[axis].astype(np.float64)
    g = _grid(a * idx)
    L, grad = orc.tv(g, weight=w, delta=1.0)
    N = np.prod(n)
    want = np.zeros(n)
    first = [slice(None)] * 3
    last = [slice(None)] * 3
    first[axis], last[axis] = 0, n[axis] - 1
    want[tuple(first)] = -2 * w / N * a
    want[tuple(last)] = 2 * w / N * a
    np.testing.assert_allclose(grad[..., 0], want, rtol=1e-12, atol=1e-15)
    # each of the (n_axis - 1) * (other sizes) edges appears twice with penalty a^2 / 2
    edges = (n[axis] - 1) * N // n[axis]
    assert L == pytest.approx(w / N * 2 * edges * 0.5 * a * a, rel=1e-12)


def test_spike_saturates(orc):
    # one vertex raised by A >> delta: the spike gets 2 w delta / N per neighbour, each
    # neighbour -2 w delta / N, everything else 0
    n, A, w, d = (5, 5, 5), 10.0, 1.0, 0.25
    v = np.zeros(n)
    v[2, 2, 2] = A
    L, grad = orc.tv(_grid(v), weight=w, delta=d)
    N = np.prod(n)
    want = np.zeros(n)
    want[2, 2, 2] = 6 * 2 * w * d / N
    for o in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        want[2 + o[0], 2 + o[1], 2 + o[2]] = -2 * w * d / N
    np.testing.assert_allclose(grad[..., 0], want, rtol=1e-12, atol=1e-15)
    assert L == pytest.approx(w / N * 12 * d * (A - d / 2), rel=1e-12)


@pytest.mark.parametrize("delta", [0.3, 1e9])
def test_gradient_matches_finite_differences(orc, delta):
    rng = np.random.default_rng(40)
    data = rng.standard_normal((4, 5, 3, 2)).astype(np.float32)
    w = 2.0
    _, grad = orc.tv(_grid(data), weight=w, delta=delta)
    eps = 1e-3
    worst = 0.0
    for idx in np.ndindex(data.shape):
        p, m = data.copy(), data.copy()
        p[idx] += eps
        m[idx] -= eps
        hp = float(np.float32(p[idx]))
        hm = float(np.float32(m[idx]))
        fd = (orc.tv(_grid(p), w, delta)[0] - orc.tv(_grid(m), w, delta)[0]) / (hp - hm)
        worst = max(worst, abs(fd - grad[idx]) / (abs(grad).max()))
    # Huber is C1; a difference within eps of +-delta adds O(eps) curvature error
    assert worst < (1e-6 if delta > 1e6 else 2e-2)


def test_quadratic_regime_is_2_homogeneous(orc):
    rng = np.random.default_rng(41)
    data = rng.standard_normal((3, 4, 5, 3))
    g = _grid(data)
    L, grad = orc.tv(g, weight=0.5, delta=1e9)
    v = g.data.astype(np.float64)
    assert float(np.sum(v * grad)) == pytest.approx(2 * L, rel=1e-12)


def test_sparse_mode_rule(orc):
    rng = np.random.default_rng(42)
    data = rng.standard_normal((5, 4, 6, 3)).astype(np.float32)
    g = _grid(data)
    incoming = np.zeros(data.shape)
    touched = rng.random(data.shape[:3]) < 0.3
    ch = rng.integers(0, 3, data.shape[:3])
    for idx in zip(*np.nonzero(touched)):
        incoming[idx + (ch[idx],)] = rng.standard_normal()
    incoming[0, 0, 0, :] = 0.0
    incoming[0, 0, 0, 1] = -0.0          # a negative zero is a zero gradient
    touched[0, 0, 0] = False
    _, dense = orc.tv(g, 0.2, 0.4, dense=True)
    _, sparse = orc.tv(g, 0.2, 0.4, dense=False, grad=incoming)
    assert np.array_equal(sparse[~touched], incoming[~touched])
    assert not touched[0, 0, 0]
    np.testing.assert_allclose(sparse[touched], incoming[touched] + dense[touched], rtol=1e-15, atol=0)
