"""Pins of the oracle's grid lookup through the unbounded-scene contraction (Eq. 4, p = inf and
p = 2, section 5.4).

An identity field on a grid with dyadic vertex positions reproduces the contracted point
exactly (trilinear interpolation is exact on linear fields), so the lookup is pinned against an
independent numpy statement of Eq. 4, against its radius law (the p-norm of the image is
1 + b - b/||x||_p outside the unit ball, and directions are kept), against continuity at the
unit sphere and the limit radius 1 + b, and the warped scatter against the warped gather by the
adjoint identity.  Inside the unit ball the warped lookup equals the plain one bit for bit.
"""
import numpy as np
import pytest

import synth


def _grid(data, b, warp):
    lo = np.full(3, -1.0 - b, np.float32)
    return synth.Grid(np.ascontiguousarray(data, np.float32), lo, -lo, warp=warp, warp_b=b)


def _identity(b, n=17):
    # n vertices over [-1-b, 1+b]: dyadic spacing for b = 1 (0.25) and b = 3 (0.5)
    ax = np.linspace(-1.0 - b, 1.0 + b, n)
    return np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1)


def _norm(x, warp):
    return np.abs(x).max(axis=-1) if warp == 1 else np.linalg.norm(x, axis=-1)


def _eq4(x, b, warp):
    n = _norm(x, warp)[:, None]
    return np.where(n <= 1.0, x, (1.0 + b - b / np.maximum(n, 1.0)) * x / np.maximum(n, 1e-300))


def _points(rng, S):
    d = rng.standard_normal((S, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = 10.0 ** rng.uniform(-1.0, 4.0, S)
    return (d * r[:, None]).astype(np.float32)


@pytest.mark.parametrize("warp", [1, 2])
@pytest.mark.parametrize("b", [1.0, 3.0])
def test_identity_field_reproduces_eq4(orc, warp, b):
    rng = np.random.default_rng(110)
    x = _points(rng, 4000)
    got = orc.gather(_grid(_identity(b), b, warp), x)
    want = _eq4(x.astype(np.float64), b, warp)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("warp", [1, 2])
def test_radius_law_and_direction(orc, warp):
    b = 1.0
    rng = np.random.default_rng(111)
    x = _points(rng, 3000).astype(np.float64)
    out = _norm(x, warp) > 1.0
    got = orc.gather(_grid(_identity(b), b, warp), x.astype(np.float32))
    xs = x.astype(np.float32).astype(np.float64)
    n = _norm(xs, warp)
    np.testing.assert_allclose(_norm(got, warp)[out], 1.0 + b - b / n[out], rtol=1e-12)
    cross = np.cross(got, xs)
    assert np.abs(cross).max() <= 1e-10 * np.abs(xs).max()
    assert (np.einsum("ij,ij->i", got, xs) > 0).all()
    # never leaves the radius-(1+b) ball, and the far field approaches it
    assert _norm(got, warp).max() < 1.0 + b
    far = orc.gather(_grid(_identity(b), b, warp), np.float32([[3e7, -1e7, 2e7]]))
    assert _norm(far, warp)[0] == pytest.approx(1.0 + b, abs=1e-6)


@pytest.mark.parametrize("warp", [1, 2])
def test_continuous_at_the_unit_sphere(orc, warp):
    b = 1.0
    d = np.array([[0.6, -0.48, 0.64], [1.0, 0.25, -0.5]])
    d /= _norm(d, warp)[:, None]
    x = np.concatenate([d * (1 - 1e-6), d * (1 + 1e-6)]).astype(np.float32)
    got = orc.gather(_grid(_identity(b), b, warp), x)
    assert np.abs(got[:2] - got[2:]).max() < 1e-5


@pytest.mark.parametrize("warp", [1, 2])
def test_inside_is_the_plain_lookup(orc, warp):
    rng = np.random.default_rng(112)
    data = rng.standard_normal((9, 10, 11, 4)).astype(np.float32)
    x = rng.uniform(-1.0, 1.0, (2000, 3))
    if warp == 2:
        x = x[np.linalg.norm(x, axis=1) <= 0.999]
    x = x.astype(np.float32)
    warped = orc.gather(_grid(data, 1.0, warp), x)
    plain = orc.gather(_grid(data, 1.0, 0), x)
    assert np.array_equal(warped, plain)


@pytest.mark.parametrize("warp", [1, 2])
def test_warped_scatter_is_the_adjoint(orc, warp):
    rng = np.random.default_rng(113)
    data = rng.standard_normal((8, 9, 10, 3)).astype(np.float32)
    g = _grid(data, 2.0, warp)
    x = _points(rng, 500)
    v = rng.standard_normal((500, 3))
    lhs = float(np.sum(orc.gather(g, x) * v))
    rhs = float(np.sum(data.astype(np.float64) * orc.scatter(g, x, v)))
    assert lhs == pytest.approx(rhs, rel=1e-12)
