"""Tolerance rule shared by the GPU parity tests.

FP32 results are compared with the FP64 oracle per output tensor x (GPU) vs y (oracle):
pass iff BOTH
  normwise     ||x - y||_2 <= rtol ||y||_2, and
  elementwise  |x_i - y_i| <= rtol * max(|y_i|, floor * ||y||_inf).
rtol is 1e-5 for forward values and 1e-4 for gradients; floor is 1e-3 for forward values
and 1e-2 for gradients.  The floor exists because per-sample density gradients carry an
inherent cancellation (T_{k+1} g_k - S_k) and because float32 transmittance underflows
for opaque rays where float64 does not; the normwise bound keeps the comparison strict.
"""
import numpy as np

FWD = dict(rtol=1e-5, floor=1e-3)
GRAD = dict(rtol=1e-4, floor=1e-2)


def close(x, y, rtol, floor, name="value", scale=None, skip=None, slack=None, elem_rtol=None):
    """scale (optional, per element): the magnitude the result is conditioned on, e.g.
    sum_c w_c |G_c| for an interpolated value whose terms cancel; the elementwise bound
    then uses max(|y_i|, floor * ||y||_inf, scale_i).  skip (optional boolean mask):
    elements at a non-differentiable point (a ReLU unit within rounding of its kink) are
    left out of the elementwise check; the normwise check still covers them.  slack
    (optional, per element): an absolute allowance added to the elementwise bound, e.g. the
    change a gradient sees when a ReLU unit at its kink switches side; its 2-norm is added to
    the normwise bound as well.  elem_rtol (optional): a separate relative bound for the
    elementwise check (the normwise check keeps rtol)."""
    x = np.asarray(x, np.float64).ravel()
    y = np.asarray(y, np.float64).ravel()
    assert x.shape == y.shape, f"{name}: shape {x.shape} vs {y.shape}"
    assert np.isfinite(x).all(), f"{name}: non-finite values"
    ny = np.linalg.norm(y)
    err = np.linalg.norm(x - y)
    # a slack (an ambiguous kink decision) may move the result by up to |slack| per element
    ns = np.linalg.norm(np.asarray(slack, np.float64)) if slack is not None else 0.0
    assert err <= rtol * ny + ns + 1e-30, f"{name}: normwise error {err / max(ny, 1e-300):.3e} > {rtol}"
    if y.size:
        er = rtol if elem_rtol is None else elem_rtol
        bound = er * np.maximum(np.abs(y), floor * np.abs(y).max())
        if scale is not None:
            bound = np.maximum(bound, er * np.asarray(scale, np.float64).ravel())
        bad = np.abs(x - y) > bound + 1e-30
        if slack is not None:
            bad &= np.abs(x - y) > bound + np.asarray(slack, np.float64).ravel()
        if skip is not None:
            bad &= ~np.asarray(skip, bool).ravel()
        if bad.any():
            excess = np.abs(x - y) - bound - (0.0 if slack is None else np.asarray(slack, np.float64).ravel())
            i = np.argmax(np.where(bad, excess, -np.inf))
            raise AssertionError(f"{name}: {bad.sum()} of {y.size} elements out of bound; worst at {i}: "
                                 f"gpu {x[i]:.9g} oracle {y[i]:.9g} bound {bound[i]:.3g}")
    return err / max(ny, 1e-300)


def close_after_adam(x, y, steps, lr, name="value", rtol=1e-5):
    """Grid parameters after `steps` Adam updates in two runs whose gradients are sums of the same
    terms added in different orders (atomics).  Adam's update is normalised (at most about lr per
    step for beta1^2 < beta2), so where a gradient nearly cancels, the reordered sum can move that
    element's update by up to lr per step in each run.  Checked: normwise within rtol; every
    element within 2 lr per step; all but 1e-4 of the elements within rtol of max(|y|, steps lr)."""
    x = np.asarray(x, np.float64).ravel()
    y = np.asarray(y, np.float64).ravel()
    assert x.shape == y.shape, f"{name}: shape {x.shape} vs {y.shape}"
    assert np.isfinite(x).all(), f"{name}: non-finite values"
    d = np.abs(x - y)
    assert d.max() <= 2 * lr * steps, f"{name}: {d.max():.3g} beyond Adam's step bound"
    assert np.linalg.norm(x - y) <= rtol * np.linalg.norm(y) + 1e-30, f"{name}: normwise"
    loose = d > rtol * np.maximum(np.abs(y), steps * lr)
    assert loose.mean() <= 1e-4, f"{name}: {loose.sum()} of {y.size} beyond rounding"
