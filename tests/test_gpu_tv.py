"""GPU parity of the total-variation gradient (dvgo_tv_add_grad) against the FP64 oracle.

Dense and sparse modes, the float4 path (12 channels) and the scalar path (1 channel; 3
channels with a padded stride, whose padding must stay untouched), small ragged shapes and
the full 160^3 x 12 feature grid of the step.  The bar is R16's forward tolerance with the
elementwise floor taken from the magnitude each sum is conditioned on (the oracle's
2 w/(N C) sum |clamp|), since the six neighbour differences cancel inside smooth regions.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from parity import FWD, close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_05085_amd as pkg
    pkg.lib()  # raises if the HIP library is missing
    from paper_2206_05085_amd import ops
    return ops


def say(*a):
    print("[case]", *a, flush=True)


def T(a, dt=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)


def _grid(data):
    return synth.Grid(np.ascontiguousarray(data, np.float32), np.full(3, -1.0, np.float32),
                      np.full(3, 1.0, np.float32))


def _run(dv, data, weight, delta, dense, incoming=None, channels=None):
    g = T(data)
    gr = torch.zeros_like(g) if incoming is None else T(incoming)
    dv.tv_add_grad(dv.DeviceGrid(g, (-1, -1, -1), (1, 1, 1), grad=gr, channels=channels), weight, delta, dense)
    torch.cuda.synchronize()
    return gr.cpu().numpy()


def _oracle(data, weight, delta, dense, incoming=None, channels=None):
    C = data.shape[3] if channels is None else channels
    # the oracle sees the used channels only; padding is compared separately
    d = np.ascontiguousarray(data[..., :C])
    inc = None if incoming is None else np.ascontiguousarray(incoming[..., :C], np.float64)
    _, grad, mag = oracle.tv(_grid(d), weight, delta, dense=dense, grad=inc, want_mag=True)
    return grad, mag


@pytest.mark.parametrize("shape,channels,delta", [((17, 18, 19, 1), None, 0.5), ((9, 10, 11, 12), None, 0.3),
                                                  ((8, 9, 7, 4), 3, 1.0), ((2, 2, 2, 12), None, 1e6)])
def test_tv_dense(dv, shape, channels, delta):
    rng = np.random.default_rng(70)
    data = rng.standard_normal(shape).astype(np.float32)
    N, C = np.prod(shape[:3]), shape[3] if channels is None else channels
    weight = N * C / 2.0          # coef = 2 w / (N C) = 1 keeps the values O(1)
    say("tv dense", shape, "channels", C, "delta", delta)
    got = _run(dv, data, weight, delta, True, channels=channels)
    want, mag = _oracle(data, weight, delta, True, channels=channels)
    close(got[..., :C], want, **FWD, name="tv grad", scale=mag)
    if C < shape[3]:
        assert not got[..., C:].any(), "padding channels touched"


def test_tv_sparse(dv):
    rng = np.random.default_rng(71)
    shape = (12, 13, 14, 12)
    data = rng.standard_normal(shape).astype(np.float32)
    incoming = np.zeros(shape, np.float32)
    touched = rng.random(shape[:3]) < 0.25
    ch = rng.integers(0, 12, shape[:3])
    for idx in zip(*np.nonzero(touched)):
        incoming[idx + (ch[idx],)] = rng.standard_normal()
    incoming[3, 3, 3, :] = 0.0
    incoming[3, 3, 3, 5] = -0.0
    touched[3, 3, 3] = False
    N = np.prod(shape[:3])
    weight = N * 12 / 2.0
    say("tv sparse", shape, int(touched.sum()), "touched vertices")
    got = _run(dv, data, weight, 0.4, False, incoming=incoming)
    want, mag = _oracle(data, weight, 0.4, False, incoming=incoming)
    assert np.array_equal(got[~touched].view(np.uint32), incoming[~touched].view(np.uint32)), "untouched changed"
    close(got[touched], want[touched], **FWD, name="tv grad (touched)",
          scale=np.maximum(mag[touched], np.abs(incoming[touched])))


@pytest.mark.parametrize("dense", [True, False])
def test_tv_feature_grid_full_size(dv, dense):
    # the step's 160^3 x 12 feature grid, paper weight 1e-6 (section 5.3 feature grid), delta 1
    wl_rng = np.random.default_rng(72)
    data = wl_rng.standard_normal((160, 160, 160, 12)).astype(np.float32)
    incoming = None
    if not dense:
        incoming = np.zeros_like(data)
        mask = wl_rng.random((160, 160, 160)) < 0.5
        incoming[mask, 0] = 1e-9
    say("tv full size 160^3 x 12, dense =", dense)
    got = _run(dv, data, 1e-6, 1.0, dense, incoming=incoming)
    want, mag = _oracle(data, 1e-6, 1.0, dense, incoming=incoming)
    scale = mag if incoming is None else np.maximum(mag, np.abs(incoming))
    close(got, want, **FWD, name="tv grad 160^3x12", scale=scale)
