"""Host-side logic of TrainStep (no GPU): construction with every option, the MLP parameter
views into one flat buffer, and the choice of the fused-gather and two-stream paths."""
import numpy as np
import pytest
import torch

import synth
from paper_2206_05085_amd import ops
from paper_2206_05085_amd.step import TrainStep


@pytest.mark.parametrize("kw", [dict(), dict(tv=(1e-5, 1e-6, 1.0, True)), dict(warp=(1, 1.0)),
                                dict(mlp_precision=1), dict(binned_scatter=False, concurrent=False)])
def test_construct_on_host(kw):
    wl = synth.config2(R=8, n=16)
    st = TrainStep(wl.density.data, (wl.density.xyz_min, wl.density.xyz_max), feat=wl.feat.data,
                   mlp=(wl.mlp.W, wl.mlp.b), device="cpu", **kw)
    assert st.binned == kw.get("binned_scatter", True) and st.concurrent == kw.get("concurrent", True)
    assert st.mlp.precision == kw.get("mlp_precision", 0)
    g = st.grid("feat")
    assert g.warp == kw.get("warp", (0, 1.0))[0] and g.data.shape == (16, 16, 16, 12)
    # MLP parameters are views of one flat buffer (one Adam launch covers them)
    flat = st.mlp_flat["p"]
    total = sum(w.size for w in wl.mlp.W) + sum(b.size for b in wl.mlp.b)
    assert flat.numel() == total
    assert all(w.data_ptr() >= flat.data_ptr() for w in st.mlp.W)
    np.testing.assert_array_equal(st.mlp.W[1].numpy(), wl.mlp.W[1])
    np.testing.assert_array_equal(st.mlp.b[2].numpy(), wl.mlp.b[2])


def test_grid_mode_on_host():
    wl = synth.config1(R=8, n=8)
    st = TrainStep(wl.density.data, (wl.density.xyz_min, wl.density.xyz_max), color=wl.color.data, device="cpu")
    assert st.grid_mode and st.grid("color").channels == 3
    assert torch.equal(st.color["p"], torch.as_tensor(wl.color.data))


def test_fused_gather_choice():
    wl = synth.config2(R=8, n=16)
    st = TrainStep(wl.density.data, (wl.density.xyz_min, wl.density.xyz_max), feat=wl.feat.data,
                   mlp=(wl.mlp.W, wl.mlp.b), device="cpu")
    assert st.fused_gather  # 12 feature channels: the gather runs inside the colour head's forward
    # three feature channels cannot move as float4 rows: the separate gather is kept
    m3 = synth.mlp_weights(np.random.default_rng(0), C=3)
    st3 = TrainStep(wl.density.data, (wl.density.xyz_min, wl.density.xyz_max), feat=wl.feat.data[..., :3],
                    mlp=(m3.W, m3.b), device="cpu")
    assert not st3.fused_gather
    assert not TrainStep(wl.density.data, (wl.density.xyz_min, wl.density.xyz_max), feat=wl.feat.data,
                         mlp=(wl.mlp.W, wl.mlp.b), fused_gather=False, device="cpu").fused_gather
