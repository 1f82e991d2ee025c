"""The distortion loss entry point that allocates nothing (its checkpoints live in the library's
fixed device array) against dvgo_distortion_loss with a caller workspace, on two calls in a row,
the second with a smaller batch; and its size limit.  Both run the same kernel, which has no
atomics, so the results must agree bit for bit."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_05085_amd as pkg
    pkg.lib()
    from paper_2206_05085_amd import ops
    return ops


def say(*a):
    print("[case]", *a, flush=True)


def T(a, dt=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)


def _case(rng, lengths):
    offs, w, m, l = synth.random_ragged(rng, lengths)
    gl = rng.standard_normal(len(lengths)).astype(np.float32)
    g0 = rng.standard_normal(int(offs[-1])).astype(np.float32)  # grad_w accumulates into this
    return offs, w, m, l, gl, g0


def test_noalloc_matches_workspace_call(dv):
    rng = np.random.default_rng(90)
    big = list(rng.integers(0, 700, 4096)) + [0, 1, 63, 64, 65, 1024]
    small = list(rng.integers(0, 130, 97)) + [0, 129]
    for name, lengths in (("large", big), ("smaller", small)):
        offs, w, m, l, gl, g0 = _case(rng, lengths)
        say("distortion no-alloc vs workspace:", name, len(lengths), "rays,", int(offs[-1]), "samples")
        args = (T(offs, torch.int32), T(w), T(m), T(l))
        ga, gb = T(g0), T(g0)
        la, _ = dv.distortion_loss_noalloc(*args, grad_loss=T(gl), grad_w=ga)
        lb, _ = dv.distortion_loss(*args, grad_loss=T(gl), grad_w=gb)
        lf, _ = dv.distortion_loss_noalloc(*args)  # forward only
        torch.cuda.synchronize()
        assert torch.equal(la, lb) and torch.equal(lf, lb)
        assert torch.equal(ga, gb)
        assert not torch.equal(ga, T(g0))


def test_noalloc_size_limit(dv):
    # n_samples / 64 + n_rays + 1 checkpoints must fit the fixed 2 MiB (262144 of 8 bytes): one ray
    # of 64 samples among 262144 rays needs 262146 and is refused; among 262142 rays it fits
    import paper_2206_05085_amd as pkg
    say("distortion no-alloc: batch beyond the fixed scratch is refused, the largest one runs")
    for R, ok in ((262144, False), (262142, True)):
        offs = np.full(R + 1, 64, np.int32)
        offs[0] = 0
        w = T(np.full(64, 1.0 / 64))
        m = T((np.arange(64) + 0.5) / 64)
        l = T(np.full(64, 1.0 / 64))
        gl = torch.zeros(R, device="cuda")
        gl[0] = 1.0
        gw = torch.zeros(64, device="cuda")
        if not ok:
            with pytest.raises(pkg.DvgoError) as err:
                dv.distortion_loss_noalloc(T(offs, torch.int32), w, m, l, grad_loss=gl, grad_w=gw)
            assert err.value.code == -3 and "fixed" in str(err.value)
            continue
        loss, _ = dv.distortion_loss_noalloc(T(offs, torch.int32), w, m, l, grad_loss=gl, grad_w=gw)
        torch.cuda.synchronize()
        # uniform weights on 64 equal intervals: D = 1/3 (the closed form of Eq. 1), other rays empty
        assert abs(float(loss[0]) - 1.0 / 3.0) < 1e-6 and not loss[1:].any()
        assert gw.abs().sum() > 0
