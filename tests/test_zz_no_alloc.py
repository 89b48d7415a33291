"""The allocation-free MLP backward (fm_mlp_backward_noalloc, gradient slots
in the library's static device scratch) against fm_mlp_backward (slots in a
context workspace it allocates) through the C ABI, on two calls in a row, the
second with a smaller input.  Up to 8,192 matches both launch the same grid,
so the gradients are bit-identical; above, the allocation-free call caps the
grid at 128 workgroups, so its float32 slot sums run in a different order and
agree to within 1e-4 of each gradient block's largest entry (at most 2,048
float32 additions per entry)."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _weights(ctx, rng):
    from paper_2505_04612_amd import api
    w = api.MlpWeights(ctx.device, mean=torch.zeros(3, device=ctx.device), std=torch.ones(3, device=ctx.device))
    for k, shp in api.MLP_SHAPES.items():
        w.views[k].copy_(torch.from_numpy(rng.normal(0.0, 0.5, size=shp).astype(np.float32)))
    return w


def _call(ctx, name, w, feats, act, dout):
    from paper_2505_04612_amd import api
    from paper_2505_04612_amd._lib import check
    g = api.MlpWeights(ctx.device)
    M = int(feats.shape[0])
    gs = w.grad_struct(g)
    fn = getattr(ctx.lib, name)
    check(ctx.handle, fn(ctx.handle, M, feats.data_ptr(), ctypes.byref(w.struct()), act.data_ptr(),
                         dout.data_ptr(), ctypes.byref(gs), torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return {k: v.clone() for k, v in g.views.items()}


@pytest.mark.parametrize("sizes", [(8000, 3001), (200_003, 5_000)])
def test_noalloc_backward_matches_allocating_backward(sizes):
    from paper_2505_04612_amd import api
    ctx = api.default_context()
    rng = np.random.default_rng(3)
    w = _weights(ctx, rng)
    for M in sizes:
        feats = torch.from_numpy(rng.normal(0.0, 1.0, size=(M, 3)).astype(np.float32)).to(ctx.device)
        dout = torch.from_numpy(rng.normal(0.0, 1.0, size=M).astype(np.float32)).to(ctx.device)
        _, act = api.mlp_forward(ctx, w, feats, keep_act=True)
        ref = _call(ctx, "fm_mlp_backward", w, feats, act, dout)
        got = _call(ctx, "fm_mlp_backward_noalloc", w, feats, act, dout)
        for k in ref:
            if M <= 8192:
                assert torch.equal(got[k], ref[k]), (M, k)
            else:
                scale = float(ref[k].abs().max())
                assert float((got[k] - ref[k]).abs().max()) <= 1e-4 * scale, (M, k)
