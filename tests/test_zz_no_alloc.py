"""The allocation-free entry point nst_loss_grad_noalloc (device scratch held by the
library) against nst_loss_grad (caller workspace) through the C ABI: two calls in a row
on one context, the second on a smaller image, each bit-identical to nst_loss_grad (the
tile batch differs, and results do not depend on it); a size whose smallest tile batch
exceeds the scratch is refused before any launch."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from gpu_common import cuda, rel

pytestmark = pytest.mark.gpu

W5 = [0.2] * 5


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def noalloc(nst, x, gt, fc, alpha, T, m, flags=3, grams_x=None):
    from paper_2212_13459_amd._lib import check, lib
    from paper_2212_13459_amd.nst import _ptr, _stream
    H, W = x.shape[1:]
    gx = torch.full_like(gt, 7.0) if grams_x is None else grams_x
    grad = torch.full_like(x, 7.0)
    en = (ctypes.c_double * (2 + len(W5)))()
    wst = (ctypes.c_double * len(W5))(*W5)
    check("nst_loss_grad_noalloc", lib().nst_loss_grad_noalloc(
        nst._h, _ptr(x), H, W, _ptr(gt), _ptr(fc), wst, alpha, T, m, flags, _ptr(gx), en, _ptr(grad),
        _stream(x.device)))
    torch.cuda.synchronize()
    return list(en), gx, grad


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_noalloc_equals_loss_grad_two_calls(prec):
    from paper_2212_13459_amd import Context
    from paper_2212_13459_amd._lib import lib
    assert lib().nst_scratch_bytes() == 256 << 20
    ws, bs = synth.vgg_weights(synth.VGG19_CONVS, synth.SEED_WEIGHTS)
    nst = Context(ws, bs, prec)
    for (H, W, Hs, Ws, T) in ((200, 328, 176, 208, 96), (136, 152, 120, 120, 64)):
        x = cuda(synth.image(H, W, 8.0, synth.SEED_X))
        c = cuda(synth.image(H, W, 8.0, synth.SEED_CONTENT))
        s = cuda(synth.image(Hs, Ws, 8.0, synth.SEED_STYLE))
        gt = nst.style_grams(s, T, 155)
        fc = nst.content_feats(c, T, 155)
        e1, g1, d1 = nst.loss_grad(x, gt, fc, W5, 1.0, T, 155)
        g1, d1 = g1.clone(), d1.clone()
        e2, g2, d2 = noalloc(nst, x, gt, fc, 1.0, T, 155)
        print(f"[noalloc {prec} {H}x{W} T={T}] energy {e2[0]:.6e} vs {e1[0]:.6e}, grad rel {rel(d2.cpu(), d1.cpu()):.1e}",
              flush=True)
        assert e1 == e2
        assert torch.equal(g1, g2) and torch.equal(d1, d2)
        # Step 2 alone from the Grams of Step 1
        _, _, d3 = noalloc(nst, x, gt, fc, 1.0, T, 155, flags=2, grams_x=g2.clone())
        assert torch.equal(d3, d1)
    nst.close()


def test_noalloc_refuses_sizes_beyond_the_scratch():
    from paper_2212_13459_amd import Context, vgg19_desc, workspace_bytes
    from paper_2212_13459_amd._lib import NstError
    H, W, T = 2048, 2048, 1024
    assert workspace_bytes(vgg19_desc(), "bf16", H, W, T, 155, 1) > 256 << 20
    ws, bs = synth.vgg_weights(synth.VGG19_CONVS, synth.SEED_WEIGHTS)
    nst = Context(ws, bs, "bf16")
    x = torch.zeros((3, H, W), dtype=torch.float32, device="cuda")
    gt = torch.zeros(sum(c * c for c in nst.gram_sizes()), dtype=torch.float64, device="cuda")
    fc = torch.zeros((H // 8, W // 8, 512), dtype=torch.float32, device="cuda")
    with pytest.raises(NstError) as ei:
        noalloc(nst, x, gt, fc, 1.0, T, 155)
    assert ei.value.status == -7
    nst.close()
