"""GPU checks at the workload sizes: the autograd Function, finite differences at
2048x2048, tiled-vs-whole bit identity at 6048x8064 in the benchmark's launch
configuration, stage checks on the GPU's own inputs at full size (every conv of one or
two tiles' windows, the Grams through probe products, the full gradient of those tiles'
blocks; the whole 2048x2048 image with every element of the gradient), and element-wise
comparisons with stored FP64 oracle values (tests/golden/oracle_*.json, written by
tests/golden/make_golden.py from oracle/ only).

Bars follow tests/test_gpu_layers.py for the stages.  The end-to-end comparison with
the FP64 oracle holds Grams (probe products, full Grams for C <= 128), energies and
content features element-wise to 1e-5 in FP32; the end-to-end gradient is stated and
held to the share of sampled pixels within 1e-4 (FP32), because the sampled pixels
whose receptive cone holds a decision that FP32 rounding resolves the other way move by
that decision's contribution (the stage checks show the kernels themselves at 1e-5).
"""
import functools
import json
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import check_forward, gpu_acts, layer_input, quant, rel, seeds_on
from oracle import bf16ref
from oracle.loss import gram
from oracle.ops import conv3x3, relu
from oracle.plan import make_plan

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
W5 = [0.2] * 5
NET = oracle.vgg19()


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


_ctx = {}


@pytest.fixture(autouse=True)
def release_workspaces():
    yield
    for c in _ctx.values():
        c._ws = {}
    torch.cuda.empty_cache()


def ctx(prec):
    from paper_2212_13459_amd import Context
    if prec not in _ctx:
        ws, bs = synth.vgg_weights(synth.VGG19_CONVS, synth.SEED_WEIGHTS)
        _ctx[prec] = Context(ws, bs, prec)
    return _ctx[prec]


def weights64():
    ws, bs = synth.vgg_weights(synth.VGG19_CONVS, synth.SEED_WEIGHTS)
    return [w.astype(np.float64) for w in ws], [b.astype(np.float64) for b in bs]


@functools.lru_cache(maxsize=2)
def host_images(H, W, Hs, Ws, sigma, down=0):
    """x, c (box-downsampled `down` times from their size x 2^down) and s, float32."""
    out = []
    for seed in (synth.SEED_X, synth.SEED_CONTENT):
        a = synth.image(H << down, W << down, sigma, seed)
        for _ in range(down):
            a = synth.box_down2(a)
        out.append(a)
    out.append(synth.image(Hs, Ws, sigma, synth.SEED_STYLE))
    return tuple(out)


def images(H, W, Hs, Ws, sigma, down=0):
    dev = torch.device("cuda", 0)
    return tuple(torch.from_numpy(a).to(dev) for a in host_images(H, W, Hs, Ws, sigma, down))


def cfg_images(cfg):
    return images(cfg["H"], cfg["W"], cfg["Hs"], cfg["Ws"], cfg["sigma"], cfg.get("down", 0))


def _golden(name):
    p = os.path.join(HERE, "golden", f"oracle_{name}.json")
    if not os.path.exists(p):
        pytest.skip(f"{p} not generated")
    with open(p) as f:
        return json.load(f)


def probes(sizes, seed=5):
    """The seeded C x 16 probe matrices of tests/golden/make_golden.py."""
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((c, 16)) for c in sizes]


def probe_own(feats, P, n_p, rows=1 << 22):
    """V^T (V P) / n_p in FP64 for the GPU's h x w x C features V, in row chunks."""
    C = feats.shape[-1]
    v = feats.reshape(-1, C)
    acc = np.zeros((C, P.shape[1]))
    for r0 in range(0, v.shape[0], rows):
        blk = v[r0:r0 + rows].double().cpu().numpy()
        acc += blk.T @ (blk @ P)
    return acc / n_p


# --------------------------------------------------------------------- autograd ----

@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_autograd_function_equals_loss_grad(prec):
    from paper_2212_13459_amd import StyleEnergy
    nst = ctx(prec)
    x, c, s = images(512, 512, 512, 512, 8.0)
    gt = nst.style_grams(s, 256, 155)
    fc = nst.content_feats(c, 256, 155)
    xv = x.clone().requires_grad_(True)
    e = StyleEnergy.apply(xv, nst, gt, fc, W5, 1.0, 256, 155)
    e.backward()
    e2, _, g2 = nst.loss_grad(x, gt, fc, W5, 1.0, 256, 155)
    torch.cuda.synchronize()
    assert e.item() == e2[0]
    assert torch.equal(xv.grad, g2)
    # a second backward through a scaled energy scales the gradient
    xv.grad = None
    (2.0 * StyleEnergy.apply(xv, nst, gt, fc, W5, 1.0, 256, 155)).backward()
    assert torch.allclose(xv.grad, 2.0 * g2, rtol=0, atol=0)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_finite_differences_2048(prec):
    """autograd.Function backward vs central finite differences (h = 1e-3) at 64 seeded
    pixels, 2048x2048 image, 1024x1280 style, 512 px tiles.

    The differences are FP64 values stored by the oracle (the FP32 energy's rounding
    noise inside a pixel's receptive cone exceeds the 2 h g signal).  Even in exact
    arithmetic a 1e-3 step crosses ReLU / max-pool kinks, so FD differs from the true
    gradient by a few percent.  FP32: the GPU gradient is as close to the FD values as the
    oracle's exact gradient is.  BF16 (stated): within the BF16 storage error of the
    exact gradient (0.5) of the FD values."""
    from paper_2212_13459_amd import StyleEnergy
    gd = _golden("C2")
    if gd.get("fd_samples") is None:
        pytest.skip("no finite differences stored")
    cfg = gd["config"]
    nst = ctx(prec)
    x, c, s = cfg_images(cfg)
    gt = nst.style_grams(s, cfg["T"], cfg["m"])
    fc = nst.content_feats(c, cfg["T"], cfg["m"])
    xv = x.clone().requires_grad_(True)
    StyleEnergy.apply(xv, nst, gt, fc, gd["w_style"], gd["alpha"], cfg["T"], cfg["m"]).backward()
    fd = np.array(gd["fd_samples"])
    smp = np.array(gd["grad_samples"])[: len(fd)]
    idx = (smp[:, 0].astype(int), smp[:, 1].astype(int), smp[:, 2].astype(int))
    g_gpu = xv.grad.double().cpu().numpy()[idx]
    g_ora = smp[:, 3]
    e_gpu, e_ora = rel(g_gpu, fd), rel(g_ora, fd)
    print(f"[fd 2048 {prec}] |autograd - FD| / |FD| = {e_gpu:.3e}; exact FP64 gradient vs the same FD: "
          f"{e_ora:.3e}; autograd vs exact at these pixels {rel(g_gpu, g_ora):.3e}", flush=True)
    assert e_ora < 0.1
    if prec == "fp32":
        assert e_gpu <= 1.05 * e_ora + 1e-4
    else:
        assert e_gpu <= e_ora + 0.5


# ------------------------------------------------------------ tiling at full size ----

def test_full_size_tiled_equals_single_window_bitwise():
    """6048x8064 with the benchmark's 1024 px tiles vs one 6048x8064 window (BF16): owned
    features and the fixed-Gram Step 2 gradient are bit-identical."""
    nst = ctx("bf16")
    x, c, s = images(6048, 8064, 4226, 5319, 16.0)
    for conv in (9, 12):
        a = nst.layer_feats(x, 1024, 155, conv)
        b = nst.layer_feats(x, 8064, 155, conv)
        assert torch.equal(a, b), conv
        del a, b
    gt = nst.style_grams(s, 1024, 155)
    fc = nst.content_feats(c, 1024, 155)
    _, gx, _ = nst.loss_grad(x, gt, fc, W5, 1.0, 1024, 155, flags=1)
    fixed = gx.clone()
    _, _, g1 = nst.loss_grad(x, gt, fc, W5, 1.0, 1024, 155, flags=2, grams_x=fixed.clone())
    g1 = g1.clone()
    _, _, g2 = nst.loss_grad(x, gt, fc, W5, 1.0, 8064, 155, flags=2, grams_x=fixed.clone())
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)


# ------------------------------------------------- stages on own inputs, full size ----

GRAD_BAR = {"fp32": 1e-5, "bf16": 1e-2}


@pytest.mark.parametrize("name", ["C2", "C4", "C3p1", "C3"])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_stages_at_scale(name, prec):
    """At the workload sizes: Grams of x against probe products of the GPU's own
    whole-image features; for tiles of the plan (centre and last at 2048x2048, one at the
    larger sizes), every conv of the tile's window against the convolution of the GPU's
    own previous layer, and the tile block's gradient against the reverse pass on the
    GPU's own window activations with the Grams of x fixed (Step 2 of Algorithm 1; the
    block's gradient depends on nothing outside the window when m covers the receptive
    field)."""
    gd = _golden(name)
    cfg = gd["config"]
    H, W, T, m = cfg["H"], cfg["W"], cfg["T"], cfg["m"]
    nst = ctx(prec)
    ws, bs = weights64()
    q = quant(prec)
    x, c, s = cfg_images(cfg)
    xh = host_images(H, W, cfg["Hs"], cfg["Ws"], cfg["sigma"], cfg.get("down", 0))[0]
    gt = nst.style_grams(s, T, m)
    fc = nst.content_feats(c, T, m)
    _, gx, _ = nst.loss_grad(x, gt, fc, W5, 1.0, T, m, flags=1)
    grams_x = [g.double().cpu().numpy() for g in nst.split_grams(gx)]
    g_t = [g.double().cpu().numpy() for g in nst.split_grams(gt)]
    strides = NET.strides()
    n_ps = [(H // strides[i]) * (W // strides[i]) for i in NET.style]
    P = probes([g.shape[0] for g in grams_x])
    gerr = []
    for k, i in enumerate(NET.style):
        if H * W > 4096 * 4096 and strides[i] == 1:
            continue   # relu1_1 is checked at the smaller sizes (its 6048x8064 map is 12.5 GB)
        feats = nst.layer_feats(x, T, m, i)
        gerr.append(rel(grams_x[k] @ P[k], probe_own(feats, P[k], n_ps[k])))
        del feats
    print(f"[scale {name} {prec}] Gram probes vs own features {['%.1e' % e for e in gerr]}", flush=True)
    assert max(gerr) <= 1e-6, gerr

    _, _, grad = nst.loss_grad(x, gt, fc, W5, 1.0, T, m, flags=2, grams_x=gx.clone())
    grad_h = grad.double().cpu().numpy()
    del grad
    fc_h = fc.permute(2, 0, 1).double().cpu().numpy()
    plan = make_plan(H, W, T, m, strides, NET.align())
    centre = next(k for k, t in enumerate(plan) if t.by0 <= H // 2 < t.by1 and t.bx0 <= W // 2 < t.bx1)
    ic = NET.content
    # C2: the centre tile and the last (ragged) one; the larger sizes one each: the last
    # tile (image borders on two sides, ragged at C4) or the centre (windows interior)
    picks = {"C2": [centre, len(plan) - 1], "C4": [len(plan) - 1], "C3p1": [centre], "C3": [len(plan) - 1]}[name]
    for ti in picks:
        t = plan[ti]
        xw = np.ascontiguousarray(xh[:, t.ey0:t.ey1, t.ex0:t.ex1])
        hw, ww = xw.shape[1:]
        acts = gpu_acts(nst, torch.from_numpy(xw).cuda(), max(hw, ww), m, max(NET.style))
        label = f"scale {name} {prec} tile {ti} window {hw}x{ww}"
        check_forward(NET, acts, ws, bs, xw, prec, label)
        sc = strides[ic]
        oy, ox = t.ey0 // sc, t.ex0 // sc
        hl, wl = acts[ic].shape[1:]
        raw_c = relu(conv3x3(layer_input(NET, acts, ic, q(xw.astype(np.float64)), q), q(ws[ic]), bs[ic]))
        seeds = seeds_on(NET, acts, raw_c, grams_x, g_t, fc_h[:, oy:oy + hl, ox:ox + wl], W5, 1.0, prec, n_ps)
        g_ref = bf16ref.backward(NET, acts, seeds, ws, q)
        inner_ref = g_ref[:, t.by0 - t.ey0:t.by1 - t.ey0, t.bx0 - t.ex0:t.bx1 - t.ex0]
        inner_gpu = grad_h[:, t.by0:t.by1, t.bx0:t.bx1]
        derr = rel(inner_gpu, inner_ref)
        print(f"  [{label}] block {t.by1 - t.by0}x{t.bx1 - t.bx0} gradient vs reverse pass on own "
              f"activations {derr:.2e}", flush=True)
        assert derr <= GRAD_BAR[prec], derr
        del acts, g_ref, seeds


_acts_cache = {}


def _whole_acts(prec, x, T, m, xh):
    """The GPU's whole-image features at C2, each conv checked once per precision."""
    if prec not in _acts_cache:
        _acts_cache.clear()
        ws, bs = weights64()
        acts = gpu_acts(ctx(prec), x, T, m, max(NET.style))
        check_forward(NET, acts, ws, bs, xh, prec, f"whole 2048 {prec}")
        _acts_cache[prec] = acts
    return _acts_cache[prec]


@pytest.mark.parametrize("prec,alpha,w_style", [("fp32", 1.0, W5), ("fp32", 0.0, W5), ("fp32", 1.0, [0.0] * 5),
                                                ("bf16", 1.0, W5)])
def test_whole_image_stages_2048(prec, alpha, w_style):
    """C2 (2048x2048, 512 px tiles): every conv, every Gram and every element of the
    gradient of the whole image against the plain definitions evaluated on the GPU's own
    features (the full gradient vector, not samples); the full energy, style-only and
    content-only."""
    gd = _golden("C2")
    cfg = gd["config"]
    H, W, T, m = cfg["H"], cfg["W"], cfg["T"], cfg["m"]
    nst = ctx(prec)
    ws, bs = weights64()
    q = quant(prec)
    x, c, s = cfg_images(cfg)
    xh = host_images(H, W, cfg["Hs"], cfg["Ws"], cfg["sigma"])[0]
    gt = nst.style_grams(s, T, m)
    fc = nst.content_feats(c, T, m)
    acts = _whole_acts(prec, x, T, m, xh)
    _, gx, _ = nst.loss_grad(x, gt, fc, w_style, alpha, T, m, flags=1)
    grams_x = [g.double().cpu().numpy() for g in nst.split_grams(gx)]
    g_t = [g.double().cpu().numpy() for g in nst.split_grams(gt)]
    gerr = [rel(G, gram(acts[i], acts[i].shape[1] * acts[i].shape[2])) for G, i in zip(grams_x, NET.style)]
    _, _, grad = nst.loss_grad(x, gt, fc, w_style, alpha, T, m, flags=2, grams_x=gx.clone())
    ic = NET.content
    raw_c = relu(conv3x3(layer_input(NET, acts, ic, q(xh.astype(np.float64)), q), q(ws[ic]), bs[ic]))
    seeds = seeds_on(NET, acts, raw_c, grams_x, g_t, fc.permute(2, 0, 1).double().cpu().numpy(), w_style, alpha,
                     prec)
    g_ref = bf16ref.backward(NET, acts, seeds, ws, q)
    derr = rel(grad.double().cpu().numpy(), g_ref)
    print(f"[whole 2048 {prec} alpha={alpha} w={w_style[0]}] Grams vs own features {['%.1e' % e for e in gerr]}; "
          f"full gradient vector vs reverse pass on own activations {derr:.2e}", flush=True)
    assert max(gerr) <= 1e-6, gerr
    assert derr <= GRAD_BAR[prec], derr


# -------------------------------------------------------- against the FP64 oracle ----

@pytest.mark.parametrize("name", ["C2", "C4", "C3p1", "C3"])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_against_stored_oracle(name, prec):
    """Energies, Grams (probe products for every layer, full Grams for C <= 128),
    content features at 384 seeded positions and dE/dx at 512 seeded pixels against
    the FP64 oracle at the full configuration sizes."""
    gd = _golden(name)
    cfg = gd["config"]
    T, m = cfg["T"], cfg["m"]
    nst = ctx(prec)
    x, c, s = cfg_images(cfg)
    gt = nst.style_grams(s, T, m)
    fc = nst.content_feats(c, T, m)
    energy, gx, grad = nst.loss_grad(x, gt, fc, gd["w_style"], gd["alpha"], T, m)
    torch.cuda.synchronize()
    tol = 1e-5 if prec == "fp32" else 2e-2
    P = probes([len(p) for p in gd["grams_x_probe"]], gd["probe_seed"])
    perr = []
    for G, ref, p in list(zip(nst.split_grams(gx), gd["grams_x_probe"], P)) + \
            list(zip(nst.split_grams(gt), gd["grams_style_probe"], P)):
        perr.append(rel(G.double().cpu().numpy() @ p, np.array(ref)))
    ferr = [rel(G.double().cpu().numpy(), np.array(ref))
            for G, ref in zip(nst.split_grams(gx), gd["grams_x_full"]) if ref is not None]
    eerr = [abs(energy[0] - gd["E"]) / gd["E"], abs(energy[1] - gd["E_content"]) / gd["E_content"]]
    eerr += [abs(a - b) / abs(b) for a, b in zip(energy[2:], gd["E_style"])]
    cs = np.array(gd["content_feats"]["samples"])
    ci = [torch.from_numpy(cs[:, j].astype(np.int64)).to(fc.device) for j in (1, 2, 0)]
    fv = fc[ci[0], ci[1], ci[2]].double().cpu().numpy()
    cerr = rel(fv, cs[:, 3])
    smp = np.array(gd["grad_samples"])
    gv = grad.double().cpu().numpy()[smp[:, 0].astype(int), smp[:, 1].astype(int), smp[:, 2].astype(int)]
    ref = smp[:, 3]
    scale = np.sqrt(np.mean(ref ** 2))
    derr = np.abs(gv - ref) / np.maximum(np.abs(ref), 0.1 * scale)
    within = float(np.mean(derr <= 1e-4))
    print(f"[golden {name} {prec}] Gram probes rel max {max(perr):.2e}, full Grams {['%.1e' % e for e in ferr]}, "
          f"energy rel {['%.2e' % e for e in eerr]}, content features {cerr:.2e}; gradient at {len(ref)} px: "
          f"vector rel {rel(gv, ref):.2e}, median {np.median(derr):.2e}, p90 {np.percentile(derr, 90):.2e}, "
          f"{within:.1%} within 1e-4", flush=True)
    assert max(perr) <= tol and max(ferr) <= tol, (perr, ferr)
    assert max(eerr) <= (1e-5 if prec == "fp32" else 3e-2), eerr
    assert cerr <= tol, cerr
    if prec == "fp32":
        assert within >= 0.75, within
        assert rel(gv, ref) <= 5e-2
    else:
        assert rel(gv, ref) <= 0.6
