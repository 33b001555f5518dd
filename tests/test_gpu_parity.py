"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

FP32 bars (relative, Frobenius / 2-norm): Grams <= 1e-5 per layer, energies <= 1e-5,
gradient <= 1e-4, checked for the full energy and separately for the style-only
(alpha = 0) and content-only (w = 0) energies, since the content term dominates both E
and its gradient at alpha = 1.

The gradient is piecewise smooth: FP32 rounding of the forward pass can resolve a
ReLU or max-pool decision that sits within ~1e-6 of its boundary the other way, which
moves the gradient by that decision's full contribution on its receptive field.  No
FP32 implementation avoids this on large images.  Where the raw FP32 gradient misses
the bar, the test removes the exact FP64 effects of flipping decisions whose margin is
below 1e-5 x RMS (oracle.flips, pinned on the CPU) and applies the bar to what
remains; the raw error and the flips used are printed.

BF16 end-to-end results are compared with two references on the same inputs:

* the FP64 oracle: the error is stated; it is the error of BF16 storage itself, which
  the BF16-storage reference (oracle/bf16ref.py, FP64 arithmetic rounded to BF16 where a
  BF16 evaluation stores a value) shows on its own.  Activation rounding (~2e-3) flips
  max-pool and ReLU decisions all over the image, which moves the image gradient by
  ~0.2-0.4 in norm.  The bar is that the GPU is no further from FP64 than that
  reference is (x 1.25 + 0.02); Grams and energies within 2e-2 / 3e-2;
* the BF16-storage reference: Grams, energies and gradient within the spread that FP32
  accumulation alone produces between two BF16-storage evaluations
  (tests/test_oracle_bf16.py: Grams 2e-3, energies 5e-4, gradient 0.2 on the full net).

Each kernel is held to tight bars on identical inputs in tests/test_gpu_layers.py.
"""

import numpy as np
import pytest
import torch

from gpu_common import (bf16ref_loss, case, cuda, fc_hwc, flat_grams, flip_corrected, oracle_loss,
                        oracle_style_means, oracle_targets, rel, to_np)

pytestmark = pytest.mark.gpu

TINY = ("tiny", 64, 64, 64, 64, 4.0)           # 64x64 images, tiny net, single tile
RAGGED = ("full", 200, 328, 176, 208, 8.0)     # full net, 3 x 4 tiles of 96 with ragged tails
W5 = (0.2, 0.2, 0.2, 0.2, 0.2)
W3 = (1 / 3, 1 / 3, 1 / 3)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.synchronize()


_ctx = {}


def ctx(kind, prec, bias=0.0):
    from paper_2212_13459_amd import Context
    key = (kind, prec, bias)
    if key not in _ctx:
        k = case(kind, 8, 8, 8, 8, 1.0, bias)
        _ctx[key] = Context(k["ws"], k["bs"], prec, tiny=(kind == "tiny"))
    return _ctx[key]


def run_gpu(spec, prec, T, m, w_style, alpha, bias=0.0, oracle_inputs=True, flags=3, msw=None):
    kind, H, W, Hs, Ws, sigma = spec
    k = case(kind, H, W, Hs, Ws, sigma, bias)
    nst = ctx(kind, prec, bias)
    ms = None
    if oracle_inputs:
        g_t, f_c = oracle_targets(kind, H, W, Hs, Ws, sigma, bias)
        gt_d = cuda(flat_grams(g_t), torch.float64)
        fc_d = cuda(fc_hwc(f_c))
        if msw is not None:
            from paper_2212_13459_amd import MeanStdTerms
            ms = MeanStdTerms(msw[0], msw[1], cuda(np.concatenate(oracle_style_means(*spec, bias)), torch.float64))
    else:
        gt_d = nst.style_grams(cuda(k["s"]), T, m)
        fc_d = nst.content_feats(cuda(k["c"]), T, m)
    energy, gx, grad = nst.loss_grad(cuda(k["x"]), gt_d, fc_d, w_style, alpha, T, m, flags=flags, ms=ms)
    torch.cuda.synchronize()
    means = None if ms is None else nst.split_means(ms.means_x)
    return energy, nst.split_grams(gx), grad, means


def compare(spec, prec, T, m, w_style, alpha, gram_tol, grad_tol, e_tol, bias=0.0, label="", msw=None):
    kind, H, W, Hs, Ws, sigma = spec
    terms, ograd = oracle_loss(kind, H, W, Hs, Ws, sigma, tuple(w_style), alpha, bias, msw)
    energy, grams, grad, means = run_gpu(spec, prec, T, m, w_style, alpha, bias, msw=msw)
    gerr = [rel(to_np(g), go) for g, go in zip(grams, terms["grams"])]
    if means is not None:
        gerr += [rel(to_np(a), b) for a, b in zip(means, terms["means"])]
    derr = rel(to_np(grad), ograd)
    eerr = [abs(energy[0] - terms["E"]) / abs(terms["E"])]
    if alpha != 0:
        eerr.append(abs(energy[1] - terms["E_content"]) / abs(terms["E_content"]))
    for a, b in zip(energy[2:], terms["E_style"]):
        if b != 0:
            eerr.append(abs(a - b) / abs(b))
    print(f"[{label} {prec} {spec} T={T} m={m} alpha={alpha} w={w_style}] gram rel {['%.2e' % e for e in gerr]}"
          f" grad rel {derr:.2e} energy rel {['%.2e' % e for e in eerr]}", flush=True)
    if prec == "bf16":
        bterms, bgrad = bf16ref_loss(kind, H, W, Hs, Ws, sigma, tuple(w_style), alpha, bias, msw)
        ref_err = rel(bgrad, ograd)
        bg = [rel(to_np(g), go) for g, go in zip(grams, bterms["grams"])]
        be = [abs(energy[0] - bterms["E"]) / abs(bterms["E"])]
        bd = rel(to_np(grad), bgrad)
        print(f"    BF16-storage reference vs FP64 grad {ref_err:.2e}; GPU vs that reference: gram "
              f"{['%.1e' % e for e in bg]} energy {be[0]:.1e} grad {bd:.2e}", flush=True)
        gram_spread, e_spread, grad_spread = (1e-4, 2e-4, 3e-2) if kind == "tiny" else (2e-3, 5e-4, 0.2)
        assert max(bg) <= gram_spread and be[0] <= e_spread and bd <= grad_spread, (bg, be, bd)
        grad_tol = 1.25 * ref_err + 0.02
    assert max(gerr) <= gram_tol, gerr
    assert max(eerr) <= e_tol, eerr
    if derr > grad_tol and prec == "fp32":
        resid, flips = flip_corrected(kind, H, W, Hs, Ws, sigma, tuple(w_style), alpha, to_np(grad), bias,
                                      msw=msw)
        print(f"    flip-corrected grad rel {resid:.2e} after {len(flips)} near-tie flips, margins/rms "
              f"{['%.1e' % f[0] for f in flips[:12]]} kinds {sorted(set((f[1], f[2]) for f in flips))}", flush=True)
        derr = resid
    assert derr <= grad_tol, derr
    return gerr, derr, eerr


# ------------------------------------------------------------------ FP32 bars ------

@pytest.mark.parametrize("alpha,w", [(1.0, W3), (0.0, W3), (1.0, (0.0, 0.0, 0.0))])
def test_tiny_single_tile_fp32(alpha, w):
    compare(TINY, "fp32", 64, 23, w, alpha, 1e-5, 1e-4, 1e-5, label="C0")


def test_tiny_with_bias_and_tiles_fp32():
    compare(TINY, "fp32", 24, 23, W3, 1.0, 1e-5, 1e-4, 1e-5, bias=0.05, label="C0-bias-tiled")


@pytest.mark.parametrize("alpha,w", [(1.0, W5), (0.0, W5), (1.0, (0.0,) * 5)])
def test_full_ragged_tiles_fp32(alpha, w):
    compare(RAGGED, "fp32", 96, 155, w, alpha, 1e-5, 1e-4, 1e-5, label="ragged")


# ------------------------------------------------------------------------ BF16 ----

@pytest.mark.parametrize("alpha,w", [(1.0, W3), (0.0, W3)])
def test_tiny_bf16(alpha, w):
    compare(TINY, "bf16", 64, 23, w, alpha, 2e-2, None, 3e-2, label="C0")


@pytest.mark.parametrize("alpha,w", [(1.0, W5), (0.0, W5)])
def test_full_ragged_bf16(alpha, w):
    compare(RAGGED, "bf16", 96, 155, w, alpha, 2e-2, None, 3e-2, label="ragged")


# -------------------------------------------------- augmented style loss (Eq. 5) ----

MSW5 = ((0.5, 1.0, 2.0, 4.0, 8.0), (2.0, 4.0, 8.0, 16.0, 32.0))


@pytest.mark.parametrize("alpha", [1.0, 0.0])
def test_full_ragged_mean_std_fp32(alpha):
    compare(RAGGED, "fp32", 96, 155, W5, alpha, 1e-5, 1e-4, 1e-5, label="ragged-ms", msw=MSW5)


def test_full_ragged_mean_std_bf16():
    compare(RAGGED, "bf16", 96, 155, W5, 1.0, 2e-2, None, 3e-2, label="ragged-ms", msw=MSW5)


def test_style_stats_means():
    """nst_style_stats: the Grams equal nst_style_grams bit for bit, the channel means
    match the FP64 oracle (FP32 path)."""
    kind, H, W, Hs, Ws, sigma = RAGGED
    k = case(*RAGGED)
    nst = ctx(kind, "fp32")
    g1 = nst.style_grams(cuda(k["s"]), 64, 155)
    g2, mu = nst.style_stats(cuda(k["s"]), 64, 155)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)
    err = [rel(to_np(a), b) for a, b in zip(nst.split_means(mu), oracle_style_means(*RAGGED))]
    print(f"[style means fp32] rel {['%.1e' % e for e in err]}", flush=True)
    assert max(err) <= 1e-6


# --------------------------------------------------------- targets and features ----

@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 5e-2)])
def test_style_grams_and_content_feats(prec, tol):
    kind, H, W, Hs, Ws, sigma = RAGGED
    k = case(*RAGGED)
    g_t, f_c = oracle_targets(*RAGGED)
    nst = ctx(kind, prec)
    g = nst.split_grams(nst.style_grams(cuda(k["s"]), 64, 155))
    f = nst.content_feats(cuda(k["c"]), 80, 155)
    torch.cuda.synchronize()
    gerr = [rel(to_np(a), b) for a, b in zip(g, g_t)]
    ferr = rel(to_np(f), fc_hwc(f_c))
    print(f"[targets {prec}] style gram rel {['%.2e' % e for e in gerr]} content feat rel {ferr:.2e}", flush=True)
    assert max(gerr) <= tol and ferr <= tol
    for a in g:   # the mirrored reduction makes every Gram exactly symmetric
        assert torch.equal(a, a.T)


# ------------------------------------------------------- tiling invariants (GPU) ---

@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_owned_features_bit_identical_tiled_vs_whole(prec):
    kind, H, W = "full", 200, 328
    k = case(*RAGGED)
    nst = ctx(kind, prec)
    x = cuda(k["x"])
    for conv in (0, 4, 9, 12):
        a = nst.layer_feats(x, 96, 155, conv)
        b = nst.layer_feats(x, 4096, 155, conv)
        assert torch.equal(a, b), conv


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_step2_with_fixed_grams_bit_identical_tiled_vs_whole(prec):
    kind, H, W, Hs, Ws, sigma = RAGGED
    k = case(*RAGGED)
    nst = ctx(kind, prec)
    g_t, f_c = oracle_targets(*RAGGED)
    gt_d = cuda(flat_grams(g_t), torch.float64)
    fc_d = cuda(fc_hwc(f_c))
    x = cuda(k["x"])
    _, gx, _ = nst.loss_grad(x, gt_d, fc_d, W5, 1.0, 4096, 155, flags=1)
    fixed = gx * 1.01
    _, _, g_whole = nst.loss_grad(x, gt_d, fc_d, W5, 1.0, 4096, 155, flags=2, grams_x=fixed.clone())
    _, _, g_tiled = nst.loss_grad(x, gt_d, fc_d, W5, 1.0, 96, 155, flags=2, grams_x=fixed.clone())
    torch.cuda.synchronize()
    assert torch.equal(g_whole, g_tiled)


def test_tiled_grams_match_whole_and_halo_too_small_shows_seams():
    k = case(*RAGGED)
    nst = ctx("full", "fp32")
    g_t, f_c = oracle_targets(*RAGGED)
    gt_d = cuda(flat_grams(g_t), torch.float64)
    fc_d = cuda(fc_hwc(f_c))
    x = cuda(k["x"])
    _, gw, dw = nst.loss_grad(x, gt_d, fc_d, W5, 1.0, 4096, 155)
    gw, dw = gw.clone(), dw.clone()
    _, gt, dt = nst.loss_grad(x, gt_d, fc_d, W5, 1.0, 96, 155)
    assert rel(to_np(gt), to_np(gw)) < 2e-6
    assert rel(to_np(dt), to_np(dw)) < 2e-6
    _, g0, d0 = nst.loss_grad(x, gt_d, fc_d, W5, 1.0, 96, 0)
    err0 = rel(to_np(d0), to_np(dw))
    print(f"[seams] zero-margin gradient rel err {err0:.3e}", flush=True)
    assert err0 > 1e-2


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_deterministic(prec):
    k = case(*RAGGED)
    nst = ctx("full", prec)
    g_t, f_c = oracle_targets(*RAGGED)
    gt_d = cuda(flat_grams(g_t), torch.float64)
    fc_d = cuda(fc_hwc(f_c))
    x = cuda(k["x"])
    e1, g1, d1 = nst.loss_grad(x, gt_d, fc_d, W5, 1.0, 96, 155)
    g1, d1 = g1.clone(), d1.clone()
    e2, g2, d2 = nst.loss_grad(x, gt_d, fc_d, W5, 1.0, 96, 155)
    assert e1 == e2 and torch.equal(g1, g2) and torch.equal(d1, d2)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_step2_reuse_equals_recompute(prec):
    """Step 2 recomputing each tile batch's forward (Algorithm 1, the default, here with
    two tile slots) and Step 2 on the activations Step 1 left resident (NST_RESIDENT, a
    slot per tile) give bit-identical energies, Grams of x and gradients (12 tiles)."""
    from paper_2212_13459_amd import Context, plan
    k = case(*RAGGED)
    recompute = Context(k["ws"], k["bs"], prec, tile_batch=2)
    resident = Context(k["ws"], k["bs"], prec, resident=True)
    assert len(plan(resident.desc, k["H"], k["W"], 96, 155)) == 12
    g_t, f_c = oracle_targets(*RAGGED)
    gt_d = cuda(flat_grams(g_t), torch.float64)
    fc_d = cuda(fc_hwc(f_c))
    x = cuda(k["x"])
    e1, g1, d1 = resident.loss_grad(x, gt_d, fc_d, W5, 1.0, 96, 155)
    g1, d1 = g1.clone(), d1.clone()
    e2, g2, d2 = recompute.loss_grad(x, gt_d, fc_d, W5, 1.0, 96, 155)
    torch.cuda.synchronize()
    assert resident.workspace(k["H"], k["W"], 96, 155).numel() > recompute.workspace(k["H"], k["W"], 96, 155).numel()
    assert e1 == e2 and torch.equal(g1, g2) and torch.equal(d1, d2)


def test_resident_needs_the_every_tile_workspace():
    """NST_RESIDENT with a workspace that holds only a tile batch is refused."""
    import ctypes
    from ctypes import c_void_p

    from paper_2212_13459_amd import NST_RESIDENT, workspace_bytes
    from paper_2212_13459_amd._lib import lib
    from paper_2212_13459_amd.nst import _ptr
    k = case(*RAGGED)
    nst = ctx("full", "fp32")
    g_t, f_c = oracle_targets(*RAGGED)
    gt_d = cuda(flat_grams(g_t), torch.float64)
    fc_d = cuda(fc_hwc(f_c))
    x = cuda(k["x"])
    nb = workspace_bytes(nst.desc, "fp32", 200, 328, 96, 155, 2)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    w = (ctypes.c_double * 5)(*W5)
    gx, grad = torch.empty_like(gt_d), torch.empty_like(x)
    st = lib().nst_loss_grad(nst._h, _ptr(x), 200, 328, _ptr(gt_d), _ptr(fc_d), w, 1.0, 96, 155, 3 | NST_RESIDENT,
                             _ptr(gx), None, _ptr(grad), _ptr(ws), nb, c_void_p())
    assert st == -7
    st = lib().nst_loss_grad(nst._h, _ptr(x), 200, 328, _ptr(gt_d), _ptr(fc_d), w, 1.0, 96, 155, 3,
                             _ptr(gx), None, _ptr(grad), _ptr(ws), nb, c_void_p())
    assert st == 0


@pytest.mark.parametrize("where", ["x", "content", "grams", "weight"])
def test_check_finite(where):
    """NST_CHECK_FINITE refuses a NaN or infinity in any input with NST_ENONFINITE and
    leaves the outputs untouched; without the flag the same finite call succeeds."""
    from paper_2212_13459_amd import NST_CHECK_FINITE
    from paper_2212_13459_amd._lib import NstError
    k = case(*RAGGED)
    nst = ctx("full", "fp32")
    g_t, f_c = oracle_targets(*RAGGED)
    gt_d = cuda(flat_grams(g_t), torch.float64)
    fc_d = cuda(fc_hwc(f_c))
    x = cuda(k["x"])
    e, _, _ = nst.loss_grad(x, gt_d, fc_d, W5, 1.0, 96, 155, flags=3 | NST_CHECK_FINITE)
    assert np.isfinite(e[0])
    w = list(W5)
    if where == "x":
        x[1, 7, 11] = float("nan")
    elif where == "content":
        fc_d[3, 2, 5] = float("inf")
    elif where == "grams":
        gt_d[100] = float("-inf")
    else:
        w[2] = float("nan")
    gx = torch.full_like(gt_d, 7.0)
    grad = torch.full_like(x, 7.0)
    with pytest.raises(NstError) as ei:
        nst.loss_grad(x, gt_d, fc_d, w, 1.0, 96, 155, flags=3 | NST_CHECK_FINITE, grams_x=gx, grad=grad)
    assert ei.value.status == -8
    torch.cuda.synchronize()
    assert bool((gx == 7.0).all()) and bool((grad == 7.0).all())


def test_zero_energy_when_x_c_s_coincide_fp32():
    k = case(*RAGGED)
    nst = ctx("full", "fp32")
    c = cuda(k["c"])
    gt = nst.style_grams(c, 96, 155)
    fc = nst.content_feats(c, 96, 155)
    e, _, d = nst.loss_grad(c, gt, fc, W5, 1.0, 96, 155)
    assert e[0] == 0.0 and e[1] == 0.0
    assert torch.count_nonzero(d).item() == 0


def test_error_paths_on_device():
    from paper_2212_13459_amd._lib import NstError
    k = case(*RAGGED)
    nst = ctx("full", "fp32")
    g_t, f_c = oracle_targets(*RAGGED)
    gt_d = cuda(flat_grams(g_t), torch.float64)
    fc_d = cuda(fc_hwc(f_c))
    x = cuda(k["x"])
    with pytest.raises(NstError) as ei:
        nst.loss_grad(x, gt_d, fc_d, W5, 1.0, 96, 100, flags=3 | 4)
    assert ei.value.status == -3
    with pytest.raises(NstError) as ei:
        nst.loss_grad(x, gt_d, None, W5, 1.0, 96, 155)
    assert ei.value.status == -1
    # workspace too small
    from ctypes import c_void_p
    from paper_2212_13459_amd._lib import lib
    from paper_2212_13459_amd.nst import _ptr
    gx = torch.empty_like(gt_d)
    tiny_ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    import ctypes
    w = (ctypes.c_double * 5)(*W5)
    st = lib().nst_loss_grad(nst._h, _ptr(x), 200, 328, _ptr(gt_d), _ptr(fc_d), w, 1.0, 96, 155, 3, _ptr(gx),
                             None, _ptr(torch.empty_like(x)), _ptr(tiny_ws), 1024, c_void_p())
    assert st == -7
