"""Shared helpers of the GPU tests: seeded cases and cached FP64 oracle results."""
import functools

import numpy as np
import torch

import oracle
import synth
from oracle import bf16ref
from oracle.loss import MeanStd, content_features, loss_grad, style_grams, style_stats
from oracle.ops import avgpool2, conv3x3, maxpool2, relu


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_np(t):
    return t.detach().double().cpu().numpy()


def cuda(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@functools.lru_cache(maxsize=None)
def case(kind, H, W, Hs, Ws, sigma, bias=0.0):
    net = oracle.vgg19_tiny() if kind == "tiny" else oracle.vgg19()
    ws, bs = synth.vgg_weights(net.convs, seed=synth.SEED_WEIGHTS, bias_std=bias)
    c = synth.image(H, W, sigma, synth.SEED_CONTENT)
    s = synth.image(Hs, Ws, sigma, synth.SEED_STYLE)
    x = synth.image(H, W, sigma, synth.SEED_X)
    return dict(net=net, ws=ws, bs=bs, c=c, s=s, x=x, H=H, W=W)


@functools.lru_cache(maxsize=None)
def oracle_targets(kind, H, W, Hs, Ws, sigma, bias=0.0):
    k = case(kind, H, W, Hs, Ws, sigma, bias)
    net = k["net"]
    ws = [w.astype(np.float64) for w in k["ws"]]
    bs = [b.astype(np.float64) for b in k["bs"]]
    g_t = style_grams(net, k["s"].astype(np.float64), ws, bs)
    f_c = content_features(net, k["c"].astype(np.float64), ws, bs)
    return g_t, f_c


@functools.lru_cache(maxsize=None)
def oracle_style_means(kind, H, W, Hs, Ws, sigma, bias=0.0):
    """Channel means of the style image's style layers (FP64 oracle)."""
    k = case(kind, H, W, Hs, Ws, sigma, bias)
    ws = [w.astype(np.float64) for w in k["ws"]]
    bs = [b.astype(np.float64) for b in k["bs"]]
    return style_stats(k["net"], k["s"].astype(np.float64), ws, bs)[1]


def mean_std(spec, msw, bias=0.0):
    """oracle.loss.MeanStd for weights msw = (w_mean tuple, w_std tuple), or None."""
    if msw is None:
        return None
    return MeanStd(msw[0], msw[1], oracle_style_means(*spec, bias))


_records = {}


@functools.lru_cache(maxsize=None)
def oracle_loss(kind, H, W, Hs, Ws, sigma, w_style, alpha, bias=0.0, msw=None):
    k = case(kind, H, W, Hs, Ws, sigma, bias)
    net = k["net"]
    ws = [w.astype(np.float64) for w in k["ws"]]
    bs = [b.astype(np.float64) for b in k["bs"]]
    g_t, f_c = oracle_targets(kind, H, W, Hs, Ws, sigma, bias)
    rec = {}
    terms, grad = loss_grad(net, k["x"].astype(np.float64), ws, bs, g_t, f_c, list(w_style), alpha, record=rec,
                            ms=mean_std((kind, H, W, Hs, Ws, sigma), msw, bias))
    _records[(kind, H, W, Hs, Ws, sigma, w_style, alpha, bias, msw)] = rec
    return terms, grad


@functools.lru_cache(maxsize=None)
def bf16ref_loss(kind, H, W, Hs, Ws, sigma, w_style, alpha, bias=0.0, msw=None):
    """The BF16-storage reference (oracle/bf16ref.py) on the oracle's FP64 targets."""
    from oracle import bf16ref
    k = case(kind, H, W, Hs, Ws, sigma, bias)
    ws = [w.astype(np.float64) for w in k["ws"]]
    bs = [b.astype(np.float64) for b in k["bs"]]
    g_t, f_c = oracle_targets(kind, H, W, Hs, Ws, sigma, bias)
    f_c32 = f_c.astype(np.float32).astype(np.float64)
    return bf16ref.loss_grad(k["net"], k["x"].astype(np.float64), ws, bs, g_t, f_c32, list(w_style), alpha,
                             ms=mean_std((kind, H, W, Hs, Ws, sigma), msw, bias))


def flip_corrected(kind, H, W, Hs, Ws, sigma, w_style, alpha, g_test, bias=0.0, delta=1e-5, msw=None):
    """Residual of g_test after removing the exact effects of flipped near-tie decisions
    (decisions whose FP64 margin is below delta x RMS); see oracle.flips."""
    from oracle.flips import flip_fit
    terms, g_ref = oracle_loss(kind, H, W, Hs, Ws, sigma, w_style, alpha, bias, msw)
    rec = _records[(kind, H, W, Hs, Ws, sigma, w_style, alpha, bias, msw)]
    k = case(kind, H, W, Hs, Ws, sigma, bias)
    ws = [w.astype(np.float64) for w in k["ws"]]
    bs = [b.astype(np.float64) for b in k["bs"]]
    r, flipped, _ = flip_fit(k["net"], k["x"].astype(np.float64), ws, bs, rec, g_ref, g_test, delta=delta)
    return float(np.linalg.norm(r) / np.linalg.norm(g_ref)), flipped


def flat_grams(gs):
    return np.concatenate([g.ravel() for g in gs])


def fc_hwc(f_c):
    return np.ascontiguousarray(np.transpose(f_c, (1, 2, 0)))


# ------------------------------------------ stage checks on the GPU's own inputs ----

def quant(prec):
    return bf16ref.round_bf16 if prec == "bf16" else bf16ref.identity


def gpu_acts(nst, x_d, T, m, top):
    """The GPU's stored post-ReLU features of conv 0..top, whole image, C x h x w FP64."""
    out = []
    for i in range(top + 1):
        f = nst.layer_feats(x_d, T, m, i)
        out.append(np.ascontiguousarray(f.permute(2, 0, 1).double().cpu().numpy()))
    return out


def layer_input(net, acts, i, x0, q=bf16ref.identity):
    """Input of conv i built from the GPU's stored features: the image, the previous
    layer, or its pool (an average pool's mean is stored rounded, like the kernels do)."""
    if i == 0:
        return x0
    if (i - 1) not in net.pool_after:
        return acts[i - 1]
    return q(avgpool2(acts[i - 1])) if net.avg_pool else maxpool2(acts[i - 1])


def bf16_units_apart(a, b):
    """Distance in BF16 units of non-negative BF16-exact values (bit patterns are monotone)."""
    ia = (a.astype(np.float32).view(np.int32) >> 16).astype(np.int64)
    ib = (b.astype(np.float32).view(np.int32) >> 16).astype(np.int64)
    return np.abs(ia - ib)


def check_forward(net, acts, ws, bs, x, prec, label):
    q = quant(prec)
    x0 = q(np.asarray(x, np.float64))
    worst = []
    for i in range(len(acts)):
        ref = q(relu(conv3x3(layer_input(net, acts, i, x0, q), q(ws[i]), bs[i])))
        a = acts[i]
        assert a.shape == ref.shape, (i, a.shape, ref.shape)
        rms = float(np.sqrt(np.mean(ref * ref))) or 1.0
        if prec == "fp32":
            e = float(np.abs(a - ref).max()) / rms
            f = float(np.linalg.norm(a - ref) / max(np.linalg.norm(ref), 1e-300))
            print(f"  [{label} fwd fp32] conv {i}: rel {f:.2e}, max|A-A*|/rms {e:.2e}", flush=True)
            worst.append(e)
            assert f <= 1e-5 and e <= 1e-4, (i, f, e)
        else:
            units = bf16_units_apart(a, ref)
            # a ReLU input within accumulation rounding of 0 may give a tiny positive value
            # on one side and 0 on the other: adjacent in value though not in BF16 units
            near0 = np.abs(a - ref) <= 1e-5 * rms
            far = int(np.count_nonzero((units > 1) & ~near0))
            frac = float(np.count_nonzero(a != ref)) / a.size
            print(f"  [{label} fwd bf16] conv {i}: {frac:.2e} of elements one BF16 unit off, "
                  f"{far} further", flush=True)
            worst.append(frac)
            assert far == 0, (i, far)
            assert frac <= 1e-3, (i, frac)
    return worst


def seeds_on(net, acts, raw_c, grams_x, g_t, f_c, w_style, alpha, prec, n_ps=None, ms=None):
    """Table 1 seeds on the given activations: style (2 w / n_p)(D + D^T) stored in the
    compute precision (with ms, an oracle.loss.MeanStd holding the means of x, plus
    diag(r) and the per-channel constant b of the mean and std rows, as
    oracle/bf16ref.py writes them), content 2 alpha (V - F_c) from the unrounded content
    value.  n_ps: whole-image feature counts per style layer (default: those of ``acts``)."""
    q = quant(prec)
    seeds = {}
    for k, i in enumerate(net.style):
        c, h, w = acts[i].shape
        n_p = h * w if n_ps is None else n_ps[k]
        d = grams_x[k] - g_t[k]
        dt = (2.0 * w_style[k] / n_p) * (d + d.T)
        b = None
        if ms is not None:
            r, b = bf16ref.ms_operands(grams_x[k], g_t[k], ms.means_x[k], ms.means_t[k], ms.w_mean[k],
                                       ms.w_std[k], n_p)
            dt = dt + np.diag(r)
        dt = q(dt)
        seeds[i] = (dt @ acts[i].reshape(c, -1)).reshape(acts[i].shape)
        if b is not None:
            seeds[i] = seeds[i] + b[:, None, None]
    if net.content is not None and alpha != 0.0:
        seeds[net.content] = seeds.get(net.content, 0.0) + 2.0 * alpha * (raw_c - f_c)
    return seeds
