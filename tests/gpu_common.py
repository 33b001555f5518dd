"""Shared helpers of the GPU tests: seeded cases and cached FP64 oracle results."""
import functools

import numpy as np
import torch

import oracle
import synth
from oracle.loss import content_features, loss_grad, style_grams


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


_records = {}


@functools.lru_cache(maxsize=None)
def oracle_loss(kind, H, W, Hs, Ws, sigma, w_style, alpha, bias=0.0):
    k = case(kind, H, W, Hs, Ws, sigma, bias)
    net = k["net"]
    ws = [w.astype(np.float64) for w in k["ws"]]
    bs = [b.astype(np.float64) for b in k["bs"]]
    g_t, f_c = oracle_targets(kind, H, W, Hs, Ws, sigma, bias)
    rec = {}
    terms, grad = loss_grad(net, k["x"].astype(np.float64), ws, bs, g_t, f_c, list(w_style), alpha, record=rec)
    _records[(kind, H, W, Hs, Ws, sigma, w_style, alpha, bias)] = rec
    return terms, grad


def flip_corrected(kind, H, W, Hs, Ws, sigma, w_style, alpha, g_test, bias=0.0, delta=1e-5):
    """Residual of g_test after removing the exact effects of flipped near-tie decisions
    (decisions whose FP64 margin is below delta x RMS); see oracle.flips."""
    from oracle.flips import flip_fit
    terms, g_ref = oracle_loss(kind, H, W, Hs, Ws, sigma, w_style, alpha, bias)
    rec = _records[(kind, H, W, Hs, Ws, sigma, w_style, alpha, bias)]
    k = case(kind, H, W, Hs, Ws, sigma, bias)
    ws = [w.astype(np.float64) for w in k["ws"]]
    bs = [b.astype(np.float64) for b in k["bs"]]
    r, flipped, _ = flip_fit(k["net"], k["x"].astype(np.float64), ws, bs, rec, g_ref, g_test, delta=delta)
    return float(np.linalg.norm(r) / np.linalg.norm(g_ref)), flipped


def flat_grams(gs):
    return np.concatenate([g.ravel() for g in gs])


def fc_hwc(f_c):
    return np.ascontiguousarray(np.transpose(f_c, (1, 2, 0)))
