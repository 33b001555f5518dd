"""Pins of the augmented style loss in the FP64 oracle (Sec. 3.2 Eq. 5, Table 1 rows
3-4, the std line of Algorithm 1 Step 1).

* std from the Gram diagonal and the mean equals the direct population std;
* the mean and std seeds equal central differences of the mean and std losses on the
  features alone (Table 1 checked by finite differences on V);
* the whole augmented energy and its image gradient equal torch CPU float64 autograd of
  an independent torch model (torch.mean / torch.std, not the oracle's formulas);
* tiled (Algorithm 1, means added block by block) equals whole-image;
* a constant (dead) channel gets a zero std seed instead of 0/0;
* planted mistakes (std seed without centring, mean seed with a wrong factor) are
  caught by the torch cross-check.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
import synth
from oracle.loss import (MeanStd, channel_mean, gram, loss_grad, mean_seed, std_from_stats, std_seed,
                         style_stats)
from oracle.net import vgg19, vgg19_tiny
from oracle.tiled import tiled_loss_grad, tiled_style_stats

torch.set_num_threads(4)


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_std_from_gram_and_mean_is_population_std():
    rng = np.random.default_rng(40)
    v = np.abs(rng.standard_normal((7, 13, 11))) * rng.uniform(0.5, 2.0, (7, 1, 1))
    n_p = 13 * 11
    g = gram(v, n_p)
    mean = channel_mean(v, n_p)
    assert rel(mean, v.reshape(7, -1).mean(axis=1)) < 1e-15
    assert rel(std_from_stats(g, mean), v.reshape(7, -1).std(axis=1)) < 1e-12


def test_table1_mean_and_std_rows_by_fd_on_features():
    rng = np.random.default_rng(41)
    cc, n_p = 5, 17
    v = np.abs(rng.standard_normal((cc, n_p, 1))) + 0.1
    mu_t = rng.uniform(0.2, 1.0, cc)
    sd_t = rng.uniform(0.2, 1.0, cc)
    w1, w2 = 0.7, 1.3

    def e_mean(vv):
        return w1 * np.sum((vv.reshape(cc, -1).mean(axis=1) - mu_t) ** 2)

    def e_std(vv):
        return w2 * np.sum((vv.reshape(cc, -1).std(axis=1) - sd_t) ** 2)

    mean = channel_mean(v, n_p)
    std = std_from_stats(gram(v, n_p), mean)
    s_mean = mean_seed(v.shape, mean, mu_t, w1, n_p)
    s_std = std_seed(v, mean, std, sd_t, w2, n_p)
    # the printed rows, written out: (2/n_p)(mean - mu) and (2/n_p)(V - mean)(std - sigma)/std
    assert rel(s_mean, (2 * w1 / n_p) * np.broadcast_to((mean - mu_t)[:, None, None], v.shape)) < 1e-15
    for idx in [(0, 3, 0), (2, 16, 0), (4, 0, 0), (1, 8, 0)]:
        for fun, sd in ((e_mean, s_mean), (e_std, s_std)):
            h = 1e-6
            vp, vm = v.copy(), v.copy()
            vp[idx] += h
            vm[idx] -= h
            fd = (fun(vp) - fun(vm)) / (2 * h)
            assert abs(fd - sd[idx]) <= 1e-8 * max(1.0, abs(fd)), (idx, fd, sd[idx])


def test_dead_channel_has_zero_std_seed():
    rng = np.random.default_rng(42)
    v = np.abs(rng.standard_normal((3, 6, 5)))
    v[1] = 0.0
    n_p = 30
    mean = channel_mean(v, n_p)
    std = std_from_stats(gram(v, n_p), mean)
    assert std[1] == 0.0
    s = std_seed(v, mean, std, np.full(3, 0.5), 1.0, n_p)
    assert np.all(np.isfinite(s)) and np.all(s[1] == 0.0) and np.any(s[0] != 0.0)


def torch_ms_energy(net, x, ws, bs, grams_t, means_t, f_c, w_style, w_mean, w_std, alpha):
    """Eq. 1-3 with the augmented style loss of Eq. 5, in torch (an independent model)."""
    a = x
    acts = {}
    top = max(list(net.style) + ([net.content] if net.content is not None else []))
    for i in range(top + 1):
        a = F.relu(F.conv2d(a, ws[i], bs[i], padding=1))
        acts[i] = a
        if i in net.pool_after:
            a = F.max_pool2d(a, 2, 2)
    e = torch.zeros((), dtype=torch.float64)
    for k, i in enumerate(net.style):
        v = acts[i][0].reshape(acts[i].shape[1], -1)
        g = v @ v.T / v.shape[1]
        e = e + w_style[k] * torch.sum((g - grams_t[k]) ** 2)
        e = e + w_mean[k] * torch.sum((v.mean(dim=1) - means_t[k]) ** 2)
        sd_t = torch.sqrt(torch.diagonal(grams_t[k]) - means_t[k] ** 2)
        e = e + w_std[k] * torch.sum((v.std(dim=1, unbiased=False) - sd_t) ** 2)
    if net.content is not None and alpha != 0.0:
        e = e + alpha * torch.sum((acts[net.content][0] - f_c) ** 2)
    return e


def _case(net, h, w, bias=0.0):
    ws, bs = synth.vgg_weights(net.convs, seed=0, bias_std=bias)
    ws = [a.astype(np.float64) for a in ws]
    bs = [a.astype(np.float64) for a in bs]
    c = synth.image(h, w, 4, 1).astype(np.float64)
    s = synth.image(h + 4, w - 4, 4, 2).astype(np.float64)
    x = synth.image(h, w, 4, 3).astype(np.float64)
    g_t, mu_t = style_stats(net, s, ws, bs)
    f_c = oracle.content_features(net, c, ws, bs)
    return ws, bs, x, g_t, mu_t, f_c


def _torch_check(net, ws, bs, x, g_t, mu_t, f_c, w_style, w_mean, w_std, alpha):
    tx = torch.from_numpy(x)[None].requires_grad_(True)
    e = torch_ms_energy(net, tx, [torch.from_numpy(v) for v in ws], [torch.from_numpy(v) for v in bs],
                        [torch.from_numpy(v) for v in g_t], [torch.from_numpy(v) for v in mu_t],
                        torch.from_numpy(f_c), w_style, w_mean, w_std, alpha)
    e.backward()
    return e.item(), tx.grad[0].numpy()


@pytest.mark.parametrize("kind", ["tiny", "full"])
def test_augmented_loss_matches_torch_autograd(kind):
    net = vgg19_tiny() if kind == "tiny" else vgg19()
    h, w = (24, 28) if kind == "tiny" else (36, 52)
    ws, bs, x, g_t, mu_t, f_c = _case(net, h, w, bias=0.03)
    ns = len(net.style)
    w_style = [0.5 / ns] * ns
    w_mean, w_std = [2.0 / ns] * ns, [3.0 / ns] * ns
    ms = MeanStd(w_mean, w_std, mu_t)
    terms, grad = loss_grad(net, x, ws, bs, g_t, f_c, w_style, 0.6, ms=ms)
    e_ref, g_ref = _torch_check(net, ws, bs, x, g_t, mu_t, f_c, w_style, w_mean, w_std, 0.6)
    assert abs(terms["E"] - e_ref) <= 1e-12 * abs(e_ref)
    assert rel(grad, g_ref) < 1e-11
    assert min(terms["E_mean"]) > 0 and min(terms["E_std"]) > 0
    # with zero mean/std weights the augmented loss is the plain one
    t0, g0 = loss_grad(net, x, ws, bs, g_t, f_c, w_style, 0.6)
    t1, g1 = loss_grad(net, x, ws, bs, g_t, f_c, w_style, 0.6, ms=MeanStd([0.0] * ns, [0.0] * ns, mu_t))
    assert t0["E"] == t1["E"] and np.array_equal(g0, g1)


@pytest.mark.parametrize("kind,h,w,t,m", [("tiny", 70, 58, 16, 23),
                                          pytest.param("full", 352, 48, 112, 155, marks=pytest.mark.slow)])
def test_tiled_equals_whole_with_mean_std(kind, h, w, t, m):
    net = vgg19_tiny() if kind == "tiny" else vgg19()
    ws, bs, x, g_t, mu_t, f_c = _case(net, h, w)
    ns = len(net.style)
    ms = MeanStd([1.0] * ns, [2.0] * ns, mu_t)
    whole, gw = loss_grad(net, x, ws, bs, g_t, f_c, [1.0 / ns] * ns, 1.0, ms=ms)
    tiled, gt = tiled_loss_grad(net, x, ws, bs, g_t, f_c, [1.0 / ns] * ns, 1.0, t, m, ms=ms)
    for a, b in zip(tiled["means"], whole["means"]):
        assert rel(a, b) < 1e-13
    assert abs(tiled["E"] - whole["E"]) <= 1e-12 * whole["E"]
    assert rel(gt, gw) < 1e-12
    s = synth.image(h + 4, w - 4, 4, 2).astype(np.float64)
    gs, ms_ = tiled_style_stats(net, s, ws, bs, t, m)
    for a, b in zip(ms_, mu_t):
        assert rel(a, b) < 1e-13


def test_pins_catch_planted_mean_std_mistakes(monkeypatch):
    """An uncentred std seed, or a mean seed with 1/n_p in place of 2/n_p, fails the
    torch cross-check."""
    import oracle.loss as L
    net = vgg19_tiny()
    ws, bs, x, g_t, mu_t, f_c = _case(net, 24, 28)
    w3 = [1 / 3.0] * 3
    ms = MeanStd([1.0] * 3, [1.0] * 3, mu_t)
    _, g_ref = _torch_check(net, ws, bs, x, g_t, mu_t, f_c, w3, [1.0] * 3, [1.0] * 3, 0.0)
    _, good = L.loss_grad(net, x, ws, bs, g_t, f_c, w3, 0.0, ms=ms)
    assert rel(good, g_ref) < 1e-11
    good_std, good_mean = L.std_seed, L.mean_seed

    def uncentred(v, mean, std, std_t, w2, n_p):
        return good_std(v, np.zeros_like(mean), std, std_t, w2, n_p)

    monkeypatch.setattr(L, "std_seed", uncentred)
    _, bad = L.loss_grad(net, x, ws, bs, g_t, f_c, w3, 0.0, ms=ms)
    assert rel(bad, g_ref) > 1e-3
    monkeypatch.setattr(L, "std_seed", good_std)
    monkeypatch.setattr(L, "mean_seed", lambda shape, mean, mt, w1, n_p: good_mean(shape, mean, mt, w1 / 2, n_p))
    _, bad = L.loss_grad(net, x, ws, bs, g_t, f_c, w3, 0.0, ms=ms)
    assert rel(bad, g_ref) > 1e-4


def test_bf16_reference_with_mean_std_and_rounding_off_is_the_oracle():
    """The BF16-storage reference writes the mean and std rows as V diag(r) + b; with
    rounding off that is the oracle's value up to FP64 regrouping."""
    from oracle import bf16ref
    for kind, (h, w) in (("tiny", (24, 28)), ("full", (36, 52))):
        net = vgg19_tiny() if kind == "tiny" else vgg19()
        ws, bs, x, g_t, mu_t, f_c = _case(net, h, w, bias=0.02)
        ns = len(net.style)
        ms = MeanStd([1.5] * ns, [2.5] * ns, mu_t)
        t0, g0 = loss_grad(net, x, ws, bs, g_t, f_c, [1.0 / ns] * ns, 0.8, ms=ms)
        t1, g1 = bf16ref.loss_grad(net, x, ws, bs, g_t, f_c, [1.0 / ns] * ns, 0.8, q=bf16ref.identity, ms=ms)
        assert abs(t0["E"] - t1["E"]) <= 1e-14 * t0["E"]
        assert rel(g1, g0) < 1e-12
        _, g2 = bf16ref.loss_grad(net, x, ws, bs, g_t, f_c, [1.0 / ns] * ns, 0.8, ms=ms)
        assert rel(g2, g0) > 1e-4
