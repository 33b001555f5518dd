"""Pins of the FP64 oracle against definitions, brute force, closed forms,
invariants and an independent library routine (torch CPU float64 autograd).

Each check is chosen so that a plausible slip in the oracle (a dropped term, a
sign, a transposed operand, a wrong index or stride) fails at least one of them.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
from oracle import naive, ops
from oracle.loss import backward, forward, gram, loss_grad, style_seed, content_seed
from oracle.net import receptive_fields, min_halo, vgg19, vgg19_tiny
from oracle.plan import make_plan
from oracle.tiled import tiled_loss_grad, tiled_style_grams, tiled_content_features
import synth

torch.set_num_threads(4)


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


# ---------------------------------------------------------------- ops ------

def test_conv_matches_loops():
    rng = np.random.default_rng(10)
    a = rng.standard_normal((3, 5, 6))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    assert rel(ops.conv3x3(a, w, b), naive.conv3x3_loops(a, w, b)) < 1e-13


def test_conv_matches_torch():
    rng = np.random.default_rng(11)
    a = rng.standard_normal((16, 13, 17))
    w = rng.standard_normal((8, 16, 3, 3))
    b = rng.standard_normal(8)
    ref = F.conv2d(torch.from_numpy(a)[None], torch.from_numpy(w), torch.from_numpy(b), padding=1)[0].numpy()
    assert rel(ops.conv3x3(a, w, b), ref) < 1e-13


def test_conv_adjoint_identity():
    rng = np.random.default_rng(12)
    u = rng.standard_normal((5, 9, 11))
    w = rng.standard_normal((7, 5, 3, 3))
    v = rng.standard_normal((7, 9, 11))
    lhs = np.sum(ops.conv3x3(u, w) * v)
    rhs = np.sum(u * ops.conv3x3_adjoint(v, w))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("hw", [(6, 8), (7, 9), (5, 4)])
def test_pool_matches_loops_and_torch(hw):
    rng = np.random.default_rng(13)
    a = rng.standard_normal((3,) + hw)
    out, arg = naive.maxpool2_loops(a)
    assert np.array_equal(ops.maxpool2(a), out)
    t = torch.from_numpy(a)[None].requires_grad_(True)
    y = F.max_pool2d(t, 2, 2)
    assert np.array_equal(y[0].detach().numpy(), out)
    dy = rng.standard_normal(out.shape)
    y.backward(torch.from_numpy(dy)[None])
    assert np.array_equal(ops.maxpool2_backward(dy, a), t.grad[0].numpy())
    # floor mode: dropped last row / col get exactly zero gradient
    da = ops.maxpool2_backward(dy, a)
    if hw[0] % 2:
        assert np.all(da[:, -1, :] == 0)
    if hw[1] % 2:
        assert np.all(da[:, :, -1] == 0)


def test_pool_tie_goes_to_first_in_window_order():
    a = np.zeros((1, 2, 2))
    a[0, 0, 1] = a[0, 1, 0] = 1.0          # tie between (0,1) and (1,0)
    da = ops.maxpool2_backward(np.ones((1, 1, 1)), a)
    assert da[0, 0, 1] == 1.0 and da[0, 1, 0] == 0.0


def test_gram_matches_loops():
    rng = np.random.default_rng(14)
    v = np.abs(rng.standard_normal((4, 3, 5)))
    assert rel(gram(v, 15), naive.gram_loops(v, 15)) < 1e-14


# --------------------------------------------------------- geometry --------

def test_receptive_field_closed_form():
    rf = receptive_fields(vgg19())
    assert rf == [(1, 1), (2, 2), (4, 5), (6, 7), (10, 13), (14, 17), (18, 21), (22, 25),
                  (30, 37), (38, 45), (46, 53), (54, 61), (70, 85)]
    assert min_halo(vgg19()) == 155
    assert min_halo(vgg19_tiny()) == 23
    assert vgg19().strides() == [1, 1, 2, 2, 4, 4, 4, 4, 8, 8, 8, 8, 16]
    assert vgg19().align() == 16 and vgg19_tiny().align() == 4


def test_receptive_field_brute_force_tiny():
    """Perturb one input row and record which feature rows change: with positive
    input and positive weights every ReLU is active, so the change pattern is
    exactly the dependency cone [s q - a, s q + b]."""
    net = vgg19_tiny()
    rng = np.random.default_rng(15)
    ws = [np.abs(rng.standard_normal((co, ci, 3, 3))) + 0.1 for ci, co in net.convs]
    bs = [np.zeros(co) for ci, co in net.convs]
    h, w = 48, 8
    x = np.abs(rng.standard_normal((3, h, w))) + 1.0
    base = forward(net, x, ws, bs)
    strides = net.strides()
    rf = receptive_fields(net)
    y0 = 21
    xp = x.copy()
    xp[:, y0, :] += 1.0
    pert = forward(net, xp, ws, bs)
    for i in range(net.n_conv):
        changed = np.nonzero(np.any(pert[i] != base[i], axis=(0, 2)))[0]
        s, (a, b) = strides[i], rf[i]
        expect = [q for q in range(base[i].shape[1]) if s * q - a <= y0 <= s * q + b]
        assert list(changed) == expect, (i, list(changed), expect)


# ------------------------------------------------------ torch cross-check --

def torch_energy(net, x, ws, bs, grams_t, f_c, w_style, alpha):
    a = x
    acts = {}
    for i in range(max(list(net.style) + [net.content])+ 1):
        a = F.relu(F.conv2d(a, ws[i], bs[i], padding=1))
        acts[i] = a
        if i in net.pool_after:
            a = F.max_pool2d(a, 2, 2)
    e = torch.zeros((), dtype=torch.float64)
    for k, i in enumerate(net.style):
        v = acts[i][0].reshape(acts[i].shape[1], -1).T
        g = v.T @ v / v.shape[0]
        e = e + w_style[k] * torch.sum((g - grams_t[k]) ** 2)
    e = e + alpha * torch.sum((acts[net.content][0] - f_c) ** 2)
    return e


def _tiny_case(h=24, w=28, bias=0.0):
    net = vgg19_tiny()
    ws, bs = synth.vgg_weights(net.convs, seed=0, bias_std=bias)
    ws = [wi.astype(np.float64) for wi in ws]
    bs = [bi.astype(np.float64) for bi in bs]
    c = synth.image(h, w, 4, 1).astype(np.float64)
    s = synth.image(h + 4, w - 4, 4, 2).astype(np.float64)
    x = synth.image(h, w, 4, 3).astype(np.float64)
    g_t = oracle.loss.style_grams(net, s, ws, bs)
    f_c = oracle.content_features(net, c, ws, bs)
    return net, ws, bs, c, s, x, g_t, f_c


@pytest.mark.parametrize("bias", [0.0, 0.05])
def test_loss_grad_matches_torch_autograd(bias):
    net, ws, bs, c, s, x, g_t, f_c = _tiny_case(bias=bias)
    w_style = [1 / 3.0, 0.5, 0.25]
    alpha = 0.7
    terms, grad = loss_grad(net, x, ws, bs, g_t, f_c, w_style, alpha)
    tx = torch.from_numpy(x)[None].requires_grad_(True)
    e = torch_energy(net, tx, [torch.from_numpy(v) for v in ws], [torch.from_numpy(v) for v in bs],
                     [torch.from_numpy(v) for v in g_t], torch.from_numpy(f_c), w_style, alpha)
    e.backward()
    assert abs(terms["E"] - e.item()) <= 1e-12 * abs(e.item())
    assert rel(grad, tx.grad[0].numpy()) < 1e-11


def test_loss_grad_full_net_matches_torch_autograd():
    net = vgg19()
    ws, bs = synth.vgg_weights(net.convs, seed=0)
    ws = [wi.astype(np.float64) for wi in ws]
    bs = [bi.astype(np.float64) for bi in bs]
    h, w = 36, 52
    c = synth.image(h, w, 4, 1).astype(np.float64)
    s = synth.image(40, 48, 4, 2).astype(np.float64)
    x = synth.image(h, w, 4, 3).astype(np.float64)
    g_t = oracle.loss.style_grams(net, s, ws, bs)
    f_c = oracle.content_features(net, c, ws, bs)
    w_style = [0.2] * 5
    terms, grad = loss_grad(net, x, ws, bs, g_t, f_c, w_style, 1.0)
    tx = torch.from_numpy(x)[None].requires_grad_(True)
    e = torch_energy(net, tx, [torch.from_numpy(v) for v in ws], [torch.from_numpy(v) for v in bs],
                     [torch.from_numpy(v) for v in g_t], torch.from_numpy(f_c), w_style, 1.0)
    e.backward()
    assert abs(terms["E"] - e.item()) <= 1e-12 * abs(e.item())
    assert rel(grad, tx.grad[0].numpy()) < 1e-11


def test_finite_differences_tiny():
    net, ws, bs, c, s, x, g_t, f_c = _tiny_case(h=16, w=20)
    w_style = [1 / 3.0] * 3
    for alpha in (1.0, 0.0):
        _, grad = loss_grad(net, x, ws, bs, g_t, f_c, w_style, alpha)
        rng = np.random.default_rng(4)
        # ReLU and max-pool kinks lie within +-1e-5 of some inputs; at h = 1e-6 the
        # central difference is smooth and its FP64 rounding error is ~E * 1e-16 / h.
        h = 1e-6
        for _ in range(6):
            ch, yy, xx = int(rng.integers(3)), int(rng.integers(16)), int(rng.integers(20))
            xp, xm = x.copy(), x.copy()
            xp[ch, yy, xx] += h
            xm[ch, yy, xx] -= h
            ep = loss_grad(net, xp, ws, bs, g_t, f_c, w_style, alpha, want_grad=False)[0]["E"]
            em = loss_grad(net, xm, ws, bs, g_t, f_c, w_style, alpha, want_grad=False)[0]["E"]
            fd = (ep - em) / (2 * h)
            assert abs(fd - grad[ch, yy, xx]) <= 3e-7 + 1e-7 * abs(fd), (alpha, fd, grad[ch, yy, xx])


def test_table1_gradients_by_fd_on_features():
    rng = np.random.default_rng(16)
    n_p, cc = 11, 4
    v = rng.standard_normal((cc, n_p, 1))
    g_ref = rng.standard_normal((cc, cc))
    g_ref = g_ref @ g_ref.T                           # symmetric target
    w_l = 0.3

    def e_gram(vv):
        return w_l * np.sum((gram(vv, n_p) - g_ref) ** 2)

    seed = style_seed(v, gram(v, n_p), g_ref, w_l, n_p)
    d = gram(v, n_p) - g_ref
    printed = (4.0 * w_l / n_p) * (d @ v.reshape(cc, -1)).reshape(v.shape)   # Table 1 form
    assert rel(seed, printed) < 1e-13
    f_ref = rng.standard_normal(v.shape)
    cseed = content_seed(v, f_ref, 0.9)
    for idx in [(0, 3, 0), (2, 7, 0), (3, 0, 0)]:
        for fun, sd in ((e_gram, seed), (lambda vv: 0.9 * np.sum((vv - f_ref) ** 2), cseed)):
            hh = 1e-5
            vp, vm = v.copy(), v.copy()
            vp[idx] += hh
            vm[idx] -= hh
            fd = (fun(vp) - fun(vm)) / (2 * hh)
            assert abs(fd - sd[idx]) <= 1e-8 * max(1.0, abs(fd))


# ------------------------------------------------------- invariants --------

def test_gram_properties():
    net, ws, bs, c, s, x, g_t, f_c = _tiny_case()
    acts = forward(net, x, ws, bs)
    for i in net.style:
        n_p = acts[i].shape[1] * acts[i].shape[2]
        g = gram(acts[i], n_p)
        assert np.array_equal(g, g.T)
        lam = np.linalg.eigvalsh(g)
        assert lam.min() >= -1e-12 * np.abs(lam).max()
        assert abs(np.trace(g) - np.sum(acts[i] ** 2) / n_p) <= 1e-12 * np.trace(g)


def test_gram_homogeneity_bit_exact():
    """Zero bias: every op commutes with scaling by 2, so G(2x) = 4 G(x) exactly."""
    net, ws, bs, c, s, x, g_t, f_c = _tiny_case()
    a1 = forward(net, x, ws, bs)
    a2 = forward(net, 2.0 * x, ws, bs)
    for i in net.style:
        n_p = a1[i].shape[1] * a1[i].shape[2]
        assert np.array_equal(gram(a2[i], n_p), 4.0 * gram(a1[i], n_p))


def test_zero_energy_at_identity():
    net, ws, bs, c, s, x, g_t, f_c = _tiny_case()
    g_c = oracle.loss.style_grams(net, c, ws, bs)
    terms, grad = loss_grad(net, c, ws, bs, g_c, f_c, [1 / 3.0] * 3, 1.0)
    assert terms["E"] == 0.0 and np.all(grad == 0.0)
    terms, grad = loss_grad(net, c, ws, bs, g_t, f_c, [1 / 3.0] * 3, 1.0)
    assert terms["E_content"] == 0.0 and terms["E"] > 0
    _, g_style = loss_grad(net, c, ws, bs, g_t, f_c, [1 / 3.0] * 3, 0.0)
    assert np.array_equal(grad, g_style)     # content gradient is exactly 0 at x = c


# ------------------------------------------------------------ plan ---------

@pytest.mark.parametrize("h,w,t,m", [(64, 64, 64, 23), (200, 328, 96, 155), (756, 1008, 1024, 155),
                                      (3024, 4032, 1000, 155), (37, 53, 8, 0), (17, 5, 4, 7)])
def test_plan_partitions(h, w, t, m):
    net = vgg19()
    strides = net.strides()
    tiles = make_plan(h, w, t, m, strides, 16)
    cover = np.zeros((h, w), np.int32)
    for tl in tiles:
        cover[tl.by0:tl.by1, tl.bx0:tl.bx1] += 1
        assert tl.ey0 % 16 == 0 and tl.ex0 % 16 == 0
        assert tl.ey1 == h or tl.ey1 % 16 == 0
        assert tl.ex1 == w or tl.ex1 % 16 == 0
        assert tl.ey0 <= max(0, tl.by0 - m) and tl.ey1 >= min(h, tl.by1 + m)
        assert tl.ex0 <= max(0, tl.bx0 - m) and tl.ex1 >= min(w, tl.bx1 + m)
    assert np.all(cover == 1)
    for i, s in enumerate(strides):
        nh, nw = h // s, w // s
        fc = np.zeros((nh, nw), np.int32)
        for tl in tiles:
            r0, r1, c0, c1 = tl.own[i]
            fc[r0:r1, c0:c1] += 1
            # owned features sit inside the window's feature extent at this layer
            if r1 > r0 and c1 > c0:
                assert tl.ey0 // s <= r0 and r1 <= tl.ey0 // s + (tl.ey1 - tl.ey0) // s
                assert tl.ex0 // s <= c0 and c1 <= tl.ex0 // s + (tl.ex1 - tl.ex0) // s
        assert np.all(fc == 1), i


def test_plan_ragged_counts():
    tiles = make_plan(3024, 4032, 1000, 155, vgg19().strides(), 16)
    assert len(tiles) == 4 * 5
    assert tiles[-1].by1 - tiles[-1].by0 == 24 and tiles[-1].bx1 - tiles[-1].bx0 == 32
    tiles = make_plan(6048, 8064, 1024, 155, vgg19().strides(), 16)
    assert len(tiles) == 6 * 8
    inner = [t for t in tiles if t.by0 > 0 and t.by1 < 6048 and t.bx0 > 0 and t.bx1 < 8064]
    assert all(t.ey1 - t.ey0 == 1344 and t.ex1 - t.ex0 == 1344 for t in inner)


# --------------------------------------------- tiled == whole (Alg. 1) -----

def _tiled_vs_whole(net, h, w, t, m, sigma=4):
    ws, bs = synth.vgg_weights(net.convs, seed=0)
    ws = [wi.astype(np.float64) for wi in ws]
    bs = [bi.astype(np.float64) for bi in bs]
    c = synth.image(h, w, sigma, 1).astype(np.float64)
    s = synth.image(h - 4, w + 8, sigma, 2).astype(np.float64)
    x = synth.image(h, w, sigma, 3).astype(np.float64)
    ns = len(net.style)
    w_style = [1.0 / ns] * ns
    g_t = oracle.loss.style_grams(net, s, ws, bs)
    f_c = oracle.content_features(net, c, ws, bs)
    whole, gw = loss_grad(net, x, ws, bs, g_t, f_c, w_style, 1.0)
    tiled, gt = tiled_loss_grad(net, x, ws, bs, g_t, f_c, w_style, 1.0, t, m)
    return whole, gw, tiled, gt, (ws, bs, c, s, x, g_t, f_c, w_style)


def test_tiled_equals_whole_tiny():
    net = vgg19_tiny()
    whole, gw, tiled, gt, (ws, bs, c, s, x, g_t, f_c, w_style) = _tiled_vs_whole(net, 70, 58, 16, 23)
    for a, b in zip(tiled["grams"], whole["grams"]):
        assert rel(a, b) < 1e-13
    assert abs(tiled["E"] - whole["E"]) <= 1e-12 * whole["E"]
    assert rel(gt, gw) < 1e-12
    # content features and style grams computed block by block
    assert rel(tiled_content_features(net, c, ws, bs, 16, 23), f_c) < 1e-14
    for a, b in zip(tiled_style_grams(net, s, ws, bs, 16, 23), g_t):
        assert rel(a, b) < 1e-13


def test_small_halo_shows_seams_tiny():
    net = vgg19_tiny()
    whole, gw, tiled0, g0, _ = _tiled_vs_whole(net, 70, 58, 16, 0)
    _, _, tiled1, g1, _ = _tiled_vs_whole(net, 70, 58, 16, 23 - 4)
    assert rel(g0, gw) > 1e-2
    assert rel(g1, gw) > 1e-8


@pytest.mark.slow
def test_tiled_equals_whole_full_net_ragged():
    net = vgg19()
    whole, gw, tiled, gt, _ = _tiled_vs_whole(net, 352, 48, 112, 155)
    for a, b in zip(tiled["grams"], whole["grams"]):
        assert rel(a, b) < 1e-13
    assert abs(tiled["E"] - whole["E"]) <= 1e-12 * whole["E"]
    assert rel(gt, gw) < 1e-12


def test_fixed_statistics_step2_is_local():
    """With the Grams fixed, Step 2 of a tiled run equals the whole-image
    backward seeded with the same Grams (Prop. 1)."""
    net = vgg19_tiny()
    whole, gw, tiled, gt, (ws, bs, c, s, x, g_t, f_c, w_style) = _tiled_vs_whole(net, 40, 44, 12, 23)
    fixed = [g * 1.01 for g in whole["grams"]]
    _, g_tiled = tiled_loss_grad(net, x, ws, bs, g_t, f_c, w_style, 1.0, 12, 23, grams_fixed=fixed)
    acts = forward(net, x, ws, bs)
    seeds = {}
    for k, i in enumerate(net.style):
        n_p = acts[i].shape[1] * acts[i].shape[2]
        seeds[i] = style_seed(acts[i], fixed[k], g_t[k], w_style[k], n_p)
    seeds[net.content] = seeds.get(net.content, 0) + content_seed(acts[net.content], f_c, 1.0)
    g_whole = backward(net, acts, seeds, ws)
    assert rel(g_tiled, g_whole) < 1e-12


# ---------------------------------------------- planted mistakes -----------

def test_pins_catch_a_dropped_transpose(monkeypatch):
    """Plant a mistake in the oracle (asymmetric-target Gram seed without the
    D^T term) and check the torch cross-check would fail."""
    import oracle.loss as L
    net, ws, bs, c, s, x, g_t, f_c = _tiny_case()
    rng = np.random.default_rng(5)
    g_t = [g + 0.1 * rng.standard_normal(g.shape) * np.abs(g).max() for g in g_t]   # asymmetric
    w_style = [1 / 3.0] * 3

    def wrong_seed(v, g, gt, w_l, n_p):
        cc = v.shape[0]
        return ((4.0 * w_l / n_p) * ((g - gt) @ v.reshape(cc, -1))).reshape(v.shape)

    tx = torch.from_numpy(x)[None].requires_grad_(True)
    e = torch_energy(net, tx, [torch.from_numpy(v) for v in ws], [torch.from_numpy(v) for v in bs],
                     [torch.from_numpy(v) for v in g_t], torch.from_numpy(f_c), w_style, 0.0)
    e.backward()
    _, good = L.loss_grad(net, x, ws, bs, g_t, f_c, w_style, 0.0)
    assert rel(good, tx.grad[0].numpy()) < 1e-11
    monkeypatch.setattr(L, "style_seed", wrong_seed)
    _, bad = L.loss_grad(net, x, ws, bs, g_t, f_c, w_style, 0.0)
    assert rel(bad, tx.grad[0].numpy()) > 1e-3


# ------------------------------------------- decision flips (FP32 comparisons) ----

def _recorded_case(h=40, w=44):
    net, ws, bs, c, s, x, g_t, f_c = _tiny_case(h, w)
    rec = {}
    w_style = [1 / 3.0] * 3
    terms, g = loss_grad(net, x, ws, bs, g_t, f_c, w_style, 1.0, record=rec)
    acts = [rec[("A", i)] for i in range(net.n_conv)]
    seeds = {}
    for k, i in enumerate(net.style):
        n_p = acts[i].shape[1] * acts[i].shape[2]
        seeds[i] = style_seed(acts[i], terms["grams"][k], g_t[k], w_style[k], n_p)
    seeds[net.content] = seeds[net.content] + content_seed(acts[net.content], f_c, 1.0) \
        if net.content in seeds else content_seed(acts[net.content], f_c, 1.0)
    return net, ws, bs, x, rec, acts, seeds, g


def test_relu_flip_effect_equals_full_backward_difference():
    from oracle.flips import flip_effect
    net, ws, bs, x, rec, acts, seeds, g = _recorded_case()
    i = 2                                          # conv2_1: not followed by a pool
    c, y, xx = map(int, np.argwhere(acts[i] == 0.0)[17])
    mod = [a.copy() for a in acts]
    mod[i][c, y, xx] = 1e-300                      # the mask now passes at this unit
    g_flip = backward(net, mod, seeds, ws)
    Y0, Y1, X0, X1, d = flip_effect(net, rec, ws, (0.0, "relu", i, c, y, xx), g.shape[1:])
    full = np.zeros_like(g)
    full[:, Y0:Y1, X0:X1] = d
    assert np.abs(g_flip - g - full).max() <= 1e-12 * np.abs(g).max()
    assert np.abs(full).max() > 0


def test_pool_flip_effect_equals_full_backward_difference():
    from oracle.flips import flip_effect
    net, ws, bs, x, rec, acts, seeds, g = _recorded_case()
    i = 1                                          # pool after conv1_2
    a = acts[i]
    h2, w2 = a.shape[1] // 2, a.shape[2] // 2
    v = np.stack([a[:, dy:2 * h2:2, dx:2 * w2:2] for dy, dx in ((0, 0), (0, 1), (1, 0), (1, 1))], -1)
    srt = np.sort(v, -1)
    ok = np.argwhere((srt[..., 2] > 0) & (srt[..., 3] > srt[..., 2]))
    c, py, px = map(int, ok[5])
    k1 = int(np.argmax(v[c, py, px]))
    rest = v[c, py, px].copy()
    rest[k1] = -np.inf
    k2 = int(np.argmax(rest))
    order = ((0, 0), (0, 1), (1, 0), (1, 1))
    mod = [t.copy() for t in acts]
    (y1, x1), (y2, x2) = [(2 * py + order[k][0], 2 * px + order[k][1]) for k in (k1, k2)]
    mod[i][c, y1, x1], mod[i][c, y2, x2] = a[c, y2, x2], a[c, y1, x1]   # routing now goes to k2
    g_flip = backward(net, mod, seeds, ws)
    Y0, Y1, X0, X1, d = flip_effect(net, rec, ws, (0.0, "pool", i, c, py, px), g.shape[1:])
    full = np.zeros_like(g)
    full[:, Y0:Y1, X0:X1] = d
    assert np.abs(g_flip - g - full).max() <= 1e-12 * np.abs(g).max()
    assert np.abs(full).max() > 0


def test_flip_fit_removes_planted_flips_and_keeps_real_errors():
    from oracle.flips import flip_effect, flip_fit, fragile_units
    net, ws, bs, x, rec, acts, seeds, g = _recorded_case()
    units = fragile_units(net, acts, ws, bs, x, 1e-3)
    pick, g_test = [], g.copy()
    for u in units[::3]:                          # three flips whose effect is not zero
        Y0, Y1, X0, X1, d = flip_effect(net, rec, ws, u, g.shape[1:])
        if np.abs(d).max() > 1e-6 * np.abs(g).max() and len(pick) < 3:
            g_test[:, Y0:Y1, X0:X1] += d
            pick.append(u)
    assert len(pick) == 3
    rng = np.random.default_rng(0)
    noise = 1e-9 * np.abs(g).max() * rng.standard_normal(g.shape)
    r, flipped, first = flip_fit(net, x, ws, bs, rec, g, g_test + noise, delta=1e-3)
    assert rel(r + g, g) < 1e-7
    assert sorted(flipped) == sorted(pick)
    # a genuine error (a dropped term) is not explained away
    bad = g_test.copy()
    bad[:, 5:9, 5:9] *= 1.5
    r2, _, _ = flip_fit(net, x, ws, bs, rec, g, bad, delta=1e-3)
    assert rel(r2 + g, g) > 1e-3
    # nothing to explain: no flips
    r3, flipped3, _ = flip_fit(net, x, ws, bs, rec, g, g + noise, delta=1e-3)
    assert flipped3 == [] and np.array_equal(r3, noise + g - g)


@pytest.mark.slow
def test_flip_fit_brings_a_plain_fp32_evaluation_under_1e4():
    """A plain FP32 evaluation of the definition (FP32 storage and FP32 accumulation, the
    FP64 oracle's own steps) misses the 1e-4 gradient bar at 200 x 328 on the full net
    because rounding moves a few near-tie decisions; after the fit it meets it.  This pins
    that the bar the FP32 GPU tests apply after the fit is reachable by a correct FP32
    evaluation, and that the fit needs only a handful of flips to get there."""
    from oracle import bf16ref
    from oracle.flips import flip_fit
    from test_oracle_bf16 import _adj_f32, _conv_f32
    net = vgg19()
    ws, bs = synth.vgg_weights(net.convs, seed=0)
    ws = [wi.astype(np.float64) for wi in ws]
    bs = [bi.astype(np.float64) for bi in bs]
    c = synth.image(200, 328, 8, 1).astype(np.float64)
    s = synth.image(176, 208, 8, 2).astype(np.float64)
    x = synth.image(200, 328, 8, 3).astype(np.float64)
    g_t = oracle.loss.style_grams(net, s, ws, bs)
    f_c = oracle.content_features(net, c, ws, bs)
    rec = {}
    _, g64 = loss_grad(net, x, ws, bs, g_t, f_c, [0.2] * 5, 0.0, record=rec)
    q32 = lambda a: np.asarray(a, np.float32).astype(np.float64)   # noqa: E731
    orig = bf16ref.conv3x3, bf16ref.conv3x3_adjoint
    bf16ref.conv3x3, bf16ref.conv3x3_adjoint = _conv_f32, _adj_f32
    try:
        _, g32 = bf16ref.loss_grad(net, x, ws, bs, g_t, f_c, [0.2] * 5, 0.0, q=q32)
    finally:
        bf16ref.conv3x3, bf16ref.conv3x3_adjoint = orig
    raw = rel(g32, g64)
    r, flipped, _ = flip_fit(net, x, ws, bs, rec, g64, g32)
    print(f"fp32 raw {raw:.2e}, after the fit {rel(r + g64, g64):.2e} with {len(flipped)} flips")
    assert raw > 1e-4 and rel(r + g64, g64) < 1e-5 and len(flipped) <= 10


def test_relu_flip_into_all_zero_pool_window():
    """A unit that turns positive inside an all-zero pooling window becomes that window's
    maximum and takes the pooled gradient: flip_effect must match a full backward."""
    from oracle.flips import flip_effect
    net, ws, bs, x, rec, acts, seeds, g = _recorded_case()
    i = 1                                          # conv1_2, followed by pool1
    a = acts[i]
    h2, w2 = a.shape[1] // 2, a.shape[2] // 2
    v = np.stack([a[:, dy:2 * h2:2, dx:2 * w2:2] for dy, dx in ((0, 0), (0, 1), (1, 0), (1, 1))], -1)
    zero = np.argwhere(v.max(-1) == 0.0)
    found = None
    for c, py, px in zero:
        if rec[("dP", i)][c, py, px] != 0.0:
            found = (int(c), int(py), int(px))
            break
    assert found is not None
    c, py, px = found
    y, xx = 2 * py + 1, 2 * px                       # third position in window order
    mod = [t.copy() for t in acts]
    mod[i][c, y, xx] = 1e-300                      # now the (only) positive value of the window
    g_flip = backward(net, mod, seeds, ws)
    Y0, Y1, X0, X1, d = flip_effect(net, rec, ws, (0.0, "relu", i, c, y, xx), g.shape[1:])
    full = np.zeros_like(g)
    full[:, Y0:Y1, X0:X1] = d
    assert np.abs(g_flip - g - full).max() <= 1e-12 * np.abs(g).max()
    assert np.abs(full).max() > 0


# ------------------------------------------------- average-pooling variant --

def test_avgpool_matches_loops_and_torch():
    rng = np.random.default_rng(50)
    for h, w in ((6, 8), (7, 9), (5, 4)):
        a = rng.standard_normal((3, h, w))
        ref = np.zeros((3, h // 2, w // 2))
        for c in range(3):
            for y in range(h // 2):
                for x in range(w // 2):
                    ref[c, y, x] = (a[c, 2 * y, 2 * x] + a[c, 2 * y, 2 * x + 1] + a[c, 2 * y + 1, 2 * x]
                                    + a[c, 2 * y + 1, 2 * x + 1]) / 4.0
        assert np.allclose(ops.avgpool2(a), ref, rtol=0, atol=1e-15)
        t = F.avg_pool2d(torch.from_numpy(a)[None], 2, 2)[0].numpy()
        assert np.allclose(ops.avgpool2(a), t, rtol=0, atol=1e-15)
        dy = rng.standard_normal((3, h // 2, w // 2))
        # adjoint identity <pool(a), dy> = <a, pool^T(dy)>; dropped rows get 0
        lhs = float(np.sum(ops.avgpool2(a) * dy))
        g = ops.avgpool2_backward(dy, a)
        assert abs(lhs - float(np.sum(a * g))) < 1e-12
        if h % 2:
            assert np.all(g[:, -1, :] == 0.0)


def torch_energy_avg(net, x, ws, bs, grams_t, f_c, w_style, alpha):
    a = x
    acts = {}
    for i in range(max(list(net.style) + [net.content]) + 1):
        a = F.relu(F.conv2d(a, ws[i], bs[i], padding=1))
        acts[i] = a
        if i in net.pool_after:
            a = F.avg_pool2d(a, 2, 2)
    e = torch.zeros((), dtype=torch.float64)
    for k, i in enumerate(net.style):
        v = acts[i][0].reshape(acts[i].shape[1], -1).T
        e = e + w_style[k] * torch.sum((v.T @ v / v.shape[0] - grams_t[k]) ** 2)
    return e + alpha * torch.sum((acts[net.content][0] - f_c) ** 2)


@pytest.mark.parametrize("kind", ["tiny", "full"])
def test_avgpool_net_loss_grad_matches_torch_autograd(kind):
    net = vgg19_tiny(avg_pool=True) if kind == "tiny" else vgg19(avg_pool=True)
    h, w = (26, 30) if kind == "tiny" else (36, 52)
    ws, bs = synth.vgg_weights(net.convs, seed=0, bias_std=0.02)
    ws = [wi.astype(np.float64) for wi in ws]
    bs = [bi.astype(np.float64) for bi in bs]
    c = synth.image(h, w, 4, 1).astype(np.float64)
    s = synth.image(h + 4, w - 4, 4, 2).astype(np.float64)
    x = synth.image(h, w, 4, 3).astype(np.float64)
    g_t = oracle.loss.style_grams(net, s, ws, bs)
    f_c = oracle.content_features(net, c, ws, bs)
    ns = len(net.style)
    w_style = [1.0 / ns] * ns
    terms, grad = loss_grad(net, x, ws, bs, g_t, f_c, w_style, 0.5)
    tx = torch.from_numpy(x)[None].requires_grad_(True)
    e = torch_energy_avg(net, tx, [torch.from_numpy(v) for v in ws], [torch.from_numpy(v) for v in bs],
                         [torch.from_numpy(v) for v in g_t], torch.from_numpy(f_c), w_style, 0.5)
    e.backward()
    assert abs(terms["E"] - e.item()) <= 1e-12 * abs(e.item())
    assert rel(grad, tx.grad[0].numpy()) < 1e-11
    # and it is not the max-pool network's value
    net_max = vgg19_tiny() if kind == "tiny" else vgg19()
    assert abs(loss_grad(net_max, x, ws, bs, g_t, f_c, w_style, 0.5, want_grad=False)[0]["E"] - terms["E"]) > 1e-6


def test_avgpool_net_tiled_equals_whole():
    net = vgg19_tiny(avg_pool=True)
    whole, gw, tiled, gt, _ = _tiled_vs_whole(net, 70, 58, 16, 23)
    for a, b in zip(tiled["grams"], whole["grams"]):
        assert rel(a, b) < 1e-13
    assert rel(gt, gw) < 1e-12


def test_avgpool_bf16_reference_with_rounding_off_is_the_oracle():
    from oracle import bf16ref
    net = vgg19_tiny(avg_pool=True)
    ws, bs = synth.vgg_weights(net.convs, seed=0, bias_std=0.02)
    ws = [wi.astype(np.float64) for wi in ws]
    bs = [bi.astype(np.float64) for bi in bs]
    x = synth.image(24, 28, 4, 3).astype(np.float64)
    c = synth.image(24, 28, 4, 1).astype(np.float64)
    s = synth.image(28, 24, 4, 2).astype(np.float64)
    g_t = oracle.loss.style_grams(net, s, ws, bs)
    f_c = oracle.content_features(net, c, ws, bs)
    t0, g0 = loss_grad(net, x, ws, bs, g_t, f_c, [1 / 3] * 3, 1.0)
    t1, g1 = bf16ref.loss_grad(net, x, ws, bs, g_t, f_c, [1 / 3] * 3, 1.0, q=bf16ref.identity)
    assert t0["E"] == t1["E"] and np.array_equal(g0, g1)
