"""Pins of the BF16-storage reference (oracle/bf16ref.py).

* its rounding is torch's float32 -> bfloat16 cast (round to nearest, ties to even);
* with rounding off it is the FP64 oracle, bit for bit;
* with rounding on it equals an independent model of the same storage points built on
  torch CPU float64 autograd (the rounding placed on values and on gradients by two
  small autograd functions, everything else differentiated by torch);
* the spread between it and the same reference with FP32 accumulation bounds the
  GPU-vs-reference bars used by the BF16 parity tests.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
import synth
from oracle import bf16ref
from oracle.loss import content_features, loss_grad, style_grams
from oracle.net import NetSpec

torch.set_num_threads(4)


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ------------------------------------------------------------ rounding -----

def test_round_bf16_matches_torch_cast():
    rng = np.random.default_rng(30)
    vals = [rng.standard_normal(20000).astype(np.float32),
            (rng.standard_normal(20000) * 1e-6).astype(np.float32),
            (rng.standard_normal(20000) * 1e5).astype(np.float32)]
    # exact halfway cases (low 16 bits 0x8000) with even and odd kept parts, carries into
    # the exponent (0x3fff8000 -> 2.0), negatives and zeros
    bits = rng.integers(0x3f000000, 0x40ffffff, 4096, dtype=np.int64).astype(np.uint32)
    ties = (bits & np.uint32(0xffff0000)) | np.uint32(0x8000)
    special = np.array([0x3fff8000, 0x3f7f8000, 0xbf808000, 0x3f818000, 0, 0x80000000], np.uint32)
    vals += [ties.view(np.float32), (ties | np.uint32(0x80000000)).view(np.float32), special.view(np.float32)]
    for v in vals:
        ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
        assert np.array_equal(bf16ref.round_bf16(v.astype(np.float64)), ref)


def test_round_bf16_properties():
    rng = np.random.default_rng(31)
    v = rng.standard_normal(10000) * np.exp(rng.uniform(-20, 20, 10000))
    r = bf16ref.round_bf16(v)
    assert np.array_equal(bf16ref.round_bf16(r), r)                  # idempotent
    m, e = np.frexp(r)
    assert np.array_equal(m * 256.0, np.rint(m * 256.0))             # 8 significant bits
    assert np.all(np.abs(r - v) <= np.ldexp(1.0, e - 9) * (1 + 1e-15))  # within half a unit
    s = np.sort(v)
    assert np.all(np.diff(bf16ref.round_bf16(s)) >= 0)              # monotone


# ------------------------------------------------ rounding off = oracle ----

def _case(net, h, w, bias=0.0, sigma=4.0):
    ws, bs = synth.vgg_weights(net.convs, seed=0, bias_std=bias)
    w64 = [a.astype(np.float64) for a in ws]
    b64 = [a.astype(np.float64) for a in bs]
    c = synth.image(h, w, sigma, 1).astype(np.float64)
    s = synth.image(h + 4, w - 4, sigma, 2).astype(np.float64)
    x = synth.image(h, w, sigma, 3).astype(np.float64)
    g_t = style_grams(net, s, w64, b64)
    f_c = content_features(net, c, w64, b64) if net.content is not None else None
    return w64, b64, x, g_t, f_c


@pytest.mark.parametrize("kind", ["tiny", "full"])
def test_identity_rounding_is_the_fp64_oracle_bitwise(kind):
    net = oracle.vgg19_tiny() if kind == "tiny" else oracle.vgg19()
    h, w = (24, 28) if kind == "tiny" else (36, 52)
    w64, b64, x, g_t, f_c = _case(net, h, w, bias=0.05)
    ns = len(net.style)
    for alpha in (1.0, 0.0):
        t0, g0 = loss_grad(net, x, w64, b64, g_t, f_c, [1.0 / ns] * ns, alpha)
        t1, g1 = bf16ref.loss_grad(net, x, w64, b64, g_t, f_c, [1.0 / ns] * ns, alpha, q=bf16ref.identity)
        assert t0["E"] == t1["E"] and t0["E_content"] == t1["E_content"] and t0["E_style"] == t1["E_style"]
        assert all(np.array_equal(a, b) for a, b in zip(t0["grams"], t1["grams"]))
        assert np.array_equal(g0, g1)


# ------------------------------------------- independent torch model -------

def _rb(t):
    m, e = torch.frexp(t)
    return torch.ldexp(torch.round(m * 256.0), e - 8)   # torch.round: halves to even


class _RoundValue(torch.autograd.Function):
    """Stored value: rounded forward, gradient passed through."""

    @staticmethod
    def forward(ctx, t):
        return _rb(t)

    @staticmethod
    def backward(ctx, g):
        return g


class _RoundGrad(torch.autograd.Function):
    """Stored adjoint: identity forward, gradient rounded."""

    @staticmethod
    def forward(ctx, t):
        return t.clone()

    @staticmethod
    def backward(ctx, g):
        return _rb(g)


class _StyleTerm(torch.autograd.Function):
    """w ||A A^T / n - Ghat||^2 with the residual operand rounded in the backward."""

    @staticmethod
    def forward(ctx, a, g_t, w, n_p):
        m = a.reshape(a.shape[0], -1)
        d = m @ m.T / n_p - g_t
        ctx.save_for_backward(m, d)
        ctx.k = (w, n_p, a.shape)
        return w * (d * d).sum()

    @staticmethod
    def backward(ctx, ge):
        m, d = ctx.saved_tensors
        w, n_p, shape = ctx.k
        return ge * (_rb((2.0 * w / n_p) * (d + d.T)) @ m).reshape(shape), None, None, None


def torch_bf16_energy(net, x, ws, bs, g_t, f_c, w_style, alpha):
    a = _RoundValue.apply(x)
    e = x.new_zeros(())
    top = max(list(net.style) + ([net.content] if net.content is not None else []))
    for i in range(top + 1):
        z = F.conv2d(a[None], _rb(ws[i]), bs[i], padding=1)[0]
        r = F.relu(_RoundGrad.apply(z))          # the masked dE/dZ is stored rounded
        ai = _RoundValue.apply(r)
        if i == net.content and alpha != 0.0:
            e = e + alpha * ((r - f_c) ** 2).sum()  # content difference from the unrounded value
        if i in net.style:
            k = net.style.index(i)
            e = e + _StyleTerm.apply(ai, g_t[k], w_style[k], ai.shape[1] * ai.shape[2])
        a = _RoundGrad.apply(F.max_pool2d(ai[None], 2, 2)[0]) if i in net.pool_after else ai
    return e


NET_A = NetSpec(convs=((3, 64), (64, 256), (256, 256), (256, 256)), pool_after=frozenset({1}), style=(0, 3),
                content=2)


@pytest.mark.parametrize("kind", ["tiny", "A"])
def test_bf16_storage_equals_torch_model(kind):
    net = oracle.vgg19_tiny() if kind == "tiny" else NET_A
    w64, b64, x, g_t, f_c = _case(net, 20, 28, bias=0.02)
    ns = len(net.style)
    wst = [0.5 / ns] * ns
    for alpha in (0.7, 0.0):
        terms, grad = bf16ref.loss_grad(net, x, w64, b64, g_t, f_c, wst, alpha)
        tx = torch.from_numpy(x).requires_grad_(True)
        e = torch_bf16_energy(net, tx, [torch.from_numpy(v) for v in w64], [torch.from_numpy(v) for v in b64],
                              [torch.from_numpy(v) for v in g_t],
                              None if f_c is None else torch.from_numpy(f_c), wst, alpha)
        e.backward()
        assert abs(terms["E"] - e.item()) <= 1e-12 * abs(e.item())
        assert rel(grad, tx.grad.numpy()) < 1e-11, rel(grad, tx.grad.numpy())
        # and it is not the FP64 oracle
        _, g64 = loss_grad(net, x, w64, b64, g_t, f_c, wst, alpha)
        assert rel(grad, g64) > 1e-4


# ------------------------------------- spread of valid BF16 evaluations ----

def _conv_f32(a, wt, b=None):
    cin, h, wd = a.shape
    ap = np.zeros((cin, h + 2, wd + 2), np.float32)
    ap[:, 1:-1, 1:-1] = a
    z = np.zeros((wt.shape[0], h * wd), np.float32)
    for ky in range(3):
        for kx in range(3):
            z += wt[:, :, ky, kx].astype(np.float32) @ ap[:, ky:ky + h, kx:kx + wd].reshape(cin, h * wd)
    if b is not None:
        z += np.asarray(b, np.float32)[:, None]
    return z.reshape(-1, h, wd).astype(np.float64)


def _adj_f32(dz, wt):
    cout, h, wd = dz.shape
    dap = np.zeros((wt.shape[1], h + 2, wd + 2), np.float32)
    d2 = dz.reshape(cout, h * wd).astype(np.float32)
    for ky in range(3):
        for kx in range(3):
            dap[:, ky:ky + h, kx:kx + wd] += (wt[:, :, ky, kx].astype(np.float32).T @ d2).reshape(-1, h, wd)
    return dap[:, 1:-1, 1:-1].astype(np.float64)


NET_B = NetSpec(convs=((3, 64), (64, 512), (512, 512), (512, 512)), pool_after=frozenset(), style=(1, 3),
                content=None)


@pytest.mark.slow
@pytest.mark.parametrize("kind,h,w,grad_bar", [("tiny", 64, 64, 3e-2), ("A", 64, 96, 3e-2), ("B", 64, 96, 3e-2),
                                               ("full", 200, 328, 0.2)])
def test_fp32_accumulation_spread_is_within_the_bf16_bars(kind, h, w, grad_bar, monkeypatch):
    """The same BF16-storage evaluation with FP32 accumulation (what the GPU does) stays
    within two thirds of the bars the GPU BF16 parity tests apply against this reference:
    gradient ``grad_bar``, Grams 1e-4 (2e-3 full net), energies 2e-4 (5e-4 full net)."""
    net = {"tiny": oracle.vgg19_tiny(), "A": NET_A, "B": NET_B, "full": oracle.vgg19()}[kind]
    w64, b64, x, g_t, f_c = _case(net, h, w, sigma=4.0 if kind != "full" else 8.0)
    ns = len(net.style)
    gram_bar, e_bar = (2e-3, 5e-4) if kind == "full" else (1e-4, 2e-4)
    for alpha in ((1.0, 0.0) if net.content is not None else (0.0,)):
        t0, g0 = bf16ref.loss_grad(net, x, w64, b64, g_t, f_c, [1.0 / ns] * ns, alpha)
        with monkeypatch.context() as mp:
            mp.setattr(bf16ref, "conv3x3", _conv_f32)
            mp.setattr(bf16ref, "conv3x3_adjoint", _adj_f32)
            t1, g1 = bf16ref.loss_grad(net, x, w64, b64, g_t, f_c, [1.0 / ns] * ns, alpha)
        ge = max(rel(a, b) for a, b in zip(t1["grams"], t0["grams"]))
        ee = abs(t1["E"] - t0["E"]) / t0["E"]
        print(f"[spread {kind} alpha={alpha}] grad {rel(g1, g0):.2e} grams {ge:.2e} energy {ee:.2e}")
        assert rel(g1, g0) < grad_bar / 1.5 and ge < gram_bar / 1.5 and ee < e_bar / 1.5
