"""Write FP64 oracle reference values for the full-size workloads (calls oracle/ only).

    python tests/golden/make_golden.py [C2|C3|C3p1|C4 ...]

For each configuration the oracle evaluates the tiled two-pass loss (Algorithm 1, its
own planner) on the seeded synthetic inputs and stores, as JSON:

* the energy terms;
* per style layer, for x and for the style image: the Gram summaries (trace, Frobenius
  norm, diagonal, first 8x8 block) and the probe products G P with P a seeded C x 16
  standard-normal matrix (seed 5, drawn layer after layer), which any wrong block of G
  changes; the full Grams of x for layers with C <= 128;
* content features: sum, sum of squares and the values at 384 seeded (c, y, x);
* dE/dx at 512 pixels of two tiles (the one holding the image centre and the last,
  ragged one), a third of them within 6 px of a block edge (Step 2 run only on those
  tiles), and for C2 central finite differences at the first 64 of them.

A tiled oracle result equals the whole-image one to ~1e-13 (pinned in
tests/test_oracle.py), so these are whole-image reference values.  C3p1 is the
3024 x 4032 level of the content pyramid (x and c box-downsampled by 2 from their
6048 x 8064 versions; the style image keeps its size).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402
from oracle.loss import energy_terms  # noqa: E402
from oracle.plan import make_plan  # noqa: E402
from oracle.loss import forward  # noqa: E402
from oracle.net import receptive_fields  # noqa: E402
from oracle.tiled import step1, step2, tiled_content_features  # noqa: E402

CONFIGS = {
    "C2": dict(H=2048, W=2048, Hs=1024, Ws=1280, sigma=8.0, T=512, m=155),
    "C3": dict(H=6048, W=8064, Hs=4226, Ws=5319, sigma=16.0, T=1024, m=155),
    "C3p1": dict(H=3024, W=4032, Hs=4226, Ws=5319, sigma=16.0, T=1024, m=155, down=1),
    "C4": dict(H=3024, W=4032, Hs=2000, Ws=2000, sigma=16.0, T=1000, m=155),
}
W_STYLE = [0.2] * 5
ALPHA = 1.0


def summarize(g):
    return {"trace": float(np.trace(g)), "fro": float(np.linalg.norm(g)),
            "diag": [float(v) for v in np.diag(g)], "block8": [[float(v) for v in r] for r in g[:8, :8]]}


def probes(sizes, seed=5):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((c, 16)) for c in sizes]


def sample_pixels(H, W, T, m, seed=4, per_tile=256, edge=6):
    """Pixels in two tiles: the one holding the image centre and the last (ragged) one;
    per tile two thirds uniform over the block and one third within ``edge`` px of one
    of its four edges."""
    net = oracle.vgg19()
    plan = make_plan(H, W, T, m, net.strides(), net.align())
    centre = next(k for k, t in enumerate(plan) if t.by0 <= H // 2 < t.by1 and t.bx0 <= W // 2 < t.bx1)
    picks = sorted({centre, len(plan) - 1})
    rng = np.random.default_rng(seed)
    out = []
    for k in picks:
        t = plan[k]
        for j in range(per_tile):
            ch = int(rng.integers(3))
            y, x = int(rng.integers(t.by0, t.by1)), int(rng.integers(t.bx0, t.bx1))
            if 3 * j >= 2 * per_tile:
                side, d = int(rng.integers(4)), int(rng.integers(edge))
                if side == 0:
                    y = t.by0 + d
                elif side == 1:
                    y = t.by1 - 1 - d
                elif side == 2:
                    x = t.bx0 + d
                else:
                    x = t.bx1 - 1 - d
            out.append((ch, y, x))
    return picks, out


def local_fd(net, x, w64, b64, g_x, g_t, f_c, px, h=1e-3):
    """Central differences (E(x + h e) - E(x - h e)) / 2h of the FP64 energy for single
    pixels, evaluated exactly from a window around the pixel: a pixel changes only the
    features whose dependency cone [s q - a, s q + b] contains it, so with the global
    Grams G(x) the energy change is
        sum_l w_l (||D_l + (S+ - S0)/n_p||^2 - ||D_l + (S- - S0)/n_p||^2)
        + alpha sum (||v+ - f||^2 - ||v- - f||^2)
    with D_l = G_l(x) - Ghat_l and S the V^T V sums over those features."""
    H, W = x.shape[1:]
    S = net.align()
    rf = receptive_fields(net)
    strides = net.strides()
    top = max(list(net.style) + [net.content])
    d = [gx - gt for gx, gt in zip(g_x, g_t)]
    out = []
    for ch, y, xx in px:
        Y0, Y1 = max(0, S * ((y - 160) // S)), min(H, S * (-(-(y + 161) // S)))
        X0, X1 = max(0, S * ((xx - 160) // S)), min(W, S * (-(-(xx + 161) // S)))
        win = x[:, Y0:Y1, X0:X1]
        acts = {}
        for key, sgn in (("0", 0.0), ("+", 1.0), ("-", -1.0)):
            xw = win.copy()
            xw[ch, y - Y0, xx - X0] += sgn * h
            acts[key] = forward(net, xw, w64, b64, upto=top)
        e = {}
        for key in ("+", "-"):
            tot = 0.0
            for k, i in enumerate(net.style):
                s, (a, b) = strides[i], rf[i]
                n_h, n_w = H // s, W // s
                r0, r1 = max(0, -(-(y - b) // s)), min(n_h - 1, (y + a) // s) + 1
                c0, c1 = max(0, -(-(xx - b) // s)), min(n_w - 1, (xx + a) // s) + 1
                oy, ox = Y0 // s, X0 // s
                sums = []
                for kk in (key, "0"):
                    v = acts[kk][i][:, r0 - oy:r1 - oy, c0 - ox:c1 - ox].reshape(acts[kk][i].shape[0], -1)
                    sums.append(v @ v.T)
                n_p = float(n_h * n_w)
                tot += W_STYLE[k] * float(np.sum((d[k] + (sums[0] - sums[1]) / n_p) ** 2))
            i = net.content
            s, (a, b) = strides[i], rf[i]
            n_h, n_w = H // s, W // s
            r0, r1 = max(0, -(-(y - b) // s)), min(n_h - 1, (y + a) // s) + 1
            c0, c1 = max(0, -(-(xx - b) // s)), min(n_w - 1, (xx + a) // s) + 1
            oy, ox = Y0 // s, X0 // s
            v = acts[key][i][:, r0 - oy:r1 - oy, c0 - ox:c1 - ox]
            tot += ALPHA * float(np.sum((v - f_c[:, r0:r1, c0:c1]) ** 2))
            e[key] = tot
        out.append((e["+"] - e["-"]) / (2 * h))
    return out


def images(cfg):
    H, W, Hs, Ws, sigma = (cfg[k] for k in ("H", "W", "Hs", "Ws", "sigma"))
    down = cfg.get("down", 0)
    xs = []
    for seed in (synth.SEED_X, synth.SEED_CONTENT):
        a = synth.image(H << down, W << down, sigma, seed)
        for _ in range(down):
            a = synth.box_down2(a)
        xs.append(a.astype(np.float64))
    s = synth.image(Hs, Ws, sigma, synth.SEED_STYLE).astype(np.float64)
    return xs[0], xs[1], s


def run(name):
    cfg = CONFIGS[name]
    H, W, T, m = (cfg[k] for k in ("H", "W", "T", "m"))
    t0 = time.time()
    net = oracle.vgg19()
    ws, bs = synth.vgg_weights(net.convs, synth.SEED_WEIGHTS)
    w64 = [w.astype(np.float64) for w in ws]
    b64 = [b.astype(np.float64) for b in bs]
    x, c, s = images(cfg)
    print(f"[{name}] inputs {time.time() - t0:.0f}s", flush=True)
    g_t, _ = step1(net, s, w64, b64, T, m)
    print(f"[{name}] style grams {time.time() - t0:.0f}s", flush=True)
    f_c = tiled_content_features(net, c, w64, b64, T, m)
    print(f"[{name}] content features {time.time() - t0:.0f}s", flush=True)
    g_x, e_c = step1(net, x, w64, b64, T, m, f_c=f_c, alpha=ALPHA)
    terms = energy_terms(g_x, g_t, W_STYLE, e_c)
    print(f"[{name}] step 1 {time.time() - t0:.0f}s E={terms['E']:.9e}", flush=True)
    picks, px = sample_pixels(H, W, T, m)
    grad = step2(net, x, w64, g_x, g_t, f_c, W_STYLE, ALPHA, T, m, b64, only=set(picks))
    print(f"[{name}] step 2 on tiles {picks} {time.time() - t0:.0f}s", flush=True)
    fd = local_fd(net, x, w64, b64, g_x, g_t, f_c, px[:64]) if name == "C2" else None
    print(f"[{name}] finite differences {time.time() - t0:.0f}s", flush=True)
    P = probes([g.shape[0] for g in g_x])
    rng = np.random.default_rng(6)
    cs, ch, cw = f_c.shape
    fsmp = [(int(rng.integers(cs)), int(rng.integers(ch)), int(rng.integers(cw))) for _ in range(384)]
    out = {
        "config": cfg, "w_style": W_STYLE, "alpha": ALPHA,
        "E": terms["E"], "E_content": terms["E_content"], "E_style": terms["E_style"],
        "grams_x": [summarize(g) for g in g_x], "grams_style": [summarize(g) for g in g_t],
        "probe_seed": 5,
        "grams_x_probe": [(g @ p).tolist() for g, p in zip(g_x, P)],
        "grams_style_probe": [(g @ p).tolist() for g, p in zip(g_t, P)],
        "grams_x_full": [g.tolist() if g.shape[0] <= 128 else None for g in g_x],
        "content_feats": {"sum": float(f_c.sum()), "sumsq": float((f_c ** 2).sum()),
                          "samples": [[a, b, d, float(f_c[a, b, d])] for a, b, d in fsmp]},
        "grad_tiles": picks,
        "grad_samples": [[ch_, y, xx, float(grad[ch_, y, xx])] for ch_, y, xx in px],
        "fd_h": 1e-3, "fd_samples": fd,
        "seconds": time.time() - t0,
    }
    with open(os.path.join(HERE, f"oracle_{name}.json"), "w") as f:
        json.dump(out, f)
    print(f"[{name}] done in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or ["C2", "C4", "C3p1", "C3"]:
        run(name)
