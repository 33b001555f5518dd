#!/usr/bin/env python3
"""Throughput of one style+content loss+gradient evaluation (both passes of
Algorithm 1) through libnst on one MI355X.

Workload (default): x and content 6048 x 8064, style 4226 x 5319 (the paper's Fig. 1
sizes), seeded synthetic images (Gaussian-blurred noise, sigma 16 px), VGG-19
conv1_1..conv5_1 with seeded He-normal weights, style layers relu{1..5}_1 with
w = 1/5, content relu4_2 with alpha = 1, tiles of 1024 px with the exact
receptive-field margin 155 (48 tiles).  The style Grams and content features are
computed once, untimed; each timed step is nst_loss_grad(STEP1 | STEP2) with all
inputs resident in HBM.  When the workspace (--ws-gib) holds every tile, Step 2 runs the
backward on the activations Step 1 left resident; --recompute sizes it for tile batches
so that Step 2 recomputes each tile's forward as Algorithm 1 prints it.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpixel/s per style+content loss+grad eval (VGG-19); BF16 vs FP32 at stated grad error"
PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3}
HBM_GBS = 8000.0
# algorithmic FLOPs of one evaluation per image pixel as Algorithm 1 prints it: two
# forwards, one data gradient, the style Grams and the style residual products (full
# VGG-19 prefix); with resident activations one of the two forwards is not executed
FLOP_PER_PX = 2 * 722304 + 722304 + 2 * 34816


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(args):
    import synth
    log(f"[bench] generating inputs x, c {args.H}x{args.W}, style {args.Hs}x{args.Ws}")
    t = time.time()
    x = synth.image(args.H, args.W, args.sigma, synth.SEED_X, threads=3)
    c = synth.image(args.H, args.W, args.sigma, synth.SEED_CONTENT, threads=3)
    s = synth.image(args.Hs, args.Ws, args.sigma, synth.SEED_STYLE, threads=3)
    ws, bs = synth.vgg_weights(synth.VGG19_CONVS, synth.SEED_WEIGHTS)
    log(f"[bench] inputs generated in {time.time() - t:.1f}s")
    return x, c, s, ws, bs


def run_precision(prec, steps, warmup, args, x, c, s, ws, bs, profile):
    import torch
    from paper_2212_13459_amd import Context, plan, vgg19_desc, workspace_bytes
    dev = torch.device("cuda", 0)
    nst = Context(ws, bs, prec, tile_batch=args.tile_batch, ws_limit=int(args.ws_gib * (1 << 30)),
                  retain=not args.recompute)
    xd = torch.from_numpy(x).to(dev)
    gt = nst.style_grams(torch.from_numpy(s).to(dev), args.T, args.m)
    fc = nst.content_feats(torch.from_numpy(c).to(dev), args.T, args.m)
    w_style = [0.2] * 5
    gx = torch.empty_like(gt)
    grad = torch.empty_like(xd)
    torch.cuda.synchronize()
    nt = len(plan(vgg19_desc(), args.H, args.W, args.T, args.m))
    wsb = nst.workspace(args.H, args.W, args.T, args.m).numel()
    resident = wsb >= workspace_bytes(vgg19_desc(), prec, args.H, args.W, args.T, args.m, nt)
    log(f"[bench] {prec}: targets ready, workspace {wsb / 2**30:.1f} GiB, "
        f"{'every tile resident (Step 2 reuses Step 1 activations)' if resident else 'tile batches (Step 2 recomputes)'}")
    for i in range(warmup):
        nst.loss_grad(xd, gt, fc, w_style, 1.0, args.T, args.m, grams_x=gx, grad=grad, want_energy=False)
        torch.cuda.synchronize()
        log(f"[bench] {prec}: warmup {i + 1}/{warmup} done")
    if profile:
        nst.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        nst.loss_grad(xd, gt, fc, w_style, 1.0, args.T, args.m, grams_x=gx, grad=grad, want_energy=False)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    stats = []
    if profile:
        stats = nst.profile_read()
        nst.profile(False)
    energy, _, _ = nst.loss_grad(xd, gt, fc, w_style, 1.0, args.T, args.m, grams_x=gx, grad=grad)
    log(f"[bench] {prec}: {steps} steps, {dt * 1e3:.1f} ms/step, E={energy[0]:.6e}")
    out = dict(ms=dt * 1e3, stats=stats, energy=energy, grad_norm=float(grad.double().norm()),
               step2="reuses Step 1 activations" if resident else "recomputes the forward per tile batch")
    del nst, xd, gt, fc, gx, grad
    torch.cuda.empty_cache()
    return out


def roofline(prec, stats, steps):
    from paper_2212_13459_amd.profsum import read_traffic
    top = stats[0]
    avg_ms = top["ms"] / top["launches"]
    if top["flops"] > 0:
        achieved = top["flops"] / top["launches"] / (avg_ms * 1e-3) / 1e12
        peak = PEAK_TFLOPS[prec]
        r = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s"}
    else:
        achieved = top["bytes"] / top["launches"] / (avg_ms * 1e-3) / 1e9
        peak = HBM_GBS
        r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": peak, "unit": "GB/s"}
    # HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary, if it was
    # taken on the current kernel sources
    tr = read_traffic(os.path.join(ROOT, "profiles"), top["name"])
    r.update({"frac": round(achieved / peak, 4), "traffic": None if tr is None else round(tr[0]),
              "kernel": top["name"], "launches_per_step": top["launches"] / steps,
              "avg_launch_ms": round(avg_ms, 4),
              "algorithmic_bytes_per_launch": round(top["bytes"] / top["launches"]),
              "algorithmic_flops_per_launch": round(top["flops"] / top["launches"])})
    if tr is not None:
        r["traffic_source"] = tr[1]
    return r


def cpu_baseline(args, x, c, s, ws, bs):
    """The FP64 oracle (whole-image loss and gradient) on a crop of the same workload."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import oracle
    from oracle.loss import content_features, loss_grad, style_grams
    n = args.cpu_sample
    net = oracle.vgg19()
    w64 = [w.astype(np.float64) for w in ws]
    b64 = [b.astype(np.float64) for b in bs]
    y0, x0 = (args.H - n) // 2, (args.W - n) // 2
    xs = x[:, y0:y0 + n, x0:x0 + n].astype(np.float64)
    cs = c[:, y0:y0 + n, x0:x0 + n].astype(np.float64)
    ys, xs0 = (args.Hs - n) // 2, (args.Ws - n) // 2
    ss = s[:, ys:ys + n, xs0:xs0 + n].astype(np.float64)
    g_t = style_grams(net, ss, w64, b64)
    f_c = content_features(net, cs, w64, b64)
    t = time.perf_counter()
    loss_grad(net, xs, w64, b64, g_t, f_c, [0.2] * 5, 1.0)
    dt = time.perf_counter() - t
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    log(f"[bench] cpu oracle: {n}x{n} crop in {dt:.1f}s with {threads} BLAS threads")
    return {"value": round(n * n / dt / 1e6, 5), "unit": "Mpixel/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle whole-image loss+gradient on a {n}x{n} centre crop of x (targets from "
                      f"crops of the content and style images), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp32"])
    ap.add_argument("--fp32-steps", type=int, default=2, help="FP32 comparison steps (0 skips it)")
    ap.add_argument("--H", type=int, default=6048)
    ap.add_argument("--W", type=int, default=8064)
    ap.add_argument("--Hs", type=int, default=4226)
    ap.add_argument("--Ws", type=int, default=5319)
    ap.add_argument("--sigma", type=float, default=16.0)
    ap.add_argument("--T", type=int, default=1024)
    ap.add_argument("--m", type=int, default=155)
    ap.add_argument("--tile-batch", type=int, default=32)
    ap.add_argument("--ws-gib", type=float, default=200.0)
    ap.add_argument("--cpu-sample", type=int, default=1440)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--recompute", action="store_true",
                    help="size the workspace for a tile batch, so that Step 2 recomputes each tile's "
                         "forward (Algorithm 1 as printed) instead of reusing Step 1's resident activations")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first launch a plain copy (negation) kernel of this many MiB three times, "
                         "as the reference for FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this implementation runs on one GPU; --gpus N with N > 1 is not supported "
              "(the tiles of one evaluation would shard across GPUs with one Gram all-reduce, which "
              "is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_2212_13459_amd import plan, vgg19_desc
    n_tiles = len(plan(vgg19_desc(), args.H, args.W, args.T, args.m))
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib << 18
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.neg(a, out=b)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 3 x {4 * n} bytes read and written")
        del a, b
    x, c, s, ws, bs = make_inputs(args)

    main_res = run_precision(args.precision, args.steps, args.warmup, args, x, c, s, ws, bs, profile=True)
    ms = main_res["ms"]
    value = args.H * args.W / (ms * 1e-3) / 1e6
    peak = PEAK_TFLOPS[args.precision]
    result = {
        "metric": METRIC, "value": round(value, 3), "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"loss+grad x {args.H}x{args.W}, style {args.Hs}x{args.Ws}, "
                               f"tiles {args.T} px margin {args.m} ({n_tiles} tiles), VGG-19 conv1_1..conv5_1",
                   "H": args.H, "W": args.W, "style_H": args.Hs, "style_W": args.Ws, "T": args.T, "m": args.m,
                   "tiles": n_tiles, "style_weight": 0.2, "alpha": 1.0, "step2": main_res["step2"]},
        "roofline": roofline(args.precision, main_res["stats"], args.steps),
        "effective_mfma_frac": round(FLOP_PER_PX * args.H * args.W / (ms * 1e-3) / 1e12 / peak, 4),
        "kernels": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()}
                    for st in main_res["stats"]],
        "energy": main_res["energy"],
    }
    if args.fp32_steps > 0 and args.precision != "fp32":
        r32 = run_precision("fp32", args.fp32_steps, 1, args, x, c, s, ws, bs, profile=False)
        result["fp32"] = {"value": round(args.H * args.W / (r32["ms"] * 1e-3) / 1e6, 3),
                          "ms_per_step": round(r32["ms"], 3), "step2": r32["step2"],
                          "speedup_of_bf16": round(r32["ms"] / ms, 3),
                          "energy_rel_diff_bf16_vs_fp32": abs(main_res["energy"][0] - r32["energy"][0]) / abs(r32["energy"][0]),
                          "grad_norm_rel_diff": abs(main_res["grad_norm"] - r32["grad_norm"]) / r32["grad_norm"]}
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args, x, c, s, ws, bs)
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
