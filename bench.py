#!/usr/bin/env python3
"""Throughput of one style+content loss+gradient evaluation (both passes of
Algorithm 1) through libnst on one MI355X.

Workload (default): x and content 6048 x 8064, style 4226 x 5319 (the paper's Fig. 1
sizes), seeded synthetic images (Gaussian-blurred noise, sigma 16 px), VGG-19
conv1_1..conv5_1 with seeded He-normal weights, style layers relu{1..5}_1 with
w = 1/5, content relu4_2 with alpha = 1, tiles of 1024 px with the exact
receptive-field margin 155 (48 tiles).  The style Grams and content features are
computed once, untimed; each timed step is nst_loss_grad(STEP1 | STEP2) with all
inputs resident in HBM.  Step 2 recomputes each tile batch's forward as Algorithm 1
prints it (memory: one batch of 24 tiles; batches of 1, 8 and 16 tiles are timed beside it).
The same evaluation with every tile's activations resident (NST_RESIDENT) is reported
beside it, as are the whole image as one window (a single tile, which one GPU's HBM
holds), FP32, the smaller scales of the content pyramid and the ragged 1000 px tiling of
a 3024 x 4032 image.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpixel/s per style+content loss+grad eval (VGG-19); BF16 vs FP32 at stated grad error"
PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3}
HBM_GBS = 8000.0
# algorithmic FLOPs of one evaluation per image pixel: two forwards, one data gradient,
# the style Grams and the style residual products (full VGG-19 prefix)
FLOP_PER_PX = 2 * 722304 + 722304 + 2 * 34816
W_STYLE = [0.2] * 5


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_images(H, W, Hs, Ws, sigma):
    import synth
    t = time.time()
    x = synth.image(H, W, sigma, synth.SEED_X, threads=3)
    c = synth.image(H, W, sigma, synth.SEED_CONTENT, threads=3)
    s = synth.image(Hs, Ws, sigma, synth.SEED_STYLE, threads=3)
    log(f"[bench] images x, c {H}x{W}, style {Hs}x{Ws} generated in {time.time() - t:.1f}s")
    return x, c, s


class Eval:
    """One precision's context, targets and inputs on the GPU for one workload."""

    def __init__(self, prec, ws, bs, x, c, s, T, m, resident=False, tile_batch=32, ws_gib=200.0):
        import torch
        from paper_2212_13459_amd import Context
        self.dev = torch.device("cuda", 0)
        self.prec, self.T, self.m = prec, T, m
        self.H, self.W = x.shape[1:]
        self.nst = Context(ws, bs, prec, tile_batch=tile_batch, ws_limit=int(ws_gib * (1 << 30)),
                           resident=resident)
        self.x = torch.from_numpy(x).to(self.dev)
        self.gt = self.nst.style_grams(torch.from_numpy(s).to(self.dev), T, m)
        self.fc = self.nst.content_feats(torch.from_numpy(c).to(self.dev), T, m)
        self.gx = torch.empty_like(self.gt)
        self.grad = torch.empty_like(self.x)
        torch.cuda.synchronize()

    def step(self, want_energy=False):
        e, _, _ = self.nst.loss_grad(self.x, self.gt, self.fc, W_STYLE, 1.0, self.T, self.m, grams_x=self.gx,
                                     grad=self.grad, want_energy=want_energy)
        return e

    def timed(self, steps, warmup, label, profile=False):
        import torch
        for i in range(warmup):
            self.step()
            torch.cuda.synchronize()
            log(f"[bench] {label}: warmup {i + 1}/{warmup} done")
        if profile:
            self.nst.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            self.step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        stats = []
        if profile:
            stats = self.nst.profile_read()
            self.nst.profile(False)
        energy = self.step(want_energy=True)
        log(f"[bench] {label}: {steps} steps, {dt * 1e3:.1f} ms/step, E={energy[0]:.6e}")
        return dt * 1e3, stats, energy

    def workspace_gib(self):
        return self.nst.workspace(self.H, self.W, self.T, self.m).numel() / 2 ** 30

    def close(self):
        import torch
        self.nst._ws = {}
        self.nst.close()
        del self.x, self.gt, self.fc, self.gx, self.grad
        torch.cuda.empty_cache()


def kernel_frac(st, prec):
    """The kernel's bound from its algorithmic intensity (FLOP per byte) against the ridge
    point of the MFMA peak over the HBM peak, and its fraction of that bound's peak; both
    fractions are listed."""
    sec = st["ms"] * 1e-3
    mfma = st["flops"] / sec / 1e12 / PEAK_TFLOPS[prec]
    hbm = st["bytes"] / sec / 1e9 / HBM_GBS
    ridge = PEAK_TFLOPS[prec] * 1e12 / (HBM_GBS * 1e9)
    bound = "mfma" if st["bytes"] == 0 or st["flops"] / st["bytes"] >= ridge else "hbm"
    return {"bound": bound, "frac": round(mfma if bound == "mfma" else hbm, 4),
            "mfma_frac": round(mfma, 4), "hbm_frac": round(hbm, 4)}


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


def golden_errors(name, energy, grad):
    """Energies and sampled gradient values against the stored FP64 oracle values
    (tests/golden/oracle_<name>.json, written from oracle/ only)."""
    import numpy as np
    import torch
    p = os.path.join(ROOT, "tests", "golden", f"oracle_{name}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        gd = json.load(f)
    smp = np.array(gd["grad_samples"])
    idx = [torch.from_numpy(smp[:, j].astype(np.int64)).to(grad.device) for j in range(3)]
    gv = grad[idx[0], idx[1], idx[2]].double().cpu().numpy()
    ref = smp[:, 3]
    terms = [abs(energy[0] - gd["E"]) / abs(gd["E"]), abs(energy[1] - gd["E_content"]) / abs(gd["E_content"])]
    terms += [abs(a - b) / abs(b) for a, b in zip(energy[2:], gd["E_style"])]
    return {"energy_rel": float("%.3e" % terms[0]), "energy_terms_rel_max": float("%.3e" % max(terms)),
            "grad_samples": int(len(ref)),
            "grad_samples_vector_rel": float("%.3e" % (np.linalg.norm(gv - ref) / np.linalg.norm(ref)))}


def multiscale_runs(args, ws, bs, x, c, s):
    """Whole style transfers (Algorithm 2): x starts from the content image downscaled to
    the first of 4 scales; each scale runs its L-BFGS iterations (history 100 at the
    first scale, 10 after), one loss + gradient evaluation per iteration."""
    import torch
    from paper_2212_13459_amd import Context
    from paper_2212_13459_amd.multiscale import iteration_schedule, style_transfer
    nst = Context(ws, bs, args.precision, tile_batch=args.tile_batch, ws_limit=int(args.ws_gib * (1 << 30)))
    dev = torch.device("cuda", 0)
    c_d, s_d = torch.from_numpy(c).to(dev), torch.from_numpy(s).to(dev)
    out = {}
    modes = ["fast", "full"] if args.multiscale == "both" else [args.multiscale]
    for mode in modes:
        its = iteration_schedule(4, fast=(mode == "fast"))

        def progress(scale, n, e):
            if n % 100 == 0:
                log(f"[bench] multiscale {mode}: scale {scale + 1}, evaluation {n}, E={e:.6e}")

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        img, recs = style_transfer(nst, c_d, s_d, n_scales=4, iterations=its, T=args.T, callback=progress)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        log(f"[bench] multiscale {mode}: {dt:.1f} s")
        out["SPST-fast" if mode == "fast" else "SPST"] = {
            "seconds": round(dt, 2), "iterations": its,
            "scales": [{"size": list(r["size"]), "evaluations": r["evaluations"], "seconds": round(r["seconds"], 3),
                        "E_first": r["E_first"], "E_last": r["E_last"]} for r in recs]}
        del img
    nst._ws = {}
    nst.close()
    del c_d, s_d
    torch.cuda.empty_cache()
    return out


def cpu_baseline(args, x, c, s, ws, bs):
    """The FP64 oracle's tiled two-pass evaluation (Algorithm 1) on a bounded sample of
    the workload: Step 1 and Step 2 of the one tile that holds the image centre."""
    import numpy as np
    import psutil
    from threadpoolctl import threadpool_info

    import oracle
    from oracle.loss import backward, forward, gram, style_seed, content_seed
    from oracle.plan import make_plan
    net = oracle.vgg19()
    w64 = [w.astype(np.float64) for w in ws]
    b64 = [b.astype(np.float64) for b in bs]
    plan = make_plan(args.H, args.W, args.T, args.m, net.strides(), net.align())
    k = next(i for i, t in enumerate(plan) if t.by0 <= args.H // 2 < t.by1 and t.bx0 <= args.W // 2 < t.bx1)
    t = plan[k]
    xw = x[:, t.ey0:t.ey1, t.ex0:t.ex1].astype(np.float64)
    strides = net.strides()
    ic = net.content
    f_c = np.zeros((net.convs[ic][1], (t.ey1 - t.ey0) // strides[ic], (t.ex1 - t.ex0) // strides[ic]))
    t0 = time.perf_counter()
    # Step 1: forward over the window, owned-feature Gram sums
    acts = forward(net, xw, w64, b64)
    sums = []
    for i in net.style:
        sy, sx = t.ey0 // strides[i], t.ex0 // strides[i]
        r0, r1, c0, c1 = t.own[i]
        v = acts[i][:, r0 - sy:r1 - sy, c0 - sx:c1 - sx].reshape(acts[i].shape[0], -1)
        sums.append(v @ v.T)
    t1 = time.perf_counter()
    # Step 2: forward again, seeds, reverse pass (the values of the global statistics do
    # not change the work; the tile's own sums stand in for them)
    acts = forward(net, xw, w64, b64)
    seeds = {}
    for k_, i in enumerate(net.style):
        n_p = acts[i][0].size
        seeds[i] = style_seed(acts[i], gram(acts[i], n_p), sums[k_] / n_p, 0.2, n_p)
    seeds[ic] = seeds.get(ic, 0.0) + content_seed(acts[ic], f_c, 1.0)
    backward(net, acts, seeds, w64)
    dt = time.perf_counter() - t0
    px = (t.by1 - t.by0) * (t.bx1 - t.bx0)
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    log(f"[bench] cpu oracle: tile {k} ({t.ey1 - t.ey0}x{t.ex1 - t.ex0} window, {px} owned px) in {dt:.1f}s "
        f"(Step 1 {t1 - t0:.1f}s) with {threads} BLAS threads")
    return {"value": round(px / dt / 1e6, 5), "unit": "Mpixel/s", "cores": threads, "kind": "oracle",
            "cpu_model": model, "physical_cores": psutil.cpu_count(logical=False),
            "logical_cpus": psutil.cpu_count(logical=True),
            "sample": f"FP64 oracle, Algorithm 1 Step 1 + Step 2 of tile {k} of {len(plan)} (the centre tile: "
                      f"{t.ey1 - t.ey0}x{t.ex1 - t.ex0} px window, {px} owned px) of the headline workload, "
                      f"{dt:.1f} s; rate = owned px / time"}


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
    ap.add_argument("--tile-batch", type=int, default=32, help="tiles per launch at most (48 tiles: 2 batches of 24)")
    ap.add_argument("--tile-batch-sweep", default="1,8,16",
                    help="other tile batches timed beside the headline (memory against speed; '' skips)")
    ap.add_argument("--ws-gib", type=float, default=200.0)
    ap.add_argument("--resident-steps", type=int, default=3,
                    help="steps of the same evaluation with every tile's activations resident (0 skips)")
    ap.add_argument("--one-window-steps", type=int, default=3,
                    help="steps of the same evaluation with the whole image as one window (0 skips)")
    ap.add_argument("--no-scales", action="store_true", help="skip the pyramid scales and the ragged tiling")
    ap.add_argument("--multiscale", default="none", choices=["none", "fast", "full", "both"],
                    help="also time whole style transfers (Algorithm 2, 4 scales, L-BFGS): SPST-fast "
                         "(600, 200, 66, 30 iterations), SPST (600, 300, 300, 300) or both")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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

    import numpy as np
    import torch

    import synth
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
    x, c, s = make_images(args.H, args.W, args.Hs, args.Ws, args.sigma)
    ws, bs = synth.vgg_weights(synth.VGG19_CONVS, synth.SEED_WEIGHTS)
    full = (args.H, args.W, args.Hs, args.Ws, args.T) == (6048, 8064, 4226, 5319, 1024)

    # headline: Algorithm 1, Step 2 recomputing each tile batch's forward
    ev = Eval(args.precision, ws, bs, x, c, s, args.T, args.m, tile_batch=args.tile_batch, ws_gib=args.ws_gib)
    log(f"[bench] {args.precision}: workspace {ev.workspace_gib():.1f} GiB (tile batches; Step 2 recomputes)")
    ms, stats, energy = ev.timed(args.steps, args.warmup, args.precision, profile=True)
    value = args.H * args.W / (ms * 1e-3) / 1e6
    peak = PEAK_TFLOPS[args.precision]
    executed = sum(st["flops"] for st in stats) / args.steps
    result = {
        "metric": METRIC, "value": round(value, 3), "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"loss+grad x {args.H}x{args.W}, style {args.Hs}x{args.Ws}, "
                               f"tiles {args.T} px margin {args.m} ({n_tiles} tiles), VGG-19 conv1_1..conv5_1",
                   "H": args.H, "W": args.W, "style_H": args.Hs, "style_W": args.Ws, "T": args.T, "m": args.m,
                   "tiles": n_tiles, "tile_batch": args.tile_batch, "style_weight": 0.2, "alpha": 1.0,
                   "step2": "recomputes each tile batch's forward (Algorithm 1)",
                   "workspace_gib": round(ev.workspace_gib(), 2)},
        "roofline": roofline(args.precision, stats, args.steps),
        # algorithmic FLOPs (both forwards, the data gradient, Grams, residual products; no
        # halo recompute, no padding) over the step time
        "effective_mfma_frac": round(FLOP_PER_PX * args.H * args.W / (ms * 1e-3) / 1e12 / peak, 4),
        # FLOPs the kernels execute (halo recompute included, padding not) over the step time
        "executed_mfma_frac": round(executed / (ms * 1e-3) / 1e12 / peak, 4),
        "executed_over_algorithmic": round(executed / (FLOP_PER_PX * args.H * args.W), 4),
        "kernels": [dict({k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()},
                         **kernel_frac(st, args.precision)) for st in stats],
        "energy": energy,
    }
    g_main = ev.grad.clone()
    if full:
        result["oracle_C3"] = {args.precision: golden_errors("C3", energy, g_main)}
    ev.close()

    if args.resident_steps > 0:
        ev = Eval(args.precision, ws, bs, x, c, s, args.T, args.m, resident=True, ws_gib=args.ws_gib)
        ms_r, _, _ = ev.timed(args.resident_steps, 1, f"{args.precision} resident")
        result["resident"] = {"ms_per_step": round(ms_r, 3), "value": round(args.H * args.W / (ms_r * 1e-3) / 1e6, 3),
                              "workspace_gib": round(ev.workspace_gib(), 2),
                              "step2": "reuses Step 1's activations (NST_RESIDENT)"}
        ev.close()

    if args.tile_batch_sweep:
        sweep = {}
        for tb in [int(v) for v in args.tile_batch_sweep.split(",") if v]:
            ev = Eval(args.precision, ws, bs, x, c, s, args.T, args.m, tile_batch=tb, ws_gib=args.ws_gib)
            ms_b, _, _ = ev.timed(3, 1, f"{args.precision} tile batch {tb}")
            sweep[str(tb)] = {"ms_per_step": round(ms_b, 3), "value": round(args.H * args.W / (ms_b * 1e-3) / 1e6, 3),
                              "workspace_gib": round(ev.workspace_gib(), 2)}
            ev.close()
        result["tile_batch_sweep"] = sweep

    if args.one_window_steps > 0:
        # the whole image as one window: a single tile (no margin inside the image, nothing
        # recomputed; Step 1 keeps its activations for Step 2), which one GPU's HBM holds
        T1 = max(args.H, args.W)
        ev = Eval(args.precision, ws, bs, x, c, s, T1, args.m, resident=True, tile_batch=1, ws_gib=args.ws_gib)
        ms_w, _, e_w = ev.timed(args.one_window_steps, 1, f"{args.precision} one window")
        dg = float((g_main.double() - ev.grad.double()).norm() / g_main.double().norm())
        result["one_window"] = {"ms_per_step": round(ms_w, 3), "value": round(args.H * args.W / (ms_w * 1e-3) / 1e6, 3),
                                "T": T1, "tiles": 1, "workspace_gib": round(ev.workspace_gib(), 2),
                                "energy_rel_diff_vs_tiled": abs(e_w[0] - energy[0]) / abs(energy[0]),
                                "grad_vector_rel_diff_vs_tiled": float("%.4e" % dg)}
        ev.close()

    if args.fp32_steps > 0 and args.precision != "fp32":
        ev = Eval("fp32", ws, bs, x, c, s, args.T, args.m, tile_batch=args.tile_batch, ws_gib=args.ws_gib)
        ms32, _, e32 = ev.timed(args.fp32_steps, 1, "fp32")
        dg = float((g_main.double() - ev.grad.double()).norm() / ev.grad.double().norm())
        result["fp32"] = {"value": round(args.H * args.W / (ms32 * 1e-3) / 1e6, 3), "ms_per_step": round(ms32, 3),
                          "step2": "recomputes each tile batch's forward (Algorithm 1)",
                          "speedup_of_bf16": round(ms32 / ms, 3),
                          "energy_rel_diff_bf16_vs_fp32": abs(energy[0] - e32[0]) / abs(e32[0]),
                          "grad_vector_rel_diff_bf16_vs_fp32": float("%.4e" % dg)}
        if full:
            result["oracle_C3"]["fp32"] = golden_errors("C3", e32, ev.grad)
        ev.close()
    del g_main

    if not args.no_scales and full:
        # the content pyramid of the Fig. 1 experiment (x and c box-downsampled by 2, 4, 8;
        # the style image keeps its size) and the ragged 1000 px tiling of a 3024 x 4032 image
        scales = {}
        xs, cs = x, c
        for lev in range(1, 4):
            xs, cs = synth.box_down2(xs), synth.box_down2(cs)
            h, w = xs.shape[1:]
            ev = Eval(args.precision, ws, bs, xs, cs, s, args.T, args.m, ws_gib=args.ws_gib)
            ms_l, _, _ = ev.timed(3, 1, f"{args.precision} {h}x{w}")
            scales[f"{h}x{w}"] = {"ms_per_step": round(ms_l, 3), "value": round(h * w / (ms_l * 1e-3) / 1e6, 3),
                                  "tiles": len(plan(vgg19_desc(), h, w, args.T, args.m))}
            ev.close()
        result["pyramid"] = scales
        x4, c4, s4 = make_images(3024, 4032, 2000, 2000, 16.0)
        rag = {"workload": "x, content 3024x4032, style 2000x2000, tiles 1000 px margin 155 (ragged 24/32 px strips)",
               "tiles": len(plan(vgg19_desc(), 3024, 4032, 1000, 155))}
        for prec, steps in ((args.precision, 3), ("fp32", 1)):
            ev = Eval(prec, ws, bs, x4, c4, s4, 1000, 155, ws_gib=args.ws_gib)
            ms4, _, e4 = ev.timed(steps, 1, f"{prec} ragged 3024x4032")
            rag[prec] = {"ms_per_step": round(ms4, 3), "value": round(3024 * 4032 / (ms4 * 1e-3) / 1e6, 3),
                         "oracle_C4": golden_errors("C4", e4, ev.grad)}
            ev.close()
        result["ragged"] = rag

    if args.multiscale != "none":
        result["multiscale"] = multiscale_runs(args, ws, bs, x, c, s)

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args, x, c, s, ws, bs)
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
