"""Text summaries of rocprofv3 output for the kernels of libnst.

    python -m paper_2212_13459_amd.profsum stats  STATS_CSV [--top N] [--cmd "..."]
    python -m paper_2212_13459_amd.profsum traffic FETCH_OUT WRITE_OUT --kernel NAME
           --copy-bytes B [--cmd-fetch "..."] [--cmd-write "..."]
    python -m paper_2212_13459_amd.profsum counters PMC_OUT [--last N] [--cmd "..."]

``stats`` formats a ``--kernel-trace --stats`` kernel_stats.csv.  ``traffic`` turns two
``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs (counter_collection.csv or *_results.db)
into HBM bytes per launch of one kernel.  Each counter is scaled by what it reads for a
plain copy kernel of B bytes read and B bytes written in the same run (the
elementwise negation kernel that bench.py --copy-calibration-mib launches), so that the
figure is in the same units as the algorithmic bytes.  The summary records a digest of
the kernel sources; bench.py reports the traffic only while the digest still matches.
"""
import argparse
import collections
import csv
import glob
import hashlib
import os
import re
import sqlite3
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ("csrc/kernels.hip", "csrc/kernels.h", "csrc/nst_api.cpp")
COPY_KERNEL = "neg_kernel"


def demangle(names):
    """Demangled kernel names.  The demanglers here do not know the __bf16 code DF16b;
    it is read as the half-precision code Dh (like it, a builtin type that takes no
    substitution slot, so later back-references keep their meaning) and the type name
    is written back, which gives the text of the library's own profile records."""
    names = list(names)
    todo = [n for n in names if n.startswith("_Z")]
    if not todo:
        return {n: n for n in names}
    out = subprocess.run(["c++filt"], input="\n".join(t.replace("DF16b", "Dh") for t in todo),
                         capture_output=True, text=True, check=True).stdout.split("\n")
    out = [re.sub(r"\bhalf\b", "__bf16", o) for o in out]
    m = {n: n for n in names}
    m.update(zip(todo, out))
    return m


def source_digest():
    h = hashlib.sha256()
    for rel in SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _find(path, pattern):
    if os.path.isfile(path):
        return path
    hits = sorted(glob.glob(os.path.join(path, "**", pattern), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no {pattern} under {path}")
    return hits[0]


def read_counters(path):
    """{kernel name: {counter: [value per dispatch, in dispatch order]}} from a --pmc run."""
    out = collections.defaultdict(lambda: collections.defaultdict(dict))
    try:
        f = _find(path, "*counter_collection.csv")
        with open(f) as fh:
            for row in csv.DictReader(fh):
                out[row["Kernel_Name"]][row["Counter_Name"]][int(row["Dispatch_Id"])] = \
                    out[row["Kernel_Name"]][row["Counter_Name"]].get(int(row["Dispatch_Id"]), 0.0) + \
                    float(row["Counter_Value"])
    except FileNotFoundError:
        f = _find(path, "*_results.db")
        con = sqlite3.connect(f)
        q = ("select coalesce(s.kernel_name, k.kernel_name), k.counter_name, k.value, k.dispatch_id "
             "from counters_collection k left join kernel_symbols s on s.kernel_id = k.kernel_id")
        for k, c, v, d in con.execute(q):
            k = k[:-3] if k.endswith(".kd") else k
            out[k][c][d] = out[k][c].get(d, 0.0) + float(v)
    dm = demangle(out)
    return {dm[k]: {c: [d[i] for i in sorted(d)] for c, d in cs.items()} for k, cs in out.items()}


def durations(path):
    """{kernel: [duration ns per dispatch, in dispatch order]} of a --pmc rocpd database."""
    con = sqlite3.connect(_find(path, "*_results.db"))
    q = ("select coalesce(s.kernel_name, k.kernel_name), k.dispatch_id, max(k.duration) from counters_collection k "
         "left join kernel_symbols s on s.kernel_id = k.kernel_id group by k.dispatch_id")
    out = collections.defaultdict(dict)
    for k, d, du in con.execute(q):
        out[k[:-3] if k.endswith(".kd") else k][d] = float(du)
    dm = demangle(out)
    return {dm[k]: [v[i] for i in sorted(v)] for k, v in out.items()}


def counters(path, last, cmd, top=20):
    """Per kernel, over its last ``last`` dispatches: duration, shader clock, MFMA-busy
    fraction, LDS bank-conflict rate (a pass with SQ_VALU_MFMA_BUSY_CYCLES, SQ_BUSY_CYCLES,
    SQ_LDS_BANK_CONFLICT, SQ_LDS_IDX_ACTIVE, GRBM_GUI_ACTIVE).  GRBM_GUI_ACTIVE sums the
    8 XCDs' busy clocks, so clock = GRBM_GUI_ACTIVE / 8 / duration, and the MFMA units'
    busy fraction = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 x 256 CUs x 4 SIMDs)."""
    cs, du = read_counters(path), durations(path)
    rows = []
    for k, c in cs.items():
        d = du.get(k, [])
        if not d or "GRBM_GUI_ACTIVE" not in c:
            continue
        n = min(last, len(d))
        mean = lambda name: sum(c.get(name, [0])[-n:]) / n  # noqa: E731
        dur = sum(d[-n:]) / n
        g = mean("GRBM_GUI_ACTIVE") / 8.0
        rows.append((sum(d), k, len(d), dur, g / dur, mean("SQ_VALU_MFMA_BUSY_CYCLES") / (g * 1024.0),
                     mean("SQ_LDS_BANK_CONFLICT") / max(mean("SQ_LDS_IDX_ACTIVE"), 1.0)))
    rows.sort(key=lambda r: -r[0])
    lines = [f"command: {cmd}", "", f"Means over each kernel's last {last} dispatches.", "",
             "| kernel | dispatches | mean ms | shader clock GHz | MFMA busy | LDS bank-conflict cycles / LDS cycles |",
             "|---|---:|---:|---:|---:|---:|"]
    for _, k, nd, dur, clk, mfma, lds in rows[:top]:
        lines.append(f"| `{k[:100]}` | {nd} | {dur / 1e6:.4f} | {clk:.2f} | {mfma:.3f} | {lds:.3f} |")
    return "\n".join(lines) + "\n"


def _pick(counters, needle):
    names = [k for k in counters if needle in k]
    if not names:
        raise KeyError(f"kernel {needle!r} not in the counter output ({len(counters)} kernels)")
    return max(names, key=lambda k: len(next(iter(counters[k].values()))))


def traffic(fetch_path, write_path, kernel, copy_bytes, last=0):
    """HBM bytes per launch of ``kernel``, averaged over its last ``last`` dispatches (all
    of them if 0)."""
    fc, wc = read_counters(fetch_path), read_counters(write_path)
    res = {}
    for tag, cs, cname in (("fetch", fc, "FETCH_SIZE"), ("write", wc, "WRITE_SIZE")):
        k = _pick(cs, kernel)
        cp = _pick(cs, COPY_KERNEL)
        vals, cvals = cs[k][cname], cs[cp][cname]
        if last:
            vals = vals[-last:]
        per = sum(vals) / len(vals)
        cper = sum(cvals) / len(cvals)
        scale = copy_bytes / 1024.0 / cper
        res[tag] = dict(kernel=kernel, rocprof_name=k, dispatches=len(vals), kib_per_dispatch=per, copy_kib=cper,
                        copy_kernel=cp, scale=scale, bytes_per_launch=per * scale * 1024.0)
    return res


def write_traffic(res, copy_bytes, cmd_fetch, cmd_write, out):
    f, w = res["fetch"], res["write"]
    total = f["bytes_per_launch"] + w["bytes_per_launch"]
    lines = [
        f"# HBM traffic of {f['kernel']}",
        "",
        f"command (FETCH_SIZE): {cmd_fetch}",
        f"command (WRITE_SIZE): {cmd_write}",
        "",
        f"kernel: {f['kernel']}",
        f"rocprof kernel name: {f['rocprof_name']}",
        f"source_digest: {source_digest()}",
        f"dispatches averaged (the last ones, the benchmark's loss+gradient evaluations): {f['dispatches']}",
        f"FETCH_SIZE KiB per dispatch (raw): {f['kib_per_dispatch']:.1f}",
        f"WRITE_SIZE KiB per dispatch (raw): {w['kib_per_dispatch']:.1f}",
        f"copy kernel: {f['copy_kernel']} reading and writing {copy_bytes} bytes per dispatch",
        f"copy FETCH_SIZE KiB (raw): {f['copy_kib']:.1f}  scale {f['scale']:.4f}",
        f"copy WRITE_SIZE KiB (raw): {w['copy_kib']:.1f}  scale {w['scale']:.4f}",
        f"fetch_bytes_per_launch: {f['bytes_per_launch']:.0f}",
        f"write_bytes_per_launch: {w['bytes_per_launch']:.0f}",
        f"traffic_bytes_per_launch: {total:.0f}",
    ]
    text = "\n".join(lines) + "\n"
    if out:
        with open(out, "w") as fh:
            fh.write(text)
    return text


def read_traffic(profiles_dir, kernel):
    """HBM bytes per launch of ``kernel`` from a summary whose digest matches the current
    sources, else None."""
    dig = source_digest()
    for p in sorted(glob.glob(os.path.join(profiles_dir, "*traffic*.txt"))):
        kv = {}
        with open(p) as fh:
            for line in fh:
                if ": " in line and not line.startswith("#"):
                    a, b = line.rstrip("\n").split(": ", 1)
                    kv[a] = b
        if kv.get("kernel") == kernel and kv.get("source_digest") == dig:
            return float(kv["traffic_bytes_per_launch"]), os.path.basename(p)
    return None


def dispatches(path):
    """[(demangled kernel name, start ns, duration ns)] in start order, from a kernel trace:
    kernel_trace.csv or a rocpd database (*_results.db)."""
    out = []
    try:
        f = _find(path, "*kernel_trace.csv")
        with open(f) as fh:
            for r in csv.DictReader(fh):
                out.append((r["Kernel_Name"], int(r["Start_Timestamp"]),
                            int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    except FileNotFoundError:
        # the mangled symbol name (rocprofv3's own demangled name garbles a __bf16 argument)
        con = sqlite3.connect(_find(path, "*_results.db"))
        q = ("select coalesce(s.kernel_name, k.name), k.start, k.end from kernels k "
             "left join kernel_symbols s on s.kernel_id = k.kernel_id")
        out = [(n[:-3] if n.endswith(".kd") else n, int(a), int(b) - int(a)) for n, a, b in con.execute(q)]
    dm = demangle({n for n, _, _ in out})
    return sorted(((dm[n], a, d) for n, a, d in out), key=lambda r: r[1])


def last_dispatches(path, kernel, n):
    """Mean duration (ms) of the last n dispatches of ``kernel``."""
    d = [x for x in dispatches(path) if kernel in x[0]]
    tail = [x[2] for x in d[-n:]]
    return len(d), sum(tail) / len(tail) / 1e6


def _agg(path):
    """Per kernel: calls, total, average, min, max (ns) and percentage of the summed time."""
    try:
        f = _find(path, "*kernel_stats.csv")
        with open(f) as fh:
            rows = list(csv.DictReader(fh))
        dm = demangle({r["Name"] for r in rows})
        return [(dm[r["Name"]], int(r["Calls"]), float(r["TotalDurationNs"]), float(r["AverageNs"]),
                 float(r["MinNs"]), float(r["MaxNs"]), float(r["Percentage"])) for r in rows]
    except FileNotFoundError:
        agg = collections.OrderedDict()
        for name, _, d in dispatches(path):
            agg.setdefault(name, []).append(d)
        tot = sum(sum(v) for v in agg.values()) or 1.0
        return [(k, len(v), float(sum(v)), sum(v) / len(v), float(min(v)), float(max(v)), 100.0 * sum(v) / tot)
                for k, v in agg.items()]


def stats(path, top, cmd, kernel="", last=0):
    rows = sorted(_agg(path), key=lambda r: -r[2])
    lines = [f"command: {cmd}", "",
             "| kernel | calls | total ms | average ms | min ms | max ms | % |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for name, calls, tot, avg, mn, mx, pct in rows[:top]:
        lines.append(f"| `{name[:110]}` | {calls} | {tot / 1e6:.3f} | {avg / 1e6:.4f} | {mn / 1e6:.4f} | "
                     f"{mx / 1e6:.4f} | {pct:.2f} |")
    if kernel and last:
        total, avg = last_dispatches(path, kernel, last)
        lines += ["", f"`{kernel}`: {total} dispatches in the run; mean of the last {last} "
                      f"(the last evaluations, all of the benchmark's configuration): {avg:.4f} ms"]
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("path")
    s.add_argument("--top", type=int, default=25)
    s.add_argument("--cmd", default="")
    s.add_argument("--kernel", default="")
    s.add_argument("--last", type=int, default=0)
    t = sub.add_parser("traffic")
    t.add_argument("fetch")
    t.add_argument("write")
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--cmd-fetch", default="")
    t.add_argument("--cmd-write", default="")
    t.add_argument("--out", default="")
    t.add_argument("--last", type=int, default=0)
    c = sub.add_parser("counters")
    c.add_argument("path")
    c.add_argument("--last", type=int, default=8)
    c.add_argument("--cmd", default="")
    c.add_argument("--top", type=int, default=20)
    a = ap.parse_args(argv)
    if a.mode == "counters":
        sys.stdout.write(counters(a.path, a.last, a.cmd, a.top))
    elif a.mode == "stats":
        sys.stdout.write(stats(a.path, a.top, a.cmd, a.kernel, a.last))
    else:
        res = traffic(a.fetch, a.write, a.kernel, a.copy_bytes, a.last)
        sys.stdout.write(write_traffic(res, a.copy_bytes, a.cmd_fetch, a.cmd_write, a.out))


if __name__ == "__main__":
    main()
