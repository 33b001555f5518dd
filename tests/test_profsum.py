"""Host logic of the rocprofv3 summaries (paper_2212_13459_amd.profsum) on synthetic
counter and trace files."""
import csv
import os

from paper_2212_13459_amd import profsum

K = "void nst::k_conv2<__bf16, 256, 2, 2, 0, false>(nst::ConvArgs, nst::Batch)"
K_MANGLED = "_ZN3nst7k_conv2IDF16bLi256ELi2ELi2ELi0ELb0EEEvNS_8ConvArgsENS_5BatchE"
COPY = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda(...)>"


def _counters(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for d, (k, v) in enumerate(rows):
            w.writerow([d + 1, k, counter, v])


def test_demangle_bf16_names():
    m = profsum.demangle([K_MANGLED, "plain"])
    assert m[K_MANGLED] == K
    assert m["plain"] == "plain"


def test_traffic_scaled_by_copy_kernel(tmp_path):
    copy_bytes = 1 << 30
    # the fetch counter reads half of the copy's bytes, the write counter all of them
    _counters(tmp_path / "f", "FETCH_SIZE",
              [(COPY, copy_bytes / 2048)] + [(K_MANGLED, 100.0)] * 3 + [(K_MANGLED, 10.0)] * 2)
    _counters(tmp_path / "w", "WRITE_SIZE",
              [(COPY, copy_bytes / 1024)] + [(K_MANGLED, 7.0)] * 3 + [(K_MANGLED, 5.0)] * 2)
    res = profsum.traffic(str(tmp_path / "f"), str(tmp_path / "w"), K, copy_bytes, last=2)
    assert abs(res["fetch"]["scale"] - 2.0) < 1e-12 and abs(res["write"]["scale"] - 1.0) < 1e-12
    assert res["fetch"]["dispatches"] == 2
    assert res["fetch"]["bytes_per_launch"] == 10.0 * 2 * 1024
    assert res["write"]["bytes_per_launch"] == 5.0 * 1024
    out = tmp_path / "prof"
    out.mkdir()
    profsum.write_traffic(res, copy_bytes, "cmd f", "cmd w", str(out / "k_traffic.txt"))
    got = profsum.read_traffic(str(out), K)
    assert got is not None and got[0] == (10.0 * 2 + 5.0) * 1024
    # a summary taken on other kernel sources is not used
    text = (out / "k_traffic.txt").read_text().replace(profsum.source_digest(), "0" * 16)
    (out / "k_traffic.txt").write_text(text)
    assert profsum.read_traffic(str(out), K) is None


def test_stats_tail_average(tmp_path):
    with open(tmp_path / "b_kernel_stats.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs"])
        w.writerow([K_MANGLED, 4, 10e6, 2.5e6, 90.0, 1e6, 4e6])
    with open(tmp_path / "b_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for i, d in enumerate([1e6, 4e6, 2e6, 3e6]):
            w.writerow([K_MANGLED, 100 * i * 10**6, int(100 * i * 10**6 + d)])
    text = profsum.stats(str(tmp_path), 5, "cmd", K, 2)
    assert K in text
    assert "mean of the last 2" in text and "2.5000 ms" in text
