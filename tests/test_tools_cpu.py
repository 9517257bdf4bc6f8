"""CPU tests of the benchmark's command-line contract and the rocprofv3 summary
parser (no GPU needed)."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def _write_csv(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_profile_summary(tmp_path):
    from paper_1609_00958_amd import profiling
    trace = tmp_path / "trace"
    fetch = tmp_path / "fetch"
    write = tmp_path / "write"
    for d in (trace, fetch, write):
        d.mkdir()
    _write_csv(trace / "x_kernel_stats.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs"], [
        ["void gjp::fwd_kernel<float, 0, false>(gjp::FwdArgs)", 2, 20e6, 10e6],
        ["void gjp::adj_gather_sep_kernel<0>(...)", 4, 8e6, 2e6],
        ["__amd_rocclr_copyBuffer", 1, 1e5, 1e5],
    ])
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    gib_kib = float(1 << 20)
    _write_csv(fetch / "x_counter_collection.csv", hdr, [
        [1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", gib_kib / 4], [1, "__amd_rocclr_copyBuffer",
                                                                   "FETCH_SIZE", gib_kib / 4],
        [2, "void gjp::fwd_kernel<float, 0, false>(gjp::FwdArgs)", "FETCH_SIZE", 1000.0],
    ])
    _write_csv(write / "x_counter_collection.csv", hdr, [
        [1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", gib_kib],
        [2, "void gjp::fwd_kernel<float, 0, false>(gjp::FwdArgs)", "WRITE_SIZE", 10.0],
    ])
    stats = profiling.kernel_stats(str(trace))
    assert stats["forward_f32"]["avg_ms"] == 10.0
    assert stats["adjoint_gather"]["calls"] == 4
    f, fs = profiling.scaled_traffic(str(fetch))
    w, ws = profiling.scaled_traffic(str(write))
    # the copy reads as half a GiB on FETCH: factor 2
    assert fs == 2.0 and ws == 1.0
    assert f["forward_f32"] == 1000.0 * 1024 * 2.0
    assert w["forward_f32"] == 10.0 * 1024
    out_md = tmp_path / "s.md"
    out_js = tmp_path / "s.json"
    subprocess.check_call([sys.executable, "-m", "paper_1609_00958_amd.profiling", "--trace",
                           str(trace), "--fetch", str(fetch), "--write", str(write), "--label",
                           "t", "--command", "c", "--out-md", str(out_md), "--out-json",
                           str(out_js)], cwd=ROOT, stdout=subprocess.DEVNULL, timeout=300)
    data = json.loads(out_js.read_text())
    assert data["source_sha256"] == profiling.source_hash()
    assert data["kernels"]["forward_f32"]["fetch_bytes_per_launch"] == 1000.0 * 1024 * 2.0



def test_profile_last_dispatches(tmp_path):
    """--last N averages the final N dispatches of each kernel (after set-up
    launches such as autotuning trials)."""
    from paper_1609_00958_amd import profiling
    trace = tmp_path / "trace"
    trace.mkdir()
    fwd = "void gjp::fwd_pair_kernel<gjp::bf16_t, 0, false, 2>(gjp::FwdArgs)"
    rows = [[i, fwd, 1000 * i, 1000 * i + d] for i, d in enumerate([900, 50, 70, 100, 100])]
    rows.append([9, "elementwise_kernel<...>", 0, 5])
    _write_csv(trace / "x_kernel_trace.csv",
               ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    stats = profiling.kernel_stats_last(str(trace), 2)
    assert list(stats) == ["forward_bf16_pairs"]
    assert stats["forward_bf16_pairs"]["calls"] == 2
    assert abs(stats["forward_bf16_pairs"]["avg_ms"] - 100e-6) < 1e-12
    assert profiling.kernel_stats_last(str(trace), 10)["forward_bf16_pairs"]["calls"] == 5


def test_profile_kernel_names():
    from paper_1609_00958_amd import profiling
    want = {
        "void gjp::fwd_kernel<float, 0, false>(gjp::FwdArgs)": "forward_f32",
        "void gjp::fwd_kernel<gjp::bf16_t, 0, false>(gjp::FwdArgs)": "forward_bf16",
        "void gjp::batched_fwd_kernel<float, 0, false>(gjp::BatchInst const*)": "batched",
        "void gjp::naive_fwd_kernel<float, 0>(gjp::GridGeom, double const*)": "forward_naive_f32",
        "void gjp::naive_fwd_kernel<gjp::f16_t, 1>(gjp::GridGeom)": "forward_naive_f16",
        "void gjp::batched_pad_kernel(gjp::BatchInst const*)": "batched_pad",
        "void gjp::fwd_pair_kernel<gjp::f16_t, 0, false, 2>(gjp::FwdArgs)": "forward_f16_pairs",
        "void gjp::fwd_kernel<gjp::f16_t, 0, false, 4>(gjp::FwdArgs)": "forward_f16",
        "void gjp::pad_kernel<unsigned int>(unsigned int const*)": "pad",
        "void gjp::adj_gather_sep_kernel<0>(gjp::GridGeom)": "adjoint_gather",
        "elementwise_kernel<...>": None,
    }
    for name, short in want.items():
        assert profiling.short_name(name) == short, name
