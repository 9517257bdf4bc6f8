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


def test_profile_counter_table(tmp_path):
    from paper_1609_00958_amd import profiling
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    k = "void gjp::fwd_kernel<float, 0, false, 4>(gjp::FwdArgs)"
    d1, d2 = tmp_path / "a", tmp_path / "b"
    d1.mkdir()
    d2.mkdir()
    # two dispatches; the last one counts: 100 waves, 5000 VALU, 50 loads
    _write_csv(d1 / "x_counter_collection.csv", hdr, [
        [1, k, "SQ_WAVES", 1.0], [1, k, "SQ_INSTS_VALU", 1.0], [1, k, "SQ_INSTS_VMEM_RD", 1.0],
        [2, k, "SQ_WAVES", 60.0], [2, k, "SQ_WAVES", 40.0], [2, k, "SQ_INSTS_VALU", 5000.0],
        [2, k, "SQ_INSTS_VMEM_RD", 50.0]])
    _write_csv(d2 / "x_counter_collection.csv", hdr, [
        [7, k, "TA_TA_BUSY_sum", 8.0e5], [7, k, "GRBM_GUI_ACTIVE", 8000.0]])
    st = profiling.counters_last([str(d1), str(d2)], 1)
    assert st["forward_f32"]["SQ_WAVES"] == 100.0
    rows = {r.split("|")[1].strip(): r.split("|")[2].strip()
            for r in profiling.counter_table(st)[2:]}
    assert rows["VALU instr / wave"] == "50"
    assert rows["load instr / wave"] == "0.5"
    # TA busy per CU: 8 * 8e5 / 8000 / 256 = 3.125 (a synthetic ratio)
    assert rows["address unit busy (TA)"] == "3.12"
    assert rows["L2 hit rate"] == "-"


def test_source_hash_ignores_comments():
    from paper_1609_00958_amd import profiling
    a = "int f(int x) {  // first\n  return x + 1; /* two\n lines */\n}\n"
    b = "// header\nint f(int x) {\n\n  return x + 1;\n}\n"
    c = "int f(int x) {\n  return x + 2;\n}\n"
    assert profiling._code_only(a) == profiling._code_only(b)
    assert profiling._code_only(a) != profiling._code_only(c)
