"""Summaries of rocprofv3 output for the projector's kernels.

    python -m paper_1609_00958_amd.profiling --trace DIR [--fetch DIR --write DIR]
        --label NAME --command "..." --out-md FILE [--out-json FILE]

`--trace` is the output directory of `rocprofv3 --kernel-trace --stats
--output-format csv`; `--fetch` / `--write` are those of two `rocprofv3 --pmc
FETCH_SIZE` and `--pmc WRITE_SIZE` runs. Hardware byte counters are scaled by
what the same counter reads for a plain device-to-device copy of 1 GiB found in
the same run (the benchmark's `--calibrate-copy` option issues one), and
reported per launch. The JSON output records a hash of the kernel sources so
that a reader can tell whether the counters still describe the current code.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/gjp_kernels.hip", "csrc/gjp_ray.h")

# First match wins: the longer kernel names come before their substrings.
SHORT = (
    ("naive_fwd_kernel<float", "forward_naive_f32"),
    ("naive_fwd_kernel<gjp::bf16_t", "forward_naive_bf16"),
    ("naive_fwd_kernel<gjp::f16_t", "forward_naive_f16"),
    ("fwd_pair_kernel<gjp::bf16_t", "forward_bf16_pairs"),
    ("fwd_pair_kernel<gjp::f16_t", "forward_f16_pairs"),
    ("fwd_triple_kernel<float", "forward_f32_triples"),
    ("fwd_triple_kernel<gjp::bf16_t", "forward_bf16_triples"),
    ("fwd_triple_kernel<gjp::f16_t", "forward_f16_triples"),
    ("batched_fwd_kernel", "batched"),
    ("batched_pad_kernel", "batched_pad"),
    ("fwd_kernel<float", "forward_f32"),
    ("fwd_kernel<gjp::bf16_t", "forward_bf16"),
    ("fwd_kernel<gjp::f16_t", "forward_f16"),
    ("adj_value_table_kernel", "adjoint_table"),
    ("adj_gather_sep_kernel", "adjoint_gather"),
    ("adj_splat_kernel", "adjoint_gather"),
    ("adj_table_kernel", "adjoint_table"),
    ("pad_kernel", "pad"),
    ("__amd_rocclr_copyBuffer", "copy"),
)


def short_name(name: str):
    for key, short in SHORT:
        if key in name:
            return short
    return None


def _code_only(text: str) -> str:
    """Source text without comments and blank lines, so that editing a comment
    does not mark measured byte counts as stale."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = []
    for line in text.splitlines():
        line = re.sub(r"//.*$", "", line).rstrip()
        if line.strip():
            out.append(line)
    return "\n".join(out)


def source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()


def _one(dirpath: str, suffix: str) -> str:
    hits = glob.glob(os.path.join(dirpath, "**", "*" + suffix), recursive=True)
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {dirpath}")
    return sorted(hits)[0]


def kernel_stats(trace_dir: str):
    out = {}
    with open(_one(trace_dir, "kernel_stats.csv")) as f:
        for row in csv.DictReader(f):
            s = short_name(row["Name"])
            if s is None:
                continue
            calls = int(row["Calls"])
            total = float(row["TotalDurationNs"])
            cur = out.setdefault(s, {"calls": 0, "total_ns": 0.0})
            cur["calls"] += calls
            cur["total_ns"] += total
    for v in out.values():
        v["avg_ms"] = v["total_ns"] / max(v["calls"], 1) / 1e6
    return out


def counter_per_dispatch(pmc_dir: str):
    """{dispatch id: (kernel name, summed counter value)} of one --pmc run."""
    vals = collections.OrderedDict()
    with open(_one(pmc_dir, "counter_collection.csv")) as f:
        for row in csv.DictReader(f):
            d = int(row["Dispatch_Id"])
            name, v = vals.get(d, (row["Kernel_Name"], 0.0))
            vals[d] = (name, v + float(row["Counter_Value"]))
    return vals


def scaled_traffic(pmc_dir: str, ref_bytes: float = float(1 << 30), last: int = 0):
    """Average scaled bytes per dispatch per kernel (over each kernel's last
    `last` dispatches if last > 0), and the copy scale factor."""
    vals = counter_per_dispatch(pmc_dir)
    ref = [v for (n, v) in vals.values() if short_name(n) == "copy"]
    if not ref:
        raise RuntimeError("no reference copy dispatch in " + pmc_dir)
    ref_kib = max(ref)
    scale = (ref_bytes / 1024.0) / ref_kib
    acc = collections.defaultdict(list)
    for d in sorted(vals):
        n, v = vals[d]
        s = short_name(n)
        if s and s != "copy":
            acc[s].append(v * 1024.0 * scale)
    if last > 0:
        acc = {k: v[-last:] for k, v in acc.items()}
    return {k: sum(v) / len(v) for k, v in acc.items()}, scale


def kernel_stats_last(trace_dir: str, n: int):
    """Per-kernel average over the last n dispatches of each kernel (from the
    per-dispatch trace), so that set-up launches such as autotuning trials
    before the timed steps do not enter the averages."""
    runs = collections.defaultdict(list)
    with open(_one(trace_dir, "kernel_trace.csv")) as f:
        for row in csv.DictReader(f):
            s = short_name(row["Kernel_Name"])
            if s is None:
                continue
            t0, t1 = int(row["Start_Timestamp"]), int(row["End_Timestamp"])
            runs[s].append((t0, t1 - t0))
    out = {}
    for s, v in runs.items():
        v.sort()
        last = v[-n:]
        total = float(sum(d for _, d in last))
        out[s] = {"calls": len(last), "total_ns": total, "avg_ms": total / len(last) / 1e6}
    return out


def counters_last(dirs, n: int):
    """{kernel: {counter: average over the kernel's last n dispatches}} from
    one or more --pmc runs of the same program (each run one pass)."""
    out = collections.defaultdict(dict)
    for d in dirs:
        per = collections.defaultdict(lambda: collections.defaultdict(float))
        names = {}
        with open(_one(d, "counter_collection.csv")) as f:
            for row in csv.DictReader(f):
                s = short_name(row["Kernel_Name"])
                if s is None:
                    continue
                disp = int(row["Dispatch_Id"])
                names[disp] = s
                per[disp][row["Counter_Name"]] += float(row["Counter_Value"])
        by_kernel = collections.defaultdict(list)
        for disp in sorted(per):
            by_kernel[names[disp]].append(per[disp])
        for k, runs in by_kernel.items():
            last = runs[-n:]
            for c in last[0]:
                out[k][c] = sum(r.get(c, 0.0) for r in last) / len(last)
    return out


# Derived figures of the counter table: (label, function of the counters).
# GRBM_GUI_ACTIVE sums the eight XCDs' clocks; per-CU unit counters sum 256 CUs.
DERIVED = (
    ("VALU instr / wave", lambda c: c["SQ_INSTS_VALU"] / c["SQ_WAVES"]),
    ("load instr / wave", lambda c: c["SQ_INSTS_VMEM_RD"] / c["SQ_WAVES"]),
    ("LDS instr / wave", lambda c: c["SQ_INSTS_LDS"] / c["SQ_WAVES"]),
    ("VALU issue (2 cycles / wave instr)",
     lambda c: 2.0 * c["SQ_INSTS_VALU"] / (1024.0 * c["GRBM_GUI_ACTIVE"] / 8.0)),
    ("address unit busy (TA)", lambda c: 8.0 * c["TA_TA_BUSY_sum"] / c["GRBM_GUI_ACTIVE"] / 256.0),
    ("data unit busy (TD)", lambda c: 8.0 * c["TD_TD_BUSY_sum"] / c["GRBM_GUI_ACTIVE"] / 256.0),
    ("TA cycles / load instr", lambda c: c["TA_TA_BUSY_sum"] / c["SQ_INSTS_VMEM_RD"]),
    ("L1 tag accesses / load instr",
     lambda c: c["TCP_TOTAL_CACHE_ACCESSES_sum"] / c["SQ_INSTS_VMEM_RD"]),
    ("L1 -> L2 requests / L1 access",
     lambda c: c["TCP_TCC_READ_REQ_sum"] / c["TCP_TOTAL_CACHE_ACCESSES_sum"]),
    ("L2 hit rate", lambda c: c["TCC_HIT_sum"] / (c["TCC_HIT_sum"] + c["TCC_MISS_sum"])),
)


def counter_table(stats):
    kernels = sorted(stats)
    lines = ["| figure | " + " | ".join(kernels) + " |",
             "|---|" + "---|" * len(kernels)]
    for label, fn in DERIVED:
        cells = []
        for k in kernels:
            try:
                cells.append(f"{fn(stats[k]):.3g}")
            except (KeyError, ZeroDivisionError):
                cells.append("-")
        lines.append(f"| {label} | " + " | ".join(cells) + " |")
    return lines


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--label", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--out-md", required=True)
    ap.add_argument("--out-json")
    ap.add_argument("--last", type=int, default=0,
                    help="average only the last N dispatches of each kernel")
    ap.add_argument("--counters", nargs="*", default=[],
                    help="--pmc run directories: adds a table of derived counter figures")
    a = ap.parse_args()
    stats = kernel_stats_last(a.trace, a.last) if a.last > 0 else kernel_stats(a.trace)
    fetch = write = None
    fscale = wscale = None
    if a.fetch and a.write:
        fetch, fscale = scaled_traffic(a.fetch, last=a.last)
        write, wscale = scaled_traffic(a.write, last=a.last)
    head = "launches" if a.last <= 0 else f"launches (last {a.last})"
    lines = [f"# {a.label}", "", "Command(s):", "", "```", a.command, "```", "",
             f"| kernel | {head} | avg ms / launch | HBM fetch GB / launch | "
             "HBM write GB / launch |",
             "|---|---|---|---|---|"]
    for k in sorted(stats, key=lambda k: -stats[k]["total_ns"]):
        f = f"{fetch[k] / 1e9:.3f}" if fetch and k in fetch else "-"
        w = f"{write[k] / 1e9:.3f}" if write and k in write else "-"
        lines.append(f"| {k} | {stats[k]['calls']} | {stats[k]['avg_ms']:.3f} | {f} | {w} |")
    if fscale:
        lines += ["", f"Byte counters scaled by the 1 GiB copy reference: FETCH_SIZE x {fscale:.3f}, "
                      f"WRITE_SIZE x {wscale:.3f}."]
    derived = {}
    if a.counters:
        cstats = counters_last(a.counters, max(a.last, 1))
        lines += ["", "Counters (last " + str(max(a.last, 1)) + " dispatches of each kernel):", ""]
        lines += counter_table(cstats)
        for k, c in cstats.items():
            for label, fn in DERIVED:
                try:
                    derived.setdefault(k, {})[label] = fn(c)
                except (KeyError, ZeroDivisionError):
                    pass
    lines += ["", f"Kernel source sha256 (code without comments): `{source_hash()}`", ""]
    with open(a.out_md, "w") as f:
        f.write("\n".join(lines))
    if a.out_json:
        data = {"label": a.label, "command": a.command, "source_sha256": source_hash(),
                "kernels": {k: {"launches": v["calls"], "avg_ms": v["avg_ms"],
                                "fetch_bytes_per_launch": fetch.get(k) if fetch else None,
                                "write_bytes_per_launch": write.get(k) if write else None,
                                "counters": derived.get(k)}
                            for k, v in stats.items()},
                "copy_scale": {"fetch": fscale, "write": wscale}}
        with open(a.out_json, "w") as f:
            json.dump(data, f, indent=1)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
