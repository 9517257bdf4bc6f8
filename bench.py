#!/usr/bin/env python3
"""Benchmark of the generalized Joseph projector hot path on one MI355X.

One step = one pass of the whole projection path over the synthetic workload
(default: 256^3 volume of 12 seeded random ellipsoids, 360 cone-beam views
over 360 degrees, 384 x 384 detector, magnification 1.5):
  1. differentiable FP32 forward  y = A x        (autograd forward)
  2. hand-written adjoint         A^T w          (autograd backward)
  3. BF16-storage forward
  4. FP16-storage forward
`value` is ray-samples per second over the whole step (each pass processes the
workload's exact sample count S). Inputs are resident in HBM before timing.
Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def measured_copy_gbs(torch, dev):
    """Device-to-device copy rate of a 2 GiB buffer (bytes read + written per
    second), a measured stream peak to set beside the nominal HBM figure."""
    src = torch.empty(1 << 29, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    gbs = 2.0 * src.numel() * 4 / (ms * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch (fetch + write) of `kernel` from the committed rocprofv3
    summary of this workload, or None if there is none or the kernel sources
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    from paper_1609_00958_amd import profiling
    with open(path) as f:
        data = json.load(f)
    if data.get("source_sha256") != profiling.source_hash():
        return None
    k = data.get("kernels", {}).get(kernel, {})
    fb, wb = k.get("fetch_bytes_per_launch"), k.get("write_bytes_per_launch")
    if fb is None or wb is None:
        return None
    return fb + wb


def cpu_baseline(cfg, vol_np, target_s: float):
    """Time the FP64 oracle forward on a bounded random sample of the workload's rays."""
    import oracle
    import workloads
    og = oracle.geometry_for(cfg)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(int(cores), 16))
    oracle.set_num_threads(cores)
    # grow a probe until it runs for about a second, then size the sample
    n_probe = 4000
    while True:
        probe = workloads.sample_rays(11, n_probe, cfg.n_views, cfg.n_u, cfg.n_v)
        t0 = time.perf_counter()
        _, c = oracle.forward_rays(og, vol_np, probe, with_counts=True)
        dt = time.perf_counter() - t0
        if dt >= 1.0 or n_probe >= cfg.n_rays:
            break
        n_probe = min(cfg.n_rays, n_probe * 4)
    rate = max(int(c.sum()), 1) / max(dt, 1e-6)
    n_rays = int(min(cfg.n_rays, max(4000, target_s * rate / max(c.mean(), 1.0))))
    rays = workloads.sample_rays(12, n_rays, cfg.n_views, cfg.n_u, cfg.n_v)
    t0 = time.perf_counter()
    _, c = oracle.forward_rays(og, vol_np, rays, with_counts=True)
    dt = time.perf_counter() - t0
    samples = int(c.sum())
    # the same oracle on one thread, over a slice of the sample sized for a few seconds
    n1 = int(min(n_rays, max(1000, 3.0 * samples / dt / cores / max(c.mean(), 1.0))))
    oracle.set_num_threads(1)
    t1 = time.perf_counter()
    _, c1 = oracle.forward_rays(og, vol_np, rays[:n1], with_counts=True)
    dt1 = time.perf_counter() - t1
    oracle.set_num_threads(cores)
    return {
        "value": samples / dt,
        "unit": "ray-samples/s",
        "cores": cores,
        "kind": "oracle",
        "value_1core": int(c1.sum()) / dt1,
        "sample": f"FP64 oracle forward of {n_rays} uniformly sampled rays of the workload "
                  f"({samples} ray-samples, {dt:.1f} s, {cpu_model()}); value_1core: the "
                  f"first {n1} of those rays on one thread ({dt1:.1f} s)",
    }


def bench_batched(args, torch, gjp, workloads, dev):
    """Batched workload: 32 uneven instances in one persistent, graph-replayed
    launch; a step is one batched FP32 forward of all instances."""
    from workloads.configs import batched_instances
    insts = batched_instances()
    t0 = time.perf_counter()
    geoms, vols, S = [], [], 0
    for cfg in insts:
        G = gjp.Geometry.from_config(cfg)
        geoms.append(G)
        vols.append(workloads.rasterize_torch(cfg.phantom_ellipsoids(), cfg.shape, dev))
        S += G.count_samples()
    log(f"{len(insts)} instances ready in {time.perf_counter() - t0:.1f} s; S = {S}")
    outs = [torch.empty(G.sino_shape, dtype=torch.float32, device=dev) for G in geoms]
    for _ in range(max(args.warmup, 1)):
        gjp.forward_batched(vols, geoms, outs)
    torch.cuda.synchronize()
    gjp.timing_reset()
    gjp.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gjp.forward_batched(vols, geoms, outs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gjp.timing_enable(False)
    b_ms, b_n = gjp.timing_read("batched")
    avg = b_ms / max(b_n, 1)
    n_rays = sum(G.n_views * G.n_u * G.n_v for G in geoms)
    alg = 16.0 * S + 4.0 * n_rays
    achieved = alg / (avg * 1e-3) / 1e9
    out = {
        "metric": "GJP ray-samples/s, batched FP32 forward of uneven instances",
        "value": S / (elapsed / args.steps),
        "unit": "ray-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c4: 32 uneven instances (edges 96-320, 90-360 views, "
                               "128^2-512^2 detectors, cone or parallel) in one batched "
                               "persistent launch; step = one batched FP32 forward",
                   "ray_samples_per_pass": S, "rays_per_pass": n_rays},
        "roofline": {"kernel": "batched", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("c4", "batched")},
    }
    print(json.dumps(out), flush=True)


# The paper's GJP_lin FP32 forward with the volume in global memory (Table I,
# Sec. IV-C geometry): ms per projection on its two GPUs.
PAPER_T1_MS = {"GTX 1080": 2.70, "GTX 970": 5.69}


def bench_t1(args, torch, gjp, workloads, dev):
    """The paper's projection-speed geometry: 512^3 box clipped to the inscribed
    cylinder, 512^2 detector, 10 degree cone, 360 views; a step is one FP32
    forward of all views (Table I reports the time per projection)."""
    cfg = workloads.config("t1")
    x = workloads.rasterize_torch(cfg.phantom_ellipsoids(), cfg.shape, dev)
    G = gjp.Geometry.from_config(cfg)
    S = G.count_samples()
    out_t = torch.empty(G.sino_shape, dtype=torch.float32, device=dev)
    if not args.no_autotune:
        log(f"autotune float32: tile_v = {gjp.autotune(x, G, out_t)}")
    for _ in range(max(args.warmup, 1)):
        gjp.forward(x, G, out_t)
    torch.cuda.synchronize()
    gjp.timing_reset()
    gjp.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gjp.forward(x, G, out_t)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gjp.timing_enable(False)
    f_ms, f_n = gjp.timing_read("forward")
    avg = f_ms / max(f_n, 1)
    ms_proj = 1e3 * elapsed / args.steps / cfg.n_views
    alg = 16.0 * S + 4.0 * cfg.n_rays
    achieved = alg / (avg * 1e-3) / 1e9
    out = {
        "metric": "GJP_lin FP32 forward, ms per projection (Table I geometry)",
        "value": ms_proj,
        "unit": "ms/projection",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": ms_proj / PAPER_T1_MS["GTX 1080"],
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "t1: 512^3 box clipped to the inscribed cylinder, 512^2 "
                               "detector, 10 degree cone, 360 views; step = one FP32 forward",
                   "ray_samples_per_pass": S, "rays_per_pass": cfg.n_rays,
                   "ray_samples_per_s": S / (elapsed / args.steps),
                   "paper_ms_per_projection": PAPER_T1_MS},
        "roofline": {"kernel": "forward_f32", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("t1", "forward_f32")},
    }
    print(json.dumps(out), flush=True)


def bench_sart(args, torch, gjp, workloads, dev):
    """SART (Sec. IV-B) on the 256^3 / 360-view workload: 20 ordered subsets of
    18 views; a step is one iteration (every subset updated once: one forward
    and one adjoint over all views plus the elementwise steps)."""
    cfg = workloads.config("c2")
    x_true = workloads.rasterize_torch(cfg.phantom_ellipsoids(), cfg.shape, dev)
    G = gjp.Geometry.from_config(cfg)
    S = G.count_samples()
    b = gjp.forward(x_true, G)
    n_subsets = 20
    t0 = time.perf_counter()
    solver = gjp.SART(G, n_subsets, lam=1.0)
    torch.cuda.synchronize()
    log(f"SART set-up (row and column sums of {n_subsets} subsets): "
        f"{time.perf_counter() - t0:.2f} s")
    x = solver.run(b, max(args.warmup, 1))
    torch.cuda.synchronize()
    r0 = float(torch.linalg.vector_norm(b - gjp.forward(x, G)))
    t0 = time.perf_counter()
    x = solver.run(b, args.steps, x0=x)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    r1 = float(torch.linalg.vector_norm(b - gjp.forward(x, G)))
    out = {
        "metric": "SART iterations: ray-samples/s (forward + adjoint per iteration)",
        "value": 2 * S / (elapsed / args.steps),
        "unit": "ray-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sart: 256^3 random-ellipsoid volume, 360 cone-beam views, "
                               "384x384 detector; 20 ordered subsets of 18 views, lambda 1; "
                               "step = one SART iteration",
                   "ray_samples_per_pass": S,
                   "residual_norm_before_after": [r0, r1]},
    }
    print(json.dumps(out), flush=True)


def bench_dtypes_512(args, torch, gjp, workloads, dev):
    """FP32, BF16 and FP16 storage at 512^3 / 720 views / 768^2: each dtype
    autotuned first (untimed); a step is one forward of each."""
    cfg = workloads.config("c3")
    G = gjp.Geometry.from_config(cfg)
    S = G.count_samples()
    if args.volume == "uniform":
        # the kernels' work does not depend on voxel values; one fill kernel
        # instead of the phantom's many small ones (for counter collection)
        x = torch.rand(cfg.shape, device=dev, generator=torch.Generator(device=dev).manual_seed(3))
    else:
        x = workloads.rasterize_torch(cfg.phantom_ellipsoids(), cfg.shape, dev)
    vols = [x, x.to(torch.bfloat16), x.to(torch.float16)]
    y = torch.empty(G.sino_shape, dtype=torch.float32, device=dev)
    tiles = [None if args.no_autotune else gjp.autotune(v, G, y) for v in vols]
    log(f"autotuned tile_v f32 / bf16 / f16: {tiles}")
    for _ in range(args.warmup):
        for v in vols:
            gjp.forward(v, G, y)
    torch.cuda.synchronize()
    gjp.timing_reset()
    gjp.timing_enable(True)
    t0 = time.perf_counter()
    per = [0.0, 0.0, 0.0]
    for _ in range(args.steps):
        for k, v in enumerate(vols):
            gjp.forward(v, G, y)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gjp.timing_enable(False)
    # per-dtype kernel times: one more launch of each, timed alone
    for k, v in enumerate(vols):
        gjp.timing_reset()
        gjp.timing_enable(True)
        gjp.forward(v, G, y)
        torch.cuda.synchronize()
        gjp.timing_enable(False)
        ms, n = gjp.timing_read("forward")
        per[k] = ms / n
    out = {
        "metric": "GJP forward ray-samples/s by volume storage type (FP32, BF16, FP16)",
        "value": 3 * S / (elapsed / args.steps),
        "unit": "ray-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/bf16/f16 storage, f32 math",
        "data": "synthetic",
        "config": {"workload": f"dtypes512: 512^3 {'uniform random' if args.volume == 'uniform' else 'Shepp-Logan-type'} "
                               "volume, 720 cone-beam views, 768x768 detector; step = FP32 + "
                               "BF16 + FP16 forward",
                   "ray_samples_per_pass": S, "tile_v": tiles,
                   "forward_ms": {"f32": per[0], "bf16": per[1], "f16": per[2]},
                   "speedup_bf16_vs_f32": per[0] / per[1],
                   "speedup_f16_vs_f32": per[0] / per[2]},
    }
    print(json.dumps(out), flush=True)


def forward_dtypes_512(args, torch, gjp, workloads, dev):
    """FP32, BF16 and FP16 forwards at 512^3 / 720 views / 768^2 (each after
    its own autotuning, untimed), two timed launches each: the storage-type
    comparison at the size the 16-bit target refers to."""
    cfg = workloads.config("c3")
    G = gjp.Geometry.from_config(cfg)
    S = G.count_samples()
    x = workloads.rasterize_torch(cfg.phantom_ellipsoids(), cfg.shape, dev)
    out = {"workload": f"{cfg.name}: {cfg.shape[0]}^3, {cfg.n_views} views, "
                       f"{cfg.n_u}x{cfg.n_v} detector", "ray_samples_per_pass": S}
    for name, dt in (("f32", torch.float32), ("bf16", torch.bfloat16), ("f16", torch.float16)):
        xv = x.to(dt)
        y = torch.empty(G.sino_shape, dtype=torch.float32, device=dev)
        tile = gjp.autotune(xv, G, y) if not args.no_autotune else None
        gjp.forward(xv, G, y)
        torch.cuda.synchronize()
        gjp.timing_reset()
        gjp.timing_enable(True)
        for _ in range(2):
            gjp.forward(xv, G, y)
        torch.cuda.synchronize()
        gjp.timing_enable(False)
        ms, n = gjp.timing_read("forward")
        out[name] = {"ms": ms / n, "ray_samples_per_s": S / (ms / n * 1e-3), "tile_v": tile}
        log(f"512^3 forward {name}: {ms / n:.2f} ms (tile_v {tile})")
        del xv, y
    out["speedup_bf16_vs_f32"] = out["f32"]["ms"] / out["bf16"]["ms"]
    out["speedup_f16_vs_f32"] = out["f32"]["ms"] / out["f16"]["ms"]
    del x
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the forward autotuning that precedes the warm-up (untimed)")
    ap.add_argument("--volume", choices=("phantom", "uniform"), default="phantom",
                    help="dtypes512 only: the Shepp-Logan-type phantom or a uniform random "
                         "volume (same work; fewer set-up kernels under a profiler)")
    ap.add_argument("--no-512", action="store_true",
                    help="skip the FP32 / BF16 / FP16 forward comparison at 512^3 (untimed "
                         "by the step clock; reported under kernels)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device copy before the steps (untimed), a "
                         "reference kernel of known traffic for hardware byte counters")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only (--gpus 1): the projector is benchmarked on one "
              "GPU's share of the work; runs over several GPUs are not supported.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1609_00958_amd as gjp
    import workloads

    dev = torch.device("cuda:0")
    if args.workload == "c4":
        return bench_batched(args, torch, gjp, workloads, dev)
    if args.workload == "t1":
        return bench_t1(args, torch, gjp, workloads, dev)
    if args.workload == "sart":
        return bench_sart(args, torch, gjp, workloads, dev)
    if args.workload == "dtypes512":
        return bench_dtypes_512(args, torch, gjp, workloads, dev)
    cfg = workloads.config(args.workload)
    log(f"workload {cfg.name}: {cfg.shape} grid, {cfg.n_views} views, {cfg.n_u}x{cfg.n_v}")
    t0 = time.perf_counter()
    ells = cfg.phantom_ellipsoids()
    if int(np.prod(cfg.shape)) <= 256 ** 3:
        vol_np = workloads.rasterize(ells, cfg.shape)
        x = torch.from_numpy(vol_np).to(dev)
    else:
        x = workloads.rasterize_torch(ells, cfg.shape, dev)
        vol_np = None
    G = gjp.Geometry.from_config(cfg)
    S = G.count_samples()
    log(f"phantom + geometry ready in {time.perf_counter() - t0:.1f} s; S = {S} ray-samples")
    x_bf16 = x.to(torch.bfloat16)
    x_f16 = x.to(torch.float16)
    xr = x.clone().requires_grad_(True)
    w = torch.rand(G.sino_shape, generator=torch.Generator().manual_seed(3)).to(dev)
    if not args.no_autotune:
        for v in (x, x_bf16, x_f16):
            log(f"autotune {v.dtype}: tile_v = {gjp.autotune(v, G)}")
    torch.cuda.synchronize()

    def step():
        xr.grad = None
        y = gjp.project(xr, G)          # FP32 forward (autograd)
        y.backward(w)                   # adjoint (hand-written backward)
        gjp.forward(x_bf16, G)          # BF16 storage
        gjp.forward(x_f16, G)           # FP16 storage

    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)   # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    gjp.timing_reset()
    gjp.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gjp.timing_enable(False)
    kern = {k: gjp.timing_read(k) for k in ("pad", "forward", "adjoint_table", "adjoint_gather")}
    ms_per_step = 1e3 * elapsed / args.steps
    samples_per_step = 4 * S
    value = samples_per_step / (elapsed / args.steps)

    # per-kernel figures (forward launches: f32, bf16, f16 in that order each step)
    fwd_ms, fwd_n = kern["forward"]
    gat_ms, gat_n = kern["adjoint_gather"]
    tab_ms, tab_n = kern["adjoint_table"]
    # per-dtype forward times: time each dtype separately, outside the timed steps
    per_dtype = {}
    for name, v, bps in (("f32", x, 16), ("bf16", x_bf16, 8), ("f16", x_f16, 8)):
        gjp.timing_reset()
        gjp.timing_enable(True)
        for _ in range(3):
            gjp.forward(v, G)
        torch.cuda.synchronize()
        gjp.timing_enable(False)
        ms, n = gjp.timing_read("forward")
        avg = ms / max(n, 1)
        per_dtype[name] = {
            "ms": avg,
            "ray_samples_per_s": S / (avg * 1e-3),
            "alg_GBps": (bps * S + 4 * G.n_views * G.n_u * G.n_v) / (avg * 1e-3) / 1e9,
        }
    # the plain one-lane-per-ray kernel on the same volumes, for context
    naive = {}
    for name, v, bps in (("f32", x, 16), ("bf16", x_bf16, 8)):
        gjp.forward_naive(v, G)
        torch.cuda.synchronize()
        gjp.timing_reset()
        gjp.timing_enable(True)
        for _ in range(2):
            gjp.forward_naive(v, G)
        torch.cuda.synchronize()
        gjp.timing_enable(False)
        ms, n = gjp.timing_read("forward_naive")
        avg = ms / max(n, 1)
        naive[name] = {
            "ms": avg,
            "ray_samples_per_s": S / (avg * 1e-3),
            "alg_GBps": (bps * S + 4 * G.n_views * G.n_u * G.n_v) / (avg * 1e-3) / 1e9,
        }
    n_rays = G.n_views * G.n_u * G.n_v
    n_vox = int(np.prod(cfg.shape))
    gat_avg = gat_ms / max(gat_n, 1)
    adj_launches_per_step = max(gat_n // args.steps, 1)
    adj_ms_step = (gat_ms + tab_ms) / args.steps
    # algorithmic bytes of one gather launch: 16 B per sample of its view chunk, 4 B per
    # ray of the chunk read and 4 B per voxel written
    gat_bytes = (16.0 * S + 4.0 * n_rays + 4.0 * n_vox * adj_launches_per_step) / \
        adj_launches_per_step
    kernels = {
        "forward_f32": per_dtype["f32"],
        "forward_bf16": per_dtype["bf16"],
        "forward_f16": per_dtype["f16"],
        "adjoint": {
            "ms": adj_ms_step,
            "ray_samples_per_s": S / (adj_ms_step * 1e-3),
            "gather_ms_per_launch": gat_avg,
            "table_ms_per_step": tab_ms / args.steps,
            "launches_per_step": adj_launches_per_step,
        },
        "speedup_bf16_vs_f32": per_dtype["f32"]["ms"] / per_dtype["bf16"]["ms"],
        "speedup_f16_vs_f32": per_dtype["f32"]["ms"] / per_dtype["f16"]["ms"],
        "forward_naive_f32": naive["f32"],
        "forward_naive_bf16": naive["bf16"],
        "speedup_f32_vs_naive_f32": naive["f32"]["ms"] / per_dtype["f32"]["ms"],
        "speedup_bf16_vs_naive_f32": naive["f32"]["ms"] / per_dtype["bf16"]["ms"],
    }
    if not args.no_512:
        # an auxiliary comparison: a failure here is reported, not fatal to the line
        try:
            kernels["forward_dtypes_512"] = forward_dtypes_512(args, torch, gjp, workloads, dev)
        except (RuntimeError, MemoryError) as e:
            kernels["forward_dtypes_512"] = {"error": str(e)[:200]}
            torch.cuda.empty_cache()
    # dominant kernel of the step
    fwd_step_ms = fwd_ms / args.steps
    if gat_ms >= fwd_ms / 3.0:
        dom = "adjoint_gather"
        achieved = gat_bytes / (gat_avg * 1e-3) / 1e9
    else:
        dom = "forward_f32"
        achieved = per_dtype["f32"]["alg_GBps"]
    # a profiled run (--calibrate-copy) keeps its 1 GiB copy the largest copy
    # dispatch, which the byte-counter scaling takes as its reference
    copy_gbs = None if args.calibrate_copy else measured_copy_gbs(torch, dev)
    roofline = {
        "kernel": dom,
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "measured_copy_GBps": copy_gbs,
        "frac_of_measured_copy": achieved / copy_gbs if copy_gbs else None,
        "traffic": measured_traffic(args.workload, "adjoint_gather" if dom == "adjoint_gather"
                                    else "forward_f32"),
    }
    out = {
        "metric": "GJP ray-samples/s and % HBM roofline (fwd, adjoint, bf16) vs plain FP32 fwd",
        "value": value,
        "unit": "ray-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{cfg.name}: {cfg.shape[0]}^3 random-ellipsoid volume, {cfg.n_views} "
                        f"cone-beam views, {cfg.n_u}x{cfg.n_v} detector; step = FP32 forward + "
                        f"adjoint + BF16 forward + FP16 forward",
            "ray_samples_per_pass": S,
            "rays_per_pass": n_rays,
            "forward_ms_per_step": fwd_step_ms,
        },
        "kernels": kernels,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        if vol_np is None:
            vol_np = x.cpu().numpy()
        log("timing the CPU oracle on a bounded ray sample")
        out["cpu_baseline"] = cpu_baseline(cfg, vol_np, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
