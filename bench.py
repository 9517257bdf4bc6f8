#!/usr/bin/env python3
"""Benchmark of the generalized Joseph projector hot path on one MI355X.

Default workload (c3): a 512^3 Shepp-Logan-type volume (builder-defined
stand-in, 10 nested ellipsoids), 720 cone-beam views over 360 degrees, 768 x
768 detector, magnification 1.5. One step = one FP32 forward projection
y = A x of all views (Algorithm 1); `value` is ray-samples per second, S / step
time, with S the exact sample count of one pass (host FP64 ray setup). Inputs
are resident in HBM before timing; the forward launch configuration is
autotuned before the untimed warm-up.

The same run then times, each after its own warm-up, and reports under
`kernels`: the FP32 adjoint A^T y (table and gather passes), BF16 and FP16
storage forwards and their speed-up over FP32, the plain one-lane-per-ray FP32
forward, 20 gradient-descent steps of the differentiable projector, one
batched launch of the 32-instance uneven workload, the paper's speed geometry
(Table I: ms per projection), a 1024^3 BF16/FP16 forward, a 2048^3 FP32
forward and SART iterations on the 256^3 workload. `roofline` refers to the FP32 forward kernel and its
binding unit (the vector-memory address path); the HBM fraction from the
committed byte counters and the paper's access rate are reported beside it.

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
# The vector-memory address path takes a wavefront load instruction whose lanes
# hit irregular 16-byte (or 8-/12-byte) locations at 4 lanes per clock per
# compute unit: 256 CUs x 2.4 GHz x 4 lane addresses.
N_CU, CLOCK_HZ, ADDR_LANES_PER_CLK = 256, 2.4e9, 4
ADDR_PEAK = N_CU * CLOCK_HZ * ADDR_LANES_PER_CLK
# The paper's GJP_lin FP32 forward, volume in global memory (Table I, Sec.
# IV-C geometry): ms per projection.
PAPER_T1_MS = {"GTX 1080": 2.70, "GTX 970": 5.69}
METRIC = "GJP ray-samples/s and % HBM roofline (fwd, adjoint, bf16) vs plain FP32 fwd"


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


def host_threads():
    """Threads the oracle may use: the environment's OpenMP setting (the
    host's CPU share for this GPU), else the affinity mask."""
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return min(int(env), aff), aff
    return aff, aff


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch (fetch, write) of `kernel` from the committed
    rocprofv3 summary of this workload, or None if there is none or the kernel
    sources changed since the counters were taken."""
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
    return fb, wb


class Timer:
    """Kernel times from the HIP events the library records around each of its
    launches on their stream, plus the wall clock around the calls."""

    def __init__(self, torch, gjp):
        self.torch, self.gjp = torch, gjp

    def run(self, fn, reps, kernels):
        torch, gjp = self.torch, self.gjp
        torch.cuda.synchronize()
        gjp.timing_reset()
        gjp.timing_enable(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        gjp.timing_enable(False)
        out = {"wall_ms": 1e3 * wall}
        for k in kernels:
            ms, n = gjp.timing_read(k)
            out[k] = {"ms_per_launch": ms / max(n, 1), "launches_per_call": n / reps,
                      "ms_per_call": ms / reps}
        return out


def cpu_baseline(cfg, G_gjp, vol_np, target_s: float):
    """The FP64 oracle forward on the host: a bounded sample of the workload's
    rays on the host's thread share (sized to about target_s seconds), and the
    seeded 1e5-ray subset on all of those threads and on one thread."""
    import oracle
    import workloads
    og = oracle.geometry_for(cfg)
    threads, aff = host_threads()
    oracle.set_num_threads(threads)
    sub = workloads.sample_rays(51, 100000, cfg.n_views, cfg.n_u, cfg.n_v)
    t0 = time.perf_counter()
    _, c = oracle.forward_rays(og, vol_np, sub, with_counts=True)
    dt_sub = time.perf_counter() - t0
    rate_sub = int(c.sum()) / dt_sub
    n_rays = int(min(cfg.n_rays, max(100000, target_s * rate_sub / max(c.mean(), 1.0))))
    rays = workloads.sample_rays(12, n_rays, cfg.n_views, cfg.n_u, cfg.n_v)
    t0 = time.perf_counter()
    _, c2 = oracle.forward_rays(og, vol_np, rays, with_counts=True)
    dt = time.perf_counter() - t0
    samples = int(c2.sum())
    oracle.set_num_threads(1)
    t1 = time.perf_counter()
    _, c1 = oracle.forward_rays(og, vol_np, sub, with_counts=True)
    dt1 = time.perf_counter() - t1
    oracle.set_num_threads(threads)
    return {
        "value": samples / dt,
        "unit": "ray-samples/s",
        "cores": threads,
        "kind": "oracle",
        "value_1core": int(c1.sum()) / dt1,
        "subset_1e5_all_threads": rate_sub,
        "sample": f"FP64 oracle forward of {n_rays} uniformly sampled rays of the {cfg.name} "
                  f"workload ({samples} ray-samples, {dt:.1f} s) on {threads} threads "
                  f"(OpenMP; affinity mask {aff} CPUs, {cpu_model()}); value_1core: the seeded "
                  f"1e5-ray subset on one thread ({dt1:.1f} s); subset_1e5_all_threads: the "
                  f"same subset on {threads} threads ({dt_sub:.2f} s)",
    }


# ---------------------------------------------------------------------------
# the auxiliary kernel figures (each a failure of its own, not of the line)
# ---------------------------------------------------------------------------
def _aux(name, fn, out):
    import torch
    free, total = torch.cuda.mem_get_info()
    log(f"{name}: start ({free / 2**30:.1f} of {total / 2**30:.1f} GiB free)")
    t0 = time.perf_counter()
    try:
        out[name] = fn()
        log(f"{name}: {json.dumps(out[name])[:300]} ({time.perf_counter() - t0:.1f} s)")
    except (RuntimeError, MemoryError, ValueError) as e:
        out[name] = {"error": str(e)[:300]}
        log(f"{name} failed: {e}")
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def aux_adjoint(T, torch, gjp, G, x, S, fwd_ms):
    y = gjp.forward(x, G)
    out = torch.empty_like(x)
    gjp.back(y, G, out)
    r = T.run(lambda: gjp.back(y, G, out), 2, ("adjoint_table", "adjoint_gather"))
    ms = r["adjoint_table"]["ms_per_call"] + r["adjoint_gather"]["ms_per_call"]
    return {"ms": ms, "wall_ms": r["wall_ms"], "ray_samples_per_s": S / (ms * 1e-3),
            "table_ms": r["adjoint_table"]["ms_per_call"],
            "gather_ms": r["adjoint_gather"]["ms_per_call"],
            "gather_launches": r["adjoint_gather"]["launches_per_call"],
            "ratio_to_f32_forward": ms / fwd_ms}


def aux_dtypes(T, torch, gjp, G, x, S, fwd_ms, autotune):
    res = {}
    y = torch.empty(G.sino_shape, device=x.device)
    for name, dt in (("bf16", torch.bfloat16), ("f16", torch.float16)):
        xv = x.to(dt)
        tile = gjp.autotune(xv, G, y) if autotune else None
        gjp.forward(xv, G, y)
        r = T.run(lambda: gjp.forward(xv, G, y), 3, ("forward",))
        ms = r["forward"]["ms_per_launch"]
        res[name] = {"ms": ms, "ray_samples_per_s": S / (ms * 1e-3), "tile_v": tile,
                     "access_rate_GBps": 8.0 * S / (ms * 1e-3) / 1e9,
                     "speedup_vs_f32": fwd_ms / ms}
        del xv
    return res


def aux_one_ray(T, torch, gjp, G, x, S, fwd_ms):
    """The FP32 forward with one ray per lane (64-wide tiles: one 16-byte load
    per sample), then the autotuned configuration again."""
    y = torch.empty(G.sino_shape, device=x.device)
    cfg = gjp.get_forward_tile(G, torch.float32)
    gjp.set_forward_tile(G, torch.float32, 64, 8, 4)
    try:
        gjp.forward(x, G, y)
        r = T.run(lambda: gjp.forward(x, G, y), 3, ("forward",))
    finally:
        gjp.set_forward_tile(G, torch.float32, *cfg)
    ms = r["forward"]["ms_per_launch"]
    return {"ms": ms, "ray_samples_per_s": S / (ms * 1e-3), "launch_config": [64, 8, 4],
            "tuned_f32_speedup": ms / fwd_ms}


def aux_naive(T, torch, gjp, G, x, S, fwd_ms):
    y = torch.empty(G.sino_shape, device=x.device)
    gjp.forward_naive(x, G, y)
    r = T.run(lambda: gjp.forward_naive(x, G, y), 2, ("forward_naive",))
    ms = r["forward_naive"]["ms_per_launch"]
    return {"ms": ms, "ray_samples_per_s": S / (ms * 1e-3), "tuned_f32_speedup": ms / fwd_ms}


def autotune_instances(torch, gjp, geoms, vols, outs):
    """The batched workload's ray-tile shapes: each instance's forward
    autotuned on its own (untimed); the batched launch runs each instance's
    choice. Returns the tile widths chosen."""
    tiles = [gjp.autotune(v, G, o) for G, v, o in zip(geoms, vols, outs)]
    torch.cuda.synchronize()
    return tiles


def aux_batched(T, torch, gjp, workloads, dev):
    from workloads.configs import batched_instances
    insts = batched_instances()
    geoms = [gjp.Geometry.from_config(cfg) for cfg in insts]
    vols = [workloads.rasterize_torch(cfg.phantom_ellipsoids(), cfg.shape, dev) for cfg in insts]
    S = sum(G.count_samples() for G in geoms)
    outs = [torch.empty(G.sino_shape, dtype=torch.float32, device=dev) for G in geoms]
    t0 = time.perf_counter()
    tiles = autotune_instances(torch, gjp, geoms, vols, outs)
    tune_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    gjp.forward_batched(vols, geoms, outs)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    gjp.forward_batched(vols, geoms, outs)
    r = T.run(lambda: gjp.forward_batched(vols, geoms, outs), 3, ("batched",))
    ms = r["batched"]["ms_per_launch"]
    return {"workload": "c4: 32 uneven instances (edges 96-320, 90-360 views, 128^2-512^2 "
                        "detectors, cone or parallel) in one persistent graph-replayed launch, "
                        "each instance's ray-tile shape autotuned",
            "ms": ms, "wall_ms": r["wall_ms"], "ray_samples": S,
            "ray_samples_per_s": S / (ms * 1e-3), "first_call_with_plan_s": plan_s,
            "autotune_s": tune_s,
            "tile_v_counts": {str(t): tiles.count(t) for t in sorted(set(tiles))}}


def aux_t1(T, torch, gjp, workloads, dev, autotune):
    cfg = workloads.config("t1")
    x = workloads.rasterize_torch(cfg.phantom_ellipsoids(), cfg.shape, dev)
    G = gjp.Geometry.from_config(cfg)
    S = G.count_samples()
    y = torch.empty(G.sino_shape, device=dev)
    tile = gjp.autotune(x, G, y) if autotune else None
    gjp.forward(x, G, y)
    r = T.run(lambda: gjp.forward(x, G, y), 3, ("forward",))
    ms = r["forward"]["ms_per_launch"]
    return {"workload": "t1: the paper's speed geometry (512^3 box clipped to the inscribed "
                        "cylinder, 512^2 detector, 10 degree cone, 360 views), FP32",
            "ms_per_projection": ms / cfg.n_views,
            "wall_ms_per_projection": r["wall_ms"] / cfg.n_views,
            "paper_ms_per_projection": PAPER_T1_MS, "ray_samples_per_s": S / (ms * 1e-3),
            "access_rate_GBps": 16.0 * S / (ms * 1e-3) / 1e9, "tile_v": tile}


def aux_c5a(T, torch, gjp, workloads, dev, tiles16):
    cfg = workloads.config("c5a")
    G = gjp.Geometry.from_config(cfg)
    S = G.count_samples()
    x = workloads.rasterize_torch(cfg.phantom_ellipsoids(), cfg.shape, dev)
    y = torch.empty(G.sino_shape, device=dev)
    res = {"workload": "c5a: 1024^3, 1440 cone-beam views, 1536^2 detector; 16-bit storage, "
                       "launch configuration of the 512^3 autotuning", "ray_samples": S}
    for name, dt in (("bf16", torch.bfloat16), ("f16", torch.float16)):
        xv = x.to(dt)
        if tiles16.get(name):
            gjp.set_forward_tile(G, dt, *tiles16[name])
        gjp.forward(xv, G, y)
        r = T.run(lambda: gjp.forward(xv, G, y), 1, ("forward",))
        ms = r["forward"]["ms_per_launch"]
        res[name] = {"ms": ms, "ray_samples_per_s": S / (ms * 1e-3)}
        del xv
    return res


def aux_c5b(T, torch, gjp, workloads, dev, tile32):
    cfg = workloads.config("c5b")
    G = gjp.Geometry.from_config(cfg)
    S = G.count_samples()
    x = workloads.rasterize_torch(cfg.phantom_ellipsoids(), cfg.shape, dev)
    y = torch.empty(G.sino_shape, device=dev)
    if tile32:
        gjp.set_forward_tile(G, torch.float32, *tile32)
    gjp.forward(x, G, y)
    r = T.run(lambda: gjp.forward(x, G, y), 1, ("forward", "pad"))
    ms = r["forward"]["ms_per_launch"]
    return {"workload": "c5b: 2048^3 FP32 (34 GB), 64 cone-beam views, 3072^2 detector; "
                        "launch configuration of the 512^3 autotuning",
            "launch_config": list(gjp.get_forward_tile(G, torch.float32)),
            "ms": ms, "pad_ms": r["pad"]["ms_per_launch"], "ray_samples": S,
            "ray_samples_per_s": S / (ms * 1e-3)}


def aux_gd(T, torch, gjp, G, x_true, steps=20):
    """The differentiable-projector run of the 512^3 workload: loss
    0.5 ||Ax - b||^2 through the autograd wrapper (forward A, backward the
    hand-written A^T), `steps` gradient-descent steps from x = 0 with step
    1/lambda (lambda from three power iterations on A^T A, untimed). b is the
    forward projection of the phantom plus seeded Gaussian noise (sigma = 1% of
    max b): the steps' cost does not depend on b's values."""
    b = gjp.forward(x_true, G)
    gen = torch.Generator(device="cpu").manual_seed(3)
    b = b + (0.01 * float(b.max())) * torch.randn(G.sino_shape, generator=gen).to(b.device)
    q = torch.rand(G.shape, generator=torch.Generator().manual_seed(32)).to(b.device)
    lam = 1.0
    for _ in range(3):
        q = gjp.back(gjp.forward(q, G), G)
        lam = float(torch.linalg.vector_norm(q))
        q = q / lam
    del q
    x = torch.zeros(G.shape, device=b.device, requires_grad=True)
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x.grad = None
        r = gjp.project(x, G) - b
        L = 0.5 * (r * r).sum()
        L.backward()
        losses.append(L.detach())
        with torch.no_grad():
            x -= x.grad / lam
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    losses = [float(v) for v in losses]
    return {"workload": "c3 differentiable projector: 512^3, 720 views, 768^2; loss "
                        "0.5||Ax - b||^2, gradient through the hand-written adjoint",
            "steps": steps, "s_total": dt, "ms_per_step": 1e3 * dt / steps,
            "loss_first_last": [losses[0], losses[-1]],
            "loss_monotone": all(l2 < l1 for l1, l2 in zip(losses, losses[1:]))}


def aux_sart(torch, gjp, workloads, dev, iters=3):
    """SART (Sec. IV-B) on the 256^3 / 360-view workload: 20 ordered subsets
    of 18 views; one iteration = every subset updated once."""
    cfg = workloads.config("c2")
    x_true = workloads.rasterize_torch(cfg.phantom_ellipsoids(), cfg.shape, dev)
    G = gjp.Geometry.from_config(cfg)
    S = G.count_samples()
    b = gjp.forward(x_true, G)
    solver = gjp.SART(G, 20, lam=1.0)
    x = solver.run(b, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x = solver.run(b, iters, x0=x)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / iters
    return {"workload": "sart: 256^3 random-ellipsoid volume, 360 cone-beam views, 384^2 "
                        "detector; 20 ordered subsets of 18 views, lambda 1",
            "ms_per_iteration": ms, "ray_samples_per_s": 2 * S / (ms * 1e-3)}


# ---------------------------------------------------------------------------
# alternative workloads for profiling runs (one JSON line each)
# ---------------------------------------------------------------------------
def bench_batched(args, torch, gjp, workloads, dev):
    """A step is one batched FP32 forward of the 32 uneven instances."""
    T = Timer(torch, gjp)
    res = aux_batched(T, torch, gjp, workloads, dev)
    from workloads.configs import batched_instances
    insts = batched_instances()
    geoms = [gjp.Geometry.from_config(cfg) for cfg in insts]
    vols = [workloads.rasterize_torch(cfg.phantom_ellipsoids(), cfg.shape, dev) for cfg in insts]
    outs = [torch.empty(G.sino_shape, device=dev) for G in geoms]
    for _ in range(max(args.warmup, 1)):
        gjp.forward_batched(vols, geoms, outs)
    r = T.run(lambda: gjp.forward_batched(vols, geoms, outs), args.steps, ("batched",))
    S = res["ray_samples"]
    print(json.dumps({
        "metric": "GJP ray-samples/s, batched FP32 forward of uneven instances",
        "value": S / (r["wall_ms"] * 1e-3), "unit": "ray-samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["wall_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "config": {"workload": res["workload"], "ray_samples_per_pass": S},
        "kernels": {"batched_ms_per_launch": r["batched"]["ms_per_launch"]}}), flush=True)


def bench_sart(args, torch, gjp, workloads, dev):
    """SART (Sec. IV-B) on the 256^3 / 360-view workload: 20 ordered subsets of
    18 views; a step is one iteration (every subset updated once)."""
    cfg = workloads.config("c2")
    x_true = workloads.rasterize_torch(cfg.phantom_ellipsoids(), cfg.shape, dev)
    G = gjp.Geometry.from_config(cfg)
    S = G.count_samples()
    b = gjp.forward(x_true, G)
    solver = gjp.SART(G, 20, lam=1.0)
    x = solver.run(b, max(args.warmup, 1))
    torch.cuda.synchronize()
    r0 = float(torch.linalg.vector_norm(b - gjp.forward(x, G)))
    t0 = time.perf_counter()
    x = solver.run(b, args.steps, x0=x)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    r1 = float(torch.linalg.vector_norm(b - gjp.forward(x, G)))
    print(json.dumps({
        "metric": "SART iterations: ray-samples/s (forward + adjoint per iteration)",
        "value": 2 * S / (elapsed / args.steps), "unit": "ray-samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sart: 256^3 random-ellipsoid volume, 360 cone-beam views, "
                               "384x384 detector; 20 ordered subsets of 18 views, lambda 1",
                   "ray_samples_per_pass": S, "residual_norm_before_after": [r0, r1]}}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3",
                    help="c3 (default), c1, c2, t1, c5a, c5b: step = one FP32 forward; "
                         "c4: one batched forward; sart: one SART iteration")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the forward autotuning that precedes the warm-up (untimed)")
    ap.add_argument("--no-aux", action="store_true",
                    help="time the steps only (no auxiliary kernel figures): profiled runs")
    ap.add_argument("--only-aux", default="",
                    help="comma list of auxiliary figures to run (adjoint, dtypes (with the "
                         "one-ray FP32 forward), naive, gd (20 gradient-descent steps, 512^3 "
                         "only), batched, t1, c5a, c5b, sart); default all")
    ap.add_argument("--volume", default="phantom", choices=("phantom", "uniform"),
                    help="phantom: the workload's ellipsoid phantom (rasterised in FP64); "
                         "uniform: seeded uniform random values in [0, 1) drawn in FP32 "
                         "(profiled runs: no double-precision kernels in the process)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device copy before the steps (untimed), a "
                         "reference dispatch of known traffic for hardware byte counters")
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
    if args.workload == "sart":
        return bench_sart(args, torch, gjp, workloads, dev)
    cfg = workloads.config(args.workload)
    log(f"workload {cfg.name}: {cfg.shape} grid, {cfg.n_views} views, {cfg.n_u}x{cfg.n_v}")
    t0 = time.perf_counter()
    if args.volume == "uniform":
        x = torch.rand(cfg.shape, generator=torch.Generator(device=dev).manual_seed(11),
                       device=dev)
    else:
        x = workloads.rasterize_torch(cfg.phantom_ellipsoids(), cfg.shape, dev)
    G = gjp.Geometry.from_config(cfg)
    S = G.count_samples()
    n_rays = cfg.n_rays
    log(f"phantom + geometry ready in {time.perf_counter() - t0:.1f} s; S = {S} ray-samples")
    y = torch.empty(G.sino_shape, dtype=torch.float32, device=dev)
    tile = None
    if not args.no_autotune:
        tile = gjp.autotune(x, G, y)
        log(f"autotune float32: tile_v = {tile}")
    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)   # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        gjp.forward(x, G, y)
    T = Timer(torch, gjp)
    r = T.run(lambda: gjp.forward(x, G, y), args.steps, ("forward", "pad"))
    step_ms = r["wall_ms"]
    fwd_ms = r["forward"]["ms_per_launch"]
    value = S / (step_ms * 1e-3)
    log(f"FP32 forward: {step_ms:.2f} ms per step (kernel {fwd_ms:.2f} ms, pad "
        f"{r['pad']['ms_per_launch']:.2f} ms); {value:.4g} ray-samples/s")

    # roofline of the FP32 forward kernel on the vector-memory address path:
    # each irregular 16-byte load of a lane is one lane address; one per sample
    # with one ray per lane, two per three samples with three rays per lane
    # (192-wide tiles, where the rays of a lane share their pair elements)
    tile_cfg = gjp.get_forward_tile(G, torch.float32)
    loads_per_sample = 2.0 / 3.0 if tile_cfg[0] == 192 else 1.0
    fwd_kernel = "forward_f32_triples" if tile_cfg[0] == 192 else "forward_f32"
    achieved = loads_per_sample * S / (fwd_ms * 1e-3)
    traffic = measured_traffic(cfg.name, fwd_kernel)
    roofline = {
        "kernel": fwd_kernel,
        "bound": "vmem_address",
        "achieved": achieved,
        "peak": ADDR_PEAK,
        "unit": "lane addresses/s",
        "lane_addresses_per_sample": loads_per_sample,
        "frac": achieved / ADDR_PEAK,
        "traffic": (traffic[0] + traffic[1]) if traffic else None,
        "hbm_GBps": ((traffic[0] + traffic[1]) / (fwd_ms * 1e-3) / 1e9) if traffic else None,
        "hbm_frac": ((traffic[0] + traffic[1]) / (fwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS)
        if traffic else None,
        "access_rate_GBps": (16.0 * S + 4.0 * n_rays) / (fwd_ms * 1e-3) / 1e9,
        "hbm_peak_GBps": HBM_PEAK_GBS,
    }
    kernels = {"forward_f32": {"ms": fwd_ms, "ray_samples_per_s": S / (fwd_ms * 1e-3),
                               "tile_v": tile, "launch_config": list(tile_cfg),
                               "pad_ms": r["pad"]["ms_per_launch"]}}
    want = set(a for a in args.only_aux.split(",") if a) or {
        "adjoint", "dtypes", "naive", "gd", "batched", "t1", "c5a", "c5b", "sart"}
    if args.no_aux:
        want = set()
    if "adjoint" in want:
        _aux("adjoint", lambda: aux_adjoint(T, torch, gjp, G, x, S, fwd_ms), kernels)
    if "dtypes" in want:
        _aux("forward_f32_one_ray", lambda: aux_one_ray(T, torch, gjp, G, x, S, fwd_ms), kernels)

        def dts():
            d = aux_dtypes(T, torch, gjp, G, x, S, fwd_ms, not args.no_autotune)
            kernels["forward_bf16"], kernels["forward_f16"] = d["bf16"], d["f16"]
            out = {"speedup_bf16_vs_f32": d["bf16"]["speedup_vs_f32"],
                   "speedup_f16_vs_f32": d["f16"]["speedup_vs_f32"]}
            one = kernels.get("forward_f32_one_ray", {}).get("ms")
            if one:
                out["speedup_bf16_vs_f32_one_ray"] = one / d["bf16"]["ms"]
                out["speedup_f16_vs_f32_one_ray"] = one / d["f16"]["ms"]
            return out
        _aux("storage_speedups", dts, kernels)
    if "naive" in want:
        _aux("forward_naive_f32", lambda: aux_naive(T, torch, gjp, G, x, S, fwd_ms), kernels)
    if "gd" in want and cfg.name == "c3":
        _aux("gd20_c3", lambda: aux_gd(T, torch, gjp, G, x), kernels)
    vol_np = None
    if not args.no_cpu_baseline:
        vol_np = x.cpu().numpy()
    del x, y
    torch.cuda.empty_cache()
    # the largest workloads first, while the device holds nothing else
    if "c5b" in want:
        tile32 = tuple(tile_cfg) if tile else None
        _aux("c5b_2048_f32", lambda: aux_c5b(T, torch, gjp, workloads, dev, tile32), kernels)
    if "c5a" in want:
        tiles16 = {}
        for name, dt in (("bf16", torch.bfloat16), ("f16", torch.float16)):
            if kernels.get(f"forward_{name}", {}).get("tile_v"):
                tiles16[name] = tuple(gjp.get_forward_tile(G, dt))
        _aux("c5a_1024_16bit", lambda: aux_c5a(T, torch, gjp, workloads, dev, tiles16), kernels)
    if "t1" in want:
        _aux("t1_table1_geometry", lambda: aux_t1(T, torch, gjp, workloads, dev,
                                                  not args.no_autotune), kernels)
    if "batched" in want:
        _aux("batched_c4", lambda: aux_batched(T, torch, gjp, workloads, dev), kernels)
    if "sart" in want:
        _aux("sart_c2", lambda: aux_sart(torch, gjp, workloads, dev), kernels)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "ray-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{cfg.name}: {cfg.shape[0]}x{cfg.shape[1]}x{cfg.shape[2]} "
                        f"{'uniform random' if args.volume == 'uniform' else ('Shepp-Logan-type stand-in' if cfg.phantom == 'sl' else 'random-ellipsoid')} "
                        f"volume, {cfg.n_views} {cfg.beam}-beam views, {cfg.n_u}x{cfg.n_v} "
                        f"detector; step = one FP32 forward projection of all views",
            "ray_samples_per_pass": S,
            "rays_per_pass": n_rays,
        },
        "roofline": roofline,
        "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded ray sample")
        out["cpu_baseline"] = cpu_baseline(cfg, G, vol_np, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
