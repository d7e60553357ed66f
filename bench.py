#!/usr/bin/env python3
"""Benchmark of the GPU spin stepper: spin-steps/s on one MI355X.

Default workload: the 3-D configuration -- a 128^3 grid of two co-located
species (water 0.8 rho, fat 0.2 rho at -440 Hz; 4,194,304 spins) in a
quadratic B0 map of +-50 Hz, a spoiled GRE with a 128-sub-step TBW-4 sinc
excitation (30 deg), TE 5 ms, TR 10 ms, 128 x 128 phase encodes (kz outer)
x 128 samples: 4,227,072 elementary intervals per spin, 2,097,152 complex
samples.  One step is one complete simulation of that request through the
C ABI (sequence compile + upload, step kernels over the time slices, FP64
finalize) with the object already resident in HBM.  Prints one JSON line.
--workload c2 selects the 2-D 256 x 256 spin-echo configuration instead.

Also reported: the step kernel's roofline position (the FP32 flops it
executes per launch / its mean HIP-event duration, against the FP32 vector
peak; a shaped pulse applied from its cached propagator counts as that
affine map), the FP64 CPU oracle timed on the host on a bounded spin subset
of the same workload (with the GPU's error against it on that subset), and
served vs one-request-per-launch latency on a prefix of the Poisson request
stream.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import platform
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X FP32 peak (published; vector and dense matrix alike)
PEAK_FP64_TFLOPS = 78.6       # MI355X FP64 vector peak (published)
FLOPS_ADC_SAMPLE = 8          # p <- p z (complex multiply) and accumulate
FLOPS_HARD_RF = 15            # 3x3 rotation of (Mx, My, Mz), eq. 3.19
FLOPS_SHAPE_SUBSTEP = 23      # rotation + complex precession/decay + Mz recovery
FLOPS_SHAPE_APPLY = 18        # cached shaped pulse: M <- A M + b (9 FMAs)


def bench_c4(args):
    """64 uneven requests: one batched call vs one launch per request."""
    import torch
    import paper_1305_6861_amd as ps
    from workloads import configs as C
    reqs = C.c4(64)
    devs = [ps.to_device(o) for o, _ in reqs]
    packs = [ps.pack_sequence(s) for _, s in reqs]
    spin_steps = float(sum(o.n_spins * s.n_steps_per_spin for o, s in reqs))
    rule_ctx = ps.Context(**CTX_KW)         # tilings of the threshold rule
    ctx = ps.Context(**CTX_KW)
    tuned = 0
    classes = []
    if not args.no_tune:                    # one tuner run per request class
        t_tune = time.perf_counter()
        for d, p in zip(devs, packs):
            r = ctx.tune(d, p)
            if not r["from_table"]:
                classes.append({"n_spins": int(d["x"].shape[0]), "spins_per_lane": r["spins_per_lane"],
                                "replicas": r["replicas"], "best_ms": r["best_ms"], "rule_ms": r["rule_ms"]})
        tuned = len(classes)
        t_tune = time.perf_counter() - t_tune
    outs = [torch.empty(2 * s.n_samples, dtype=torch.float64, device="cuda") for _, s in reqs]

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps

    res = {}
    for tag, c in (("", ctx), ("rule_", rule_ctx)):
        def one_per_launch():
            for d, p, o in zip(devs, packs, outs):
                c.simulate(d, p, out=o)

        def batched():
            return c.simulate_batch(devs, packs)
        res[tag + "one_per_launch"] = timed(one_per_launch)
        res[tag + "batched"] = timed(batched)
    rec = {"metric": "spin-steps/s", "value": spin_steps / res["batched"], "unit": "spin-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["batched"] * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "c4: 64 requests, 2-D N^2 (N log-uniform 16..256), GRE or SE, "
                                  "U{32..256} phase encodes x N samples, per-request seeds",
                      "spin_steps": spin_steps, "matrix_readout": CTX_KW.get("matrix_readout", True)},
           "one_per_launch_ms": res["one_per_launch"] * 1e3,
           "speedup_vs_one_per_launch": res["one_per_launch"] / res["batched"],
           "tiling": {"source": "autotuner" if not args.no_tune else "threshold rule",
                      "classes_tuned": tuned, "classes": classes, "tuning_s": t_tune if not args.no_tune else 0.0,
                      "threshold_rule_batched_ms": res["rule_batched"] * 1e3,
                      "threshold_rule_one_per_launch_ms": res["rule_one_per_launch"] * 1e3},
           "roofline": None, "cpu_baseline": None}
    if not args.no_cpu_baseline:
        import oracle
        got = [t.cpu().numpy() for t in ctx.simulate_batch(devs, packs)]
        t0 = time.perf_counter()
        errs = [oracle.rel_l2(g, oracle.simulate(o, s)) for g, (o, s) in zip(got, reqs)]
        dt = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": spin_steps / dt, "unit": "spin-steps/s", "cores": oracle.default_threads(),
                               "kind": "oracle", "sample": "all 64 requests", "gpu_worst_rel_l2": max(errs)}
    print(json.dumps(rec), flush=True)


def bench_kt(args):
    """The K-t engine (ps_kt_simulate) on a 256 x 256 grid of four tissue
    classes under a 256 x 256 spoiled GRE, against the isochromat stepper on
    the same spins and sequence; the same signal both ways (lattice moments,
    tissue-uniform parameters)."""
    import torch
    import paper_1305_6861_amd as ps
    from workloads import configs as C
    from workloads.phantom import kt_phantom_2d
    fov = 0.25
    obj, begin, t1, t2, dw, _ = kt_phantom_2d(256, fov)
    seq = C.spoiled_gre_2d(256, 256, fov, dwell=10e-6)
    dk = (1 / fov, 1 / fov, 0.0)
    dev = ps.to_device(obj)
    packed = ps.pack_sequence(seq)
    n_samples, n_steps = packed.count()
    ctx = ps.Context(**CTX_KW)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps, out
    t_kt, s_kt = timed(lambda: ctx.kt_simulate(dev, begin, t1, t2, dw, packed, dk))
    t_iso, s_iso = timed(lambda: ctx.simulate(dev, packed))
    import oracle
    err = oracle.rel_l2(s_kt.cpu().numpy(), s_iso.cpu().numpy())
    spin_steps = float(obj.n_spins) * n_steps
    rec = {"metric": "spin-steps/s", "value": spin_steps / t_kt, "unit": "spin-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_kt * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "K-t engine: 256x256 grid of 4 tissue classes (nested discs, %d spins), "
                                  "256x256 spoiled GRE, lattice 1/FOV" % obj.n_spins,
                      "n_spins": obj.n_spins, "n_steps_per_spin": n_steps, "n_samples": n_samples,
                      "step": "full call: population tracking on the host, spectrum and superposition kernels"},
           "isochromat_ms_per_step": t_iso * 1e3, "rel_l2_kt_vs_isochromat": err,
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(rec), flush=True)


def bench_c5(args):
    """Poisson stream: served (continuous batching) vs FIFO one launch per
    request, both replaying the same arrival schedule in real time."""
    rec = c5_replay(args.c5_requests, serve_graphs=not args.serve_direct, rate_hz=args.c5_rate,
                    frac_3d=args.c5_frac_3d)
    print(json.dumps(rec), flush=True)


def latency_block(n_requests: int) -> dict:
    """Served vs FIFO one-launch-per-request latency on the first n_requests
    of the c5 arrival schedule (Poisson, 50 requests/s)."""
    rec = c5_replay(n_requests)
    out = {"requests": n_requests, "arrivals": "c5 Poisson stream prefix, 50 requests/s, seed 5000",
           "served": rec["served"], "fifo_one_per_launch": rec["fifo_one_per_launch"],
           "served_spin_steps_per_s": rec["value"], "workload": rec["config"]["workload"]}
    return out


def c5_replay(n_requests: int, serve_graphs: bool = True, rate_hz: float = 50.0, frac_3d: float = 0.1) -> dict:
    import numpy as np
    import torch
    import paper_1305_6861_amd as ps
    from workloads import configs as C
    sched = C.c5_stream(n_requests=n_requests, rate_hz=rate_hz, frac_3d=frac_3d)
    reqs = [C.c5_request(kind, param) for _, kind, param in sched]
    devs = [ps.to_device(o) for o, _ in reqs]
    packs = [ps.pack_sequence(s) for _, s in reqs]
    torch.cuda.synchronize()
    spin_steps = float(sum(o.n_spins * s.n_steps_per_spin for o, s in reqs))
    arrivals = np.array([t for t, _, _ in sched])
    is3d = np.array([k == "3d" for _, k, _ in sched])

    def replay(submit, finish_all):
        t0 = time.perf_counter()
        handles = []
        for i, t_arr in enumerate(arrivals):
            now = time.perf_counter() - t0
            if t_arr > now:
                time.sleep(t_arr - now)
            handles.append(submit(i, time.perf_counter() - t0))
        done = finish_all(handles, t0)
        return done, time.perf_counter() - t0

    # served
    ctx = ps.Context(serve_graphs=serve_graphs, **CTX_KW)
    def s_submit(i, t):
        return (t, ctx.submit(devs[i], packs[i]))
    kernel_s, queue_s = [], []

    def s_finish(handles, t0):
        lat = []
        for t_sub, h in handles:
            h.wait(-1.0)
            st = h.stats()
            lat.append(st["t_e2e"])
            kernel_s.append(st["t_kernel"])
            queue_s.append(st["t_queue"])
        return np.array(lat)
    lat_s, wall_s = replay(s_submit, s_finish)
    served_iters = ctx.server_stats()["iterations"]
    ctx.close()
    # FIFO one launch per request: a worker thread runs requests in arrival order
    import queue, threading
    ctx2 = ps.Context(**CTX_KW)
    q = queue.Queue()
    lat_f = np.zeros(len(reqs))
    stream = torch.cuda.Stream()
    def worker(t0_holder):
        with torch.cuda.stream(stream):
            while True:
                item = q.get()
                if item is None:
                    return
                i, t_sub = item
                out = ctx2.simulate(devs[i], packs[i], stream=stream)
                stream.synchronize()
                lat_f[i] = time.perf_counter() - t0_holder[0] - t_sub
    t0h = [0.0]
    th = threading.Thread(target=worker, args=(t0h,))
    th.start()
    def f_submit(i, t):
        if i == 0:
            t0h[0] = time.perf_counter() - t
        q.put((i, t))
        return i
    def f_finish(handles, t0):
        q.put(None)
        th.join()
        return lat_f
    lat_f, wall_f = replay(f_submit, f_finish)
    ctx2.close()

    def pct(a, p):
        return float(np.percentile(a, p) * 1e3)
    rec = {"metric": "spin-steps/s", "value": spin_steps / wall_s, "unit": "spin-steps/s", "n_gpus": 1,
           "steps": 1, "warmup": 0, "ms_per_step": wall_s * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"c5: Poisson stream of {len(reqs)} requests at {rate_hz:g}/s, "
                                  f"{int(is3d.sum())} of them 3-D 2x64^3 sinc GRE, the rest c4-type",
                      "spin_steps": spin_steps, "matrix_readout": CTX_KW.get("matrix_readout", True)},
           "served": {"wall_s": wall_s, "p50_ms": pct(lat_s, 50), "p99_ms": pct(lat_s, 99),
                      "p50_2d_ms": pct(lat_s[~is3d], 50), "p99_2d_ms": pct(lat_s[~is3d], 99),
                      "p50_3d_ms": pct(lat_s[is3d], 50) if is3d.any() else None,
                      "p50_queue_ms": pct(np.array(queue_s), 50),
                      "p50_kernel_ms": pct(np.array(kernel_s), 50),
                      "iterations": served_iters, "iterations_per_s": served_iters / wall_s,
                      "launch": ("HIP graph replay per iteration, short iterations launched ahead" if serve_graphs
                                 else "one iteration at a time, direct kernel launches")},
           "fifo_one_per_launch": {"wall_s": wall_f, "p50_ms": pct(lat_f, 50), "p99_ms": pct(lat_f, 99),
                                   "p50_2d_ms": pct(lat_f[~is3d], 50), "p99_2d_ms": pct(lat_f[~is3d], 99)},
           "roofline": None, "cpu_baseline": None}
    return rec


# keyword arguments of every context the run creates (--no-matrix-readout)
CTX_KW = {}

WORKLOADS = {
    "c2": ("c2: 2-D 256x256 grid, 4 jittered isochromats/voxel (262,144 spins), "
           "spin echo 90x/180y TE 20 ms TR 500 ms, 256 phase encodes x 256 samples"),
    "c3": ("c3: 3-D 128^3 grid x two species (4,194,304 spins), quadratic B0 +-50 Hz, fat -440 Hz; "
           "GRE with 128-sub-step TBW-4 sinc (30 deg), TE 5 ms TR 10 ms, 128x128 phase encodes x 128 samples"),
    "t78-tse": ("Table 7.8 2-D turbo spin echo: 100^2 grid (10,000 spins) with the eq. 6.3 Legendre B0, "
                "128^2 matrix, echo train 16, ESP 10 ms"),
    "t78-radial": ("Table 7.8 2-D radial: 100^2 grid (10,000 spins) with the eq. 6.3 Legendre B0, "
                   "128 spokes x 128 samples, spoiled GRE"),
    "t78-epi": ("Table 7.8 2-D EPI: 100^2 grid (10,000 spins) with the eq. 6.3 Legendre B0, "
                "single shot, 128 lines x 128 samples"),
    "spiral": ("2-D spiral: the c2 object (256x256 grid, 4 jittered isochromats/voxel, 262,144 spins), "
               "32-interleave spiral spoiled GRE to k_max = 256/(2 FOV), 2048 samples per interleave at 4 us "
               "(per-sample trajectory tables), TR 20 ms"),
    "t78-se3d": ("Table 7.8 3-D spin echo: 56^3 grid (175,616 spins) with the eq. 6.3 Legendre B0, "
                 "128 samples x 128 x 64 phase encodes"),
}

# Table 7.8, PARSPIN 1.5.0 on a PVM cluster of five Sun Ultra-1 170: context only
# (different hardware, the paper's Shepp-Logan phantom instead of these grids).
PAPER_T78_SECONDS = {"t78-tse": 18.0, "t78-radial": 13.0, "t78-epi": 11.0, "t78-se3d": 4 * 3600.0}


def load_workload(name: str):
    from workloads import configs as C
    if name == "c2":
        return C.c2()
    if name == "c3":
        return C.c3()
    if name.startswith("t78-"):
        return C.table78(name[4:])
    if name == "spiral":
        obj, _ = C.c2()
        return obj, C.spiral_2d(32, 2048, res=256)
    raise ValueError(name)


def algorithmic_flops(seq, n_spins: int, n_coils: int = 1, cached_shapes: bool = False) -> float:
    """Each receive coil has its own readout pass over every spin-sample.
    cached_shapes: count each shaped pulse that recurs (five times or more,
    the library's rule for a propagator slot) as the application of its
    cached affine propagator (FLOPS_SHAPE_APPLY), plus filling the slot once:
    the three columns of the identity and the offset vector stepped through
    its sub-steps (4 x FLOPS_SHAPE_SUBSTEP per sub-step)."""
    n_rf = int(sum(1 for a in seq.rf_alpha if a != 0.0))
    uses = {}
    for sh in seq.rf_shape:
        if sh >= 0:
            uses[int(sh)] = uses.get(int(sh), 0) + 1
    shape_flops = 0.0
    for sid, n_use in uses.items():
        n_sub = seq.shapes[sid].n_sub
        if cached_shapes and n_use >= 5:
            shape_flops += 4 * FLOPS_SHAPE_SUBSTEP * n_sub + FLOPS_SHAPE_APPLY * n_use
        else:
            shape_flops += FLOPS_SHAPE_SUBSTEP * n_sub * n_use
    return float(n_spins) * (FLOPS_ADC_SAMPLE * seq.n_samples * max(n_coils, 1) + FLOPS_HARD_RF * n_rf
                             + shape_flops)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "ps_ops.h", "ps_kernels.h"):
        with open(os.path.join(ROOT, "paper_1305_6861_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload: str, spl: int):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source and tiling."""
    p = os.path.join(ROOT, "profiles", f"step_kernel_{workload}_traffic.json")
    try:
        with open(p) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_source_hash() or rec.get("spins_per_lane") != spl:
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(obj, seq, ctx, target_s: float, rx=None):
    """Oracle (FP64, all host threads) on every stride-th spin of the
    workload, stride chosen so that the run takes about target_s; rx: the
    receive-coil sensitivities (s_x, s_y) as numpy arrays, or None."""
    import numpy as np
    import oracle
    from workloads.phantom import subset
    n_steps = seq.n_steps_per_spin
    threads = oracle.default_threads()

    def sub_rx(stride):
        return None if rx is None else tuple(a[:, ::stride] for a in rx)

    probe = subset(obj, 4096)
    t0 = time.perf_counter()
    oracle.simulate(probe, seq, n_threads=threads, coils=sub_rx(4096))
    rate = probe.n_spins * n_steps / max(time.perf_counter() - t0, 1e-6)
    want = max(rate * target_s / n_steps, 64)
    stride = 1 << max(0, int(math.floor(math.log2(obj.n_spins / want))))
    sub = subset(obj, stride)
    t0 = time.perf_counter()
    ref = oracle.simulate(sub, seq, n_threads=threads, coils=sub_rx(stride))
    dt = time.perf_counter() - t0
    # one thread on a quarter of the multi-thread run's time
    stride1 = stride << max(0, int(math.ceil(math.log2(max(threads, 1) * 4))))
    sub1 = subset(obj, min(stride1, obj.n_spins))
    t1 = time.perf_counter()
    oracle.simulate(sub1, seq, n_threads=1, coils=sub_rx(min(stride1, obj.n_spins)))
    dt1 = time.perf_counter() - t1
    import torch
    got = ctx.simulate(sub, seq, coils=sub_rx(stride))
    torch.cuda.synchronize()
    err = oracle.rel_l2(got.cpu().numpy(), ref)
    return {"value": sub.n_spins * n_steps / dt, "unit": "spin-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"every {stride}th spin ({sub.n_spins} spins) through the full sequence "
                      f"({n_steps} steps/spin), {dt:.1f} s",
            "one_thread": {"value": sub1.n_spins * n_steps / dt1, "spins": sub1.n_spins, "seconds": dt1},
            "cpu_model": cpu_model(),
            "gpu_rel_l2_on_sample": err}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def valu_calibration():
    """The vector FMA rate the library's code generation attains (FP32 with
    packed FP32 disabled, and FP64) next to MI355X's published vector peaks."""
    import paper_1305_6861_amd as ps
    with ps.Context() as ctx:
        f32, f64 = ctx.valu_peak(32), ctx.valu_peak(64)
    print(json.dumps({"fma_tflops_fp32": f32, "fma_tflops_fp64": f64, "published_peak_fp32": PEAK_FP32_TFLOPS,
                      "published_peak_fp64": PEAK_FP64_TFLOPS, "fraction_fp32": f32 / PEAK_FP32_TFLOPS,
                      "fraction_fp64": f64 / PEAK_FP64_TFLOPS}), flush=True)


def copy_calibration(n_bytes: int = 1 << 30, reps: int = 5):
    """A plain copy of n_bytes (read n_bytes, write n_bytes) per launch."""
    import torch
    a = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_read": n_bytes, "copy_bytes_written": n_bytes, "reps": reps,
                      "ms_per_copy": dt * 1e3, "GB_per_s": 2 * n_bytes / dt / 1e9}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--spins-per-lane", type=int, default=0,
                    help="0 = the autotuner's choice (or the threshold rule with --no-tune)")
    ap.add_argument("--no-readout-split", action="store_true",
                    help="no readout replicas (PS_CFG_NO_READOUT_SPLIT); with --spins-per-lane, pins the "
                         "tuner's 'none' choice for a profiled run")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner: tiles from the threshold rule")
    ap.add_argument("--workload", choices=sorted(WORKLOADS) + ["c4", "c5", "kt"], default="c3",
                    help="c3 (default, the reported workload: 3-D shaped-pulse configuration), "
                         "c2 (2-D spin echo), c4 (batched vs one launch per request), "
                         "c5 (served stream vs FIFO)")
    ap.add_argument("--c5-requests", type=int, default=2000)
    ap.add_argument("--serve-direct", action="store_true",
                    help="c5: the served loop runs one iteration at a time with direct kernel launches "
                         "(default: HIP graph replay, short iterations launched ahead)")
    ap.add_argument("--c5-frac-3d", type=float, default=0.1,
                    help="c5: share of 3-D 2x64^3 jobs in the stream (the configuration's is 0.1)")
    ap.add_argument("--c5-rate", type=float, default=50.0,
                    help="c5: mean arrival rate of the Poisson stream, requests/s (the configuration's is 50)")
    ap.add_argument("--latency-requests", type=int, default=300,
                    help="requests of the c5 stream prefix replayed served and FIFO for the latency block "
                         "of the default run (0: leave the block out)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle time for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plan", action="store_true",
                    help="time replays of a compiled plan (HIP graph: no host compile or upload per step)")
    ap.add_argument("--coils", type=int, default=0,
                    help="receive with this many loop coils on a ring around the object (0: one homogeneous coil)")
    ap.add_argument("--no-matrix-readout", action="store_true",
                    help="sum every readout with the vector recurrence (PS_CFG_NO_MATRIX_READOUT), for comparison")
    ap.add_argument("--no-shape-cache", action="store_true",
                    help="step recurring shaped pulses sub-step by sub-step (default: propagator cache)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="instead of the workload, run a plain 1 GiB device-to-device copy 5 times "
                         "(reference kernel for scaling HBM byte counters)")
    ap.add_argument("--precision", type=int, choices=(32, 64), default=32,
                    help="32: FP32 stepping with FP64 phases and sums (default); 64: FP64 throughout")
    ap.add_argument("--valu-calibration", action="store_true",
                    help="instead of the workload, measure the attainable vector FMA rate (FP32 and FP64)")
    args = ap.parse_args()
    if args.no_matrix_readout:
        CTX_KW["matrix_readout"] = False
    if args.copy_calibration:
        copy_calibration()
        return
    if args.valu_calibration:
        valu_calibration()
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on exactly one GPU; --gpus N with N > 1 is not supported "
              "(the spin domain would shard across GPUs with one reduction of the partial signals, "
              "which is not built here)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c4":
        return bench_c4(args)
    if args.workload == "c5":
        return bench_c5(args)
    if args.workload == "kt":
        return bench_kt(args)

    import torch
    import paper_1305_6861_amd as ps
    from workloads import configs as C

    obj, seq = load_workload(args.workload)
    dev = ps.to_device(obj)
    cache = not args.no_shape_cache
    ctx = ps.Context(kernel_timing=True, spins_per_lane=args.spins_per_lane, shape_cache=cache, **CTX_KW,
                     precision=args.precision, readout_split=not args.no_readout_split)
    fp64 = args.precision == 64
    peak = PEAK_FP64_TFLOPS if fp64 else PEAK_FP32_TFLOPS
    packed = ps.pack_sequence(seq)
    n_samples, n_steps = packed.count()
    rx, rx_np = None, None
    if args.coils > 0:
        from workloads import coils as coil_maps
        rx_np = coil_maps.loop_ring(obj, args.coils, ring_radius=0.2, coil_radius=0.06)
        rx = tuple(torch.from_numpy(a).cuda() for a in rx_np)
    out = torch.empty(2 * n_samples * max(args.coils, 1), dtype=torch.float64, device="cuda")
    tune = None
    if args.spins_per_lane == 0 and not args.no_tune:
        tune = ctx.tune(dev, packed, coils=rx)
    tiling = ctx.tile_for(obj.n_spins, packed, args.coils)
    spl = tiling["spins_per_lane"]
    tiling["source"] = ("fixed" if args.spins_per_lane else "autotuner" if tiling["tuned"] else "threshold rule")
    if tune is not None:
        tiling["tuner"] = {k: tune[k] for k in ("best_ms", "rule_ms", "probe_events", "candidates")}
        tiling["tuner"]["gain_over_rule_on_probe"] = tune["rule_ms"] / tune["best_ms"]

    if args.plan:
        plan = ctx.plan(dev, packed, coils=rx)

        def step():
            plan.launch()
    else:
        def step():
            ctx.simulate(dev, packed, out=out, coils=rx)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.kernel_times()                     # forget warm-up launches

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    step_ms, fin_ms = ctx.kernel_times()
    if args.plan:
        # a replay is one graph launch on torch's current stream: bracket each
        # with events there (step and finalize kernels together)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        for a_ev, b_ev in evs:
            a_ev.record()
            step()
            b_ev.record()
        torch.cuda.synchronize()
        step_ms = [a_ev.elapsed_time(b_ev) for a_ev, b_ev in evs]
        fin_ms = 0.0

    spin_steps = float(obj.n_spins) * n_steps
    ms_per_step = 1e3 * elapsed / args.steps
    value = spin_steps * args.steps / elapsed
    shaped = any(int(x) >= 0 for x in seq.rf_shape)
    # the flops the kernel executes: a recurring shaped pulse is applied from
    # its cached propagator (when the cache is on)
    flops = algorithmic_flops(seq, obj.n_spins, args.coils, cached_shapes=cache)
    # a long sequence runs as several time slices (launches) per step: the
    # step's kernel time is the sum over its launches
    launches = len(step_ms) // max(args.steps, 1)
    k_ms = sum(step_ms) / max(args.steps, 1)
    achieved = flops / (k_ms * 1e-3) / 1e12
    # which kernel and units sum the readouts: FP32 readouts at one spin per
    # lane run on the matrix cores (dense FP32 matrix peak = FP32 vector
    # peak on MI355X, 157.3 TFLOP/s)
    path = ctx.readout_path(obj.n_spins, packed, spl, args.coils)
    variant = ""
    if not fp64 and spl == 1:
        variant = ",matrix-only" if path["matrix_only"] else ",vector-only" if path["matrix"] == 0 else ""
    kernel = "step_kernel<%s,%d%s>" % ("double" if fp64 else "float", spl, variant)
    roof = {"bound": "mfma" if path["matrix"] > 0 else "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": (traffic_from_profiles(args.workload, spl) if args.coils == 0 and not fp64 else None),
            "kernel": kernel, "readout_path": path, "kernel_ms": k_ms,
            "launches_per_step": launches,
            "kernel_ms_per_launch": k_ms / max(launches, 1),
            "flops_per_step": flops, "flops_per_launch": flops / max(launches, 1),
            "flops_basis": ("executed: 8 per ADC spin-sample, 15 per hard pulse, 23 per shaped-pulse sub-step "
                            "stepped" + (", 18 per shaped pulse applied from its cached propagator plus the "
                                         "fill (4 x 23 per sub-step, once)" if cache and shaped else "")),
            "finalize_ms_per_step": fin_ms / max(args.steps, 1)}
    if args.workload == "spiral":
        roof["flops_basis"] = ("8 per spin-sample, the unit of the recurrence readout; tabulated samples are "
                               "evaluated directly (FP32 offset phase from an FP64 anchor per 8 samples, "
                               "hardware cos/sin, the decay stepped by one multiply per sample on the "
                               "regular raster) at several times that cost")
    if args.plan:
        roof["kernel"] += " + finalize (one graph replay per step)"
        roof["timing"] = "HIP events around each graph replay on its stream"
    if cache and shaped:
        # side figure: the sub-step path's flops over the same time (what the
        # cache saves), not a roofline position
        effective = algorithmic_flops(seq, obj.n_spins, args.coils, cached_shapes=False)
        roof["effective"] = {"flops_per_step": effective, "tflops": effective / (k_ms * 1e-3) / 1e12,
                             "basis": "every shaped pulse counted as its %d-flop sub-steps, which the cached "
                                      "propagator replaces; a rate, not a fraction of the peak"
                                      % FLOPS_SHAPE_SUBSTEP}
    rec = {"metric": "spin-steps/s", "value": value, "unit": "spin-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64" if fp64 else "f32",
           "data": "synthetic",
           "config": {"workload": WORKLOADS[args.workload], "n_spins": obj.n_spins, "n_steps_per_spin": n_steps,
                      "n_samples": n_samples, "spins_per_lane": spl, "tiling": tiling,
                      "matrix_readout": CTX_KW.get("matrix_readout", True),
                      "precision": "fp64 throughout" if fp64 else "fp32 stepping, fp64 phases and cross-block sums",
                      "shape_cache": cache,
                      "receive_coils": args.coils or "one homogeneous coil",
                      "step": "plan replay (HIP graph)" if args.plan else "full call: compile, upload, kernels"},
           "eta_spins_per_s": obj.n_spins / (ms_per_step * 1e-3),
           "roofline": roof}
    if args.workload in PAPER_T78_SECONDS:
        t_paper = PAPER_T78_SECONDS[args.workload]
        rec["paper_context"] = {"t_sim_s": t_paper, "source": "Table 7.8, PARSPIN 1.5.0",
                                "hardware": "PVM cluster of 5 Sun Ultra-1 170",
                                "speedup_of_this_run": t_paper / (ms_per_step * 1e-3)}
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(obj, seq, ctx, args.cpu_seconds, rx_np)
    else:
        rec["cpu_baseline"] = None
    ctx.close()
    if args.latency_requests > 0 and not args.plan and args.coils == 0 and not fp64:
        del dev
        torch.cuda.empty_cache()
        rec["latency"] = latency_block(args.latency_requests)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
