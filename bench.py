"""Benchmark: decomposition + recomposition throughput at 513^3 on one GPU.

One step = decompose + recompose of a 513x513x513 field (full decomposition,
8 level steps) with the library's HIP path; inputs are resident in HBM before
the timed region.  Throughput = input bytes per direction / time, the
refactoring throughput the paper reports (Sec. IV-C), so one step counts
2 * N * sizeof(dtype) bytes.

Prints one JSON line.  Besides the headline (float32, sinusoid-plus-noise
field) it reports float64, the Gaussian-blob field, separate decompose and
recompose times, the single-pass copy bandwidth, the roofline of the
dominant kernel (HIP events around its launches in the timed region) and the
CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
SHAPE = (513, 513, 513)
SEED_SIN, SEED_BLOB = 1, 2

# Dominant kernel and its algorithmic bytes per level-0 launch: the method's
# floor for one level step, reading the level grid once and writing every
# node once, 2 V s.  This design's intermediates (the packed coarse values
# and the load vector, Vc each) are not part of the floor: they show up in
# the measured traffic instead.
DOMINANT = "stream_dec"


def algorithmic_bytes(kernel, shape, s):
    V = int(np.prod(shape))
    if kernel in ("stream_dec", "interp_recompose", "adjoint"):
        return 2 * V * s
    raise ValueError(kernel)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--quick", action="store_true", help="sinusoid field only, no other workloads")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the 96-field batch against serial calls (for profiling it); prints its own JSON")
    ap.add_argument("--other-only", action="store_true",
                    help="only the other plain-method workloads, --steps timed steps each; prints its own JSON "
                         "(the default run measures them this way, in a child process)")
    ap.add_argument("--dtypes", default="f32,f64", help="comma-separated subset of f32,f64 (default both; "
                                                        "--quick alone means f32)")
    return ap.parse_args()


def timed_steps(mgr, torch, x, y, r, steps, warmup, on_start=None):
    for _ in range(warmup):
        mgr.mgr_decompose(x, y)
        mgr.mgr_recompose(y, r)
    torch.cuda.synchronize()
    if on_start:
        on_start()
    t0 = time.perf_counter()
    for _ in range(steps):
        mgr.mgr_decompose(x, y)
        mgr.mgr_recompose(y, r)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def split_times(mgr, torch, x, y, r, reps=5):
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    td, tr = [], []
    for _ in range(reps):
        e[0].record()
        mgr.mgr_decompose(x, y)
        e[1].record()
        mgr.mgr_recompose(y, r)
        e[2].record()
        torch.cuda.synchronize()
        td.append(e[0].elapsed_time(e[1]))
        tr.append(e[1].elapsed_time(e[2]))
    return float(np.median(td)), float(np.median(tr))


def copy_bandwidth(mgr, torch, nbytes=1 << 30, reps=10):
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        mgr.mgr_bench_copy(a, b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        mgr.mgr_bench_copy(a, b)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del a, b
    return 2.0 * nbytes / dt / 1e9  # read + write bytes per second


def event_ms(torch, fn, reps=5, warmup=2):
    """Median milliseconds of fn() on the current stream (HIP events)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b))
    return float(np.median(out))


def batched_vs_serial(mgr, torch, synth):
    """The 96-field float32 workload: the batched launches (eager and as a
    replayed HIP graph, after autotuning) against 96 serial mgr_decompose
    calls on the same stream."""
    shapes = [s for s, _ in synth.batched_shapes()]
    xs = [torch.from_numpy(synth.batched_field(i)).to(torch.float32).cuda() for i in range(len(shapes))]
    ys = [torch.empty_like(x) for x in xs]
    nbytes = sum(x.numel() * 4 for x in xs)
    for x in xs:
        mgr.mgr_prepare(torch.float32, tuple(x.shape))

    def serial():
        for x, y in zip(xs, ys):
            mgr.mgr_decompose(x, y)

    t_serial = event_ms(torch, serial)
    plan = mgr.BatchPlan(shapes, torch.float32)
    out = {"fields": len(xs), "input_bytes": nbytes, "serial_ms": round(t_serial, 4),
           "serial_GBps": round(nbytes / t_serial / 1e6, 2)}
    want = [mgr.decompose(x) for x in xs]
    # the autotuner picks the tile geometry, launch form and chunk (model
    # fitted to probe runs of each, top three timed); both forms are then timed at the
    # best chunk of a plain sweep as well
    tuned_chunk, _, _ = plan.autotune(xs, ys, top_k=3)
    tuned_form, model = plan.tuning()
    # the sweeps below keep the tile geometry the autotuner chose
    out["autotune"] = {"form": "persistent" if tuned_form else "waves", "chunk": tuned_chunk,
                       "tile": "wide" if plan.tile() else "narrow",
                       "model_ms_a_perbyte_peritem_perdepthplane": {k: [float(f"{v:.4g}") for v in m]
                                                                     for k, m in model.items()}}
    for mode in ("waves", "persistent"):
        plan.set_mode(mode == "persistent")
        sweep = {}
        for c in (2, 4, 8, 16, 32, 64, 128):
            plan.set_config(c)
            sweep[c] = event_ms(torch, lambda: plan.decompose(xs, ys), reps=3, warmup=1)
        plan.check()
        chunk = min(sweep, key=sweep.get)
        plan.set_config(chunk)
        _, launches, items = plan.config()
        t_batch = event_ms(torch, lambda: plan.decompose(xs, ys))
        g = torch.cuda.CUDAGraph()
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            with torch.cuda.graph(g, stream=st):
                plan.decompose(xs, ys)
        t_graph = event_ms(torch, g.replay)
        plan.check()
        ok = all(torch.equal(y, w) for y, w in zip(ys, want))
        del g
        out[mode] = {"batched_ms": round(t_batch, 4), "graph_ms": round(t_graph, 4),
                     "graph_GBps": round(nbytes / t_graph / 1e6, 2),
                     "speedup_vs_serial": round(t_serial / t_graph, 3), "chunk": chunk,
                     "chunk_sweep_ms": {str(c): round(v, 3) for c, v in sweep.items()},
                     "launches": launches, "items": items,
                     "matches_serial_bitwise": bool(ok)}
    plan.close()
    best = min(("waves", "persistent"), key=lambda m: out[m]["graph_ms"])
    out["best"] = best
    out["graph_ms"] = out[best]["graph_ms"]
    out["graph_GBps"] = out[best]["graph_GBps"]
    out["speedup_vs_serial"] = out[best]["speedup_vs_serial"]
    return out


def adjoint_timing(mgr, torch, synth, oracle_free=True):
    """257^3 float32 Gaussian-blob field through the autograd function with
    the level-weighted loss sum_l 2^l ||class l||^2: forward + backward
    against the plain decomposition, and the adjoint alone."""
    shape = (257, 257, 257)
    u, _ = synth.blob_field(shape, 5)
    x = torch.from_numpy(u).to(torch.float32).cuda()
    w = torch.from_numpy(np.power(2.0, mgr.mgr_class_map(shape)).astype(np.float32)).cuda()
    y = torch.empty_like(x)
    g = torch.empty_like(x)
    mgr.mgr_prepare(torch.float32, shape)
    t_dec = event_ms(torch, lambda: mgr.mgr_decompose(x, y))
    t_adj = event_ms(torch, lambda: mgr.mgr_decompose_adjoint(x, g))

    def fwd_bwd():
        xr = x.detach().requires_grad_(True)
        out = mgr.Decompose.apply(xr, None, -1)
        (w * out * out).sum().backward()

    t_fb = event_ms(torch, fwd_bwd)
    nbytes = x.numel() * 4
    return {"shape": list(shape), "dtype": "f32", "decompose_ms": round(t_dec, 4), "adjoint_ms": round(t_adj, 4),
            "fwd_bwd_ms": round(t_fb, 4), "adjoint_GBps": round(nbytes / t_adj / 1e6, 2),
            "fwd_bwd_over_decompose": round(t_fb / t_dec, 3)}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_threads():
    """Threads the all-core leg uses: the cores this process may run on,
    capped by OMP_NUM_THREADS when it is set."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_baseline(u_sin):
    """The CPU oracle (plain C, FP64) on one step of the headline workload:
    the 513^3 sinusoid-plus-noise field (rounded to float32, as the GPU sees
    it) decomposed and recomposed once, on all the host cores this process
    may use (OpenMP over independent fibres and nodes; bitwise the same
    output as one thread) and on one thread.  Rate in the metric's unit:
    float32 input bytes (4 per node) per direction, as for the GPU."""
    import oracle

    u = u_sin.astype(np.float32).astype(np.float64)
    n = u.size
    legs = {}
    for threads in (cpu_threads(), 1):
        prev = oracle.set_threads(threads)
        t0 = time.perf_counter()
        d = oracle.decompose(u)
        oracle.recompose(d)
        legs[threads] = time.perf_counter() - t0
        oracle.set_threads(prev)
        del d
    nt = cpu_threads()
    t_all, t_one = legs[nt], legs[1]
    return {"value": round(2 * n * 4 / t_all / 1e9, 4), "unit": "GB/s", "cores": nt, "kind": "oracle",
            "sample": f"one decompose+recompose of the full 513^3 sinusoid field (FP64 oracle, "
                      f"{nt} threads, {t_all:.1f} s; one thread {t_one:.1f} s); GB/s counted as float32 "
                      f"input bytes per direction",
            "single_thread_value": round(2 * n * 4 / t_one / 1e9, 4),
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


# The other plain-method workloads (parity cases in the tests), timed for
# their throughput: (name, shape, dtype, generator, seed, nonuniform).
OTHER_WORKLOADS = [
    ("65^3_f64_sinusoid", (65, 65, 65), "f64", "sinusoid", 0, False),
    ("8193^2_f64_nonuniform", (8193, 8193), "f64", "sinusoid", 3, True),
    ("1025x1025x257_f32_nonuniform", (1025, 1025, 257), "f32", "sinusoid", 4, True),
]


def other_workloads(mgr, torch, synth, steps, warmup):
    out = {}
    for name, shape, dtn, gen, seed, nu in OTHER_WORKLOADS:
        print(f"[bench] {name}: {warmup} warmup + {steps} steps", file=sys.stderr, flush=True)
        dt = torch.float32 if dtn == "f32" else torch.float64
        s = 4 if dtn == "f32" else 8
        u, coords = getattr(synth, gen + "_field")(shape, seed, nonuniform=nu)
        x = torch.from_numpy(u).to(dt).cuda()
        del u
        y, r = torch.empty_like(x), torch.empty_like(x)
        mgr.mgr_prepare(dt, shape, coords)

        def dec():
            mgr.mgr_decompose(x, y, coords)

        def rec():
            mgr.mgr_recompose(y, r, coords)

        for _ in range(warmup):
            dec()
            rec()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_host = 0.0
        for _ in range(steps):
            h0 = time.perf_counter()
            dec()
            rec()
            t_host += time.perf_counter() - h0
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        td = event_ms(torch, dec)
        tr = event_ms(torch, rec)
        ts = event_ms(torch, lambda: (dec(), rec()))
        err = float((r - x).abs().max().item() / x.abs().max().item())
        n = x.numel()
        out[name] = {"GBps": round(2 * n * s / sec / 1e9, 2), "ms_per_step": round(sec * 1e3, 4),
                     "t_decompose_ms": round(td, 4), "t_recompose_ms": round(tr, 4),
                     "event_ms_per_step": round(ts, 4), "host_enqueue_ms_per_step": round(t_host / steps * 1e3, 4),
                     "roundtrip_max_rel_err": err}
        del x, y, r
        torch.cuda.empty_cache()
    return out


def other_workloads_isolated(steps, warmup):
    """other_workloads in a child process with a runtime state of its own.
    In the bench process, after the headline runs' split timings and the
    copy-kernel runs, the 8193^2 workload's host enqueue time grew about ten
    times (0.3 -> 3.6 ms per step, removing either earlier part removed the
    growth), which made its wall-clock rate a measure of the bench's history
    rather than of the library."""
    import subprocess
    cmd = [sys.executable, "-u", os.path.abspath(__file__), "--other-only", "--steps", str(steps),
           "--warmup", str(warmup), "--no-cpu"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"other workloads: child process exited with {r.returncode}")
    return json.loads(r.stdout.strip().splitlines()[-1])["other_workloads"]


# HBM traffic of the dominant kernel, from rocprofv3 FETCH_SIZE / WRITE_SIZE
# passes scaled by the same counters on a copy kernel of known size; valid
# only while the kernel source matches the one the counters were taken on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stream_dec_513cube_{}_counters.md")
KERNEL_SRCS = [os.path.join(ROOT, "paper_2007_04457_amd", "csrc", f) for f in (
    "mgr_internal.h", "mgr_stream_dev.h", "mgr_stream.hip")]


def measured_traffic(dt_name):
    import hashlib
    try:
        text = open(TRAFFIC_FILE.format(dt_name)).read()
        h = hashlib.sha256()
        for f in KERNEL_SRCS:
            h.update(open(f, "rb").read())
        src = h.hexdigest()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines() if line.startswith(("traffic_bytes", "source_sha256")))
    if fields.get("source_sha256", "").strip() != src:
        return None
    return int(fields["traffic_bytes"].strip())


# HBM traffic of all library kernels of one decompose + recompose step, from
# the same counter runs; valid only while no library source has changed.
STEP_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "decompose_recompose_513cube_f32_step_traffic.md")
CSRC = os.path.join(ROOT, "paper_2007_04457_amd", "csrc")


def measured_step_traffic():
    import hashlib
    try:
        text = open(STEP_TRAFFIC_FILE).read()
        h = hashlib.sha256()
        for f in sorted(os.listdir(CSRC)):
            if f.endswith((".h", ".hip", ".cpp")):
                h.update(open(os.path.join(CSRC, f), "rb").read())
        src = h.hexdigest()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines() if line.startswith(("step_bytes", "source_sha256")))
    if fields.get("source_sha256", "").strip() != src:
        return None
    return int(fields["step_bytes"].strip())


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "a multi-GPU path is not built", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2007_04457_amd as mgr
    from paper_2007_04457_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.batched_only:
        print(json.dumps({"batched": batched_vs_serial(mgr, torch, synth)}), flush=True)
        return
    if args.other_only:
        print(json.dumps({"other_workloads": other_workloads(mgr, torch, synth, args.steps, args.warmup)}),
              flush=True)
        return
    N = int(np.prod(SHAPE))
    L = mgr.mgr_max_levels(SHAPE)

    print(f"[bench] generating 513^3 fields", file=sys.stderr, flush=True)
    u_sin, _ = synth.sinusoid_field(SHAPE, SEED_SIN)
    u_blob = None if args.quick else synth.blob_field(SHAPE, SEED_BLOB)[0]

    results = {}
    roofs = {}
    dtypes = [d.strip() for d in args.dtypes.split(",") if d.strip()]
    if args.quick and "--dtypes" not in " ".join(sys.argv):
        dtypes = ["f32"]
    for dt_name, dt in (("f32", torch.float32), ("f64", torch.float64)):
        if dt_name not in dtypes:
            continue
        s = 4 if dt == torch.float32 else 8
        for fname, u in (("sinusoid", u_sin), ("blobs", u_blob)):
            if u is None:
                continue
            x = torch.from_numpy(u).to(dt).to(dev)
            y = torch.empty_like(x)
            r = torch.empty_like(x)
            mgr.mgr_prepare(dt, SHAPE)
            # the dominant kernel is timed in the sinusoid runs of both dtypes
            headline = (fname == "sinusoid")
            print(f"[bench] {dt_name} {fname}: {args.warmup} warmup + {args.steps} steps",
                  file=sys.stderr, flush=True)
            def start_timing():
                mgr.mgr_timing_read()  # clear
                mgr.mgr_timing_enable(DOMINANT, 0)
            sec = timed_steps(mgr, torch, x, y, r, args.steps, args.warmup,
                              start_timing if headline else None)
            if headline:
                ms_tot, launches = mgr.mgr_timing_read()
                mgr.mgr_timing_disable()
                if launches == 0:
                    raise RuntimeError(f"kernel {DOMINANT} was not launched at level 0")
                per_launch_ms = ms_tot / launches
                ab = algorithmic_bytes(DOMINANT, SHAPE, s)
                achieved = ab / (per_launch_ms * 1e-3) / 1e9
                roofs[dt_name] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                                  "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                                  "traffic": measured_traffic(dt_name),
                                  "kernel": DOMINANT, "level": 0, "launch_ms": round(per_launch_ms, 4),
                                  "launches": launches, "algorithmic_bytes": ab}
            td, tr = split_times(mgr, torch, x, y, r)
            torch.cuda.synchronize()
            err = float((r - x).abs().max().item() / x.abs().max().item())
            results[(dt_name, fname)] = {
                "GBps": round(2 * N * s / sec / 1e9, 2), "ms_per_step": round(sec * 1e3, 4),
                "t_decompose_ms": round(td, 4), "t_recompose_ms": round(tr, 4),
                "roundtrip_max_rel_err": err}
            del x, y, r
            torch.cuda.empty_cache()

    head_dt = "f32" if ("f32", "sinusoid") in results else dtypes[0]
    head = results[(head_dt, "sinusoid")]
    copy_gbps = copy_bandwidth(mgr, torch)
    extra = {}
    if not args.quick:
        extra["other_workloads"] = other_workloads_isolated(max(3, args.steps // 2), args.warmup)
        print("[bench] batched 96 fields vs serial", file=sys.stderr, flush=True)
        extra["batched"] = batched_vs_serial(mgr, torch, synth)
        print("[bench] adjoint / autograd at 257^3", file=sys.stderr, flush=True)
        extra["adjoint"] = adjoint_timing(mgr, torch, synth)
    out = {
        "metric": "decompose+recompose GB/s at 513^3 fp32/fp64; % HBM peak; batched vs serial",
        "value": head["GBps"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": head_dt, "data": "synthetic",
        "config": {"workload": "513^3 uniform grid, sinusoid-plus-noise field (seed 1), "
                               f"full decomposition ({L} level steps) then recomposition",
                   "shape": list(SHAPE), "nlevels": L},
        "roofline": roofs.get("f32"),
        "roofline_f64": roofs.get("f64"),
        "t_decompose_ms": head["t_decompose_ms"], "t_recompose_ms": head["t_recompose_ms"],
        "roundtrip_max_rel_err": head["roundtrip_max_rel_err"],
        "copy_kernel_GBps": round(copy_gbps, 1),
        # the paper's peak model (Sec. IV-C): achievable single-pass bandwidth
        # divided by its 8.43 passes per direction
        "paper_model_peak_GBps": round(copy_gbps / 8.43, 1),
        "frac_of_paper_model_peak": round(head["GBps"] / (copy_gbps / 8.43), 4),
        "variants": {f"{k[0]}_{k[1]}": v for k, v in results.items()},
    }
    step_bytes = measured_step_traffic()
    out["step_traffic"] = None if step_bytes is None else {
        # counter-measured bytes of every kernel of the step, as passes over
        # the field per direction (the paper's design: 8.43) and as a rate
        # over the measured step time
        "bytes": step_bytes,
        "passes_per_direction": round(step_bytes / 2 / (2 * N * 4), 3),  # float32 step
        "GBps": round(step_bytes / (head["ms_per_step"] * 1e-3) / 1e9, 1),
        "frac_of_peak": round(step_bytes / (head["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}
    out.update(extra)
    if not args.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(u_sin)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
