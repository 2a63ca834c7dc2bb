"""Benchmark of the PIV hot path on one MI355X.

A step is one pass of the whole path (predict -> validate predictor ->
correct -> validate -> vorticity) over one batch of synthetic 1 MP u8 pairs
resident in HBM (1024 x 1024, 0.04 ppp, Lamb-Oseen vortex with 20 px peak
displacement and 10% particle dropout; 16 x 16 windows at step 8 -> 128 x 128
vectors; +-4 px correction search; 3-level predictor with radii 6/2).
Pairs are independent, so by default two batches are in flight, each on
its own HIP stream with its own plan and buffers (step k on stream k mod 2):
the memory-bound stages of one batch then run beside the ALU-bound
correlation of the other.  The one-stream rate is reported beside it.

Prints ONE JSON line with pairs/s (value), Mvectors/s, p50/p99 latency of
the batched step and of a single pair, the step's accuracy against the
analytic truth, the HBM-roofline fraction of the whole step, the roofline
of the dominant kernel (the correlation stage) measured with HIP events on
its stream, the FP64 CPU oracle timed on a bounded sample of the same
workload (all cores and one thread, with its agreement with the GPU on
that pair), and the other forms of the path: the 256^2 config (plain
correction and L = 1 path), HIP-graph batches of 8, pre-processing
(high-pass, CLAHE), the 500-pair 4K u16 stream in graph batches of 8, the
differentiable SSD and its refinement, the largest image the paper runs
(8192 x 4096), the low-seeding study (fixed-centre stencil against the
argmax search), and continuous batching of a served mix of sizes against
the plain per-pair FIFO form over a sweep of offered loads.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector (dense)
PAPER_PAIRS_PER_S = 1150.0     # the paper's 1 MP pair throughput (Sec. 4.1)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--distinct", type=int, default=8, help="distinct rendered pairs in the batch")
    ap.add_argument("--streams", type=int, default=2,
                    help="batches in flight: each HIP stream has its own plan and buffers, step k runs on "
                         "stream k mod S")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the graph/serving/stream/SSD forms")
    ap.add_argument("--forms", default="all",
                    help="comma-separated forms to run beside the headline (default all): cfg1_256, "
                         "graph_batched_cfg2, preprocess_cfg2, sgm_predictor_cfg2, stream_cfg3, ssd_cfg4, "
                         "largest_8192x4096, low_seeding_wake, served_cfg5")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="seconds of arrivals per load point")
    ap.add_argument("--serve-first-scale", type=float, default=3.0,
                    help="the first (3,000 pairs/s) load point runs this many times longer")
    ap.add_argument("--serve-rates", type=float, nargs="+", default=[3000.0, 6000.0, 12000.0, 24000.0],
                    help="offered loads (pairs/s, all 12 streams together)")
    ap.add_argument("--form-reps", type=int, default=None, metavar="K",
                    help="timed repetitions in the pre-processing, semi-global and SSD forms (default: "
                         "each form's own; a small K keeps counter-collection runs short)")
    ap.add_argument("--cfg3-pairs", type=int, default=500, metavar="N",
                    help="pairs through the 4K u16 stream form (default 500; a few keep counter runs short)")
    ap.add_argument("--render-workers", type=int, default=16,
                    help="processes that render the synthetic inputs (1: in this process, e.g. under a profiler)")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run three plain device-to-device copies of MIB MiB (a known-size "
                         "reference for memory counters)")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def algorithmic(W, H, nx, ny, r):
    """Per-pair algorithmic bytes and FP32 flops of the correlation stage and
    of the whole path (what the method must touch/compute, not what a kernel
    happens to do)."""
    S = (2 * r + 1) ** 2
    xcorr_flop = 2.0 * S * W * H            # one FMA per pixel-shift product (shared by windows)
    combine_flop = 25.0 * S * nx * ny       # window sums -> coefficient, argmax
    warp_flop = 20.0 * W * H                # bilinear deformation of B
    corr_flop = xcorr_flop + combine_flop + warp_flop
    path_bytes = 2.0 * W * H + nx * ny * 17.0  # A, B in; disp 8, flags 1, omega 4, peak 4 out
    return dict(corr_flop=corr_flop, path_bytes=path_bytes)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A, B, log_fn, strip_rows=16):
    """The FP64 oracle (as it stands) on a bounded sample of one 1 MP pair of
    the workload, on the host's cores.

    All cores (OpenMP, the thread count the runtime takes): the whole path on
    the full pair (predictor, its validation, correction, validation,
    vorticity).  One thread: the full predictor, then the correction on a
    strip of `strip_rows` window rows scaled to the 128 rows of the pair,
    validation and vorticity on the full grid.  Runs before the GPU is
    touched.  Returns the baseline and the all-core run's outputs (checked
    against the GPU's results for the same pair afterwards)."""
    import ctypes

    import oracle
    gomp = ctypes.CDLL("libgomp.so.1")
    nproc = os.cpu_count() or 1
    threads = int(gomp.omp_get_max_threads())
    t0 = time.perf_counter()
    ref = oracle.run(A, B, win=16, step=8, r=4, levels=3, Rc=6, Rf=2)
    t_all = time.perf_counter() - t0
    gomp.omp_set_num_threads(1)
    try:
        t0 = time.perf_counter()
        pred = oracle.predict(A, B, 8, 16, 3, 6, 2).astype(np.float64)
        pred, _ = oracle.validate(pred, None)
        t_pred = time.perf_counter() - t0
        ys = slice(512 - 8 * strip_rows // 2 - 4, 512 + 8 * strip_rows // 2 + 4)
        ps = np.ascontiguousarray(pred[:, 64 - strip_rows // 2:64 + strip_rows // 2 + 1])
        t0 = time.perf_counter()
        oracle.correct(A[ys], B[ys], 16, 8, 4, ps)
        t_corr = (time.perf_counter() - t0) * 128.0 / (strip_rows + 1)
        t0 = time.perf_counter()
        f = ref["disp_raw"].copy()
        oracle.validate(f, ref["flags_raw"].copy())
        oracle.vorticity(f, 8)
        t_post = time.perf_counter() - t0
    finally:
        gomp.omp_set_num_threads(threads)
    t_one = t_pred + t_corr + t_post
    log_fn(f"cpu oracle ({_cpu_model()}, nproc {nproc}): all {threads} threads {t_all:.2f} s per pair; "
           f"one thread {t_one:.2f} s per pair (predict {t_pred:.2f} s, correct scaled {t_corr:.2f} s)")
    base = {"value": round(1.0 / t_all, 5), "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": "one 1024x1024 pair of the workload, the whole path, all cores",
            "single_thread": {"value": round(1.0 / t_one, 5), "unit": "pairs/s", "cores": 1,
                              "sample": f"full predictor + validation + vorticity; correction on {strip_rows + 1} "
                                        "of 128 window rows, scaled"},
            "nproc": nproc, "cpu_model": _cpu_model(),
            "vectors_per_s": round(128 * 128 / t_all, 1)}
    return base, ref


def _render(job):
    """One rendered input (runs in a worker process before the GPU is
    touched): ("cfg2", seed) | ("cfg3", k) | ("cfg5", stream, k) | ("cfg1", seed)
    | ("cfg4", k) | ("wake", seed, ppp)."""
    from paper_2504_17987_amd import synth
    kind = job[0]
    if kind == "cfg2":
        A, B, _ = synth.cfg2_pair(job[1])
        return A, B
    if kind == "cfg3":
        A, B, _ = synth.cfg3_pair(job[1])
        return A, B
    if kind == "cfg5":
        A, B, _ = synth.cfg5_pair(job[1], job[2])
        return A, B
    if kind == "cfg1":
        A, B, _ = synth.cfg1_pair(job[1])
        return A, B
    if kind == "cfg4":
        A, B, _ = synth.cfg4_pair(job[1])
        return A, B
    if kind == "wake":
        flow = synth.cylinder_wake(1024, 512)
        A, B = synth.make_pair(1024, 512, flow, job[2], noise=2.0, seed=job[1])
        return A, B
    raise KeyError(kind)


def render_all(jobs, log_fn, workers=16):
    """Render every input in a pool of worker processes (forked before the
    GPU is initialised; the workers only run numpy); workers <= 1 renders in
    this process."""
    import multiprocessing as mp
    t0 = time.perf_counter()
    n = min(workers, os.cpu_count() or 1, len(jobs))
    if n <= 1:
        out = [_render(j) for j in jobs]
    else:
        with mp.get_context("fork").Pool(n) as pool:
            out = pool.map(_render, jobs, chunksize=1)
    log_fn(f"rendered {len(jobs)} inputs in {time.perf_counter() - t0:.1f} s")
    return dict(zip(jobs, out))


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_correct_bands_cfg2_b64_traffic.txt")
CORR_SRC = os.path.join(ROOT, "paper_2504_17987_amd", "csrc", "correct.hip")


def measured_traffic():
    """Bytes per launch of the correlation kernel beyond L2 (fetch + write),
    from the committed counter summary, scaled there by a plain copy of known
    size; None when the summary is missing or was taken on another version of
    the kernel source."""
    import hashlib
    try:
        kv = {}
        with open(TRAFFIC_FILE) as f:
            for ln in f:
                if ":" in ln and not ln.startswith("#"):
                    k, v = ln.split(":", 1)
                    kv[k.strip()] = v.strip()
        with open(CORR_SRC, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
        if kv.get("source_sha256") != sha:
            return None
        return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def events(torch, n):
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def graph_batched(torch, api, A, B, kw, args):
    """Config-2 pairs through one captured HIP graph of 8 slots."""
    from paper_2504_17987_amd.serve import GraphRunner
    run = GraphRunner(api.Plan(1024, 1024, max_batch=8, **kw), 8)
    run.capture()
    n = A.shape[0]
    reps = max(8, args.steps)
    for _ in range(3):
        run.replay(8)
    torch.cuda.synchronize()
    ev = events(torch, reps + 1)
    ev[0].record(run.stream)
    for k in range(reps):
        lo = (8 * k) % n
        with torch.cuda.stream(run.stream):
            run.A.copy_(A[lo:lo + 8])
            run.B.copy_(B[lo:lo + 8])
        run.replay(8)
        ev[k + 1].record(run.stream)
    torch.cuda.synchronize()
    ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(reps)])
    # the same with a second graph (own plan and slots), replays alternating
    # between the two graphs' streams: two batches in flight
    run2 = GraphRunner(api.Plan(1024, 1024, max_batch=8, **kw), 8)
    run2.capture()
    run2.replay(8)
    runs = (run, run2)
    main = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0, e1 = events(torch, 2)
    e0.record(main)
    for r in runs:
        r.stream.wait_stream(main)
    for k in range(reps):
        lo, r = (8 * k) % n, runs[k % 2]
        with torch.cuda.stream(r.stream):
            r.A.copy_(A[lo:lo + 8])
            r.B.copy_(B[lo:lo + 8])
        r.replay(8)
    for r in runs:
        main.wait_stream(r.stream)
    e1.record(main)
    torch.cuda.synchronize()
    return {"slots": 8, "pairs_per_s": round(8 * reps / (ev[0].elapsed_time(ev[-1]) / 1e3), 1),
            "replay_p50_ms": round(float(np.percentile(ms, 50)), 4),
            "replay_p99_ms": round(float(np.percentile(ms, 99)), 4),
            "pairs_per_s_two_in_flight": round(8 * reps / (e0.elapsed_time(e1) / 1e3), 1),
            "includes": "device-to-device copy of the 8 input pairs into the graph's slots"}


def _fifo_outputs(torch, p):
    return dict(pred=torch.empty((1, 2, p.ny, p.nx), device="cuda"),
                disp=torch.empty((1, 2, p.ny, p.nx), device="cuda"),
                peak=torch.empty((1, p.ny, p.nx), device="cuda"),
                flags=torch.empty((1, p.ny, p.nx), dtype=torch.uint8, device="cuda"),
                omega=torch.empty((1, p.ny, p.nx), device="cuda"))


SERVE_SIZES = {"s": (512, 512, 16), "m": (1024, 1024, 8), "l": (2048, 2048, 4)}
SERVE_PER_STREAM = 16


def served(torch, api, synth, kw, args, log_fn, inputs):
    """The serving mix: 12 streams (4 x 512^2, 4 x 1024^2, 4 x 2048^2 u8;
    solid-body or shear flows, 0.03 ppp), each with 16 device-resident
    pairs, Poisson arrivals.  Continuous batching (per-class graphs on their
    own streams, HBM-budget admission) against the plain per-pair form (one
    eager run at a time in arrival order) on the same traces, over a sweep
    of the offered load from 3,000 pairs/s past the plain form's
    saturation; at each point p50/p99 latency, completed pairs/s and the
    batch sizes the server launched.  Then one run with a budget too small
    for every class (admission refuses the 2048^2 streams)."""
    from paper_2504_17987_amd.serve import latency_stats, make_gpu_server, poisson_trace, run_fifo, serve_trace
    per = SERVE_PER_STREAM
    cls_of = {512: "s", 1024: "m", 2048: "l"}
    stream_class, pairs = {}, {}
    for s in range(12):
        W = synth.CFG5_SIZES[s]
        stream_class[s] = cls_of[W]
        a, b = zip(*[inputs[("cfg5", s, k)] for k in range(per)])
        pairs[s] = (torch.from_numpy(np.stack(a)).cuda(), torch.from_numpy(np.stack(b)).cuda())
    free, _ = torch.cuda.mem_get_info()
    sched, ex = make_gpu_server(SERVE_SIZES, pairs, stream_class, budget=int(0.5 * free), plan_kw=kw)
    plans = {c: api.Plan(W, H, max_batch=1, **kw) for c, (W, H, _) in SERVE_SIZES.items()}
    for p in plans.values():
        p._fifo_out = _fifo_outputs(torch, p)
    streams = list(stream_class.items())
    serve_trace(sched, poisson_trace(streams, 250.0, 0.3, per, seed=6), time.perf_counter, poll=0)   # warm-up
    run_fifo(lambda c: plans[c], pairs, poisson_trace(streams, 250.0, 0.1, per, seed=7), time.perf_counter)
    r4 = lambda d: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}
    sweep = []
    for rate_total in args.serve_rates:
        secs = args.serve_seconds * (args.serve_first_scale if rate_total == args.serve_rates[0] else 1.0)
        trace = poisson_trace(streams, rate_total / 12.0, secs, per, seed=int(rate_total))
        sched.finished.clear()
        b0 = len(ex.batch_sizes)
        serve_trace(sched, trace, time.perf_counter, poll=0, deadline=60.0 + 20 * secs)
        torch.cuda.synchronize()
        st = latency_stats(trace)
        hist = np.bincount(np.array(ex.batch_sizes[b0:], dtype=np.int64), minlength=17)
        fifo = [type(r)(r.rid, r.stream, r.cls, r.item, r.arrival) for r in trace]
        run_fifo(lambda c: plans[c], pairs, fifo, time.perf_counter, deadline=120.0 + 40 * secs)
        sf = latency_stats(fifo)
        log_fn(f"served at {rate_total:.0f}/s offered ({secs:.0f} s): {st['pairs_per_s']:.0f} pairs/s, p50 "
               f"{st['p50_ms']:.3f} / p99 {st['p99_ms']:.3f} ms, {len(ex.batch_sizes) - b0} batches; plain FIFO "
               f"{sf['pairs_per_s']:.0f} pairs/s, p50 {sf['p50_ms']:.3f} / p99 {sf['p99_ms']:.3f} ms")
        sweep.append({"offered_pairs_per_s": rate_total, "seconds": secs,
                      "continuous_batching": r4(st), "plain_per_pair_fifo": r4(sf),
                      "batch_size_histogram": {str(k): int(v) for k, v in enumerate(hist) if v}})
    # admission under a budget that holds classes s and m but not l
    c = sched.classes
    budget = sum(2 * c[k].slot_bytes + 4 * c[k].stream_bytes for k in ("s", "m"))
    del sched, ex
    torch.cuda.synchronize()
    sched2, ex2 = make_gpu_server(SERVE_SIZES, pairs, stream_class, budget=budget, plan_kw=kw)
    trace = poisson_trace(streams, 250.0, min(args.serve_seconds, 3.0), per, seed=99)
    refused = serve_trace(sched2, trace, time.perf_counter, poll=0, deadline=120.0)
    torch.cuda.synchronize()
    sa = latency_stats(trace)
    admission = {"budget_bytes": budget, "admitted_streams": len(sched2.admitted),
                 "waiting_streams": len(sched2.waiting), "refused_requests": len(refused),
                 "classes_built": sorted(ex2.runners), **r4(sa)}
    log_fn(f"admission under {budget / 2**20:.0f} MiB: {len(sched2.admitted)} streams admitted, "
           f"{len(refused)} requests refused, p99 {sa['p99_ms']:.3f} ms")
    del sched2, ex2
    return {"mix": "4x512^2, 4x1024^2, 4x2048^2 u8, 16 resident pairs per stream", "sweep": sweep,
            "admission_budget": admission}


def stream_cfg3(torch, api, synth, log_fn, inputs, npairs=500, distinct=16):
    """The 3840x2160 u16 (12-bit) stream, 24/12 windows: 500 pairs in graph
    replays of 8 (62 full and one of 4), each replay preceded by the copy of
    its pairs into the graph's slots (device to device, on the graph's
    stream).  The stream cycles `distinct` rendered pairs of the advected
    flow (pair k at advection 0.5 k px), resident in HBM.  Two captured
    graphs (own plans and slots) alternate on their own streams, so two
    batches are in flight; the one-graph rate is reported beside it."""
    from paper_2504_17987_amd.serve import GraphRunner
    kw = dict(dtype="u16", win=24, step=12, radius=4, levels=3, radius_coarse=6, radius_fine=2)
    prs = [inputs[("cfg3", k)] for k in range(distinct)]
    A = torch.stack([torch.from_numpy(p[0].view(np.int16)) for p in prs]).cuda().view(torch.uint16)
    B = torch.stack([torch.from_numpy(p[1].view(np.int16)) for p in prs]).cuda().view(torch.uint16)
    runs = []
    for _ in range(2):
        run = GraphRunner(api.Plan(3840, 2160, max_batch=8, **kw), 8)
        run.capture()
        run.replay(8)
        runs.append(run)
    torch.cuda.synchronize()
    main = torch.cuda.current_stream()
    batches = [(lo, min(8, npairs - lo)) for lo in range(0, npairs, 8)]

    def timed(rs):
        e0, e1 = events(torch, 2)
        beg, end = events(torch, len(batches)), events(torch, len(batches))
        e0.record(main)
        for r in rs:
            r.stream.wait_stream(main)
        for k, (lo, n) in enumerate(batches):
            r = rs[k % len(rs)]
            beg[k].record(r.stream)
            with torch.cuda.stream(r.stream):
                for i in range(n):
                    r.A[i].copy_(A[(lo + i) % distinct], non_blocking=True)
                    r.B[i].copy_(B[(lo + i) % distinct], non_blocking=True)
            r.replay(n)
            end[k].record(r.stream)
        for r in rs:
            main.wait_stream(r.stream)
        e1.record(main)
        torch.cuda.synchronize()
        ms = np.array([beg[k].elapsed_time(end[k]) for k in range(len(batches))])
        return npairs / (e0.elapsed_time(e1) / 1e3), ms

    timed(runs)   # warm-up
    one, ms1 = timed(runs[:1])
    pps, ms = timed(runs)
    log_fn(f"cfg3 stream: {npairs} pairs in {len(batches)} replays, {pps:.0f} pairs/s with two graphs in flight "
           f"(one graph {one:.0f} pairs/s, replay p50 {np.percentile(ms1, 50):.3f} ms, with the slot copies)")
    return {"pairs": npairs, "replays": len(batches), "distinct_rendered_pairs": distinct,
            "pairs_per_s": round(pps, 1), "one_graph_pairs_per_s": round(one, 1),
            "replay_p50_ms": round(float(np.percentile(ms1, 50)), 4),
            "replay_p99_ms": round(float(np.percentile(ms1, 99)), 4),
            "replay_p50_ms_two_in_flight": round(float(np.percentile(ms, 50)), 4), "slots": 8,
            "mvec_per_s": round(pps * 320 * 180 / 1e6, 2),
            "includes": "device-to-device copy of each replay's pairs into the graph's slots"}


def cfg1_forms(torch, api, log_fn, inputs, reps=1000):
    """Config 1: one 256x256 u8 pair, 32x32 windows at step 16 (16x16
    vectors), +-8 search.  The plain correction with no predictor
    (piv_correct, pred = NULL) and the whole path with a one-level predictor
    (radius 8), each timed with HIP events around every one of `reps`
    calls."""
    A, B = inputs[("cfg1", 1000)]
    Ad, Bd = torch.from_numpy(A[None]).cuda(), torch.from_numpy(B[None]).cuda()
    P = api.Plan(256, 256, max_batch=1, win=32, step=16, radius=8, levels=1, radius_coarse=8)
    disp, peak, flags = P.correct(Ad, Bd, None)
    out = P.run(Ad, Bd)
    stream = torch.cuda.current_stream()
    res = {}
    for name, call in (("plain_correct", lambda: P.correct(Ad, Bd, None, disp, peak, flags)),
                       ("path_L1", lambda: P.run(Ad, Bd, out))):
        for _ in range(20):
            call()
        torch.cuda.synchronize()
        beg, end = events(torch, reps), events(torch, reps)
        for k in range(reps):
            beg[k].record(stream)
            call()
            end[k].record(stream)
        torch.cuda.synchronize()
        ms = np.array([beg[k].elapsed_time(end[k]) for k in range(reps)])
        res[name] = {"p50_ms": round(float(np.percentile(ms, 50)), 4), "p99_ms": round(float(np.percentile(ms, 99)), 4),
                     "reps": reps}
    log_fn(f"cfg1 256^2: plain correction p50 {res['plain_correct']['p50_ms']:.4f} ms, whole path (L=1) p50 "
           f"{res['path_L1']['p50_ms']:.4f} ms")
    return res


def largest(torch, api, synth, kw, log_fn, n=4, reps=10):
    """The largest image the paper runs (8192 x 4096 u8, 33.6 MP), batches of
    4 pairs through the whole path; the frames tile a rendered 1 MP pair."""
    A1, B1, _ = synth.cfg2_pair(2600)
    A = torch.from_numpy(np.tile(A1, (4, 8))).cuda().expand(n, -1, -1).contiguous()
    B = torch.from_numpy(np.tile(B1, (4, 8))).cuda().expand(n, -1, -1).contiguous()
    P = api.Plan(8192, 4096, max_batch=n, **kw)
    out = P.run(A, B)
    torch.cuda.synchronize()
    e0, e1 = events(torch, 2)
    e0.record()
    for _ in range(reps):
        P.run(A, B, out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    pps = n / (ms / 1e3)
    # two batches in flight: a second plan and outputs, batches alternating
    # between two streams
    P2, s2, main = api.Plan(8192, 4096, max_batch=n, **kw), torch.cuda.Stream(), torch.cuda.current_stream()
    with torch.cuda.stream(s2):
        out2 = P2.run(A, B)
    torch.cuda.synchronize()
    jobs = ((P, out, main), (P2, out2, s2))
    e0, e1 = events(torch, 2)
    e0.record(main)
    s2.wait_stream(main)
    for k in range(2 * reps):
        p, o, s = jobs[k % 2]
        with torch.cuda.stream(s):
            p.run(A, B, o)
    main.wait_stream(s2)
    e1.record(main)
    torch.cuda.synchronize()
    pps2 = 2 * reps * n / (e0.elapsed_time(e1) / 1e3)
    log_fn(f"8192x4096: {pps:.0f} pairs/s ({ms:.2f} ms per batch of {n}; two in flight {pps2:.0f} pairs/s)")
    return {"pairs_per_s": round(pps, 1), "ms_per_batch": round(ms, 3), "batch": n,
            "pairs_per_s_two_in_flight": round(pps2, 1), "mvec_per_s": round(pps * 1024 * 512 / 1e6, 1)}


def ssd_cfg4(torch, api, log_fn, inputs, n=64, distinct=8, reps=20):
    """64 pairs of 512x512 f32: forward and backward of the windowed SSD,
    and 10 steps of the on-device refinement (piv_ssd_refine) with its
    loss history."""
    from paper_2504_17987_amd import synth
    prs = [inputs[("cfg4", k)] for k in range(distinct)]
    A = torch.stack([torch.from_numpy(prs[i % distinct][0]) for i in range(n)]).cuda()
    B = torch.stack([torch.from_numpy(prs[i % distinct][1]) for i in range(n)]).cuda()
    flows = [synth.smooth_random_flow(512, 512, 16.0, 6.0, seed=4000 + 10000 + k) for k in range(distinct)]
    U = torch.stack([torch.from_numpy(synth.truth(flows[i % distinct], 512, 512, 8).astype(np.float32))
                     for i in range(n)]).cuda()
    P = api.Plan(512, 512, max_batch=n, dtype="f32", levels=1)
    g = torch.ones((n, 64, 64), device="cuda")
    loss = P.ssd_forward(A, B, U)
    gU, D = P.ssd_backward(A, B, U, g)
    Ur = U.clone()
    hist = torch.empty((n, 11), device="cuda")
    P.ssd_refine(A, B, Ur, steps=10, hist=hist)
    torch.cuda.synchronize()
    e = events(torch, 4)
    nref = min(3, reps)
    e[0].record()
    for _ in range(reps):
        P.ssd_forward(A, B, U, loss)
    e[1].record()
    for _ in range(reps):
        P.ssd_backward(A, B, U, g, gU, D)
    e[2].record()
    for _ in range(nref):
        Ur.copy_(U)
        P.ssd_refine(A, B, Ur, steps=10, hist=hist)
    e[3].record()
    torch.cuda.synchronize()
    f_ms, b_ms = e[0].elapsed_time(e[1]) / reps, e[1].elapsed_time(e[2]) / reps
    r_ms = e[2].elapsed_time(e[3]) / nref
    img = 512 * 512 * 4
    fwd_bytes = n * (2 * img + 2 * 64 * 64 * 4 + 64 * 64 * 4)
    bwd_bytes = n * (2 * img + 2 * 64 * 64 * 4 + 64 * 64 * 4 + 4 * 64 * 64 * 4)
    gbs = (fwd_bytes + bwd_bytes) / ((f_ms + b_ms) / 1e3) / 1e9
    log_fn(f"ssd: forward {f_ms:.3f} ms, backward {b_ms:.3f} ms, {gbs:.0f} GB/s algorithmic; "
           f"10 refinement steps {r_ms:.3f} ms")
    return {"batch": n, "forward_ms": round(f_ms, 4), "backward_ms": round(b_ms, 4),
            "forward_gbs": round(fwd_bytes / (f_ms / 1e3) / 1e9, 1),
            "backward_gbs": round(bwd_bytes / (b_ms / 1e3) / 1e9, 1),
            "achieved_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "refine_10_steps_ms": round(r_ms, 4),
            "refine_loss_first_last": [round(float(hist[:, 0].sum()), 2), round(float(hist[:, -1].sum()), 2)]}


def preprocess_cfg2(torch, api, A, log_fn, reps=20):
    """Pre-processing of 64 frames of the headline workload (1024^2 u8):
    high-pass background removal (radius 7) and CLAHE (8 x 8 tiles, clip 2),
    each timed with HIP events; HBM roofline by algorithmic bytes (high-pass
    reads and writes each frame once; CLAHE reads it twice and writes it
    once)."""
    n = A.shape[0]
    P = api.Plan(1024, 1024, max_batch=n, workspace=False)
    hp = torch.empty_like(A)
    cl = torch.empty_like(A)
    lut = torch.empty(P.clahe_lut_bytes(n, 8, 8), dtype=torch.uint8, device="cuda")
    P.highpass(A, hp, radius=7)
    P.clahe(hp, cl, tiles=(8, 8), clip_factor=2.0, lut=lut)
    torch.cuda.synchronize()
    e = events(torch, 3)
    e[0].record()
    for _ in range(reps):
        P.highpass(A, hp, radius=7)
    e[1].record()
    for _ in range(reps):
        P.clahe(hp, cl, tiles=(8, 8), clip_factor=2.0, lut=lut)
    e[2].record()
    torch.cuda.synchronize()
    h_ms, c_ms = e[0].elapsed_time(e[1]) / reps, e[1].elapsed_time(e[2]) / reps
    frame = 1024 * 1024
    h_gbs = n * 2 * frame / (h_ms / 1e3) / 1e9
    c_gbs = n * 3 * frame / (c_ms / 1e3) / 1e9
    log_fn(f"pre-processing 64 x 1 MP: high-pass {h_ms:.3f} ms ({h_gbs:.0f} GB/s), CLAHE {c_ms:.3f} ms "
           f"({c_gbs:.0f} GB/s)")
    return {"frames": n, "highpass_ms": round(h_ms, 4), "highpass_gbs": round(h_gbs, 1),
            "highpass_hbm_frac": round(h_gbs / HBM_PEAK_GBS, 4), "clahe_ms": round(c_ms, 4),
            "clahe_gbs": round(c_gbs, 1), "clahe_hbm_frac": round(c_gbs / HBM_PEAK_GBS, 4),
            "frames_per_s_both": round(n / ((h_ms + c_ms) / 1e3), 1)}


def sgm_predictor(torch, api, A, B, kw, T, nd, args, log_fn):
    """The headline workload with the predictor's coarsest level searched by
    semi-global matching (penalties 2 and 16 per block pixel) instead of
    block matching: the whole path per batch of 64 and the predictor alone,
    with the accuracy against the truth beside the block-matching path's."""
    nb = A.shape[0]
    res = {}
    for name, extra in (("block_matching", {}), ("semi_global", dict(sgm=True, sgm_p1=2, sgm_p2=16))):
        P = api.Plan(1024, 1024, max_batch=nb, **kw, **extra)
        out = P.run(A, B)
        pred = P.predict(A, B)
        torch.cuda.synchronize()
        e = events(torch, 3)
        reps = args.form_reps or max(5, args.steps // 2)
        e[0].record()
        for _ in range(reps):
            P.run(A, B, out)
        e[1].record()
        for _ in range(reps):
            P.predict(A, B, pred)
        e[2].record()
        torch.cuda.synchronize()
        run_ms, pred_ms = e[0].elapsed_time(e[1]) / reps, e[1].elapsed_time(e[2]) / reps
        err = (out["disp"][:nd].cpu().numpy() - T[None])[:, :, 2:-2, 2:-2]
        res[name] = {"path_ms": round(run_ms, 4), "pairs_per_s": round(nb / (run_ms / 1e3), 1),
                     "predictor_ms": round(pred_ms, 4), "rms_vs_truth_px": round(float(np.sqrt((err ** 2).mean())), 4)}
    log_fn(f"semi-global predictor: path {res['semi_global']['path_ms']:.3f} ms per 64 pairs (block matching "
           f"{res['block_matching']['path_ms']:.3f}), rms {res['semi_global']['rms_vs_truth_px']:.3f} px "
           f"(block matching {res['block_matching']['rms_vs_truth_px']:.3f})")
    return {"batch": nb, "penalties_per_block_pixel": [2, 16], **res}


def low_seeding_study(torch, api, log_fn, inputs, seeds):
    """The paper's low-seeding case (Sec. 3.2, Sec. 4.3: a cylinder wake at
    low particle concentration, 32 x 32 windows at 50% step-over), on a
    synthetic cylinder-like wake at 0.002 ppp: the a-priori 5-point stencil
    centred at zero shift against the +-4 argmax search, both after the
    same predictor and validation.  Reports, over interior nodes, the RMS
    error against the analytic truth and the share of vectors off by more
    than 1 px, before validation (raw correction) and after it."""
    from paper_2504_17987_amd import synth
    flow = synth.cylinder_wake(1024, 512)
    T = synth.truth(flow, 1024, 512, 16)
    A = torch.from_numpy(np.stack([inputs[("wake", s, 0.002)][0] for s in seeds])).cuda()
    B = torch.from_numpy(np.stack([inputs[("wake", s, 0.002)][1] for s in seeds])).cuda()
    n = len(seeds)
    res = {}
    inner = (slice(None), slice(None), slice(2, -2), slice(2, -2))
    for mode in ("fixed", "argmax"):
        P = api.Plan(1024, 512, max_batch=n, win=32, step=16, radius=4, levels=2, radius_coarse=6,
                     radius_fine=2, peak=mode)
        out = P.run(A, B)
        raw, _, _ = P.correct(A, B, out["pred"])
        torch.cuda.synchronize()
        r = {}
        for name, f in (("raw", raw), ("validated", out["disp"])):
            err = (f.cpu().numpy() - T[None])[inner]
            mag = np.sqrt((err ** 2).sum(axis=1))
            r[name] = {"rms_px": round(float(np.sqrt((err ** 2).mean())), 4),
                       "beyond_1px": round(float((mag > 1.0).mean()), 4)}
        r["outlier_share"] = round(float(((out["flags"].cpu().numpy() & 8) != 0).mean()), 4)
        res[mode] = r
    log_fn(f"low seeding (0.002 ppp, 32/16): fixed centre rms {res['fixed']['validated']['rms_px']:.3f} px, "
           f"{res['fixed']['raw']['beyond_1px']:.1%} raw beyond 1 px; argmax rms "
           f"{res['argmax']['validated']['rms_px']:.3f} px, {res['argmax']['raw']['beyond_1px']:.1%} raw beyond 1 px")
    return {"ppp": 0.002, "image": "1024x512 u8", "windows": "32x32 step 16, +-4 (argmax)", "pairs": n,
            "flow": "cylinder-like wake: 6 px free stream, 3 px deficit, alternating vortices of 2.5 px",
            **res}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the path runs on a single MI355X (asked for {args.gpus}); "
              "pairs are independent, so N GPUs would each run this benchmark on their own stream of pairs.",
              file=sys.stderr)
        sys.exit(2)
    lg = lambda *a: log(args, *a)
    W = H = 1024
    kw = dict(win=16, step=8, radius=4, levels=3, radius_coarse=6, radius_fine=2)
    nb, nd = args.batch, min(args.distinct, args.batch)
    # every input is rendered, and the CPU oracle timed, before the GPU is
    # touched (the renderers run in forked worker processes)
    jobs = [("cfg2", 2000 + i) for i in range(nd)]
    if not args.no_extras:
        want = None if args.forms == "all" else set(args.forms.split(","))
        need = lambda name: want is None or name in want
        if need("cfg1_256"):
            jobs += [("cfg1", 1000)]
        if need("stream_cfg3"):
            jobs += [("cfg3", k) for k in range(16)]
        if need("ssd_cfg4"):
            jobs += [("cfg4", k) for k in range(8)]
        if need("served_cfg5"):
            jobs += [("cfg5", s, k) for s in range(12) for k in range(SERVE_PER_STREAM)]
        if need("low_seeding_wake"):
            jobs += [("wake", 7000 + k, 0.002) for k in range(4)]
    inputs = render_all(jobs, lg, args.render_workers)
    pairs = [inputs[("cfg2", 2000 + i)] for i in range(nd)]
    cpu = ref0 = None
    if not args.no_cpu_baseline:
        cpu, ref0 = cpu_baseline(pairs[0][0], pairs[0][1], lg)

    import torch
    from paper_2504_17987_amd import api, synth

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    A = torch.empty((nb, H, W), dtype=torch.uint8, device=dev)
    B = torch.empty((nb, H, W), dtype=torch.uint8, device=dev)
    for i in range(nb):
        A[i].copy_(torch.from_numpy(pairs[i % nd][0]))
        B[i].copy_(torch.from_numpy(pairs[i % nd][1]))
    plan = api.Plan(W, H, max_batch=nb, **kw)
    nx, ny = plan.nx, plan.ny

    def outputs():
        return dict(pred=torch.empty((nb, 2, ny, nx), device=dev), disp=torch.empty((nb, 2, ny, nx), device=dev),
                    peak=torch.empty((nb, ny, nx), device=dev),
                    flags=torch.empty((nb, ny, nx), dtype=torch.uint8, device=dev),
                    omega=torch.empty((nb, ny, nx), device=dev))

    out = outputs()
    stream = torch.cuda.current_stream(dev)
    # one job per stream: independent batches of the same workload, each with
    # its own plan (workspace), inputs and outputs
    S = max(1, args.streams)
    jobs = [(plan, A, B, out, stream)]
    for _ in range(1, S):
        jobs.append((api.Plan(W, H, max_batch=nb, **kw), A.clone(), B.clone(), outputs(),
                     torch.cuda.Stream(dev)))
    torch.cuda.synchronize()
    if args.copy_probe > 0:
        src = torch.zeros(args.copy_probe << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def timed(js):
        """K steps, step k on job k mod len(js); returns (ms in total, per-step ms, wall s)."""
        for _ in range(args.warmup):
            for p, a, b, o, s in js:
                with torch.cuda.stream(s):
                    p.run(a, b, o)
        torch.cuda.synchronize()
        e0, e1 = events(torch, 2)
        beg, end = events(torch, args.steps), events(torch, args.steps)
        t0 = time.perf_counter()
        e0.record(stream)
        for _, _, _, _, s in js:
            s.wait_stream(stream)
        for k in range(args.steps):
            p, a, b, o, s = js[k % len(js)]
            beg[k].record(s)
            with torch.cuda.stream(s):
                p.run(a, b, o)
            end[k].record(s)
        for _, _, _, _, s in js:
            stream.wait_stream(s)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return e0.elapsed_time(e1), np.array([beg[k].elapsed_time(end[k]) for k in range(args.steps)]), wall

    single = None
    if S > 1:
        one_ms, _, _ = timed(jobs[:1])
        single = {"pairs_per_s": round(nb * args.steps / (one_ms / 1e3), 1),
                  "ms_per_step": round(one_ms / args.steps, 4)}
        lg(f"one stream: step {one_ms / args.steps:.3f} ms, {single['pairs_per_s']:.0f} pairs/s")
    total_ms, step_ms, wall = timed(jobs)
    ms_per_step = total_ms / args.steps
    pairs_s = nb * args.steps / (total_ms / 1e3)
    lg(f"{S} streams: step {ms_per_step:.3f} ms ({wall / args.steps * 1e3:.3f} ms wall), {pairs_s:.0f} pairs/s")

    # accuracy of the step's field against the analytic truth (interior
    # nodes of the distinct pairs) and, on the oracle's sample pair, its
    # agreement with the FP64 oracle
    T = synth.truth(synth.cfg2_flow(), W, H, 8)
    got = out["disp"][:nd].cpu().numpy()
    err = (got - T[None])[:, :, 2:-2, 2:-2]
    accuracy = {"rms_px": round(float(np.sqrt((err ** 2).mean())), 4),
                "p99_abs_px": round(float(np.percentile(np.abs(err), 99)), 4),
                "nodes": int(err[:, 0].size), "pairs": nd,
                "truth": "Lamb-Oseen displacement at the node centres, interior nodes (2 from each edge)"}
    lg(f"accuracy vs truth: rms {accuracy['rms_px']:.3f} px")
    if ref0 is not None:
        g0 = {k: v[0].cpu().numpy() for k, v in out.items()}
        d = np.abs(g0["disp"] - ref0["disp"]).max(axis=0)
        cpu["parity_on_sample"] = {
            "predictor_bit_exact": bool(np.array_equal(g0["pred"], ref0["pred"].astype(np.float32))),
            "max_abs_disp_px": float(d.max()), "vectors_beyond_0.01px": int((d > 0.01).sum()),
            "flags_equal": int((g0["flags"] == ref0["flags"]).sum()), "vectors": int(d.size),
            # vectors that would need one of the parity tests' explained
            # exemptions (near-tie, near-flat, near-threshold): those beyond
            # the tolerance or with another flag
            "exemptions_needed": int(((d > 0.01) | (g0["flags"] != ref0["flags"])).sum()),
            "omega_max_rel": float(np.abs(g0["omega"] - ref0["omega"]).max() / np.abs(ref0["omega"]).max())}
        lg(f"parity on the oracle's sample pair: max |d disp| {d.max():.2e} px, "
           f"{int((d > 0.01).sum())} vectors beyond 0.01 px")

    # dominant kernel: the correlation stage, timed alone with events on its stream
    pred = out["pred"].clone()
    disp, peakb, flags = out["disp"], out["peak"], out["flags"]
    for _ in range(3):
        plan.correct(A, B, pred, disp, peakb, flags)
    torch.cuda.synchronize()
    e0, e1 = events(torch, 2)
    e0.record(stream)
    for _ in range(args.steps):
        plan.correct(A, B, pred, disp, peakb, flags)
    e1.record(stream)
    torch.cuda.synchronize()
    corr_ms = e0.elapsed_time(e1) / args.steps
    alg = algorithmic(W, H, nx, ny, kw["radius"])
    corr_tflops = alg["corr_flop"] * nb / (corr_ms / 1e3) / 1e12
    lg(f"correct kernel {corr_ms:.3f} ms/launch, {corr_tflops:.2f} TFLOP/s algorithmic")

    lat = {}
    if not args.no_latency:
        # single pair, plain per-pair form
        p1 = api.Plan(W, H, max_batch=1, **kw)
        o1 = {k: v[:1].clone() for k, v in out.items()}
        a1, b1 = A[:1].clone(), B[:1].clone()
        for _ in range(5):
            p1.run(a1, b1, o1)
        torch.cuda.synchronize()
        xs = []
        for _ in range(100):
            s0, s1 = events(torch, 2)
            s0.record(stream)
            p1.run(a1, b1, o1)
            s1.record(stream)
            s1.synchronize()
            xs.append(s0.elapsed_time(s1))
        xs = np.array(xs)
        lat = {"pair_p50_ms": round(float(np.percentile(xs, 50)), 4),
               "pair_p99_ms": round(float(np.percentile(xs, 99)), 4)}
    lat.update({"batch_p50_ms": round(float(np.percentile(step_ms, 50)), 4),
                "batch_p99_ms": round(float(np.percentile(step_ms, 99)), 4)})

    forms = {}
    if not args.no_extras:
        want = None if args.forms == "all" else set(args.forms.split(","))
        run = lambda name: want is None or name in want
        if run("cfg1_256"):
            forms["cfg1_256"] = cfg1_forms(torch, api, lg, inputs)
        if run("graph_batched_cfg2"):
            forms["graph_batched_cfg2"] = graph_batched(torch, api, A, B, kw, args)
            lg(f"graph batches of 8: {forms['graph_batched_cfg2']['pairs_per_s']:.0f} pairs/s "
               f"(two graphs in flight {forms['graph_batched_cfg2']['pairs_per_s_two_in_flight']:.0f})")
        if run("preprocess_cfg2"):
            forms["preprocess_cfg2"] = preprocess_cfg2(torch, api, A, lg, reps=args.form_reps or 20)
        if run("sgm_predictor_cfg2"):
            forms["sgm_predictor_cfg2"] = sgm_predictor(torch, api, A, B, kw, T, nd, args, lg)
        if run("stream_cfg3"):
            forms["stream_cfg3"] = stream_cfg3(torch, api, synth, lg, inputs, npairs=args.cfg3_pairs)
        if run("ssd_cfg4"):
            forms["ssd_cfg4"] = ssd_cfg4(torch, api, lg, inputs, reps=args.form_reps or 20)
        if run("largest_8192x4096"):
            forms["largest_8192x4096"] = largest(torch, api, synth, kw, lg)
        if run("low_seeding_wake"):
            forms["low_seeding_wake"] = low_seeding_study(torch, api, lg, inputs, [7000 + k for k in range(4)])
        if run("served_cfg5"):
            forms["served_cfg5"] = served(torch, api, synth, kw, args, lg, inputs)

    path_gbs = alg["path_bytes"] * nb / (ms_per_step / 1e3) / 1e9
    line = {
        "metric": "1MP image-pair fields/sec + Mvectors/s; p50/p99 latency; % HBM roofline",
        "value": round(pairs_s, 1),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": round(pairs_s / PAPER_PAIRS_PER_S, 2),
        "baseline": {"value": PAPER_PAIRS_PER_S, "unit": "pairs/s",
                     "source": "the paper's full pipeline on 1 MP pairs, 16x16 windows at 50% overlap, "
                               "RTX 4080 (other hardware and predictor: context, not a target)"},
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1024x1024 u8 particle-image pairs (0.04 ppp, Lamb-Oseen 20 px peak, "
                               "10% dropout), 16x16 windows step 8 (128x128 vectors), +-4 px search, "
                               "3-level SAD predictor (radii 6/2), full path per step",
                   "global_batch": nb, "distinct_pairs": nd, "parallelism": "single GPU",
                   "batches_in_flight": S},
        "single_stream": single,
        "mvec_per_s": round(pairs_s * nx * ny / 1e6, 2),
        "latency": lat,
        "accuracy_vs_truth": accuracy,
        "hbm_roofline": {"achieved_gbs": round(path_gbs, 1), "peak_gbs": HBM_PEAK_GBS,
                         "frac": round(path_gbs / HBM_PEAK_GBS, 5),
                         "bytes_per_pair": alg["path_bytes"]},
        "roofline": {"kernel": "k_correct_bands (deformation + correlation + fit)", "bound": "alu",
                     "achieved": round(corr_tflops, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(corr_tflops / FP32_PEAK_TFLOPS, 5), "traffic": measured_traffic(),
                     "ms_per_launch": round(corr_ms, 4), "flop_per_pair": alg["corr_flop"],
                     "pairs_per_launch": nb},
        "forms": forms,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
