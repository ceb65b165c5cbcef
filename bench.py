"""Benchmark of the MI355X template matcher.

Default workload (config3): 4096 independent int8 +-1 instances of uneven
size (N = 2^U(16,20), K = 2^U(9,12), flips U[5%, 15%]), one tm_match_batch
per step, 1.45 GB of signals resident in HBM (every step reads all of them,
more than the 256 MB memory-side cache holds).  Other workloads: config1
(N = 2^16 int8, one match per launch), config2 (N = 2^22 +-1 stored fp32, one
match per launch), config4 (request server: open-loop p50/p99 at the offered
rate and saturation vs plain launch), config5a (N = 2^24 fp32, K = 2^14 at
-3 dB with FP32/BF16/FP16 fold storage, error against FP64), config5b (1024
signals sharing one template: tm_match_many's per-signal int8 products against
its shared-template GEMM and the FFT path).

Prints one JSON line: whole-job matches/s over the timed steps; per-step
times (HIP events on the launch stream); `roofline` for the dominant kernel
and `roofline_other` for the next one, each from HIP events carried on the
kernels' own dispatches during the timed region: the fold against 8 TB/s with
its algorithmic bytes (x read once), the correlation with the method's FFT
flops (10 P log2 P + 6 P per instance) against the FP32 vector peak whatever
route computed it (the int8 product's own executed operations are reported
beside); `serving` (default run: a short request-server sample of the serving
workload); and `cpu_baseline`, the oracle's FP64 FFT path timed on host cores
on a bounded sample of the same workload, compared with the GPU's results.
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
INT8_PEAK_TOPS = 5000.0      # dense int8 MFMA
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
METRIC = "template matches/sec + fold GB/s vs HBM peak; served p50/p99 vs plain launch"
KERNELS_SRC = os.path.join(ROOT, "paper_1509_04863_amd", "csrc", "tm_kernels.hip")

# HBM bytes per launch (FETCH_SIZE + WRITE_SIZE from rocprofv3 --pmc, each
# scaled by a plain copy's reading; summaries under profiles/), valid only for
# the kernel source they were taken on: `traffic` is null for any other.
TRAFFIC_SRC_SHA = "34199b9ee538f0be"
TRAFFIC_BYTES = {"k_fold_s8/config3": 1609298807, "corr/config3": 326735633}


def kernels_sha() -> str:
    with open(KERNELS_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_for(key):
    if not TRAFFIC_SRC_SHA or kernels_sha() != TRAFFIC_SRC_SHA:
        return None
    return TRAFFIC_BYTES.get(key)


def fft_flops(plans):
    """The method's correlation work (steps 4-6): one complex transform of
    length P each way per instance, 10 P log2 P + 6 P flops."""
    total = 0.0
    for p in plans:
        P = 1 << p.info["fft_log2"]
        total += 10.0 * P * math.log2(P) + 6.0 * P
    return total


def corr_roofline(plans, corr_ms, corr_n, traffic=None, name=None):
    """The correlation kernel against the method's FFT work: the FFT flops of
    the instances of one launch over its average duration, against the FP32
    vector peak (the precision the method's transform needs for real data).
    For the int8 product route the executed MFMA operations (2 K (M1 + M2)
    per instance and digit) are reported beside it."""
    avg_s = corr_ms / corr_n / 1e3
    info = plans[0].info
    flops = fft_flops(plans)
    achieved = flops / avg_s / 1e12
    out = {"kernel": name or ("k_cgemm" if info["corr_gemm"] else "k_finish"), "bound": "alu",
           "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
           "traffic": traffic, "avg_kernel_us": avg_s * 1e6, "algorithmic_flops_per_launch": flops}
    if info["corr_gemm"]:
        ops = sum(2.0 * p.k * (p.m1 + p.m2) for p in plans)
        out["mfma_int8_ops_per_launch_one_digit"] = ops
        out["mfma_int8_tops_one_digit"] = ops / avg_s / 1e12
    return out


def fold_roofline(kernel, fold_ms, fold_n, x_bytes, traffic=None):
    avg_s = fold_ms / fold_n / 1e3
    achieved = x_bytes / avg_s / 1e9
    return {"kernel": kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "avg_kernel_us": avg_s * 1e6,
            "algorithmic_bytes_per_launch": x_bytes}


def pick_roofline(line, fold_roof, corr_roof):
    """`roofline` is the kernel with the larger average launch time; the other
    goes into `roofline_other`."""
    roofs = [r for r in (fold_roof, corr_roof) if r is not None]
    if not roofs:
        return
    roofs.sort(key=lambda r: -r["avg_kernel_us"])
    line["roofline"] = roofs[0]
    if len(roofs) > 1:
        line["roofline_other"] = roofs[1]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 20 batches for config3, 2000 matches for config1/2)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="config3",
                    choices=["config1", "config2", "config3", "config4", "config5a", "config5b", "copy"])
    ap.add_argument("--pool", type=int, default=1024, help="device signals in the config4 pool")
    ap.add_argument("--templates", type=int, default=2048, help="distinct config4 requests (plans)")
    ap.add_argument("--rate", type=float, default=20000.0, help="config4 offered load, requests/s")
    ap.add_argument("--duration", type=float, default=10.0, help="config4 open-loop seconds")
    ap.add_argument("--batch", type=int, default=4096, help="instances per step for config3")
    ap.add_argument("--rotate-mib", type=int, default=1024)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-workers", type=int, default=0, help="oracle processes (0: the host cores, at most 16)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="config3: skip the serving sample")
    ap.add_argument("--no-profile", action="store_true", help="no kernel timing events")
    ap.add_argument("--streams", type=int, default=4, help="streams for single-match launch sequences")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 2000 if args.config in ("config1", "config2") else 20
    return args


def workload(name):
    from paper_1509_04863_amd import datagen as G
    from paper_1509_04863_amd import tm
    if name == "config2":
        return dict(make=G.config2, flags=tm.TM_F_EXACT, fold_mult=1,
                    desc="N=2^22 +-1 stored fp32, K=4096, 10% flips, one match per launch")
    return dict(make=lambda i: G.config1(i, 1), flags=0, fold_mult=1,
                desc="N=65536 +-1 int8, K=1024, 5% flips, M1=K")


def _step_stats(ms):
    import numpy as np
    a = np.asarray(ms, dtype=np.float64)
    return {"windows": int(a.size), "median_ms": float(np.median(a)), "min_ms": float(a.min()),
            "max_ms": float(a.max())}


def run_batched(args):
    """config3: every step is one tm_match_batch over the whole uneven batch;
    the fold and correlation kernels carry timing events during the timed
    steps themselves."""
    import torch

    from paper_1509_04863_amd import datagen as G
    from paper_1509_04863_amd import tm

    insts = G.config3_batch(args.batch)
    plans = [tm.Plan(s.t, n=s.n) for s in insts]
    xs = [torch.from_numpy(s.x).cuda() for s in insts]
    batch = tm.Batch(plans, xs)
    out = torch.zeros(tm.RESULT_BYTES * len(insts), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    profile = not args.no_profile
    # warmup with the timing events on as well, for as many steps as are
    # timed: every event the timed steps use is created here and reused
    tm.profile_enable(profile)
    for _ in range(max(1, args.warmup, args.steps if profile else 0)):
        batch.run(out, stream)
    torch.cuda.synchronize()
    tm.profile_enable(False)
    if profile:
        tm.profile_read(reset=True)
        tm.profile_read_corr(reset=True)
        tm.profile_enable(True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record(stream)
    h0 = time.perf_counter()
    for i in range(args.steps):
        batch.run(out, stream)
        ev[i + 1].record(stream)
    host_ms = (time.perf_counter() - h0) * 1e3 / args.steps
    torch.cuda.synchronize()
    if profile:
        tm.profile_enable(False)
    total_ms = ev[0].elapsed_time(ev[-1])
    steps_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]
    fold_ms, fold_n = tm.profile_read(reset=True) if profile else (0.0, 0)
    corr_ms, corr_n = tm.profile_read_corr(reset=True) if profile else (0.0, 0)
    results = tm.results_from_device(out)
    x_bytes = sum(s.x.nbytes for s in insts)
    t_bytes = sum(s.t.nbytes for s in insts)
    ms_per_step = total_ms / args.steps
    exact_gemm = all(p.info["corr_gemm"] for p in plans)
    line = {
        "metric": METRIC,
        "value": len(insts) * args.steps / (total_ms / 1e3), "unit": "matches/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i8 in, i32 fold, i8 MFMA correlation (i32/i64 sums)" if exact_gemm else "i8 in, i32 fold, f64 fft",
        "data": "synthetic",
        "config": {"workload": "config3: %d uneven int8 +-1 instances, N=2^U(16,20), K=2^U(9,12), "
                               "flips U[5%%,15%%], one tm_match_batch per step" % len(insts),
                   "instances": len(insts), "batch_x_bytes": x_bytes, "batch_t_bytes": t_bytes,
                   "timed_bytes": args.steps * x_bytes, "kernel_timing": "events on the timed steps' dispatches"},
        "step_times": _step_stats(steps_ms),
        "host_enqueue_ms_per_step": host_ms,
        "path_roofline": {"bound": "hbm", "achieved": (x_bytes + t_bytes) / (ms_per_step / 1e3) / 1e9,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": (x_bytes + t_bytes) / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS,
                          "algorithmic_bytes_per_step": x_bytes + t_bytes},
        "planted_recovered": "%d/%d" % (sum(int(r.shift == s.shift) for r, s in zip(results, insts)),
                                        len(insts)),
    }
    fold_roof = corr_roof = None
    if fold_n:
        fold_roof = fold_roofline("k_fold_s8", fold_ms, fold_n, x_bytes, traffic_for("k_fold_s8/config3"))
    if corr_n:
        corr_roof = corr_roofline(plans, corr_ms, corr_n, traffic_for("corr/config3"), name="k_cgemm_ring")
    pick_roofline(line, fold_roof, corr_roof)
    line["graph_replay"] = graph_replay(plans, xs, out, results, args.steps, stream)
    line["fft_route"] = fft_route(insts, xs, results, max(3, args.steps // 4), stream)
    del batch, xs
    torch.cuda.empty_cache()
    if not args.no_serving:
        line["serving"] = serving_sample(pool_size=160, templates=320, rate=args.rate, duration=2.0)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_pool("config3", args.cpu_seconds, results, args.cpu_workers)
    print(json.dumps(line), flush=True)


def graph_replay(plans, xs, out, results, steps, stream):
    """The same batch through a reusable batch (tm_batch_*: its launch
    sequence captured once in a HIP graph, one graph launch per step)."""
    import torch

    from paper_1509_04863_amd import tm
    g_out = torch.zeros_like(out)
    g = tm.BatchGraph(plans, xs, g_out, stream)
    for _ in range(2):
        g.run(stream)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    h0 = time.perf_counter()
    for _ in range(steps):
        g.run(stream)
    host_ms = (time.perf_counter() - h0) * 1e3 / steps
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    same = tm.results_from_device(g_out) == results
    g.close()
    return {"ms_per_step": ms, "matches_per_s": len(plans) / (ms / 1e3), "host_enqueue_ms_per_step": host_ms,
            "results_equal_eager": bool(same)}


def fft_route(insts, xs, results, steps, stream):
    """The same instances with the correlation by the exact FFT of steps 4-6
    (TM_F_FFT plans: FP64 transform in one workgroup's LDS) instead of the
    int8 product, for comparison."""
    import torch

    from paper_1509_04863_amd import tm
    plans = [tm.Plan(s.t, n=s.n, flags=tm.TM_F_FFT) for s in insts]
    out = torch.zeros(tm.RESULT_BYTES * len(plans), dtype=torch.uint8, device="cuda")
    batch = tm.Batch(plans, xs)
    batch.run(out, stream)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        batch.run(out, stream)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    same = sum(int(x == y) for x, y in zip(tm.results_from_device(out), results))
    return {"ms_per_step": ms, "matches_per_s": len(plans) / (ms / 1e3), "steps": steps,
            "same_results": "%d/%d" % (same, len(plans))}


def serving_sample(pool_size, templates, rate, duration, plain_rounds=3):
    """The serving workload through the request server: open-loop Poisson
    arrivals at `rate` for `duration` seconds (p50/p99 latency from
    submission to result), then closed-loop saturation throughput of the
    server and of the plain path (one synchronous tm_match per request), and
    whether every served result equals the plain one."""
    import threading

    import numpy as np
    import torch

    from paper_1509_04863_amd import datagen as G
    from paper_1509_04863_amd import tm

    pool = G.config4_pool(pool_size)
    xs = [torch.from_numpy(s.x).cuda() for s in pool]
    reqs = G.config4_requests(pool, templates, rate_hz=rate)
    plans = [tm.Plan(r.t, n=pool[r.pool_id].n, x_dtype=tm.tm_dtype_of(pool[r.pool_id].x)) for r in reqs]
    req_x = [xs[r.pool_id] for r in reqs]
    torch.cuda.synchronize()
    nreq = len(reqs)
    rng = np.random.default_rng(7)
    count = max(1, int(rate * duration))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=count))
    lat = np.zeros(count)
    with tm.Server(budget_bytes=2 << 30, max_batch=512, max_inflight=3) as srv:
        for i in range(min(64, nreq)):                      # warm-up
            srv.wait(srv.submit(plans[i], req_x[i]))
        tickets = [None] * count
        ready = threading.Semaphore(0)

        def consume():
            for i in range(count):
                ready.acquire()
                _, lat[i] = srv.wait(tickets[i])

        th = threading.Thread(target=consume)
        th.start()
        t0 = time.perf_counter()
        for i in range(count):
            while time.perf_counter() - t0 < arrivals[i]:
                pass
            j = i % nreq
            tickets[i] = srv.submit(plans[j], req_x[j])
            ready.release()
        th.join()
        open_s = time.perf_counter() - t0
        open_stats = srv.stats()
        # closed loop: the whole request set queued at once, several rounds
        rounds = 10
        t0 = time.perf_counter()
        ts = [srv.submit(plans[i % nreq], req_x[i % nreq]) for i in range(rounds * nreq)]
        served = [srv.wait(t)[0] for t in ts]
        served_s = time.perf_counter() - t0
        held = srv.stats()
    for i in range(min(16, nreq)):
        tm.match(plans[i], req_x[i])
    t0 = time.perf_counter()
    plain = [tm.match(plans[i], req_x[i]) for i in range(nreq)]
    for _ in range(plain_rounds - 1):
        for i in range(nreq):
            tm.match(plans[i], req_x[i])
    plain_s = (time.perf_counter() - t0) / plain_rounds
    same = sum(int(a == b) for a, b in zip(served[:nreq], plain))
    served_rate = rounds * nreq / served_s
    plain_rate = nreq / plain_s
    lat_ms = lat / 1e6
    return {"workload": "config4: Poisson %.0f req/s for %.1f s over %d distinct requests on a pool of %d "
                        "signals (N=2^U(14,24), 70%% int8 +-1 / 30%% fp32 N(0,1)), K=2^U(8,13), templates at 0 dB"
                        % (rate, duration, nreq, len(pool)),
            "pool_bytes": int(sum(s.x.nbytes for s in pool)),
            "offered_rate": rate, "open_loop_requests": count, "open_loop_s": open_s,
            "achieved_open_rate": count / open_s,
            "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
            "mean_batch": open_stats["completed"] / max(1, open_stats["batches"]),
            "served_matches_per_s": served_rate, "plain_matches_per_s": plain_rate,
            "served_vs_plain": served_rate / plain_rate,
            "served_equals_plain": "%d/%d" % (same, nreq),
            "server_peak_inflight_bytes": held["peak_inflight_bytes"],
            "planted_recovered": "%d/%d" % (sum(int(r.shift == q.shift) for r, q in zip(plain, reqs)), nreq)}


def run_serving(args):
    """config4 at its stated shape: the request server under open-loop
    Poisson arrivals, then saturation against the plain path."""
    sv = serving_sample(pool_size=args.pool, templates=args.templates, rate=args.rate, duration=args.duration)
    line = {
        "metric": METRIC, "value": sv["served_matches_per_s"], "unit": "matches/s", "n_gpus": 1,
        "steps": 10, "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "i32 fold (int8 signals), f32 fold (fp32 signals), f32 fft", "data": "synthetic",
        "config": {"workload": sv["workload"], "pool_bytes": sv["pool_bytes"]},
        "serving": sv,
    }
    print(json.dumps(line), flush=True)


def run_precision(args):
    """config5a: one N = 2^24 fp32 N(0,1) signal per match, K = 2^14 at -3 dB,
    for each fold storage (FP32, BF16, FP16): matches/s over signals rotated
    beyond 1 GiB, the fold kernel's HBM rate, and against the oracle's FP64
    correlation the normwise error of r and the argmax agreement."""
    import numpy as np
    import torch

    from paper_1509_04863_amd import datagen as G
    from paper_1509_04863_amd import tm

    rot = max(1, min(32, math.ceil(args.rotate_mib * 2 ** 20 / (4 << 24))))
    insts = [G.config5a(i) for i in range(rot)]
    xs = [torch.from_numpy(s.x).cuda() for s in insts]
    x_bytes = insts[0].x.nbytes
    stream = torch.cuda.current_stream()
    stores = {"f32": tm.TM_F32, "bf16": tm.TM_BF16, "f16": tm.TM_F16}
    per = {}
    for name, st in stores.items():
        plans = [tm.Plan(s.t, n=s.n, fold_store=st) for s in insts]
        out = torch.zeros(tm.RESULT_BYTES * rot, dtype=torch.uint8, device="cuda")
        for i in range(max(args.warmup, rot)):
            tm.match_into(plans[i % rot], xs[i % rot], out, i % rot, stream)
        torch.cuda.synchronize()
        tm.profile_read(reset=True)
        tm.profile_read_corr(reset=True)
        tm.profile_enable(not args.no_profile)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for i in range(args.steps):
            tm.match_into(plans[i % rot], xs[i % rot], out, i % rot, stream)
        b.record(stream)
        torch.cuda.synchronize()
        tm.profile_enable(False)
        ms = a.elapsed_time(b)
        fold_ms, fold_n = tm.profile_read(reset=True)
        entry = {"matches_per_s": args.steps / (ms / 1e3), "ms_per_match": ms / args.steps,
                 "timed_signals": min(args.steps, rot), "timed_bytes": min(args.steps, rot) * x_bytes}
        if fold_n:
            entry["fold"] = fold_roofline("k_fold_band", fold_ms, fold_n, x_bytes)
        if not args.no_cpu:
            entry.update(cpu_precision_leg(plans, xs, insts, 2))
        per[name] = entry
        del plans
    f32 = per["f32"]
    line = {
        "metric": METRIC, "value": f32["matches_per_s"], "unit": "matches/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": f32["ms_per_match"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (fold storage f32; bf16 and f16 beside)",
        "data": "synthetic",
        "config": {"workload": "config5a: N=2^24 fp32 N(0,1), K=2^14, template at -3 dB, one match per launch",
                   "signals_rotated": rot, "rotated_bytes": rot * x_bytes},
        "storage": per,
    }
    if "fold" in f32:
        line["roofline"] = f32["fold"]
    print(json.dumps(line), flush=True)


def cpu_precision_leg(plans, xs, insts, count):
    """The oracle's FP64 path on the first `count` signals of the precision
    workload (timed at one core), against the GPU's intermediates through the
    C ABI: normwise error of r and agreement of the argmaxes and the shift."""
    import numpy as np

    from oracle import ftm as O
    from paper_1509_04863_amd import tm
    errs, agree, busy, bounds = [], 0, 0.0, []
    for i in range(min(count, len(plans))):
        res, y1, y2, r1, r2 = tm.match_intermediates(plans[i], xs[i])
        bounds.append(res.err_bound)
        t0 = time.perf_counter()
        ref = O.ftm(insts[i].x.astype(np.float64), insts[i].t.astype(np.float64), plans[i].m1, plans[i].m2,
                    correlation="fft")
        busy += time.perf_counter() - t0
        errs.append(max(float(np.max(np.abs(r1 - ref.r1)) / np.max(np.abs(ref.r1))),
                        float(np.max(np.abs(r2 - ref.r2)) / np.max(np.abs(ref.r2)))))
        agree += int((res.m1_tilde, res.m2_tilde, res.shift) == (ref.m1_tilde, ref.m2_tilde, ref.shift))
    return {"normwise_r_error_vs_fp64": errs, "result_err_bound": bounds,
            "argmax_and_shift_agree_with_fp64": "%d/%d" % (agree, len(errs)),
            "oracle_matches_per_s_one_core": len(errs) / busy if busy > 0 else None}


def run_shared(args):
    """config5b: 1024 int8 +-1 signals of N=2^18 sharing one K=1024 template,
    one tm_match_many per step (its default route: one int8 MFMA product per
    signal in one batch); the same call with the shared-template GEMM
    (TM_MANY_GEMM=1) and through the FFT correlation (TM_F_FFT) for
    comparison."""
    import torch

    from paper_1509_04863_amd import datagen as G
    from paper_1509_04863_amd import tm

    insts = G.config5b_batch(count=1024)
    plan = tm.Plan(insts[0].t, n=insts[0].n)
    xs = [torch.from_numpy(s.x).cuda() for s in insts]
    many = tm.Many(plan, xs)
    out = torch.zeros(tm.RESULT_BYTES * len(xs), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def timed(steps):
        for _ in range(args.warmup):
            many.run(out, stream)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            many.run(out, stream)
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    ms_batch = timed(args.steps)            # the default: per-signal int8 products in one batch
    res_batch = tm.results_from_device(out)
    os.environ["TM_MANY_GEMM"] = "1"        # one GEMM against the shared template
    ms_gemm = timed(args.steps)
    res_gemm = tm.results_from_device(out)
    os.environ.pop("TM_MANY_GEMM")
    many = tm.Many(tm.Plan(insts[0].t, n=insts[0].n, flags=tm.TM_F_FFT), xs)
    ms_fft = timed(max(5, args.steps // 4))  # the FFT correlation of steps 4-6
    res_fft = tm.results_from_device(out)
    x_bytes = sum(s.x.nbytes for s in insts)
    hits = sum(int(r.shift == s.shift) for r, s in zip(res_batch, insts))
    line = {
        "metric": "template matches/sec + fold GB/s vs HBM peak; served p50/p99 vs plain launch",
        "value": len(xs) / (ms_batch / 1e3), "unit": "matches/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_batch, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "i8 MFMA (i32/i64 sums)", "data": "synthetic",
        "config": {"workload": "config5b: 1024 int8 +-1 signals, N=2^18, shared K=1024 template, "
                               "one tm_match_many per step", "batch_x_bytes": x_bytes},
        "fft_path": {"ms_per_step": ms_fft, "matches_per_s": len(xs) / (ms_fft / 1e3),
                     "speedup_over_fft": ms_fft / ms_batch,
                     "same_results": "%d/%d" % (sum(int(a == b) for a, b in zip(res_batch, res_fft)), len(xs))},
        "shared_template_gemm": {"ms_per_step": ms_gemm, "matches_per_s": len(xs) / (ms_gemm / 1e3),
                                 "same_results": "%d/%d" % (sum(int(a == b) for a, b in zip(res_batch, res_gemm)),
                                                            len(xs))},
        "planted_recovered": "%d/%d" % (hits, len(xs)),
    }
    print(json.dumps(line), flush=True)


def _oracle_make(name):
    from paper_1509_04863_amd import datagen as G
    return {"config1": lambda i: G.config1(i, 1), "config2": G.config2, "config3": G.config3}[name]


def _oracle_worker(job):
    """One oracle process: instances wid, wid + stride, ... of the named
    workload through the oracle's FP64 FFT path (steps 2-9) until `budget_s`
    seconds of oracle time or `limit`; generating an instance is not timed."""
    name, wid, stride, budget_s, limit = job
    from oracle import ftm as O
    make = _oracle_make(name)
    busy, done, i = 0.0, [], wid
    while i < limit and (busy < budget_s or not done):
        inst = make(i)
        m1, m2 = O.choose_moduli(inst.n, inst.k)
        t0 = time.perf_counter()
        ref = O.ftm(inst.x, inst.t, m1, m2, correlation="fft")
        busy += time.perf_counter() - t0
        done.append((i, int(ref.shift), int(ref.m1_tilde), int(ref.m2_tilde)))
        i += stride
    return busy, done


def _agreement(done, gpu_results):
    agree = checked = 0
    for i, shift, m1t, m2t in done:
        if i < len(gpu_results):
            g = gpu_results[i]
            checked += 1
            agree += int((g.shift, g.m1_tilde, g.m2_tilde) == (shift, m1t, m2t))
    return "%d/%d" % (agree, checked)


def cpu_baseline_pool(name, budget_s, gpu_results, workers=0):
    """The oracle's vectorised path (fold, FP64 numpy FFT correlation, argmax,
    resolve) on the batch's own instances, spread over the host cores in
    separate processes; the rate is the sum of the processes' rates."""
    import concurrent.futures
    import multiprocessing
    cores = workers or min(16, len(os.sched_getaffinity(0)))
    ctx = multiprocessing.get_context("spawn")      # fresh interpreters: nothing of the GPU process
    jobs = [(name, w, cores, budget_s, len(gpu_results)) for w in range(cores)]
    t0 = time.perf_counter()
    with concurrent.futures.ProcessPoolExecutor(max_workers=cores, mp_context=ctx) as ex:
        parts = list(ex.map(_oracle_worker, jobs))
    wall = time.perf_counter() - t0
    done = [d for _, ds in parts for d in ds]
    rate = sum(len(ds) / b for b, ds in parts if b > 0)
    return {"value": rate, "unit": "matches/s", "cores": cores, "kind": "oracle",
            "sample": "%d instances of the timed batch (indices strided over %d processes), oracle steps 2-9 "
                      "with the FP64 numpy FFT correlation, %.1f s of oracle time per process at most "
                      "(%.1f s wall); instance generation not timed" % (len(done), cores, budget_s, wall),
            "gpu_agrees_on": _agreement(done, gpu_results)}


def cpu_baseline_single(name, budget_s, gpu_results):
    """Single-instance workloads: the oracle's FFT path at one core."""
    busy, done = _oracle_worker((name, 0, 1, budget_s, 1 << 30))
    return {"value": len(done) / busy, "unit": "matches/s", "cores": 1, "kind": "oracle",
            "sample": "%d instances of the same workload (seeds 0..%d), oracle steps 2-9 with the FP64 numpy "
                      "FFT correlation, %.1f s" % (len(done), len(done) - 1, busy),
            "gpu_agrees_on": _agreement(done, gpu_results)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the matcher has no multi-GPU path (matches are "
              "independent; a deployment runs one process per GPU)", file=sys.stderr)
        sys.exit(2)
    # one hardware queue for each launch stream plus the main stream (read by
    # the HIP runtime when it starts, so set before torch touches the GPU):
    # with fewer, two streams share a queue and their kernels serialise
    want_queues = args.streams + 1
    if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < want_queues:
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(want_queues, 16))

    import numpy as np
    import torch

    from paper_1509_04863_amd import tm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.config == "copy":          # calibration for rocprofv3 FETCH_SIZE / WRITE_SIZE
        a = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(max(1, args.steps)):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": a.numel() * 4, "launches": max(1, args.steps)}))
        return
    if args.config == "config3":
        run_batched(args)
        return
    if args.config == "config4":
        run_serving(args)
        return
    if args.config == "config5a":
        run_precision(args)
        return
    if args.config == "config5b":
        run_shared(args)
        return
    wl = workload(args.config)
    first = wl["make"](0)
    x_bytes = first.x.nbytes
    rot = max(1, min(256, math.ceil(args.rotate_mib * 2 ** 20 / x_bytes)))
    insts = [first] + [wl["make"](i) for i in range(1, rot)]
    plans = [tm.Plan(s.t, n=s.n, fold_mult=wl["fold_mult"], flags=wl["flags"]) for s in insts]
    xs = [torch.from_numpy(s.x).cuda() for s in insts]
    out = torch.zeros(tm.RESULT_BYTES * rot, dtype=torch.uint8, device="cuda")
    main_stream = torch.cuda.current_stream()
    # independent single-match launch sequences, round-robin over the streams:
    # one match's one-workgroup finish overlaps the next match's fold
    streams = [torch.cuda.Stream() for _ in range(max(1, args.streams))]

    def issue(count, first_i=0):
        for i in range(count):
            j = (first_i + i) % rot
            tm.match_into(plans[j], xs[j], out, j, streams[i % len(streams)])

    def fence_in():
        for st in streams:
            st.wait_stream(main_stream)

    def fence_out():
        for st in streams:
            main_stream.wait_stream(st)

    fence_in()
    # every (signal, stream) pair of the timed region at least once
    warm_matches = max(args.warmup, min(args.steps, math.lcm(rot, len(streams))))
    issue(warm_matches)
    fence_out()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(main_stream)
    fence_in()
    issue(args.steps)
    fence_out()
    stop.record(main_stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)

    # fold kernel alone: HIP events around every fold launch, one stream, after the timed run
    fold_ms, fold_n, corr_ms, corr_n = 0.0, 0, 0.0, 0
    if not args.no_profile:
        tm.profile_read(reset=True)
        tm.profile_read_corr(reset=True)
        tm.profile_enable(True)
        for i in range(min(args.steps, 100)):
            j = i % rot
            tm.match_into(plans[j], xs[j], out, j, main_stream)
        torch.cuda.synchronize()
        tm.profile_enable(False)
        fold_ms, fold_n = tm.profile_read(reset=True)
        corr_ms, corr_n = tm.profile_read_corr(reset=True)

    # every rotated signal once more (untimed), so that each result slot the
    # oracle comparison reads holds a match
    for j in range(rot):
        tm.match_into(plans[j], xs[j], out, j, main_stream)
    torch.cuda.synchronize()
    results = tm.results_from_device(out)
    planted_ok = sum(int(r.shift == s.shift) for r, s in zip(results, insts))
    ms_per_step = total_ms / args.steps
    value = args.steps / (total_ms / 1e3)
    info = plans[0].info
    p_len = 1 << info["fft_log2"]
    timed_signals = min(args.steps, rot)
    line = {
        "metric": METRIC,
        "value": value, "unit": "matches/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": ("i32 fold, i8 MFMA correlation (exact)" if info["corr_gemm"] else "i32 fold, f64 fft")
        if info["exact"] else "f32",
        "data": "synthetic",
        "config": {"workload": args.config + ": " + wl["desc"], "n": first.n, "k": first.k,
                   "m1": info["m1"], "m2": info["m2"], "fft_len": p_len,
                   "x_dtype": str(first.x.dtype), "signals_rotated": rot,
                   "timed_signals": timed_signals, "timed_distinct_bytes": timed_signals * x_bytes,
                   "streams": len(streams), "warmup_matches": warm_matches,
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
                   "fold_kernel": "k_fold_band" if info["fold_bands"] else
                                  ("k_fold_s8" if info["fold_segments"] else "k_fold"),
                   "kernel_timing": "events on the dispatches of a single-stream pass after the timed region"},
        "planted_recovered": "%d/%d" % (planted_ok, rot),
    }
    fold_roof = corr_roof = None
    if fold_n:
        fold_roof = fold_roofline(line["config"]["fold_kernel"], fold_ms, fold_n, x_bytes,
                                  traffic_for(line["config"]["fold_kernel"] + "/" + args.config))
    if corr_n:
        corr_roof = corr_roofline([plans[0]], corr_ms, corr_n, traffic_for("corr/" + args.config))
    pick_roofline(line, fold_roof, corr_roof)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_single(args.config, args.cpu_seconds, results)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
