"""Benchmark of the MI355X template matcher.

Default workload (config2): one large instance per step (N = 2^22 +-1 values
stored as fp32, K = 4096, 10% template sign flips, M1 = 4096, M2 = 4097), one
match per launch sequence, sequences issued round-robin over a few streams,
inputs resident in HBM and rotated over >= 1 GiB of distinct signals so the
256 MB memory-side cache does not serve them.  Other workloads: config1
(N = 2^16 int8), config3 (4096 uneven int8 instances per launch), config4
(request server: open-loop p50/p99 and saturation vs plain launch), config5b
(1024 signals sharing one template: int8 MFMA GEMM vs the FFT path).

Prints one JSON line: whole-job matches/s; the roofline of the dominant
kernel, the fold (HBM bytes against 8 TB/s) or the correlation (int8 matrix
product: 2 K (M1 + M2) operations per match against 5 POP/s; FFT finish: its
FFT flops against the FP64 or FP32 vector peak), both timed by HIP events
carried on the kernels' own dispatches in a separate single-stream run, the
other one reported beside it; and the CPU oracle timed on a bounded sample of
the same workload.  Single-match warmup runs every rotated signal's plan once
on each stream the timed region uses it on: a plan's first match on a stream
uploads its device copy of the instance.
"""

import argparse
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

# HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE, scaled by a
# plain copy's readings (profiles/hbm_traffic_config2_config3.txt): the fold
# kernel (key = workload) and the int8 correlation kernel (workload + "_corr"),
# valid for the kernels as those counters saw them
TRAFFIC_BYTES = {"config2": 1.828e7, "config3": 1.561e9, "config2_corr": 8.602e5, "config3_corr": 7.52e8}


def corr_roofline(plans, corr_ms, corr_n, traffic=None):
    """The correlation kernel's roofline from its average launch time: the
    int8 matrix product against the int8 MFMA peak (algorithmic operations
    2 K (M1 + M2) per match), or the FFT finish against the vector peak of its
    precision (2 transforms of 5 P log2 P flops plus 6 P per match)."""
    avg_s = corr_ms / corr_n / 1e3
    info = plans[0].info
    if info["corr_gemm"]:
        ops = sum(2.0 * p.k * (p.m1 + p.m2) for p in plans)
        achieved = ops / avg_s / 1e12
        return {"kernel": "k_cgemm", "bound": "mfma", "achieved": achieved, "peak": INT8_PEAK_TOPS,
                "unit": "TOP/s", "frac": achieved / INT8_PEAK_TOPS, "traffic": traffic,
                "avg_kernel_us": avg_s * 1e6, "algorithmic_ops_per_launch": ops}
    flops = 0.0
    for p in plans:
        P = 1 << p.info["fft_log2"]
        flops += 10.0 * P * math.log2(P) + 6.0 * P
    peak = FP64_PEAK_TFLOPS if info["exact"] else FP32_PEAK_TFLOPS
    achieved = flops / avg_s / 1e12
    return {"kernel": "k_finish", "bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": traffic, "avg_kernel_us": avg_s * 1e6,
            "algorithmic_flops_per_launch": flops}


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
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="config2",
                    choices=["config1", "config2", "config3", "config4", "config5b", "copy"])
    ap.add_argument("--pool", type=int, default=96, help="device signals in the config4 pool")
    ap.add_argument("--templates", type=int, default=384, help="distinct config4 requests (plans)")
    ap.add_argument("--rate", type=float, default=20000.0, help="config4 offered load, requests/s")
    ap.add_argument("--duration", type=float, default=2.0, help="config4 open-loop seconds")
    ap.add_argument("--batch", type=int, default=4096, help="instances per step for config3")
    ap.add_argument("--rotate-mib", type=int, default=1024)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the fold-kernel event timing")
    ap.add_argument("--streams", type=int, default=4, help="streams for single-match launch sequences")
    ap.add_argument("--traffic-bytes", type=float, default=None,
                    help="HBM bytes per fold launch from rocprofv3 FETCH_SIZE + WRITE_SIZE (scaled)")
    return ap.parse_args()


def workload(name):
    from paper_1509_04863_amd import datagen as G
    from paper_1509_04863_amd import tm
    if name == "config2":
        return dict(make=G.config2, flags=tm.TM_F_EXACT, fold_mult=1,
                    desc="N=2^22 +-1 stored fp32, K=4096, 10% flips, one match per launch")
    return dict(make=lambda i: G.config1(i, 1), flags=0, fold_mult=1,
                desc="N=65536 +-1 int8, K=1024, 5% flips, M1=K")


def run_batched(args):
    """config3: every step is one tm_match_batch over the whole uneven batch."""
    import numpy as np
    import torch

    from paper_1509_04863_amd import datagen as G
    from paper_1509_04863_amd import tm

    insts = G.config3_batch(args.batch)
    plans = [tm.Plan(s.t, n=s.n) for s in insts]
    xs = [torch.from_numpy(s.x).cuda() for s in insts]
    batch = tm.Batch(plans, xs)
    out = torch.zeros(48 * len(insts), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        batch.run(out, stream)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(args.steps):
        batch.run(out, stream)
    stop.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    fold_ms, fold_n, corr_ms, corr_n = 0.0, 0, 0.0, 0
    if not args.no_profile:
        tm.profile_read(reset=True)
        tm.profile_read_corr(reset=True)
        tm.profile_enable(True)
        for _ in range(args.steps):
            batch.run(out, stream)
        torch.cuda.synchronize()
        tm.profile_enable(False)
        fold_ms, fold_n = tm.profile_read(reset=True)
        corr_ms, corr_n = tm.profile_read_corr(reset=True)
    results = tm.results_from_device(out)
    x_bytes = sum(s.x.nbytes for s in insts)
    ms_per_step = total_ms / args.steps
    line = {
        "metric": "template matches/sec + fold GB/s vs HBM peak; served p50/p99 vs plain launch",
        "value": len(insts) * args.steps / (total_ms / 1e3), "unit": "matches/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i32 fold, i8 MFMA correlation (exact)" if all(p.info["corr_gemm"] for p in plans)
        else "i32 fold, f64 fft", "data": "synthetic",
        "config": {"workload": "config3: %d uneven int8 +-1 instances, N=2^U(16,20), K=2^U(9,12), "
                               "flips U[5%%,15%%], one batch per step" % len(insts),
                   "instances": len(insts), "batch_x_bytes": x_bytes},
        "planted_recovered": "%d/%d" % (sum(int(r.shift == s.shift) for r, s in zip(results, insts)),
                                        len(insts)),
    }
    fold_roof = corr_roof = None
    if fold_n:
        avg_s = fold_ms / fold_n / 1e3
        achieved = x_bytes / avg_s / 1e9
        fold_roof = {"kernel": "k_fold_s8", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": args.traffic_bytes if args.traffic_bytes is not None
                     else TRAFFIC_BYTES.get("config3"),
                     "avg_kernel_us": avg_s * 1e6, "algorithmic_bytes_per_launch": x_bytes}
    if corr_n:
        corr_roof = corr_roofline(plans, corr_ms, corr_n, TRAFFIC_BYTES.get("config3_corr"))
    pick_roofline(line, fold_roof, corr_roof)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(lambda i: insts[i], args.cpu_seconds, results)
    print(json.dumps(line), flush=True)


def run_serving(args):
    """config4: open-loop Poisson arrivals into the request server (p50/p99
    latency), then closed-loop saturation throughput of the server and of the
    plain path (one synchronous tm_match per request)."""
    import threading

    import numpy as np
    import torch

    from paper_1509_04863_amd import datagen as G
    from paper_1509_04863_amd import tm

    pool = G.config4_pool(args.pool)
    xs = [torch.from_numpy(s.x).cuda() for s in pool]
    reqs = G.config4_requests(pool, args.templates, rate_hz=args.rate)
    plans = [tm.Plan(r.t, n=pool[r.pool_id].n, x_dtype=tm.tm_dtype_of(pool[r.pool_id].x)) for r in reqs]
    req_x = [xs[r.pool_id] for r in reqs]
    torch.cuda.synchronize()
    nreq = len(reqs)

    # open loop at the offered rate
    rng = np.random.default_rng(7)
    count = max(1, int(args.rate * args.duration))
    arrivals = np.cumsum(rng.exponential(1.0 / args.rate, size=count))
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
        rounds = 20
        t0 = time.perf_counter()
        ts = [srv.submit(plans[i % nreq], req_x[i % nreq]) for i in range(rounds * nreq)]
        served = [srv.wait(t)[0] for t in ts]
        served_s = time.perf_counter() - t0
    # plain path on the same requests
    for i in range(min(16, nreq)):
        tm.match(plans[i], req_x[i])
    t0 = time.perf_counter()
    plain = [tm.match(plans[i], req_x[i]) for i in range(nreq)]
    for _ in range(2):
        for i in range(nreq):
            tm.match(plans[i], req_x[i])
    plain_s = (time.perf_counter() - t0) / 3
    same = sum(int(a == b) for a, b in zip(served[:nreq], plain))
    recovered = sum(int(r.shift == q.shift) for r, q in zip(plain, reqs))
    served_rate = rounds * nreq / served_s
    plain_rate = nreq / plain_s
    lat_ms = lat / 1e6
    line = {
        "metric": "template matches/sec + fold GB/s vs HBM peak; served p50/p99 vs plain launch",
        "value": served_rate, "unit": "matches/s", "n_gpus": 1, "steps": rounds, "warmup": 1,
        "ms_per_step": served_s / rounds * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "i32 fold + f32 fft (real templates)", "data": "synthetic",
        "config": {"workload": "config4: serving, %d distinct requests over a pool of %d signals "
                               "(N=2^U(14,24), 70%% int8 +-1 / 30%% fp32 N(0,1)), K=2^U(8,13), "
                               "templates at 0 dB" % (nreq, len(pool)),
                   "pool_bytes": int(sum(s.x.nbytes for s in pool))},
        "serving": {"offered_rate": args.rate, "open_loop_requests": count, "open_loop_s": open_s,
                    "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
                    "mean_batch": open_stats["completed"] / max(1, open_stats["batches"]),
                    "served_matches_per_s": served_rate, "plain_matches_per_s": plain_rate,
                    "served_vs_plain": served_rate / plain_rate,
                    "served_equals_plain": "%d/%d" % (same, nreq)},
        "planted_recovered": "%d/%d" % (recovered, nreq),
    }
    print(json.dumps(line), flush=True)


def run_shared(args):
    """config5b: 1024 int8 +-1 signals of N=2^18 sharing one K=1024 template,
    one tm_match_many per step (one int8 MFMA GEMM against the shared
    template); the same signals as independent matches (TM_MANY_BATCH=1:
    per-instance int8 products) and through the FFT correlation (TM_F_FFT) for
    comparison."""
    import torch

    from paper_1509_04863_amd import datagen as G
    from paper_1509_04863_amd import tm

    insts = G.config5b_batch(count=1024)
    plan = tm.Plan(insts[0].t, n=insts[0].n)
    xs = [torch.from_numpy(s.x).cuda() for s in insts]
    many = tm.Many(plan, xs)
    out = torch.zeros(48 * len(xs), dtype=torch.uint8, device="cuda")
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

    ms_gemm = timed(args.steps)             # one GEMM against the shared template
    res_gemm = tm.results_from_device(out)
    os.environ["TM_MANY_BATCH"] = "1"       # independent matches: per-instance int8 products
    ms_batch = timed(args.steps)
    res_batch = tm.results_from_device(out)
    os.environ.pop("TM_MANY_BATCH")
    many = tm.Many(tm.Plan(insts[0].t, n=insts[0].n, flags=tm.TM_F_FFT), xs)
    ms_fft = timed(max(5, args.steps // 4))  # the FFT correlation of steps 4-6
    res_fft = tm.results_from_device(out)
    x_bytes = sum(s.x.nbytes for s in insts)
    hits = sum(int(r.shift == s.shift) for r, s in zip(res_gemm, insts))
    line = {
        "metric": "template matches/sec + fold GB/s vs HBM peak; served p50/p99 vs plain launch",
        "value": len(xs) / (ms_gemm / 1e3), "unit": "matches/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_gemm, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "i8 MFMA (i32/i64 sums)", "data": "synthetic",
        "config": {"workload": "config5b: 1024 int8 +-1 signals, N=2^18, shared K=1024 template, "
                               "one tm_match_many per step", "batch_x_bytes": x_bytes},
        "fft_path": {"ms_per_step": ms_fft, "matches_per_s": len(xs) / (ms_fft / 1e3),
                     "gemm_speedup": ms_fft / ms_gemm,
                     "same_results": "%d/%d" % (sum(int(a == b) for a, b in zip(res_gemm, res_fft)), len(xs))},
        "per_instance_gemm_batch": {"ms_per_step": ms_batch, "matches_per_s": len(xs) / (ms_batch / 1e3),
                                    "same_results": "%d/%d" % (sum(int(a == b) for a, b in zip(res_gemm, res_batch)),
                                                               len(xs))},
        "planted_recovered": "%d/%d" % (hits, len(xs)),
    }
    print(json.dumps(line), flush=True)


def cpu_baseline(make, budget_s, gpu_results):
    """The oracle as it stands, on instances of the same workload, for about
    budget_s seconds of single-threaded CPU work."""
    from oracle import ftm as O
    done, t0, agree = 0, time.perf_counter(), 0
    elapsed = 0.0
    while elapsed < budget_s or done == 0:
        inst = make(done)
        m1, m2 = O.choose_moduli(inst.n, inst.k)
        s = time.perf_counter()
        ref = O.ftm(inst.x, inst.t, m1, m2)
        elapsed += time.perf_counter() - s
        if done < len(gpu_results):
            g = gpu_results[done]
            agree += int(g.shift == ref.shift and g.m1_tilde == ref.m1_tilde and g.m2_tilde == ref.m2_tilde)
        done += 1
        if time.perf_counter() - t0 > 4 * budget_s + 60:
            break
    return {"value": done / elapsed, "unit": "matches/s", "cores": 1, "kind": "oracle",
            "sample": "%d instances of the same workload (fresh seeds 0..%d), oracle steps 2-9 with "
                      "direct O(MK) correlation, %.1f s" % (done, done - 1, elapsed),
            "gpu_agrees_on": "%d/%d" % (agree, min(done, len(gpu_results)))}


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
    out = torch.zeros(48 * rot, dtype=torch.uint8, device="cuda")
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
    line = {
        "metric": "template matches/sec + fold GB/s vs HBM peak; served p50/p99 vs plain launch",
        "value": value, "unit": "matches/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": ("i32 fold, i8 MFMA correlation (exact)" if info["corr_gemm"] else "i32 fold, f64 fft")
        if info["exact"] else "f32",
        "data": "synthetic",
        "config": {"workload": args.config + ": " + wl["desc"], "n": first.n, "k": first.k,
                   "m1": info["m1"], "m2": info["m2"], "fft_len": p_len,
                   "x_dtype": str(first.x.dtype), "signals_rotated": rot,
                   "rotated_bytes": rot * x_bytes, "streams": len(streams), "warmup_matches": warm_matches,
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
                   "fold_kernel": "k_fold_band" if info["fold_bands"] else
                                  ("k_fold_s8" if info["fold_segments"] else "k_fold")},
        "planted_recovered": "%d/%d" % (planted_ok, rot),
    }
    fold_roof = corr_roof = None
    if fold_n:
        avg_s = fold_ms / fold_n / 1e3
        achieved = x_bytes / avg_s / 1e9
        fold_roof = {"kernel": line["config"]["fold_kernel"], "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": args.traffic_bytes if args.traffic_bytes is not None
                     else TRAFFIC_BYTES.get(args.config), "avg_kernel_us": avg_s * 1e6,
                     "algorithmic_bytes_per_launch": x_bytes}
    if corr_n:
        corr_roof = corr_roofline([plans[0]], corr_ms, corr_n, TRAFFIC_BYTES.get(args.config + "_corr"))
    pick_roofline(line, fold_roof, corr_roof)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(wl["make"], args.cpu_seconds, results)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
