"""Section 5 experiments on the GPU, with the matcher's C ABI.

Table 1: noiseless +-1 signals, N = 2^23 .. 2^27, K = N / 2^10, M1 = K,
M2 = K + 1, the template cut cyclically from x at a uniform shift; the success
rate is the fraction of trials whose recovered shift equals the planted one.
Table 2: N = 2^26, K = M1 = 2^16 (M2 = K + 1), the signal observed with additive
Gaussian noise at a given SNR (unit signal power) while the template comes from
the clean signal.

Signals, shifts and noise are drawn on the device from seeded torch generators
(one stream per table, point and trial); every match runs through tm_plan /
tm_match.  Each point reports the success rate with its binomial standard
error, the paper's printed value, and (Table 1) the Theorem 5 success bound.

  python -m paper_1509_04863_amd.tables --table 1 --trials 1000 [--top-t 4]

--top-t T re-scores the candidates of the T x T runner-up pairs (an option
beyond the paper's step 9).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

# the paper's printed success rates (Section 5, Tables 1 and 2)
PAPER_T1 = {23: 0.05, 24: 0.21, 25: 0.85, 26: 1.0, 27: 1.0}
PAPER_T2 = {20: 1.0, 10: 1.0, 6: 0.95, 1: 0.72, -2: 0.48, -6: 0.06}
SEED = 150904863


def _gen(table: int, point: int, trial: int):
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(((SEED * 1_000_003 + table * 10_007 + point) * 1_000_003 + trial) % (1 << 63))
    return g


def _rademacher(n: int, g):
    import torch
    return (torch.randint(0, 2, (n,), generator=g, device="cuda", dtype=torch.int8) * 2 - 1).to(torch.int8)


def _window(x, m: int, k: int):
    import torch
    n = x.numel()
    idx = (torch.arange(k, device="cuda", dtype=torch.int64) + m) % n
    return x[idx].contiguous()


def thm5_success_bound(n: int, k: int, m1: int, m2: int) -> float:
    """Theorem 5: each fold fails with probability at most M e^{-K/(8L)} +
    4(L-1)/K, L = ceil(N/M) (Chernoff and Chebyshev terms of the proof); the
    success bound is the product of the two complements, each clamped to
    [0, 1] since the bound can exceed 1."""
    out = 1.0
    for m in (m1, m2):
        L = -(-n // m)
        f = m * math.exp(-k / (8.0 * L)) + 4.0 * (L - 1) / k
        out *= 1.0 - min(1.0, max(0.0, f))
    return out


def table1(trials: int, log2ns=(23, 24, 25, 26, 27), progress=True, top_t=1):
    import torch

    from paper_1509_04863_amd import tm
    rows = []
    for p in log2ns:
        n, k = 1 << p, (1 << p) >> 10
        m1, m2 = k, k + 1
        hits = 0
        t0 = time.perf_counter()
        for trial in range(trials):
            g = _gen(1, p, trial)
            x = _rademacher(n, g)
            m = int(torch.randint(0, n, (1,), generator=g, device="cuda").item())
            t = _window(x, m, k)
            plan = tm.Plan(t, n=n, m1=m1, m2=m2, top_t=top_t)
            r = tm.match(plan, x)
            hits += int(r.shift == m)
            del plan
        rate = hits / trials
        se = math.sqrt(max(rate * (1 - rate), 1e-12) / trials)
        row = {"log2_n": p, "n": n, "k": k, "m1": m1, "m2": m2, "top_t": top_t, "trials": trials, "success": rate,
               "stderr": se, "paper": PAPER_T1[p], "thm5_success_bound": thm5_success_bound(n, k, m1, m2),
               "seconds": time.perf_counter() - t0}
        rows.append(row)
        if progress:
            print(json.dumps(row), flush=True)
    return rows


def table2_trial(snr: float, trial: int, n: int, k: int):
    """One trial of the noise experiment on the device: a +-1 signal x, a
    uniform shift m, the template t cut from the clean x at m, and the observed
    signal x_e = x + e with e ~ N(0, sigma^2), sigma = 10^(-SNR/20) for the unit
    power of x.  Returns (x_e, t, m) with x_e and t as fp32 device tensors."""
    import torch
    sigma = 10.0 ** (-snr / 20.0)
    g = _gen(2, int(snr) + 100, trial)
    x = _rademacher(n, g)
    m = int(torch.randint(0, n, (1,), generator=g, device="cuda").item())
    t = _window(x, m, k).to(torch.float32)
    xe = x.to(torch.float32) + sigma * torch.randn(n, generator=g, device="cuda", dtype=torch.float32)
    return xe, t, m


def table2(trials: int, snrs=(20, 10, 6, 1, -2, -6), log2n=26, log2k=16, progress=True, top_t=1):
    from paper_1509_04863_amd import tm
    n, k = 1 << log2n, 1 << log2k
    m1, m2 = k, k + 1
    rows = []
    for snr in snrs:
        hits = 0
        t0 = time.perf_counter()
        for trial in range(trials):
            xe, t, m = table2_trial(snr, trial, n, k)
            plan = tm.Plan(t, n=n, m1=m1, m2=m2, top_t=top_t)
            r = tm.match(plan, xe)
            hits += int(r.shift == m)
            del plan, xe
        rate = hits / trials
        row = {"snr_db": snr, "n": n, "k": k, "top_t": top_t, "trials": trials, "success": rate,
               "stderr": math.sqrt(max(rate * (1 - rate), 1e-12) / trials), "paper": PAPER_T2[snr],
               "seconds": time.perf_counter() - t0}
        rows.append(row)
        if progress:
            print(json.dumps(row), flush=True)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--table", type=int, choices=[1, 2], required=True)
    ap.add_argument("--trials", type=int, default=1000)
    ap.add_argument("--points", default="", help="comma list of log2 N (table 1) or SNR dB (table 2)")
    ap.add_argument("--top-t", type=int, default=1, help="top-T re-scoring (1: the paper's step 9)")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "the Section 5 tables run on the GPU"
    pts = [int(v) for v in args.points.split(",") if v]
    if args.table == 1:
        table1(args.trials, tuple(pts) if pts else (23, 24, 25, 26, 27), top_t=args.top_t)
    else:
        table2(args.trials, tuple(pts) if pts else (20, 10, 6, 1, -2, -6), top_t=args.top_t)


if __name__ == "__main__":
    main()
