"""Parity on the launch shapes the headline workloads run.

* The product kernels that launches of 512 or more product workgroups run (a
  batch of uneven int8 instances, N up to 2^20 and K up to 2^12): the
  per-instance kernel with its operands in LDS and the per-row-tile kernel's
  4-wave variant, each forced onto single matches of every digit count,
  swapped and explicit moduli and top-T, and reached by a batch of 160 uneven
  instances.  Every result field against the oracle (Algorithm 1 steps 2-9),
  and y / r bit for bit on a sample.
* The precision workload at its stated size: N = 2^24 fp32 N(0,1), K = 2^14,
  template at -3 dB, the fold stored as FP32, BF16 or FP16; r normwise against
  the oracle's FP64 correlation of the same stored fold values, and the argmax
  agreement.
"""

import numpy as np
import pytest

from oracle import ftm as O
from paper_1509_04863_amd import datagen as G
from paper_1509_04863_amd import tm

from _util import assert_exact_parity, normwise, to_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _case(*a):
    print("case:", *a, flush=True)


# ------------------------------------------------------------ 4-wave product

# the product kernels a batch can run, each forced onto single matches: the
# band of a row tile split over 4 waves, per instance with its operands in
# LDS, and one wave per row tile
KERNELS = {"row-tile 4 waves": ("TM_CGEMM_WAVES", "4"), "per instance": ("TM_CGEMM_KIND", "2"),
           "wave per row tile": ("TM_CGEMM_KIND", "3"), "wave per row tile, LDS ring": ("TM_CGEMM_KIND", "4")}


@pytest.fixture(params=list(KERNELS))
def product_kernel(request, monkeypatch):
    monkeypatch.setenv(*KERNELS[request.param])
    return request.param


@pytest.mark.parametrize("lo,hi,n,k,label", [
    (-1, 2, 60000, 700, "1-2 digits"),
    (-128, 128, 3 << 16, 700, "3 digits (int8 extremes)"),
    (-1, 2, 1 << 20, 4096, "config-3 largest shape"),
    (-1, 2, 70000, 512, "one row tile per fold (split band)"),
    (-1, 2, 3000, 37, "tiny"),
])
def test_four_wave_product_int8(lo, hi, n, k, label, product_kernel):
    rng = np.random.default_rng(n + k + 1)
    x = rng.integers(lo, hi, n).astype(np.int8)
    if hi > 2:
        x[: n // 3] = 127
    x[x == 0] = 1
    t = x[1234:1234 + k].copy()
    t[rng.choice(k, k // 10, replace=False)] *= -1
    _case(product_kernel, label, n, k)
    assert_exact_parity(x, t)


@pytest.mark.parametrize("n,k", [(200000, 300), (60000, 500)])
def test_folds_with_different_digit_counts(n, k, product_kernel):
    # every M1-th sample is 127: one bucket of the M1 fold sums L of them
    # (three base-128 digits) while the M2 fold spreads them over distinct
    # buckets (two digits), so the two folds of one instance use different
    # digit counts, with the band split over waves (one or two row tiles)
    m1, _ = O.choose_moduli(n, k)
    rng = np.random.default_rng(n + k)
    x = rng.choice(np.array([-1, 1], dtype=np.int8), n)
    x[::m1] = 127
    t = x[777:777 + k].copy()
    _case(product_kernel, "unequal digits", n, k, m1)
    assert_exact_parity(x, t)


@pytest.mark.parametrize("scale,label", [(3000, "4 digits"), (1000000, "5 digits")])
def test_four_wave_product_wide_digits(scale, label, product_kernel):
    # fp32 integer signals whose folds need four and five base-128 digits
    rng = np.random.default_rng(scale + 7)
    n, k = 200000, 500
    x = np.full(n, scale, dtype=np.float32)
    x[rng.choice(n, n // 100, replace=False)] = -scale
    t = np.zeros(k, dtype=np.float32)
    t[rng.choice(k, 5, replace=False)] = rng.choice([-127.0, 127.0], 5)
    _case(product_kernel, label)
    assert_exact_parity(x, t, flags=tm.TM_F_EXACT)


def test_four_wave_product_moduli_and_top_t(product_kernel):
    inst = G.planted_pm1(300000, 600, config_id=93, index=0, flip_frac=0.05, shift=299000)
    _case(product_kernel, "swapped")
    assert_exact_parity(inst.x, inst.t, m1=701, m2=700)
    _case(product_kernel, "non-consecutive")
    assert_exact_parity(inst.x, inst.t, m1=1000, m2=1003)
    for top_t in (2, 4):
        plan = tm.Plan(inst.t, n=inst.n, top_t=top_t)
        assert plan.info["corr_gemm"] == 1
        _case(product_kernel, "top-T", top_t)
        res, y1, y2, r1, r2 = tm.match_intermediates(plan, to_device(inst.x))
        ref = O.ftm(inst.x, inst.t, plan.m1, plan.m2, top_t=top_t)
        assert np.array_equal(r1, ref.r1.astype(np.float64))
        assert np.array_equal(r2, ref.r2.astype(np.float64))
        assert (res.shift, res.n_candidates, res.m1_tilde, res.m2_tilde) == \
            (ref.shift, ref.n_candidates, ref.m1_tilde, ref.m2_tilde)


def _uneven_batch(count, seed):
    """Seeded instances of the batched workload's recipe (N = 2^U(16,20),
    K = 2^U(9,12), flips U[5%, 15%]); the first one at the largest shape so the
    launch holds well over 512 product workgroups."""
    rng = np.random.default_rng(seed)
    insts = [G.planted_pm1(1 << 20, 4096, 94, 0, flip_frac=0.1)]
    for i in range(1, count):
        n = int(round(2 ** rng.uniform(16, 20)))
        k = int(round(2 ** rng.uniform(9, 12)))
        insts.append(G.planted_pm1(n, k, 94, i, flip_frac=float(rng.uniform(0.05, 0.15))))
    return insts


def _row_tiles(m):
    """Product workgroups of one fold: tiles of 16 rows of 64 shifts."""
    rows = (m + 63) // 64
    return (rows + 15) // 16


@pytest.mark.parametrize("kind", ["1", "2", "3", "4"],
                         ids=["split band", "per-instance kernel", "wave per row tile", "LDS ring"])
def test_large_batch_four_wave_route(kind, monkeypatch):
    monkeypatch.setenv("TM_CGEMM_KIND", kind)
    insts = _uneven_batch(160, 11)
    plans = [tm.Plan(s.t, n=s.n) for s in insts]
    assert all(p.info["corr_gemm"] for p in plans)
    tasks = max(_row_tiles(p.m1) + _row_tiles(p.m2) for p in plans)
    assert len(plans) * tasks >= 512, "the launch must take the 4-wave variant"
    xs = [to_device(s.x) for s in insts]
    _case("large batch", kind, len(insts), "product workgroups", len(plans) * tasks)
    batch = tm.match_batch(plans, xs)
    single = [tm.match(p, x) for p, x in zip(plans, xs)]
    assert batch == single
    for b, inst, p in zip(batch, insts, plans):
        ref = O.ftm(inst.x, inst.t, p.m1, p.m2, correlation="fft")
        assert (b.shift, b.m1_tilde, b.m2_tilde, b.n_candidates) == \
            (ref.shift, ref.m1_tilde, ref.m2_tilde, ref.n_candidates), inst.index
        assert b.peak1 == float(ref.peak1) and b.peak2 == float(ref.peak2)
        assert b.score == float(ref.score if ref.score is not None else 0)
        assert b.flags & tm.TM_R_EXACT


def test_large_batch_intermediates_sample(product_kernel):
    # the intermediates of a sample of the batch's shapes, bit for bit, on the
    # kernels a large batch runs (a single match would otherwise take 8 waves)
    insts = _uneven_batch(160, 11)
    for inst in (insts[0], insts[17], insts[101]):
        _case(product_kernel, "sample", inst.index, inst.n, inst.k)
        assert_exact_parity(inst.x, inst.t)


# ------------------------------------------------------ precision workload

@pytest.mark.parametrize("store,name,bound", [(tm.TM_F32, "f32", 1e-5), (tm.TM_BF16, "bf16", 8 * 2.0 ** -8),
                                              (tm.TM_F16, "f16", 8 * 2.0 ** -11)])
def test_precision_workload_full_size(store, name, bound):
    inst = G.config5a(0)                      # N = 2^24 fp32, K = 2^14, -3 dB
    assert inst.n == 1 << 24 and inst.k == 1 << 14
    plan = tm.Plan(inst.t, n=inst.n, fold_store=store)
    assert plan.info["exact"] == 0 and plan.info["fft_log2"] == 15
    _case("precision workload", name)
    res, y1, y2, r1, r2 = tm.match_intermediates(plan, to_device(inst.x))
    ref = O.ftm(inst.x.astype(np.float64), inst.t.astype(np.float64), plan.m1, plan.m2, correlation="fft")
    k = inst.k
    # the stored fold against FP64: one rounding to the storage format
    e_y = max(normwise(y1, ref.y1[:plan.m1 + k - 1]), normwise(y2, ref.y2[:plan.m2 + k - 1]))
    # the correlation of the stored values against the FP64 correlation of
    # those same values isolates the FP32 transform
    r1_same = O.correlate_fft(y1, inst.t.astype(np.float64), plan.m1)
    r2_same = O.correlate_fft(y2, inst.t.astype(np.float64), plan.m2)
    e_fft = max(normwise(r1, r1_same), normwise(r2, r2_same))
    e_r = max(normwise(r1, ref.r1), normwise(r2, ref.r2))
    agree = (res.m1_tilde, res.m2_tilde) == (ref.m1_tilde, ref.m2_tilde)
    print("precision", name, "fold err", e_y, "fft err", e_fft, "r err vs fp64", e_r,
          "argmax agrees", agree, "shift", res.shift, "oracle", ref.shift, "planted", inst.shift, flush=True)
    assert e_fft <= 1e-5
    assert e_r <= bound
    # the result's own error bound holds for the transform of the stored folds
    # and, with the storage rounding, against the FP64 folds (half storage:
    # the FP32 fold sums' own rounding is far below the storage rounding)
    d_same = max(np.max(np.abs(r1 - r1_same)), np.max(np.abs(r2 - r2_same)))
    d_64 = max(np.max(np.abs(r1 - ref.r1)), np.max(np.abs(r2 - ref.r2)))
    print("err_bound", res.err_bound, "transform error", d_same, "error vs fp64", d_64, flush=True)
    assert 0 < res.err_bound and d_same <= res.err_bound
    if store != tm.TM_F32:
        assert d_64 <= res.err_bound
    if store != tm.TM_F32:                    # one rounding to 8 or 11 significant bits
        assert e_y <= 1.01 * bound / 8
    gap1 = O.top2_gap(ref.r1) / np.max(np.abs(ref.r1))
    gap2 = O.top2_gap(ref.r2) / np.max(np.abs(ref.r2))
    if min(gap1, gap2) > 2 * bound:
        assert agree and res.shift == ref.shift
