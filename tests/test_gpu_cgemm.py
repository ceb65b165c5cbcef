"""The correlation of exact plans as an int8 MFMA matrix product: limb counts
from one to five digits, extreme int8 values, templates given as float,
batches that mix it with the FFT correlations, and agreement with TM_F_FFT
and with the oracle on every intermediate."""

import numpy as np
import pytest

from oracle import ftm as O
from paper_1509_04863_amd import datagen as G
from paper_1509_04863_amd import tm

from _util import assert_exact_parity, to_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _case(*a):
    print("case:", *a, flush=True)


def test_plan_reports_gemm_route():
    t = np.ones(512, dtype=np.int8)
    assert tm.Plan(t, n=1 << 16).info["corr_gemm"] == 1
    assert tm.Plan(t, n=1 << 16, flags=tm.TM_F_FFT).info["corr_gemm"] == 0
    tf = np.full(512, 300.0, dtype=np.float32)           # outside int8: FFT route
    assert tm.Plan(tf, n=1 << 16, x_dtype=tm.TM_F32, flags=tm.TM_F_EXACT).info["corr_gemm"] == 0
    tf[:] = -128.0
    assert tm.Plan(tf, n=1 << 16, x_dtype=tm.TM_F32, flags=tm.TM_F_EXACT).info["corr_gemm"] == 1
    assert tm.Plan(tf, n=1 << 16, x_dtype=tm.TM_F32).info["corr_gemm"] == 0   # real path


@pytest.mark.parametrize("lo,hi,n,k,label", [
    (-1, 2, 60000, 700, "1-2 digits"),
    (-128, 128, 3 << 16, 700, "3 digits (int8 extremes)"),
    (-128, 128, 1 << 20, 300, "3 digits, raised M"),
])
def test_int8_value_ranges(lo, hi, n, k, label):
    rng = np.random.default_rng(n + k)
    x = rng.integers(lo, hi, n).astype(np.int8)
    x[: n // 3] = 127 if hi > 2 else x[: n // 3]          # long runs: large fold values
    t = rng.integers(lo, hi, k).astype(np.int8)
    t[:5] = -128 if lo <= -128 else t[:5]
    _case(label, n, k)
    assert_exact_parity(x, t)


@pytest.mark.parametrize("scale,label", [(3000, "4 digits"), (1000000, "5 digits")])
def test_fp32_integer_signals_need_more_digits(scale, label):
    # nearly constant signals: every fold entry is close to L * scale
    # (L = 400: 1.2e6 needs four base-128 digits, 4e8 five); a sparse template
    # keeps the FFT variant's exactness bound below 1/2 as well
    rng = np.random.default_rng(scale)
    n, k = 200000, 500
    x = np.full(n, scale, dtype=np.float32)
    x[rng.choice(n, n // 100, replace=False)] = -scale
    t = np.zeros(k, dtype=np.float32)
    t[rng.choice(k, 5, replace=False)] = rng.choice([-127.0, 127.0], 5)
    _case(label, n, k)
    assert_exact_parity(x, t, flags=tm.TM_F_EXACT)


def test_swapped_and_explicit_moduli():
    inst = G.planted_pm1(300000, 600, config_id=91, index=0, flip_frac=0.05, shift=299000)
    _case("swapped")
    assert_exact_parity(inst.x, inst.t, m1=701, m2=700)
    _case("non-consecutive")
    assert_exact_parity(inst.x, inst.t, m1=1000, m2=1003)


def test_small_moduli_and_tiny_signals():
    for n, k in [(10, 3), (64, 64), (200, 7), (1000, 1)]:
        inst = G.planted_pm1(n, k, config_id=91, index=n, flip_frac=0.0, shift=n // 3)
        _case("tiny", n, k)
        assert_exact_parity(inst.x, inst.t)


def test_mixed_batch_gemm_fft_real():
    rng = np.random.default_rng(5)
    plans, xs, refs = [], [], []
    for i in range(24):
        n = int(rng.integers(3000, 200000))
        k = int(rng.integers(1, min(n, 3000)))
        kind = i % 4
        inst = G.planted_pm1(n, k, config_id=92, index=i, flip_frac=0.05)
        if kind == 0:                        # int8: GEMM
            x, t, flags = inst.x, inst.t, 0
        elif kind == 1:                      # int8 forced FFT
            x, t, flags = inst.x, inst.t, tm.TM_F_FFT
        elif kind == 2:                      # fp32 exact: GEMM
            x, t, flags = inst.x.astype(np.float32), inst.t.astype(np.float32), tm.TM_F_EXACT
        else:                                # fp32 real: FFT in FP32
            x = rng.standard_normal(n).astype(np.float32)
            t, flags = x[:k].copy(), 0
        plans.append(tm.Plan(t, n=n, x_dtype=tm.tm_dtype_of(x), flags=flags))
        xs.append(to_device(x))
        refs.append((x, t, kind))
    _case("mixed batch")
    out = tm.match_batch(plans, xs)
    single = [tm.match(p, x) for p, x in zip(plans, xs)]
    assert out == single
    for (x, t, kind), p, r in zip(refs, plans, out):
        if kind == 3:
            continue
        ref = O.ftm(x.astype(np.int64), t.astype(np.int64), p.m1, p.m2)
        assert (r.shift, r.m1_tilde, r.m2_tilde, r.n_candidates) == \
            (ref.shift, ref.m1_tilde, ref.m2_tilde, ref.n_candidates)
        assert r.peak1 == float(ref.peak1) and r.peak2 == float(ref.peak2)
        assert r.flags & tm.TM_R_EXACT


def test_repeat_determinism_and_bucket_reset():
    inst = G.config2(0)
    plan = tm.Plan(inst.t.astype(np.float32), n=inst.x.shape[0], x_dtype=tm.TM_F32, flags=tm.TM_F_EXACT)
    assert plan.info["corr_gemm"] == 1
    xd = to_device(inst.x.astype(np.float32))
    _case("config2 repeat")
    first = tm.match(plan, xd)
    for _ in range(5):
        assert tm.match(plan, xd) == first
    ref = O.ftm(inst.x, inst.t, plan.m1, plan.m2, correlation="fft")
    assert (first.shift, first.m1_tilde, first.m2_tilde) == (ref.shift, ref.m1_tilde, ref.m2_tilde)


@pytest.mark.parametrize("split", ["1", "3", "7", "1000"])
@pytest.mark.parametrize("top_t", [1, 3])
def test_band_split_over_workgroups(split, top_t, monkeypatch):
    # a single match's band may be shared by several workgroups whose shares
    # are summed into r (exact int64): every split, including more parts than
    # steps, gives the oracle's correlations and result
    monkeypatch.setenv("TM_CGEMM_SPLIT", split)
    rng = np.random.default_rng(int(split) + 10 * top_t)
    n, k = 90001, 1500
    x = rng.integers(-128, 128, n).astype(np.int8)
    t = rng.integers(-3, 4, k).astype(np.int8)
    x[4321:4321 + k] = t
    _case("split", split, "top_t", top_t)
    plan = tm.Plan(t, n=n, top_t=top_t)
    assert plan.info["corr_gemm"] == 1
    res, y1, y2, r1, r2 = tm.match_intermediates(plan, to_device(x))
    ref = O.ftm(x, t, plan.m1, plan.m2, top_t=top_t)
    assert np.array_equal(r1, ref.r1.astype(np.float64))
    assert np.array_equal(r2, ref.r2.astype(np.float64))
    assert res.shift == ref.shift and res.n_candidates == ref.n_candidates
    assert (res.m1_tilde, res.m2_tilde) == (ref.m1_tilde, ref.m2_tilde)
    plain = tm.match(plan, to_device(x))
    assert plain == res


@pytest.mark.parametrize("kind", ["0", "4"], ids=["automatic product", "LDS ring"])
def test_batch_mixes_digit_counts(kind, monkeypatch):
    # one batch whose instances need 1, 2 and 3 digits (the ring kernel takes
    # the digit count per workgroup, and a workgroup may hold row tiles of
    # both folds): every result equals the single match and the oracle's
    monkeypatch.setenv("TM_CGEMM_KIND", kind)
    rng = np.random.default_rng(77)
    plans, xs, refs = [], [], []
    for i in range(18):
        n = int(rng.integers(40000, 300000))
        k = int(rng.choice([300, 700, 1500, 2600]))
        if i % 3 == 0:
            x = rng.integers(-1, 2, n).astype(np.int8)         # small folds
            t = rng.choice(np.array([-1, 1], dtype=np.int8), k)
        elif i % 3 == 1:
            x = rng.choice(np.array([-1, 1], dtype=np.int8), n)
            t = rng.choice(np.array([-1, 1], dtype=np.int8), k)
        else:
            x = rng.integers(-128, 128, n).astype(np.int8)     # three digits
            x[: n // 3] = 127
            t = rng.integers(-128, 128, k).astype(np.int8)
        plans.append(tm.Plan(t, n=n))
        xs.append(to_device(x))
        refs.append((x, t))
    assert all(p.info["corr_gemm"] for p in plans)
    _case("mixed digit counts", kind, len(plans))
    batch = tm.match_batch(plans, xs)
    monkeypatch.setenv("TM_CGEMM_KIND", "0")
    single = [tm.match(p, x) for p, x in zip(plans, xs)]
    assert batch == single
    for (x, t), p, r in list(zip(refs, plans, batch))[::2]:
        ref = O.ftm(x, t, p.m1, p.m2)
        assert (r.shift, r.m1_tilde, r.m2_tilde, r.n_candidates) == \
            (ref.shift, ref.m1_tilde, ref.m2_tilde, ref.n_candidates)
        assert r.peak1 == float(ref.peak1) and r.peak2 == float(ref.peak2)


@pytest.mark.parametrize("kind", ["3", "4"], ids=["wave per row tile", "LDS ring"])
def test_batch_top_t_on_per_wave_kernels(kind, monkeypatch):
    # top-T re-scoring in a batch on the per-wave product kernels (the ring
    # kernel clears the bucket zone itself, the final kernel then takes the
    # top-T branch): equal to single matches and to the oracle
    monkeypatch.setenv("TM_CGEMM_KIND", kind)
    rng = np.random.default_rng(5 + int(kind))
    plans, xs, refs = [], [], []
    for i in range(8):
        n = int(rng.integers(50000, 200000))
        k = int(rng.choice([400, 1100, 2000]))
        x = rng.integers(-128, 128, n).astype(np.int8)
        t = rng.integers(-3, 4, k).astype(np.int8)
        at = int(rng.integers(0, n - k))
        x[at:at + k] = t
        plans.append(tm.Plan(t, n=n, top_t=3))
        xs.append(to_device(x))
        refs.append((x, t))
    _case("batch top_t", kind, len(plans))
    batch = tm.match_batch(plans, xs)
    monkeypatch.setenv("TM_CGEMM_KIND", "0")
    assert batch == [tm.match(p, x) for p, x in zip(plans, xs)]
    for (x, t), p, r in zip(refs, plans, batch):
        ref = O.ftm(x, t, p.m1, p.m2, top_t=3)
        assert (r.shift, r.m1_tilde, r.m2_tilde, r.n_candidates) == \
            (ref.shift, ref.m1_tilde, ref.m2_tilde, ref.n_candidates)
