"""Theorem 2 variant (TM_F_ZERO_PAD): the zero-padded partition folds, the
circular length-M correlations, the cut candidate sets and the shift of the
HIP path against the oracle's variant="zero_pad", bit for bit on integer data,
through every fold and finish kernel (streaming int8, band, tiles; FFT in LDS
and through global memory; the shared-template GEMM; batches)."""

import numpy as np
import pytest

from oracle import ftm as O
from paper_1509_04863_amd import datagen as G
from paper_1509_04863_amd import tm

from _util import normwise, to_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

ZP = tm.TM_F_ZERO_PAD


def _case(*a):
    print("case:", *a, flush=True)


def _periodic(y, m, length):
    return y[np.arange(length) % m]


def _zp_exact(x, t, m1=0, m2=0, fold_mult=1, flags=0):
    plan = tm.Plan(t, n=x.shape[0], m1=m1, m2=m2, fold_mult=fold_mult, x_dtype=tm.tm_dtype_of(x),
                   flags=flags | ZP)
    res, y1, y2, r1, r2 = tm.match_intermediates(plan, to_device(x))
    ref = O.ftm(x, t, plan.m1, plan.m2, variant="zero_pad")
    k = t.shape[0]
    assert np.array_equal(y1, _periodic(ref.y1, plan.m1, plan.m1 + k - 1).astype(np.float64)), "fold M1"
    assert np.array_equal(y2, _periodic(ref.y2, plan.m2, plan.m2 + k - 1).astype(np.float64)), "fold M2"
    assert np.array_equal(r1, ref.r1.astype(np.float64)), "correlation M1"
    assert np.array_equal(r2, ref.r2.astype(np.float64)), "correlation M2"
    assert (res.m1_tilde, res.m2_tilde, res.n_candidates, res.shift) == \
        (ref.m1_tilde, ref.m2_tilde, ref.n_candidates, ref.shift)
    assert res.peak1 == float(ref.peak1) and res.peak2 == float(ref.peak2)
    if ref.shift != O.NOMATCH:
        assert res.score == float(ref.score)
    assert bool(res.flags & tm.TM_R_NOMATCH) == (ref.shift == O.NOMATCH)
    assert not res.flags & tm.TM_R_RESCORED
    assert res.flags & tm.TM_R_EXACT
    return plan, res, ref


CASES = [
    # (name, n, k, shift, flip, m1, m2, fold_mult)
    ("int8 stream fold, M !| N", 65536 + 123, 1024, 777, 0.05, 0, 0, 1),
    ("int8 stream fold, c=2", 65536 + 5, 1024, 65536 - 2000, 0.0, 0, 0, 2),
    ("int8 wrap template (lost by the variant)", 50000, 2000, 50000 - 1000, 0.0, 0, 0, 1),
    ("int8 M1 | N", 4096 * 16, 4096, 12345, 0.1, 0, 0, 1),
    ("int8 tiles + global FFT (M > 4608)", 200000, 5000, 150000, 0.05, 0, 0, 1),
    ("int8 L=1 (N<M)", 100, 80, 10, 0.0, 0, 0, 2),
    ("int8 explicit non-consecutive moduli", 500000, 900, 400000, 0.05, 1000, 1003, 1),
    ("int8 swapped moduli", 300000, 600, 299000, 0.05, 701, 700, 1),
    ("int8 raised M (K(K+1)<=N)", 1 << 20, 300, 123456, 0.05, 0, 0, 1),
]


@pytest.mark.parametrize("name,n,k,shift,flip,m1,m2,c", CASES, ids=[c[0] for c in CASES])
def test_zero_pad_int8(name, n, k, shift, flip, m1, m2, c):
    inst = G.planted_pm1(n, k, shift=shift, flip_frac=flip, config_id=90, index=n + k)
    _case(name, n, k, shift)
    plan, res, ref = _zp_exact(inst.x, inst.t, m1, m2, c)
    if flip == 0.0 and shift + k <= n and res.shift != O.NOMATCH:
        assert res.shift == shift


def test_zero_pad_fp32_pm1_band_fold():
    inst = G.planted_pm1((1 << 20) + 77, 1024, shift=5000, flip_frac=0.05, config_id=90, index=3)
    x = inst.x.astype(np.float32)
    t = inst.t.astype(np.float32)
    _case("fp32 +-1 band fold", x.shape[0])
    _zp_exact(x, t, flags=tm.TM_F_EXACT)


def test_zero_pad_equals_default_when_moduli_divide_n():
    # N = M1 M2: both variants are the same computation
    m1, m2, k = 1024, 1025, 1000
    inst = G.planted_pm1(m1 * m2, k, shift=777777, flip_frac=0.05, config_id=90, index=5)
    a = tm.match(tm.Plan(inst.t, n=m1 * m2, m1=m1, m2=m2), to_device(inst.x))
    b = tm.match(tm.Plan(inst.t, n=m1 * m2, m1=m1, m2=m2, flags=ZP), to_device(inst.x))
    _case("M1 M2 = N", m1, m2)
    assert a == b


def test_zero_pad_real_path():
    rng = np.random.default_rng(11)
    n, k = 300007, 700
    x = rng.standard_normal(n).astype(np.float32)
    m = 123457
    t = (x[(m + np.arange(k)) % n] + 0.5 * rng.standard_normal(k)).astype(np.float32)
    plan = tm.Plan(t, n=n, x_dtype=tm.TM_F32, flags=ZP)
    _case("real zero pad", n, k)
    res, y1, y2, r1, r2 = tm.match_intermediates(plan, to_device(x))
    ref = O.ftm(x.astype(np.float64), t.astype(np.float64), plan.m1, plan.m2, variant="zero_pad")
    assert normwise(y1[:plan.m1], ref.y1) <= 1e-5 and normwise(y2[:plan.m2], ref.y2) <= 1e-5
    assert np.array_equal(y1[plan.m1:], y1[:k - 1]) and np.array_equal(y2[plan.m2:], y2[:k - 1])
    assert normwise(r1, ref.r1) <= 1e-5 and normwise(r2, ref.r2) <= 1e-5
    if not res.flags & tm.TM_R_NEAR_TIE:
        assert (res.m1_tilde, res.m2_tilde, res.shift) == (ref.m1_tilde, ref.m2_tilde, ref.shift)
    assert res.n_candidates <= 1


def test_zero_pad_shared_template_gemm_and_batch():
    insts = G.config5b_batch(count=40, n=(1 << 16) + 333, k=512, flip_frac=0.05)
    n = insts[0].x.shape[0]
    plan = tm.Plan(insts[0].t, n=n, flags=ZP)
    xs = [to_device(s.x) for s in insts]
    _case("many zero pad", len(insts), n)
    many = tm.Many(plan, xs).match()
    single = [tm.match(plan, x) for x in xs]
    assert many == single
    batch = tm.match_batch([plan] * len(xs), xs)
    assert batch == single
    for s, r in list(zip(insts, many))[::5]:
        ref = O.ftm(s.x, s.t, plan.m1, plan.m2, variant="zero_pad")
        assert (r.shift, r.m1_tilde, r.m2_tilde, r.n_candidates) == \
            (ref.shift, ref.m1_tilde, ref.m2_tilde, ref.n_candidates)
        assert r.peak1 == float(ref.peak1) and r.peak2 == float(ref.peak2)


def test_zero_pad_mixed_batch():
    # zero-padded and default plans side by side in one batch
    insts = [G.planted_pm1(20000 + 97 * i, 256 + 16 * i, shift=19000, flip_frac=0.05, config_id=90, index=i) for i in range(12)]
    plans = [tm.Plan(s.t, n=s.x.shape[0], flags=ZP if i % 2 else 0) for i, s in enumerate(insts)]
    xs = [to_device(s.x) for s in insts]
    _case("mixed batch")
    out = tm.match_batch(plans, xs)
    for i, (s, r) in enumerate(zip(insts, out)):
        ref = O.ftm(s.x, s.t, plans[i].m1, plans[i].m2, variant="zero_pad" if i % 2 else "cyclic")
        assert (r.shift, r.m1_tilde, r.m2_tilde, r.n_candidates) == \
            (ref.shift, ref.m1_tilde, ref.m2_tilde, ref.n_candidates)
