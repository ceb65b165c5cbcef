"""Top-T re-scoring (tm_plan_desc.top_t, a robustness option beyond the
paper): the union of the candidate sets of the T x T runner-up pairs, re-scored
by (Tx)_c, against the oracle's ftm(..., top_t=T) on every correlation route
(int8 matrix product, FFT in LDS exact and FP32, four-step FFT through global
memory), with the zero-padded variant, and in a batch of mixed T."""

import numpy as np
import pytest

from oracle import ftm as O
from paper_1509_04863_amd import datagen as G
from paper_1509_04863_amd import tm

from _util import to_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _case(*a):
    print("case:", *a, flush=True)


def _noisy_pm1(n, k, flip, index):
    # flips high enough that the argmax is often wrong and the runners-up matter
    return G.planted_pm1(n, k, config_id=93, index=index, flip_frac=flip)


def _exact_check(inst, top_t, flags=0, m1=0, m2=0, x=None, t=None):
    x = inst.x if x is None else x
    t = inst.t if t is None else t
    plan = tm.Plan(t, n=x.shape[0], m1=m1, m2=m2, x_dtype=tm.tm_dtype_of(x), flags=flags, top_t=top_t)
    res = tm.match(plan, to_device(x))
    variant = "zero_pad" if flags & tm.TM_F_ZERO_PAD else "cyclic"
    corr = "direct" if plan.m1 * x.shape[0] < 4e8 else "fft"
    ref = O.ftm(inst.x.astype(np.int64), inst.t.astype(np.int64), plan.m1, plan.m2, variant=variant,
                top_t=top_t, correlation=corr)
    assert (res.m1_tilde, res.m2_tilde) == (ref.m1_tilde, ref.m2_tilde)
    assert res.n_candidates == ref.n_candidates
    assert res.shift == ref.shift
    if ref.shift != O.NOMATCH:
        assert res.score == float(ref.score)
    assert bool(res.flags & tm.TM_R_RESCORED) == (ref.n_candidates > 1)
    return plan, res, ref


@pytest.mark.parametrize("top_t", [2, 3, 4])
@pytest.mark.parametrize("route", ["gemm", "fft"])
def test_top_t_exact_routes(top_t, route):
    flags = tm.TM_F_FFT if route == "fft" else 0
    hits1 = hitst = 0
    for i in range(6):
        inst = _noisy_pm1(60000 + 977 * i, 700 + 37 * i, 0.3, i)
        _case(route, top_t, i)
        plan, res, ref = _exact_check(inst, top_t, flags)
        assert plan.info["corr_gemm"] == (route == "gemm")
        base = O.ftm(inst.x, inst.t, plan.m1, plan.m2)
        hits1 += int(base.shift == inst.shift)
        hitst += int(res.shift == inst.shift)
    assert hitst >= hits1


def test_top_t_zero_pad_and_explicit_moduli():
    inst = _noisy_pm1(300007, 600, 0.25, 11)
    _case("zero pad top-T")
    _exact_check(inst, 4, tm.TM_F_ZERO_PAD)
    _case("explicit moduli top-T")
    _exact_check(inst, 3, 0, m1=701, m2=700)


def test_top_t_small_folds():
    # M smaller than T on one side is impossible (M >= K >= 1); tiny folds with T = 4
    for n, k in [(30, 5), (12, 12), (100, 3)]:
        inst = G.planted_pm1(n, k, config_id=93, index=n, flip_frac=0.2)
        _case("tiny top-T", n, k)
        _exact_check(inst, 4)
        _exact_check(inst, 4, tm.TM_F_FFT)


def test_top_t_global_fft_exact():
    inst = _noisy_pm1(1 << 20, 6000, 0.3, 21)
    _case("global fft exact top-T")
    plan, res, ref = _exact_check(inst, 3, tm.TM_F_FFT)
    assert plan.info["fft_global"] == 1


def _real_case(n, k, snr_db, index, top_t, expect_global):
    inst = G.planted_gauss(n, k, snr_db, 94, index)
    plan = tm.Plan(inst.t, n=n, x_dtype=tm.TM_F32, top_t=top_t)
    assert plan.info["fft_global"] == expect_global
    res = tm.match(plan, to_device(inst.x))
    ref = O.ftm(inst.x.astype(np.float64), inst.t.astype(np.float64), plan.m1, plan.m2, correlation="fft",
                top_t=top_t)

    def clear(r):   # the top T + 1 values are well separated: the runner-up lists agree
        v = np.sort(np.asarray(r, np.float64))[::-1][:top_t + 1]
        return np.all(np.diff(-v) > 1e-4 * np.max(np.abs(r)))
    if clear(ref.r1) and clear(ref.r2):
        assert (res.m1_tilde, res.m2_tilde, res.n_candidates, res.shift) == \
            (ref.m1_tilde, ref.m2_tilde, ref.n_candidates, ref.shift)
        if ref.shift != O.NOMATCH:
            assert abs(res.score - float(ref.score)) <= 1e-9 * max(1.0, abs(float(ref.score)))
        return 1
    return 0


def test_top_t_real_lds_fft():
    checked = 0
    for i in range(6):
        _case("real lds top-T", i)
        checked += _real_case(1 << 18, 1024, -4.0, i, 4, 0)
    assert checked >= 3


def test_top_t_real_global_fft():
    checked = 0
    for i in range(3):
        _case("real global top-T", i)
        checked += _real_case(1 << 20, 1 << 14, -6.0, i, 2, 1)
    assert checked >= 1


def test_top_t_mixed_batch():
    insts = [_noisy_pm1(20000 + 97 * i, 300 + 16 * i, 0.3, 40 + i) for i in range(12)]
    plans = [tm.Plan(s.t, n=s.x.shape[0], top_t=1 + i % 4, flags=tm.TM_F_FFT if i % 3 == 0 else 0)
             for i, s in enumerate(insts)]
    xs = [to_device(s.x) for s in insts]
    _case("mixed top-T batch")
    out = tm.match_batch(plans, xs)
    single = [tm.match(p, x) for p, x in zip(plans, xs)]
    assert out == single
    for i, (s, r) in enumerate(zip(insts, out)):
        ref = O.ftm(s.x, s.t, plans[i].m1, plans[i].m2, top_t=1 + i % 4)
        assert (r.shift, r.m1_tilde, r.m2_tilde, r.n_candidates) == \
            (ref.shift, ref.m1_tilde, ref.m2_tilde, ref.n_candidates)


def test_top_t_many_falls_back_to_batch():
    insts = G.config5b_batch(count=20, n=1 << 16, k=512, flip_frac=0.3)
    plan = tm.Plan(insts[0].t, n=1 << 16, top_t=3)
    xs = [to_device(s.x) for s in insts]
    _case("many top-T")
    many = tm.Many(plan, xs).match()
    single = [tm.match(plan, x) for x in xs]
    assert many == single
