"""Single matches keep each plan's instance record in device memory, one copy
per stream.  The copy has to follow every change of the record: the stream's
workspace moved by a larger plan, intermediates requested or not.  It has to
serve more streams than the plan's preallocated slots, and carry each match's
own signal and result slot."""

import numpy as np
import pytest

from oracle import ftm as O
from paper_1509_04863_amd import tm

from _util import to_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _case(*a):
    print("case:", *a, flush=True)


def _signal(seed, n, k, shift):
    rng = np.random.default_rng(seed)
    t = rng.choice(np.array([-1, 1], dtype=np.int8), k)
    x = rng.choice(np.array([-1, 1], dtype=np.int8), n)
    x[shift:shift + k] = t
    return x, t


def _same(res, x, t, plan):
    ref = O.ftm(x, t, plan.m1, plan.m2)
    assert (res.m1_tilde, res.m2_tilde) == (ref.m1_tilde, ref.m2_tilde)
    assert res.shift == ref.shift
    assert res.n_candidates == ref.n_candidates
    assert res.peak1 == float(ref.peak1) and res.peak2 == float(ref.peak2)


@pytest.mark.parametrize("flags", [0, tm.TM_F_FFT])
def test_workspace_moves_between_matches(flags):
    s = torch.cuda.Stream()
    xa, ta = _signal(1, 60000, 700, 123)
    xb, tb = _signal(2, 1 << 20, 4096, 5000)
    pa = tm.Plan(ta, n=xa.shape[0], flags=flags)
    pb = tm.Plan(tb, n=xb.shape[0], flags=flags)
    da, db = to_device(xa), to_device(xb)
    _case("small plan, then a larger one on the same stream, then the small one again", flags)
    _same(tm.match(pa, da, s), xa, ta, pa)
    _same(tm.match(pb, db, s), xb, tb, pb)     # the stream's workspace grows
    _same(tm.match(pa, da, s), xa, ta, pa)     # the small plan's record must follow it


def test_intermediates_then_plain_matches():
    x, t = _signal(3, 70000, 900, 777)
    plan = tm.Plan(t, n=x.shape[0])
    d = to_device(x)
    _case("intermediates, plain, intermediates on one stream")
    ref = O.ftm(x, t, plan.m1, plan.m2)
    res, y1, y2, r1, r2 = tm.match_intermediates(plan, d)
    assert np.array_equal(r1, ref.r1.astype(np.float64)) and np.array_equal(r2, ref.r2.astype(np.float64))
    _same(res, x, t, plan)
    _same(tm.match(plan, d), x, t, plan)
    res, y1, y2, r1, r2 = tm.match_intermediates(plan, d)
    assert np.array_equal(y1, ref.y1[:plan.m1 + t.shape[0] - 1].astype(np.float64))
    _same(res, x, t, plan)


def test_many_streams_interleaved_signals():
    # one plan on twelve streams (more than its preallocated slots), three
    # signals in turn, nothing waited for between the matches
    k, n = 600, 50000
    rng = np.random.default_rng(4)
    t = rng.choice(np.array([-1, 1], dtype=np.int8), k)
    xs = []
    for i in range(3):
        x = rng.choice(np.array([-1, 1], dtype=np.int8), n)
        x[1000 * (i + 1):1000 * (i + 1) + k] = t
        xs.append(x)
    plan = tm.Plan(t, n=n)
    dx = [to_device(x) for x in xs]
    streams = [torch.cuda.Stream() for _ in range(12)]
    out = torch.zeros(tm.RESULT_BYTES * 36, dtype=torch.uint8, device="cuda")
    _case("12 streams x 3 rounds, 3 signals")
    torch.cuda.synchronize()
    for r in range(3):
        for i, st in enumerate(streams):
            tm.match_into(plan, dx[(i + r) % 3], out, 12 * r + i, st)
    torch.cuda.synchronize()
    got = tm.results_from_device(out)
    want = [O.ftm(x, t, plan.m1, plan.m2) for x in xs]
    for r in range(3):
        for i in range(12):
            res, ref = got[12 * r + i], want[(i + r) % 3]
            assert res.shift == ref.shift and (res.m1_tilde, res.m2_tilde) == (ref.m1_tilde, ref.m2_tilde)
            assert res.peak1 == float(ref.peak1) and res.peak2 == float(ref.peak2)
