"""tm_match_noalloc, the single match for callers that cannot allocate device
memory: through the C ABI, against tm_match (bit for bit) and the oracle, on
two calls in a row whose second input is smaller, on every correlation
route; plans above the scratch maximum and host result pointers are refused
before anything is launched."""

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


def _route(label, flags, x_dtype):
    big = G.planted_pm1(1 << 20, 4096, 98, 0, flip_frac=0.1, x_dtype=x_dtype)
    small = G.planted_pm1(70001, 700, 98, 1, flip_frac=0.05, x_dtype=x_dtype)
    return label, flags, big, small


ROUTES = [
    _route("int8 product", 0, np.int8),
    _route("int8 fft in lds", tm.TM_F_FFT, np.int8),
    _route("fp32 +-1 product", tm.TM_F_EXACT, np.float32),
]


def _plan(inst, flags):
    return tm.Plan(inst.t, n=inst.n, x_dtype=tm.tm_dtype_of(inst.x), flags=flags)


@pytest.mark.parametrize("label,flags,big,small", ROUTES, ids=[r[0] for r in ROUTES])
def test_two_calls_in_a_row_match_tm_match(label, flags, big, small):
    pb, ps = _plan(big, flags), _plan(small, flags)
    xb, xs = to_device(big.x), to_device(small.x)
    out = torch.zeros(tm.RESULT_BYTES * 2, dtype=torch.uint8, device="cuda")
    _case("noalloc", label)
    tm.match_noalloc(pb, xb, out, 0)
    tm.match_noalloc(ps, xs, out, 1)          # same stream, no wait in between
    got = tm.results_from_device(out)
    assert got[0] == tm.match(pb, xb)
    assert got[1] == tm.match(ps, xs)
    for r, inst, p in ((got[0], big, pb), (got[1], small, ps)):
        ref = O.ftm(inst.x.astype(np.int64), inst.t.astype(np.int64), p.m1, p.m2)
        assert (r.shift, r.m1_tilde, r.m2_tilde, r.n_candidates) == \
            (ref.shift, ref.m1_tilde, ref.m2_tilde, ref.n_candidates)
        assert r.peak1 == float(ref.peak1) and r.peak2 == float(ref.peak2)
        assert r.flags & tm.TM_R_EXACT


def test_real_and_global_fft_routes():
    # real path (fp32 FFT in LDS), then the four-step FFT through global memory
    a = G.planted_gauss(1 << 20, 2048, 0.0, 99, 0)
    b = G.config5a(2, n=1 << 21, k=1 << 14)
    pa, pb = tm.Plan(a.t, n=a.n), tm.Plan(b.t, n=b.n)
    assert pb.info["fft_global"] == 1
    xa, xb = to_device(a.x), to_device(b.x)
    out = torch.zeros(tm.RESULT_BYTES * 2, dtype=torch.uint8, device="cuda")
    _case("noalloc real + global fft")
    tm.match_noalloc(pb, xb, out, 0)          # larger workspace first
    tm.match_noalloc(pa, xa, out, 1)
    got = tm.results_from_device(out)
    assert got[0] == tm.match(pb, xb)
    assert got[1] == tm.match(pa, xa)


def test_repeat_after_other_plans_clears_buckets():
    # the scratch keeps the last call's contents: a repeat after a different
    # plan must still start from zeroed buckets
    insts = [G.config1(i) for i in range(3)]
    plans = [tm.Plan(s.t, n=s.n) for s in insts]
    xs = [to_device(s.x) for s in insts]
    out = torch.zeros(tm.RESULT_BYTES * 6, dtype=torch.uint8, device="cuda")
    _case("noalloc repeats")
    for rep in range(2):
        for i in range(3):
            tm.match_noalloc(plans[i], xs[i], out, 3 * rep + i)
    got = tm.results_from_device(out)
    for i in range(3):
        want = tm.match(plans[i], xs[i])
        assert got[i] == want and got[3 + i] == want


def test_refusals_launch_nothing():
    inst = G.config1(0)
    plan = tm.Plan(inst.t, n=inst.n)
    x = to_device(inst.x)
    res = tm.Result()
    st = tm.lib().tm_match_noalloc(plan.handle, x.data_ptr(), tm.ctypes.addressof(res), None)
    assert st == tm.TM_ERR_INVALID                      # host result pointer
    # a four-step exact FFT of 2^20 points needs 16 MiB of working values alone
    big_k = 1 << 19
    t = np.ones(big_k, dtype=np.int8)
    bp = tm.Plan(t, n=1 << 20, flags=tm.TM_F_FFT)
    assert bp.info["workspace_bytes"] > 16 << 20
    xb = torch.ones(1 << 20, dtype=torch.int8, device="cuda")
    out = torch.zeros(48, dtype=torch.uint8, device="cuda")
    _case("noalloc refusal")
    st = tm.lib().tm_match_noalloc(bp.handle, xb.data_ptr(), out.data_ptr(), None)
    assert st == tm.TM_ERR_UNSUPPORTED
    assert "scratch" in tm.lib().tm_last_error().decode()
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
