"""Reusable batches (tm_batch_*): the launch sequence of a fixed batch captured
once in a HIP graph.  Every replay, with eager work and synchronisations in
between, equals tm_match_batch on the same plans and signals bit for bit;
new signal contents at the same addresses are matched; the exact instances
agree with the oracle."""

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


def _mixed(count, seed):
    """int8 exact (product route), int8 on the FFT route, fp32 real signals,
    and one exact FFT above one workgroup's LDS (four-step route)."""
    rng = np.random.default_rng(seed)
    plans, xs, insts = [], [], []
    for i in range(count):
        kind = i % 4
        n = int(round(2 ** rng.uniform(14, 19)))
        k = min(n, int(round(2 ** rng.uniform(7, 11))))
        if i == 3:
            inst, flags = G.planted_pm1(1 << 20, 6000, 99, i, flip_frac=0.1), tm.TM_F_FFT
        elif kind == 2:
            inst, flags = G.planted_gauss(n, k, 0.0, 99, i), 0
        else:
            inst = G.planted_pm1(n, k, 99, i, flip_frac=float(rng.uniform(0.05, 0.15)))
            flags = tm.TM_F_FFT if kind == 1 else 0
        plans.append(tm.Plan(inst.t, n=inst.n, x_dtype=tm.tm_dtype_of(inst.x), flags=flags))
        xs.append(to_device(inst.x))
        insts.append(inst)
    return plans, xs, insts


@pytest.mark.parametrize("kind", ["0", "2", "3", "4"], ids=["automatic product", "per-instance product",
                                                           "wave per row tile", "LDS ring"])
def test_graph_replays_equal_eager(kind, monkeypatch):
    monkeypatch.setenv("TM_CGEMM_KIND", kind)
    plans, xs, insts = _mixed(40, 3)
    assert sum(p.info["fft_global"] for p in plans) >= 1
    eager = tm.match_batch(plans, xs)
    out = torch.zeros(tm.RESULT_BYTES * len(plans), dtype=torch.uint8, device="cuda")
    _case("graph", kind)
    g = tm.BatchGraph(plans, xs, out)
    for rep in range(4):
        out.zero_()
        g.run()
        torch.cuda.synchronize()
        assert tm.results_from_device(out) == eager, rep
        # eager work of the program between replays
        assert tm.match_batch(plans[:7], xs[:7]) == eager[:7]
        torch.cuda.synchronize()
    for r, inst, p in zip(eager, insts, plans):
        if p.info["exact"] and p.info["corr_gemm"]:
            ref = O.ftm(inst.x, inst.t, p.m1, p.m2)
            assert (r.shift, r.m1_tilde, r.m2_tilde, r.n_candidates) == \
                (ref.shift, ref.m1_tilde, ref.m2_tilde, ref.n_candidates)
    g.close()


def test_graph_sees_new_signal_contents():
    insts = [G.planted_pm1(1 << 16, 512, 100, i, flip_frac=0.05) for i in range(12)]
    plans = [tm.Plan(s.t, n=s.n) for s in insts]
    xs = [to_device(s.x) for s in insts]
    out = torch.zeros(tm.RESULT_BYTES * len(plans), dtype=torch.uint8, device="cuda")
    _case("graph new contents")
    g = tm.BatchGraph(plans, xs, out)
    g.run()
    torch.cuda.synchronize()
    first = tm.results_from_device(out)
    assert first == tm.match_batch(plans, xs)
    # instance 0's signal replaced in place by instance 1's bytes
    xs[0].copy_(xs[1])
    torch.cuda.synchronize()
    g.run()
    torch.cuda.synchronize()
    second = tm.results_from_device(out)
    assert second[0] == tm.match(plans[0], xs[0])
    ref = O.ftm(insts[1].x, insts[0].t, plans[0].m1, plans[0].m2)
    assert (second[0].shift, second[0].m1_tilde, second[0].m2_tilde) == (ref.shift, ref.m1_tilde, ref.m2_tilde)
    assert second[1:] == first[1:]
    g.close()


def test_graph_refusals():
    inst = G.config1(0)
    plan = tm.Plan(inst.t, n=inst.n)
    x = to_device(inst.x)
    handle = tm.ctypes.c_void_p()
    parr = (tm.ctypes.c_void_p * 1)(plan.handle.value)
    xarr = (tm.ctypes.c_void_p * 1)(x.data_ptr())
    res = tm.Result()
    st = tm.lib().tm_batch_create(1, parr, xarr, tm.ctypes.addressof(res), None, tm.ctypes.byref(handle))
    assert st == tm.TM_ERR_INVALID and not handle.value          # host result memory
    out = torch.zeros(tm.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    st = tm.lib().tm_batch_create(0, parr, xarr, out.data_ptr(), None, tm.ctypes.byref(handle))
    assert st == tm.TM_ERR_INVALID
    three = tm.Plan(inst.t, n=inst.n, m3=-1)
    parr3 = (tm.ctypes.c_void_p * 1)(three.handle.value)
    st = tm.lib().tm_batch_create(1, parr3, xarr, out.data_ptr(), None, tm.ctypes.byref(handle))
    assert st == tm.TM_ERR_UNSUPPORTED


def test_eager_batch_table_follows_the_arguments():
    """tm_match_batch keeps the last batch's instance table on the device and
    skips its upload when plans, signals and results are the same: a batch with
    other signals, a subset, or single matches in between on the same stream
    must still get their own results."""
    insts = [G.planted_pm1(1 << 16, 512, 101, i, flip_frac=0.05) for i in range(24)]
    plans = [tm.Plan(s.t, n=s.n) for s in insts]
    xs = [to_device(s.x) for s in insts]
    _case("eager table reuse")
    first = tm.match_batch(plans, xs)
    for r, inst, p in zip(first, insts, plans):
        ref = O.ftm(inst.x, inst.t, p.m1, p.m2)
        assert (r.shift, r.m1_tilde, r.m2_tilde, r.n_candidates) == \
            (ref.shift, ref.m1_tilde, ref.m2_tilde, ref.n_candidates)
    assert tm.match_batch(plans, xs) == first                      # the same table again
    swapped = xs[::-1]
    other = tm.match_batch(plans, swapped)                         # same plans, other signals
    single = [tm.match(p, x) for p, x in zip(plans, swapped)]      # single matches on the stream
    assert other == single
    assert tm.match_batch(plans, xs) == first                      # after the single matches
    assert tm.match_batch(plans[:10], xs[:10]) == first[:10]       # a subset
    assert tm.match_batch(plans, xs) == first
