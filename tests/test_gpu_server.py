"""The request server (continuous batching, HBM admission): every result is
the same alone and in the mix, the workspace in flight stays within the
budget, and every submitted request completes."""

import threading

import numpy as np
import pytest

from oracle import ftm as O
from paper_1509_04863_amd import datagen as G
from paper_1509_04863_amd import tm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _mix(count, seed):
    """Uneven int8 exact, int8 with real template, fp32 real requests."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(2 ** rng.uniform(12, 19)))
        k = min(n, int(round(2 ** rng.uniform(6, 11))))
        kind = i % 3
        if kind == 0:
            inst = G.planted_pm1(n, k, 98, i, flip_frac=0.1)
        elif kind == 1:
            inst = G.planted_pm1(n, k, 98, i, flip_frac=0.1)
            inst.t = (inst.t.astype(np.float32) + 0.5 * rng.standard_normal(k)).astype(np.float32)
        else:
            inst = G.planted_gauss(n, k, 0.0, 98, i)
        out.append(inst)
    return out


def test_results_same_alone_and_in_mix():
    insts = _mix(60, 1)
    plans = [tm.Plan(s.t, n=s.n, x_dtype=tm.tm_dtype_of(s.x)) for s in insts]
    xs = [torch.from_numpy(s.x).cuda() for s in insts]
    alone = [tm.match(p, x) for p, x in zip(plans, xs)]
    print("case: server mix", flush=True)
    with tm.Server(max_batch=16, max_inflight=3) as srv:
        tickets = [None] * len(insts)

        def submit(idx):
            for i in idx:
                tickets[i] = srv.submit(plans[i], xs[i])

        th = threading.Thread(target=submit, args=(range(1, 60, 2),))
        th.start()
        submit(range(0, 60, 2))
        th.join()
        got = [srv.wait(t) for t in tickets]
        st = srv.stats()
    for (r, lat), a in zip(got, alone):
        assert r == a                         # bit for bit
        assert lat > 0
    assert st["submitted"] == st["completed"] == 60 and st["failed"] == 0
    for r, inst, p in zip(alone[::3], insts[::3], plans[::3]):   # exact ones against the oracle
        ref = O.ftm(inst.x, inst.t, p.m1, p.m2)
        assert (r.shift, r.m1_tilde, r.m2_tilde) == (ref.shift, ref.m1_tilde, ref.m2_tilde)


def test_budget_bounds_workspace_in_flight():
    insts = _mix(40, 2)
    plans = [tm.Plan(s.t, n=s.n, x_dtype=tm.tm_dtype_of(s.x)) for s in insts]
    xs = [torch.from_numpy(s.x).cuda() for s in insts]
    fps = [p.info["workspace_bytes"] + 48 + 512 for p in plans]   # + result slot and instance record
    budget = 3 * int(np.median(fps))
    print("case: server budget", budget, flush=True)
    with tm.Server(budget_bytes=budget, max_batch=64, max_inflight=4) as srv:
        tickets = [srv.submit(p, x) for p, x in zip(plans, xs)]
        got = [srv.wait(t)[0] for t in tickets]
        st = srv.stats()
    assert st["peak_inflight_bytes"] <= max(budget, max(fps))
    # the device memory the server's streams held at any launch: the budget
    # (plus the alignment of a few pool blocks), or one oversized request
    assert 0 < st["peak_held_bytes"] <= max(budget, max(fps)) + 4 * 4 * 4096
    assert st["batches"] >= sum(fps) // max(budget, max(fps))
    alone = [tm.match(p, x) for p, x in zip(plans, xs)]
    assert got == alone


def test_poll_and_drain_on_close():
    insts = _mix(12, 3)
    plans = [tm.Plan(s.t, n=s.n, x_dtype=tm.tm_dtype_of(s.x)) for s in insts]
    xs = [torch.from_numpy(s.x).cuda() for s in insts]
    srv = tm.Server(max_batch=4, max_inflight=2)
    tickets = [srv.submit(p, x) for p, x in zip(plans, xs)]
    done = {}
    while len(done) < len(tickets):
        for t in tickets:
            if t not in done:
                ok, r, lat = srv.poll(t)
                if ok:
                    done[t] = r
    with pytest.raises(tm.TMError):
        srv.poll(tickets[0])                  # consumed
    later = [srv.submit(p, x) for p, x in zip(plans, xs)]
    srv.close()                               # drains the queued requests
    assert len(later) == len(plans)
    assert [done[t] for t in tickets] == [tm.match(p, x) for p, x in zip(plans, xs)]


def test_create_destroy_frees_device_memory():
    # every slot's workspace pool, pinned staging and events go with the
    # server: device memory in use returns to its level after each cycle
    insts = _mix(18, 4)
    plans = [tm.Plan(s.t, n=s.n, x_dtype=tm.tm_dtype_of(s.x)) for s in insts]
    xs = [torch.from_numpy(s.x).cuda() for s in insts]
    alone = [tm.match(p, x) for p, x in zip(plans, xs)]
    torch.cuda.synchronize()
    print("case: server create/destroy", flush=True)

    def used():
        free, total = torch.cuda.mem_get_info()
        return total - free

    def cycle():
        with tm.Server(budget_bytes=64 << 20, max_batch=8, max_inflight=3) as srv:
            got = [srv.wait(srv.submit(p, x))[0] for p, x in zip(plans, xs)]
            held = srv.stats()["peak_held_bytes"]
        assert got == alone
        return held

    cycle()                                   # the runtime's own first-use allocations
    torch.cuda.synchronize()
    base = used()
    for _ in range(3):
        held = cycle()
        torch.cuda.synchronize()
        assert held > 0
        assert used() <= base + (2 << 20), "a server left device memory behind"
