"""The streaming int8 fold (k_fold_s8) against the oracle, bit for bit.

The streaming fold reads x in 16-byte chunks addressed from x rounded down to
16 bytes, so these cases vary x's byte offset, the segment length (several
segments, several LDS pieces per segment, rows straddling segment and piece
ends), the word count of a row (1 to 9 slots per lane, M up to 4608) and both
orientations of the moduli, and check that the tiled fold gives the same.
"""

import numpy as np
import pytest

from oracle import ftm as O
from paper_1509_04863_amd import datagen as G
from paper_1509_04863_amd import tm

from _util import assert_exact_parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _case(*a):
    print("case:", *a, flush=True)


def _offset_view(x, off):
    """x on the device starting `off` bytes into a fresh allocation."""
    buf = torch.zeros(x.shape[0] + 64, dtype=torch.int8, device="cuda")
    buf[off:off + x.shape[0]] = torch.from_numpy(x).cuda()
    return buf[off:off + x.shape[0]]


def _plan_kind(n, k, **kw):
    return tm.plan_params(n, k, **kw)


@pytest.mark.parametrize("off", [0, 1, 2, 3, 5, 8, 13, 15])
def test_unaligned_signal(off):
    inst = G.planted_pm1(100003, 700, 80, off, flip_frac=0.05)
    info = _plan_kind(inst.n, inst.k)
    assert info["fold_segments"] > 0 and info["fold_tiles"] == 0
    _case("offset", off)
    assert_exact_parity(inst.x, inst.t, x_dev=_offset_view(inst.x, off))


SHAPES = [
    # (n, k, m1, m2, shift): slot counts 1..9, non-dual, swapped, M = 4608
    (70000, 16, 0, 0, 5),           # M = 265 (m0), one slot
    (300000, 512, 0, 0, 299999),    # M = 548
    (400000, 1000, 0, 0, 17),       # two slots
    (500000, 1536, 0, 0, 123),      # three (mb = 1537 -> four)
    (800000, 3000, 0, 0, 799000),   # six
    (1 << 20, 4096, 0, 0, 4095),    # eight and nine
    (1 << 20, 3000, 4607, 4608, 1), # M = 4607 / 4608, nine
    (60000, 100, 211, 307, 5000),   # non-consecutive moduli
    (200000, 500, 700, 699, 77),    # swapped
]


@pytest.mark.parametrize("seg", [16, 1008, 16384, 40000, 0])
@pytest.mark.parametrize("n,k,m1,m2,shift", SHAPES)
def test_segments_and_slots(n, k, m1, m2, shift, seg, monkeypatch):
    monkeypatch.setenv("TM_SEG_BYTES", str(seg))
    inst = G.planted_pm1(n, k, 81, n + seg, flip_frac=0.08, shift=shift)
    info = _plan_kind(n, k, m1=m1, m2=m2)
    assert info["fold_segments"] > 0
    _case("seg", seg, n, k, m1, m2, info["fold_segments"])
    assert_exact_parity(inst.x, inst.t, m1=m1, m2=m2, x_dev=_offset_view(inst.x, (n + seg) % 16))


def test_general_bytes_and_extremes():
    """All 256 byte values, long runs of -128 and 127 (largest lane sums)."""
    rng = np.random.default_rng(9)
    n, k = 600000, 2300
    x = rng.integers(-128, 128, n).astype(np.int8)
    x[1000:300000] = -128
    x[300000:590000] = 127
    t = rng.integers(-128, 128, k).astype(np.int8)
    _case("extremes")
    assert_exact_parity(x, t, x_dev=_offset_view(x, 7))


def test_row_limit_per_segment(monkeypatch):
    """Segments of exactly 256 rows of 127 (a 16-bit lane's largest sum)."""
    monkeypatch.setenv("TM_SEG_BYTES", str(1 << 30))      # capped at 256 rows
    n, k = 2048 * 600, 2048
    x = np.full(n, 127, dtype=np.int8)
    t = np.ones(k, dtype=np.int8)
    info = _plan_kind(n, k)
    assert info["fold_segments"] == -(-((n + 15) // 16) // (256 * info["m1"] // 16 - 1))
    _case("row limit")
    assert_exact_parity(x, t)


@pytest.mark.parametrize("n,k,m1,m2", [(65536, 1024, 0, 0), (1 << 20, 4096, 0, 0), (99991, 300, 0, 0),
                                       (4609 * 3, 3000, 4609, 4610)])
def test_stream_and_tile_paths_agree(n, k, m1, m2, monkeypatch):
    inst = G.planted_pm1(n, k, 82, n, flip_frac=0.1)
    plan_s = tm.Plan(inst.t, n=n, m1=m1, m2=m2)
    monkeypatch.setenv("TM_FOLD_STREAM", "0")
    plan_t = tm.Plan(inst.t, n=n, m1=m1, m2=m2)
    assert plan_t.info["fold_segments"] == 0
    assert (plan_s.info["fold_segments"] > 0) == (max(plan_s.m1, plan_s.m2) <= 4608)
    x = torch.from_numpy(inst.x).cuda()
    _case("paths", n, k)
    rs, y1s, y2s, r1s, r2s = tm.match_intermediates(plan_s, x)
    rt, y1t, y2t, r1t, r2t = tm.match_intermediates(plan_t, x)
    assert rs == rt
    for a, b in ((y1s, y1t), (y2s, y2t), (r1s, r1t), (r2s, r2t)):
        assert np.array_equal(a, b)


def test_batch_mixing_stream_and_tile_instances():
    """One batch: streamed int8, tiled int8 (M > 4608), fp32 and real instances."""
    shapes = [(70000, 600, 0, 0), (300000, 3000, 4801, 4802), (1 << 18, 2048, 0, 0), (40000, 40, 0, 0),
              (1 << 20, 4096, 0, 0), (9000, 3000, 4700, 4699)]
    insts = [G.planted_pm1(n, k, 83, i, flip_frac=0.07) for i, (n, k, _, _) in enumerate(shapes)]
    plans = [tm.Plan(s.t, n=s.n, m1=m1, m2=m2) for s, (_, _, m1, m2) in zip(insts, shapes)]
    assert any(p.info["fold_segments"] for p in plans) and any(p.info["fold_tiles"] for p in plans)
    xs = [torch.from_numpy(s.x).cuda() for s in insts]
    g = G.planted_gauss(50000, 300, 0.0, 84, 0)
    plans.append(tm.Plan(g.t, n=g.n))
    xs.append(torch.from_numpy(g.x).cuda())
    _case("mixed batch")
    batch = tm.match_batch(plans, xs)
    single = [tm.match(p, x) for p, x in zip(plans, xs)]
    assert all(b == s for b, s in zip(batch, single))
    for b, inst, p in zip(batch, insts, plans):
        ref = O.ftm(inst.x, inst.t, p.m1, p.m2)
        assert (b.shift, b.m1_tilde, b.m2_tilde, b.n_candidates) == \
            (ref.shift, ref.m1_tilde, ref.m2_tilde, ref.n_candidates)
