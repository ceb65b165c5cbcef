"""The band fold of 4-byte signals (k_fold_band) against the oracle.

Integer-valued fp32 signals on the exact path must match bit for bit; real
signals within the normwise 1e-5 of the FP64 oracle.  Cases vary the rows per
band task (ragged last row block), the band count (M not a multiple of 64),
consecutive and non-consecutive moduli, both ways of folding a consecutive
pair (two column-sum views, the default, or TM_BAND_DIAG=1: fold B from the
diagonals of view A), and compare with the tiled fold.
"""

import numpy as np
import pytest

from oracle import ftm as O
from paper_1509_04863_amd import datagen as G
from paper_1509_04863_amd import tm

from _util import assert_exact_parity, gpu_match, normwise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _case(*a):
    print("case:", *a, flush=True)


SHAPES = [
    # (n, k, m1, m2, shift)
    (1 << 20, 2048, 0, 0, 77),
    (300007, 1000, 0, 0, 300000),     # M = 1000: 16 bands, the last one partial
    (70001, 33, 0, 0, 5),             # M = m0 = 265
    (50000, 100, 211, 307, 4999),     # non-consecutive: two views
    (90000, 300, 301, 300, 12345),    # swapped
    (5000, 4000, 0, 0, 4999),         # L = 2
    (1, 1, 0, 0, 0),
]


@pytest.mark.parametrize("diag", ["0", "1"])
@pytest.mark.parametrize("rows", [0, 16, 48, 256])
@pytest.mark.parametrize("n,k,m1,m2,shift", SHAPES)
def test_band_exact_fp32_storage(n, k, m1, m2, shift, rows, diag, monkeypatch):
    monkeypatch.setenv("TM_BAND_ROWS", str(rows))
    monkeypatch.setenv("TM_BAND_DIAG", diag)
    inst = G.planted_pm1(n, k, 90, n + rows, flip_frac=0.1, shift=shift, x_dtype=np.float32)
    info = tm.plan_params(n, k, m1=m1, m2=m2, x_dtype=tm.TM_F32, flags=tm.TM_F_EXACT)
    assert info["fold_bands"] > 0 and info["fold_tiles"] == 0
    _case("band exact", n, k, m1, m2, rows, "diag", diag)
    assert_exact_parity(inst.x, inst.t, m1=m1, m2=m2, flags=tm.TM_F_EXACT,
                        x_oracle=inst.x.astype(np.int64), t_oracle=inst.t.astype(np.int64))


@pytest.mark.parametrize("diag", ["0", "1"])
@pytest.mark.parametrize("rows", [0, 16, 256])
@pytest.mark.parametrize("n,k,m1,m2", [(1 << 20, 4096, 0, 0), (99991, 700, 0, 0), (60000, 90, 257, 263)])
def test_band_real(n, k, m1, m2, rows, diag, monkeypatch):
    monkeypatch.setenv("TM_BAND_ROWS", str(rows))
    monkeypatch.setenv("TM_BAND_DIAG", diag)
    inst = G.planted_gauss(n, k, 0.0, 91, n + rows)
    _case("band real", n, k, m1, m2, rows, "diag", diag)
    res, y1, y2, r1, r2, plan = gpu_match(inst.x, inst.t, m1=m1, m2=m2)
    assert plan.info["fold_bands"] > 0
    ref = O.ftm(inst.x.astype(np.float64), inst.t.astype(np.float64), plan.m1, plan.m2)
    assert normwise(y1, ref.y1[:plan.m1 + k - 1]) <= 1e-5
    assert normwise(y2, ref.y2[:plan.m2 + k - 1]) <= 1e-5
    assert normwise(r1, ref.r1) <= 1e-5 and normwise(r2, ref.r2) <= 1e-5


def test_band_real_is_deterministic():
    inst = G.planted_gauss(1 << 21, 2000, 0.0, 92, 0)
    plan = tm.Plan(inst.t, n=inst.n)
    x = torch.from_numpy(inst.x).cuda()
    first = tm.match_intermediates(plan, x)
    for _ in range(3):
        again = tm.match_intermediates(plan, x)
        assert again[0] == first[0]
        for a, b in zip(again[1:], first[1:]):
            assert np.array_equal(a, b)


def test_band_and_tile_paths_agree_exact(monkeypatch):
    inst = G.planted_pm1(1 << 21, 3000, 93, 0, flip_frac=0.1, x_dtype=np.float32)
    plan_b = tm.Plan(inst.t, n=inst.n, x_dtype=tm.TM_F32, flags=tm.TM_F_EXACT)
    monkeypatch.setenv("TM_FOLD_BAND", "0")
    plan_t = tm.Plan(inst.t, n=inst.n, x_dtype=tm.TM_F32, flags=tm.TM_F_EXACT)
    assert plan_b.info["fold_bands"] > 0 and plan_t.info["fold_bands"] == 0
    x = torch.from_numpy(inst.x).cuda()
    rb = tm.match_intermediates(plan_b, x)
    rt = tm.match_intermediates(plan_t, x)
    assert rb[0] == rt[0]
    for a, b in zip(rb[1:], rt[1:]):
        assert np.array_equal(a, b)


def test_consecutive_pair_fold_choice(monkeypatch):
    """A consecutive pair folds as two views by default; TM_BAND_DIAG=1 takes
    fold B from view A's diagonals.  Both give the same literal folds."""
    inst = G.planted_gauss(1 << 20, 1000, 0.0, 94, 0)
    plan_v = tm.Plan(inst.t, n=inst.n)
    monkeypatch.setenv("TM_BAND_DIAG", "1")
    plan_d = tm.Plan(inst.t, n=inst.n)
    assert plan_v.info["dual"] == 0 and plan_d.info["dual"] == 1
    assert plan_v.m2 == plan_v.m1 + 1
    x = torch.from_numpy(inst.x).cuda()
    _case("fold choice")
    rv = tm.match_intermediates(plan_v, x)
    rd = tm.match_intermediates(plan_d, x)
    ref = O.ftm(inst.x.astype(np.float64), inst.t.astype(np.float64), plan_v.m1, plan_v.m2)
    for r in (rv, rd):
        assert normwise(r[1], ref.y1[:plan_v.m1 + inst.k - 1]) <= 1e-5
        assert normwise(r[2], ref.y2[:plan_v.m2 + inst.k - 1]) <= 1e-5
