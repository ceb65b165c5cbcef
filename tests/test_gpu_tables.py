"""Section 5 on the GPU, few trials: success rates inside a binomial band
around the paper's printed Table 1 and Table 2 values (the full 1000-trial
runs are `python -m paper_1509_04863_amd.tables`)."""

import math

import pytest

from paper_1509_04863_amd import tables

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _band(p_paper, trials, paper_trials=1000, z=4.0):
    se = math.sqrt(max(p_paper * (1 - p_paper), 0.01) * (1.0 / trials + 1.0 / paper_trials))
    return p_paper - z * se, p_paper + z * se


def test_table1_small():
    print("case: table 1", flush=True)
    rows = tables.table1(80, log2ns=(24, 25), progress=False)
    for r in rows:
        lo, hi = _band(r["paper"], r["trials"])
        print(r, flush=True)
        assert lo <= r["success"] <= hi


def test_table2_small():
    print("case: table 2", flush=True)
    rows = tables.table2(25, snrs=(20, -6), progress=False)
    for r in rows:
        lo, hi = _band(r["paper"], r["trials"])
        print(r, flush=True)
        assert lo <= r["success"] <= hi
