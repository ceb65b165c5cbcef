"""Shared helpers for the GPU tests: run an instance through the HIP path and
through the oracle on the same seeded bytes."""

import numpy as np

from oracle import ftm as O
from paper_1509_04863_amd import tm


def to_device(arr):
    import torch
    return torch.from_numpy(np.ascontiguousarray(arr)).cuda()


def gpu_match(x, t, m1=0, m2=0, fold_mult=1, flags=0, fold_store=tm.TM_F32, x_dev=None):
    """(result, y1, y2, r1, r2, plan) from the HIP path."""
    plan = tm.Plan(t, n=x.shape[0], m1=m1, m2=m2, fold_mult=fold_mult,
                   x_dtype=tm.tm_dtype_of(x) if x_dev is None else tm.tm_dtype_of(x_dev),
                   fold_store=fold_store, flags=flags)
    xd = to_device(x) if x_dev is None else x_dev
    res, y1, y2, r1, r2 = tm.match_intermediates(plan, xd)
    return res, y1, y2, r1, r2, plan


def assert_exact_parity(x, t, m1=0, m2=0, fold_mult=1, flags=0, x_oracle=None, t_oracle=None, x_dev=None):
    """Bit-exact comparison of every intermediate and output (integer data).
    When the plan computes the correlation by the int8 matrix product, the FFT
    correlation (TM_F_FFT) is checked as well: both must match the oracle."""
    xo = x if x_oracle is None else x_oracle
    to = t if t_oracle is None else t_oracle
    ref = None
    out = None
    variants = [flags] if flags & tm.TM_F_FFT else [flags, flags | tm.TM_F_FFT]
    for fl in variants:
        res, y1, y2, r1, r2, plan = gpu_match(x, t, m1, m2, fold_mult, fl, x_dev=x_dev)
        if ref is None:
            ref = O.ftm(xo, to, plan.m1, plan.m2)
        k = t.shape[0]
        assert np.array_equal(y1, ref.y1[:plan.m1 + k - 1].astype(np.float64)), "fold M1"
        assert np.array_equal(y2, ref.y2[:plan.m2 + k - 1].astype(np.float64)), "fold M2"
        assert np.array_equal(r1, ref.r1.astype(np.float64)), "correlation M1"
        assert np.array_equal(r2, ref.r2.astype(np.float64)), "correlation M2"
        assert (res.m1_tilde, res.m2_tilde) == (ref.m1_tilde, ref.m2_tilde)
        assert res.n_candidates == ref.n_candidates
        assert res.shift == ref.shift
        assert res.peak1 == float(ref.peak1) and res.peak2 == float(ref.peak2)
        if ref.shift != O.NOMATCH:
            assert res.score == float(ref.score)
        assert bool(res.flags & tm.TM_R_NOMATCH) == (ref.shift == O.NOMATCH)
        assert bool(res.flags & tm.TM_R_RESCORED) == (ref.n_candidates > 1)
        assert res.flags & tm.TM_R_EXACT
        if out is None:
            out = res
        else:
            assert res == out, "GEMM and FFT correlations disagree"
        if not plan.info["corr_gemm"]:
            break
    return out, ref


def normwise(a, b):
    scale = max(float(np.max(np.abs(b))), 1e-300)
    return float(np.max(np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64)))) / scale
