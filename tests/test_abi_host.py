"""Host-side checks of the C ABI: the library loads, exports every symbol that
include/tm.h declares, and its host-only plan logic (tm_plan_params) follows
the same reading of Algorithm 1 step 2 as the oracle.  No GPU is touched."""

import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import ftm as O
from paper_1509_04863_amd import tm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "tm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tm_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = tm.lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert set(tm.EXPORTS) <= set(names)


def test_status_strings_and_version():
    L = tm.lib()
    assert L.tm_status_string(0) == b"ok"
    assert L.tm_status_string(1) == b"invalid argument"
    assert re.match(rb"^\d+\.\d+\.\d+$", L.tm_version())


@pytest.mark.parametrize("n,k", [(65536, 1024), (1 << 22, 4096), (1 << 20, 512), (1 << 16, 4096),
                                  (12345, 7), (1, 1), (100, 100), (1 << 24, 256), (99991, 300)])
@pytest.mark.parametrize("c", [1, 2])
def test_auto_moduli_follow_oracle_rule(n, k, c):
    info = tm.plan_params(n, k, fold_mult=c)
    m1, m2 = O.choose_moduli(n, k, c)
    assert (info["m1"], info["m2"]) == (m1, m2)
    assert info["l1"] == -(-n // m1) and info["l2"] == -(-n // m2)
    P = 1 << info["fft_log2"]
    assert P >= m2 + k - 1 and (P // 2 < m2 + k - 1 or P == 2)
    assert info["dual"] == 1 and info["exact"] == 1


def test_explicit_moduli_and_orientation():
    info = tm.plan_params(1000, 10, 33, 32)           # swapped consecutive pair
    assert (info["m1"], info["m2"], info["dual"]) == (33, 32, 1)
    info = tm.plan_params(1000, 10, 31, 37)           # general co-prime pair
    assert (info["m1"], info["m2"], info["dual"]) == (31, 37, 0)


@pytest.mark.parametrize("kw", [
    dict(n=100, k=101),                      # K > N
    dict(n=100, k=0),                        # K < 1
    dict(n=100, k=10, m1=10, m2=12),         # gcd 2
    dict(n=200, k=10, m1=10, m2=11),         # M1 M2 < N
    dict(n=100, k=12, m1=10, m2=11),         # M < K
    dict(n=100, k=10, m1=5, m2=0),           # only one explicit modulus
    dict(n=100, k=10, fold_mult=3),
    dict(n=100, k=10, x_dtype=7),
    dict(n=100, k=10, fold_store=1 << 5),
    dict(n=100, k=10, flags=0x100),
    dict(n=100, k=10, flags=tm.TM_F_EXACT | tm.TM_F_REAL),
    dict(n=100, k=10, flags=0x10),
    dict(n=100, k=10, top_t=5),
    dict(n=100, k=10, top_t=-1),
    dict(n=100, k=10, m3=-2),                      # bad third modulus
    dict(n=100, k=3, m1=3, m2=5, m3=9),            # gcd(3, 9) = 3
    dict(n=1000, k=3, m1=3, m2=4, m3=5),           # product 60 < N
    dict(n=100, k=10, m3=-1, top_t=2),             # three moduli with top-T
    dict(n=100, k=10, m3=-1, flags=tm.TM_F_ZERO_PAD),
    dict(n=100, k=3, m3=-1, m1=3),                 # automatic with an explicit modulus
])
def test_invalid_plans_are_rejected(kw):
    with pytest.raises(tm.TMError) as e:
        tm.plan_params(**kw)
    assert e.value.status == tm.TM_ERR_INVALID
    assert tm.lib().tm_last_error()


def test_three_moduli_params():
    # automatic: (m, m + 1, m + 2), m the least odd >= K with a product above N
    info = tm.plan_params(1 << 20, 300, m3=-1)
    assert (info["m1"], info["m2"], info["m3"]) == (301, 302, 303)
    info = tm.plan_params(1 << 26, 100, m3=-1)
    m = info["m1"]
    assert m % 2 == 1 and m * (m + 1) * (m + 2) > 1 << 26 >= (m - 2) * (m - 1) * m
    two = tm.plan_params(1 << 20, 300)
    assert two["m3"] == 0 and two["m1"] == 1024          # two moduli must reach m0(N)
    explicit = tm.plan_params(1 << 20, 200, m1=211, m2=223, m3=227)
    assert (explicit["m1"], explicit["m2"], explicit["m3"]) == (211, 223, 227)


def test_modes():
    assert tm.plan_params(1000, 10)["exact"] == 1
    assert tm.plan_params(1000, 10, x_dtype=tm.TM_F32, t_dtype=tm.TM_F32)["exact"] == 0
    assert tm.plan_params(1000, 10, x_dtype=tm.TM_F32, t_dtype=tm.TM_F32,
                          flags=tm.TM_F_EXACT)["exact"] == 1
    assert tm.plan_params(1000, 10, flags=tm.TM_F_REAL)["exact"] == 0
    assert tm.plan_params(1000, 10, x_dtype=tm.TM_I8, t_dtype=tm.TM_F32)["exact"] == 0


def test_fft_length_limits():
    # exact path keeps P <= 2^13 in one workgroup's LDS, the real path P <= 2^14;
    # above that the four-step transform through global memory takes over, up to 2^21
    # (TM_F_FFT: exact plans with an int8 template otherwise take the int8 matrix product)
    F = tm.TM_F_FFT
    info = tm.plan_params(1 << 22, 4096, flags=F)
    assert info["fft_in_lds"] == 1 and info["fft_global"] == 0 and info["corr_gemm"] == 0
    info = tm.plan_params(1 << 24, 8192, flags=F)
    assert info["fft_in_lds"] == 0 and info["fft_global"] == 1
    assert tm.plan_params(1 << 24, 8192, x_dtype=tm.TM_F32, t_dtype=tm.TM_F32)["fft_in_lds"] == 1
    info = tm.plan_params(1 << 24, 1 << 14, x_dtype=tm.TM_F32, t_dtype=tm.TM_F32)
    assert info["fft_log2"] == 15 and info["fft_global"] == 1
    assert tm.plan_params(1 << 26, 1 << 16)["fft_global"] == 1          # Section 5 tables: P = 2^17
    info = tm.plan_params(1 << 30, 1 << 21)                              # P = 2^22: no path
    assert info["fft_in_lds"] == 0 and info["fft_global"] == 0


def test_correlation_route():
    # exact int8 plans: the int8 matrix product up to (M1 + M2)(K + 63) <= 2^32
    # and K <= 2^17; then the FFT; never on the real path
    info = tm.plan_params(1 << 22, 4096)
    assert info["corr_gemm"] == 1 and info["fft_global"] == 0
    assert tm.plan_params(1 << 24, 8192)["corr_gemm"] == 1
    assert tm.plan_params(1 << 25, 1 << 15)["corr_gemm"] == 1
    assert tm.plan_params(1 << 26, 1 << 16)["corr_gemm"] == 0
    assert tm.plan_params(1 << 22, 4096, flags=tm.TM_F_REAL)["corr_gemm"] == 0
    assert tm.plan_params(1 << 22, 4096, x_dtype=tm.TM_F32, t_dtype=tm.TM_F32)["corr_gemm"] == 0
    # the workspace holds the digit rows: more than the FFT route needs
    a = tm.plan_params(1 << 22, 4096)["workspace_bytes"]
    b = tm.plan_params(1 << 22, 4096, flags=tm.TM_F_FFT)["workspace_bytes"]
    assert a > b


def test_plan_create_without_device_fails_cleanly():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    desc = tm._desc(1000, 10)
    h = ctypes.c_void_p()
    t = np.ones(10, dtype=np.int8)
    st = tm.lib().tm_plan_create(ctypes.byref(desc), t.ctypes.data, 0, None, ctypes.byref(h))
    assert st in (tm.TM_ERR_DEVICE, tm.TM_ERR_NOMEM)
    assert not h.value


def test_admission_rule_first_in_first_out():
    fp = [100, 200, 300, 50, 5000, 10, 10, 10]
    b = tm.admit_batches(fp, budget_bytes=600, max_batch=3)
    # batches in order, never above the budget or max_batch, oversized alone
    assert list(b) == [0, 0, 0, 1, 2, 3, 3, 3]
    b = tm.admit_batches(fp, budget_bytes=10 ** 9, max_batch=2)
    assert list(b) == [0, 0, 1, 1, 2, 2, 3, 3]


def test_admission_rule_invariants_random():
    rng = np.random.default_rng(4)
    for _ in range(200):
        n = int(rng.integers(0, 60))
        fp = rng.integers(1, 1000, n)
        budget = int(rng.integers(1, 3000))
        mb = int(rng.integers(1, 9))
        b = tm.admit_batches(fp, budget, mb)
        assert np.all(np.diff(b) >= 0) and (n == 0 or b[0] == 0)
        for j in range(int(b.max()) + 1 if n else 0):
            members = fp[b == j]
            assert 1 <= members.size <= mb
            assert members.sum() <= budget or members.size == 1
            nxt = np.nonzero(b == j + 1)[0]
            if nxt.size and members.size < mb:       # the next request did not fit
                assert members.sum() + fp[nxt[0]] > budget
