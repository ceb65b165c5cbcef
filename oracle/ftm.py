"""Plain CPU oracle for Fast Template Matching by Subsampled Circulant Matrix
(Hsieh, Lu, Pei, arXiv 1509.04863).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
CPU-baseline leg call this module.  The product path (the HIP library and its
Python binding) never imports it, and it imports nothing from the product.

Arithmetic is int64 when both the signal and the template are integer arrays,
float64 otherwise.  The code follows the paper's definitions and the steps of
its Algorithm 1 in the paper's order; it is meant to be checked against the
paper by eye, not to be fast.

Readings taken where the paper is silent, ambiguous or inconsistent
(each one is cited again where it is used):

  R1  Eq. (1) writes 0 < k < N; shifts range over all of [0, N).
  R3  Algorithm 1 step 6 writes IFFT(t~ .* y~), a convolution, while the
      quantity the method needs (Section 3, definition of (Tx)_k and the
      matrix T^ = circ([t 0]) of Theorem 1) is a cross-correlation.  The
      oracle computes the correlation r[k] = sum_j t_j y[k+j].
  R4  When M does not divide N the fold keeps the cyclic indices of
      Algorithm 1 step 3 (Section 2: indices are taken mod N), not the
      zero padding that Section 3.2 suggests for Theorem 2.  The zero-padded
      variant is available as ftm(..., variant="zero_pad") (reading R4z).
  R4z Theorem 2 variant: x is padded with zeros to L M (L = ceil(N/M)), the
      fold is y = [I_M ... I_M] x_pad of length M (the circulant block Phi_M
      of Theorem 2 taken as the identity, the choice that makes y the
      partition fold), the correlation is the circular one of length M with
      T^ = circ([t 0]) read as a correlation (R3), and the candidate set is
      {m~ + i M : i < L} restricted to [0, N) (positions of the padding are
      not shifts of x).
  R5  Only r[0..M) is used, so the fold is evaluated for k = 0..M+K-1 and the
      correlation for k = 0..M-1 (both as in step 3 / Theorem 1 with D_{M+K}).
  R6  Step 7 writes i <= M; Section 3.3 writes k < M.  The argmax ranges over
      [0, M).
  R7  Ties in any argmax go to the lowest index.
  R8  The candidate sets of step 8 are taken mod N, i.e. S is the support of
      row m~ of the sampling matrix Phi of Eq. (3).
  R9  Step 9 assumes a single common element.  With several, each candidate c
      is re-scored by (Tx)_c and the largest wins (lowest index on ties);
      with none, the result is -1 ("no match").
  R9T Top-T re-scoring (a robustness option beyond the paper, off by
      default): the T largest entries of each correlation (lowest index on
      ties) give T x T residue pairs; the union of their candidate sets is
      re-scored by (Tx)_c as in R9.  T = 1 is step 9 itself.
  R11a Three pairwise co-prime moduli (Theorem 4 with alpha = 3), for the
      regime K (K + 1) <= N where two moduli near K cannot cover N: each fold,
      correlation and argmax as for two, the candidate set the intersection
      of the three sets; the automatic choice is (m, m + 1, m + 2) with m the
      least odd number >= c K whose product exceeds N (consecutive numbers
      with m odd are pairwise co-prime).
  R11 Step 2 asks for M1 M2 > N with M1 = K, M2 = K + 1 (Section 4); when
      K (K + 1) <= N that choice is infeasible, and the automatic rule raises
      M1 to the least m with m (m + 1) > N.  fold_mult c in {1, 2} scales the
      K term: M1 = max(c K, m0(N)), M2 = M1 + 1.

Functions that have no pin other than themselves say so in their docstring
("parity unpinned").
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

NOMATCH = -1


# --------------------------------------------------------------------------
# arithmetic type
# --------------------------------------------------------------------------

def work_dtype(x: np.ndarray, t: np.ndarray):
    """int64 when both inputs are integer arrays, float64 otherwise."""
    if np.issubdtype(x.dtype, np.integer) and np.issubdtype(t.dtype, np.integer):
        return np.int64
    return np.float64


# --------------------------------------------------------------------------
# Section 2 / Section 3: circulant matrices and the full-search correlation
# --------------------------------------------------------------------------

def circ(v: np.ndarray) -> np.ndarray:
    """circ(v) of Section 2: row 0 is v, each next row is the previous one
    rotated right by one place, so circ(v)[r, c] = v[(c - r) mod n]."""
    n = v.shape[0]
    out = np.empty((n, n), dtype=v.dtype)
    for r in range(n):
        for c in range(n):
            out[r, c] = v[(c - r) % n]
    return out


def template_matrix(t: np.ndarray, n: int) -> np.ndarray:
    """T = circ([t 0_{N-K}]) of Section 3 (requires K <= N)."""
    k = t.shape[0]
    return circ(np.concatenate([t, np.zeros(n - k, dtype=t.dtype)]))


def sampling_matrix(n: int, m: int, rows: int, dtype=np.int64) -> np.ndarray:
    """Phi = D_rows(circ(r)) of Eq. (3): r_k = 1 iff k mod M = 0 (k < N), and
    D_rows keeps the first `rows` rows (rows = M, or M + K for strategy 1 of
    Section 3.2).  Requires rows <= N."""
    r = np.array([1 if (k % m) == 0 else 0 for k in range(n)], dtype=dtype)
    return circ(r)[:rows, :]


def full_correlation(x: np.ndarray, t: np.ndarray) -> np.ndarray:
    """(Tx)_k = sum_{i<K} t_i x_{(k+i) mod N} for every k in [0, N)
    (Section 3, first paragraph; cyclic indices from Section 2).  O(N K)."""
    dt = work_dtype(x, t)
    xv = x.astype(dt)
    tv = t.astype(dt)
    n = xv.shape[0]
    out = np.zeros(n, dtype=dt)
    k_idx = np.arange(n, dtype=np.int64)
    for i in range(tv.shape[0]):
        out += tv[i] * xv[(k_idx + i) % n]
    return out


def correlation_at(x: np.ndarray, t: np.ndarray, k: int):
    """(Tx)_k for one shift k, summed in index order (int64 or float64)."""
    dt = work_dtype(x, t)
    n = x.shape[0]
    idx = (int(k) + np.arange(t.shape[0], dtype=np.int64)) % n
    prods = t.astype(dt) * x[idx].astype(dt)
    acc = dt(0)
    for p in prods:           # plain left-to-right sum
        acc += p
    return acc


def argmax_lowest(v: np.ndarray) -> int:
    """Index of the maximum, lowest index on ties (reading R7)."""
    best = 0
    for i in range(1, v.shape[0]):
        if v[i] > v[best]:
            best = i
    return best


def full_search(x: np.ndarray, t: np.ndarray) -> int:
    """Ground truth m = argmax_k (Tx)_k over k in [0, N) (Eq. (1), reading R1;
    Section 3, first paragraph)."""
    return int(np.argmax(full_correlation(x, t)))  # np.argmax returns the first maximum


# --------------------------------------------------------------------------
# Algorithm 1 step 2: choice of the co-prime pair
# --------------------------------------------------------------------------

def least_m0(n: int) -> int:
    """The least m >= 1 with m (m + 1) > N."""
    m = max(1, math.isqrt(int(n)))
    while m > 1 and (m - 1) * m > n:
        m -= 1
    while m * (m + 1) <= n:
        m += 1
    return m


def choose_moduli(n: int, k: int, fold_mult: int = 1):
    """Automatic (M1, M2): M1 = max(c K, m0(N)), M2 = M1 + 1 (reading R11;
    Algorithm 1 step 2 and Section 4's M1 = K, M2 = K + 1)."""
    m1 = max(int(fold_mult) * int(k), least_m0(n))
    return m1, m1 + 1


def check_moduli(n: int, k: int, m1: int, m2: int) -> Optional[str]:
    """Conditions of Algorithm 1 step 2 (Theorem 4's product >= N is enough for
    uniqueness in [0, N)); returns an error message or None."""
    if k < 1 or n < k:
        return "need 1 <= K <= N"
    if m1 < k or m2 < k:
        return "need M1 >= K and M2 >= K"
    if math.gcd(m1, m2) != 1:
        return "M1 and M2 must be co-prime"
    if m1 * m2 < n:
        return "need M1 * M2 >= N"
    return None


# --------------------------------------------------------------------------
# Algorithm 1 step 3 / Eq. (2): the fold (downsampling)
# --------------------------------------------------------------------------

def fold(x: np.ndarray, m: int, k: int, dt=None) -> np.ndarray:
    """y[s] = sum_{i=0}^{ceil(N/M)-1} x[(s + i M) mod N] for s = 0..M+K-1
    (Algorithm 1 step 3, Eq. (2); cyclic indices, reading R4)."""
    n = x.shape[0]
    if dt is None:
        dt = np.int64 if np.issubdtype(x.dtype, np.integer) else np.float64
    xv = x.astype(dt)
    L = -(-n // m)
    s = np.arange(m + k, dtype=np.int64)
    y = np.zeros(m + k, dtype=dt)
    for i in range(L):
        y += xv[(s + i * m) % n]
    return y


# --------------------------------------------------------------------------
# Algorithm 1 steps 4-6: correlation in the folded space
# --------------------------------------------------------------------------

def correlate(y: np.ndarray, t: np.ndarray, m: int) -> np.ndarray:
    """r[k] = sum_{j<K} t_j y[k+j] for k in [0, M), by direct summation
    (steps 4-6 read as a cross-correlation, readings R3 and R5)."""
    dt = np.result_type(y.dtype, np.int64 if np.issubdtype(t.dtype, np.integer) else np.float64)
    yv = y.astype(dt)
    tv = t.astype(dt)
    r = np.zeros(m, dtype=dt)
    for j in range(tv.shape[0]):
        r += tv[j] * yv[j:j + m]
    return r


def correlate_fft(y: np.ndarray, t: np.ndarray, m: int) -> np.ndarray:
    """The same r[0..M) through a float64 FFT of length >= M + K - 1
    (Algorithm 1 steps 5-6 with the correlation reading).  Integer inputs are
    rounded to the nearest integer.  A fast cross-check of `correlate`, used by
    the statistics tests where the direct O(M K) sum is too slow."""
    k = t.shape[0]
    size = 1
    while size < m + k - 1:
        size *= 2
    yp = np.zeros(size)
    yp[:min(y.shape[0], m + k - 1)] = y[:m + k - 1]
    tp = np.zeros(size)
    tp[:k] = t
    c = np.fft.ifft(np.conj(np.fft.fft(tp)) * np.fft.fft(yp)).real[:m]
    if np.issubdtype(y.dtype, np.integer) and np.issubdtype(t.dtype, np.integer):
        return np.rint(c).astype(np.int64)
    return c


def fold_zero_pad(x: np.ndarray, m: int, dt=None) -> np.ndarray:
    """Theorem 2 variant (Section 3.2, reading R4z): x padded with zeros to
    L M, L = ceil(N/M), then y[s] = sum_{i<L} x_pad[s + i M] for s in [0, M),
    i.e. y = [I_M I_M ... I_M] x_pad."""
    n = x.shape[0]
    if dt is None:
        dt = np.int64 if np.issubdtype(x.dtype, np.integer) else np.float64
    L = -(-n // m)
    xp = np.zeros(L * m, dtype=dt)
    xp[:n] = x.astype(dt)
    y = np.zeros(m, dtype=dt)
    for i in range(L):
        y += xp[i * m:(i + 1) * m]
    return y


def correlate_circular(y: np.ndarray, t: np.ndarray, m: int) -> np.ndarray:
    """r[k] = sum_{j<K} t_j y[(k + j) mod M] for k in [0, M): the M x M
    circulant T^ = circ([t 0_{M-K}]) of Theorem 2 applied to y, read as a
    correlation (R3), by direct summation."""
    dt = np.result_type(y.dtype, np.int64 if np.issubdtype(t.dtype, np.integer) else np.float64)
    yv = y[:m].astype(dt)
    tv = t.astype(dt)
    r = np.zeros(m, dtype=dt)
    for j in range(tv.shape[0]):
        r += tv[j] * np.roll(yv, -j)
    return r


# --------------------------------------------------------------------------
# Algorithm 1 steps 7-9: argmax, candidate sets, intersection
# --------------------------------------------------------------------------

def candidate_set(m_tilde: int, m: int, n: int) -> set:
    """S = {(m~ + i M) mod N : i = 0..ceil(N/M)-1} (step 8, reading R8)."""
    L = -(-n // m)
    return {(m_tilde + i * m) % n for i in range(L)}


def candidate_set_zero_pad(m_tilde: int, m: int, n: int) -> set:
    """S = {m~ + i M : i = 0..ceil(N/M)-1} with the members inside [0, N)
    (step 8 as printed, for the zero-padded variant, reading R4z)."""
    L = -(-n // m)
    return {m_tilde + i * m for i in range(L) if m_tilde + i * m < n}


def top_indices(r: np.ndarray, count: int) -> List[int]:
    """The `count` largest entries of r by value, lowest index first among
    equal values (R7 extended to the runners-up, reading R9T)."""
    order = sorted(range(r.shape[0]), key=lambda i: (-r[i], i))
    return [int(i) for i in order[:count]]


def resolve(x: np.ndarray, t: np.ndarray, m1_tilde, m2_tilde, m1: int, m2: int,
            variant: str = "cyclic"):
    """Step 9: C = S_{M1} cap S_{M2} by literal set intersection; several
    members are re-scored by (Tx)_c (reading R9).  m1_tilde and m2_tilde may
    be lists of residues (top-T, reading R9T): C is then the union over all
    pairs.  Returns (shift, sorted candidates, score of the shift or None)."""
    n = x.shape[0]
    cs = candidate_set if variant == "cyclic" else candidate_set_zero_pad
    a_list = m1_tilde if isinstance(m1_tilde, (list, tuple)) else [m1_tilde]
    b_list = m2_tilde if isinstance(m2_tilde, (list, tuple)) else [m2_tilde]
    common = set()
    for a in a_list:
        for b in b_list:
            common |= cs(a, m1, n) & cs(b, m2, n)
    common = sorted(common)
    if not common:
        return NOMATCH, common, None
    best, best_score = None, None
    for c in common:                      # ascending, so ties keep the lowest
        sc = correlation_at(x, t, c)
        if best is None or sc > best_score:
            best, best_score = c, sc
    return int(best), common, best_score


@dataclasses.dataclass
class OracleResult:
    shift: int
    m1_tilde: int
    m2_tilde: int
    candidates: List[int]
    score: object
    peak1: object
    peak2: object
    m1: int
    m2: int
    y1: np.ndarray
    y2: np.ndarray
    r1: np.ndarray
    r2: np.ndarray

    @property
    def n_candidates(self) -> int:
        return len(self.candidates)


def ftm(x: np.ndarray, t: np.ndarray, m1: Optional[int] = None, m2: Optional[int] = None,
        fold_mult: int = 1, correlation: str = "direct", variant: str = "cyclic",
        top_t: int = 1) -> OracleResult:
    """Algorithm 1 (FTM) end to end, in the paper's step order.

    correlation="direct" is the oracle proper; "fft" swaps in the float64 FFT
    cross-check of steps 5-6 for large statistical runs.
    variant="cyclic" is Algorithm 1 as printed (fold of length M + K with
    indices mod N, Theorem 1); "zero_pad" is the Theorem 2 variant (fold of
    the zero-padded x of length M, circular correlation of length M, reading
    R4z).  In the zero_pad result y1, y2 have length M.
    top_t > 1 re-scores the candidates of the T x T pairs of runners-up
    (reading R9T); m1_tilde and m2_tilde stay the argmaxes of step 7."""
    if variant not in ("cyclic", "zero_pad"):
        raise ValueError("variant must be 'cyclic' or 'zero_pad'")
    n, k = x.shape[0], t.shape[0]
    # step 2
    if m1 is None or m2 is None:
        m1, m2 = choose_moduli(n, k, fold_mult)
    err = check_moduli(n, k, m1, m2)
    if err:
        raise ValueError(err)
    dt = work_dtype(x, t)
    # step 3
    if variant == "cyclic":
        y1 = fold(x, m1, k, dt)
        y2 = fold(x, m2, k, dt)
    else:
        y1 = fold_zero_pad(x, m1, dt)
        y2 = fold_zero_pad(x, m2, dt)
    # steps 4-6
    if variant == "cyclic":
        corr = correlate if correlation == "direct" else correlate_fft
        r1 = corr(y1, t, m1)
        r2 = corr(y2, t, m2)
    else:
        r1 = correlate_circular(y1, t, m1)
        r2 = correlate_circular(y2, t, m2)
    # step 7
    i1 = argmax_lowest(r1) if correlation == "direct" else int(np.argmax(r1))
    i2 = argmax_lowest(r2) if correlation == "direct" else int(np.argmax(r2))
    # steps 8-9
    if top_t > 1:
        a_list, b_list = top_indices(r1, top_t), top_indices(r2, top_t)
        if correlation == "direct":
            assert a_list[0] == i1 and b_list[0] == i2
        else:
            i1, i2 = a_list[0], b_list[0]
        shift, cands, score = resolve(x, t, a_list, b_list, m1, m2, variant)
    else:
        shift, cands, score = resolve(x, t, i1, i2, m1, m2, variant)
    return OracleResult(shift=shift, m1_tilde=i1, m2_tilde=i2, candidates=cands, score=score,
                        peak1=r1[i1], peak2=r2[i2], m1=m1, m2=m2, y1=y1, y2=y2, r1=r1, r2=r2)


def choose_moduli3(n: int, k: int, fold_mult: int = 1):
    """(m, m + 1, m + 2): m the least odd number >= c K with m (m + 1) (m + 2)
    > N (reading R11a)."""
    m = max(fold_mult * k, 1)
    if m % 2 == 0:
        m += 1
    while m * (m + 1) * (m + 2) <= n:
        m += 2
    return m, m + 1, m + 2


def ftm_multi(x: np.ndarray, t: np.ndarray, moduli: Sequence[int]) -> dict:
    """Algorithm 1 with alpha pairwise co-prime moduli (Theorem 4, reading
    R11a): for each M, the fold of step 3, the correlation of steps 4-6 and
    the argmax of step 7; the candidate set of step 8 is the intersection of
    the alpha sets (mod N), several members re-scored by (Tx)_c (R9)."""
    n, k = x.shape[0], t.shape[0]
    for i, a in enumerate(moduli):
        if a < k:
            raise ValueError("every modulus must be >= K")
        for b in moduli[i + 1:]:
            if math.gcd(a, b) != 1:
                raise ValueError("moduli must be pairwise co-prime")
    if math.prod(moduli) < n:
        raise ValueError("the product of the moduli must be >= N")
    dt = work_dtype(x, t)
    tildes, peaks, rs = [], [], []
    common = None
    for m in moduli:
        y = fold(x, m, k, dt)
        r = correlate(y, t, m)
        i = argmax_lowest(r)
        tildes.append(i)
        peaks.append(r[i])
        rs.append(r)
        s = candidate_set(i, m, n)
        common = s if common is None else common & s
    cands = sorted(common)
    best, best_score = NOMATCH, None
    for c in cands:
        sc = correlation_at(x, t, c)
        if best_score is None or sc > best_score:
            best, best_score = c, sc
    return {"shift": int(best), "tildes": tildes, "peaks": peaks, "candidates": cands,
            "score": best_score, "r": rs}


def top2_gap(r: np.ndarray) -> float:
    """Difference between the largest and the second-largest entry of r (the
    distance of an argmax from a tie).  Parity unpinned: a reporting aid."""
    if r.shape[0] < 2:
        return math.inf
    s = np.sort(np.asarray(r, dtype=np.float64))
    return float(s[-1] - s[-2])


# --------------------------------------------------------------------------
# Theorem 5: success bound (proof's explicit form)
# --------------------------------------------------------------------------

def thm5_failure_bound(n: int, k: int, m: int) -> float:
    """P_F^M <= M exp(-K / (8 ceil(N/M))) + 4 (ceil(N/M) - 1) / K
    (Theorem 5 proof, Chernoff and Chebyshev terms)."""
    L = -(-n // m)
    return m * math.exp(-k / (8.0 * L)) + 4.0 * (L - 1) / k


def thm5_success_bound(n: int, k: int, m1: int, m2: int) -> float:
    """(1 - P_F^{M1}) (1 - P_F^{M2}), each factor clamped to [0, 1]
    (Theorem 5 proof, last step; clamping because the bound can be vacuous)."""
    f1 = min(1.0, max(0.0, thm5_failure_bound(n, k, m1)))
    f2 = min(1.0, max(0.0, thm5_failure_bound(n, k, m2)))
    return (1.0 - f1) * (1.0 - f2)
