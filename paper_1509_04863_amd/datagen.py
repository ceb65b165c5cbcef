"""Seeded synthetic inputs for template matching.

This module only draws random numbers and arranges them into signals and
templates; it holds none of the matching arithmetic.  Both the CPU oracle
and the GPU path are fed from the arrays produced here, so the two always
see identical bytes.

The paper's own workload (Section 5, test procedure) is a uniform +-1 signal
with the template cut out of it at a uniformly drawn shift.  The other
generators add what the benchmark configurations ask for: exact-count sign
flips in the template, Gaussian noise at a given SNR, log-uniform sizes and
Poisson arrivals.

Seeding: every configuration has a root ``SeedSequence(150904863 + config_id)``;
instance ``i`` uses child ``i`` of that root, and inside an instance the
signal, the shift, the flips and the noise each draw from their own
grandchild stream, so changing one recipe never perturbs the others.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

ROOT_SEED = 150904863

# grandchild stream slots inside one instance
_S_SIGNAL, _S_SHIFT, _S_FLIPS, _S_NOISE, _S_SIZE, _S_DTYPE = range(6)


def instance_streams(config_id: int, index: int, n_streams: int = 6) -> List[np.random.Generator]:
    """Independent generators for one instance of one configuration."""
    root = np.random.SeedSequence(ROOT_SEED + int(config_id))
    # SeedSequence.spawn is stateful; derive the child by its spawn key instead
    child = np.random.SeedSequence(root.entropy, spawn_key=(int(index),))
    return [np.random.default_rng(s) for s in child.spawn(n_streams)]


def rademacher(n: int, rng: np.random.Generator, dtype=np.int8) -> np.ndarray:
    """Uniform +-1 vector (the paper's spreading code)."""
    bits = rng.integers(0, 2, size=int(n), dtype=np.int8)
    return (2 * bits - 1).astype(dtype, copy=False)


def gaussian(n: int, rng: np.random.Generator, dtype=np.float32) -> np.ndarray:
    return rng.standard_normal(int(n)).astype(dtype)


def cyclic_window(x: np.ndarray, start: int, length: int) -> np.ndarray:
    """x[(start + j) mod N] for j < length (the planted template)."""
    n = x.shape[0]
    idx = (int(start) + np.arange(int(length), dtype=np.int64)) % n
    return x[idx].copy()


def plant(x: np.ndarray, t: np.ndarray, start: int) -> np.ndarray:
    """Write t into x cyclically from position start (returns a copy)."""
    out = x.copy()
    n = out.shape[0]
    idx = (int(start) + np.arange(t.shape[0], dtype=np.int64)) % n
    out[idx] = t.astype(out.dtype)
    return out


def flip_exact(t: np.ndarray, frac: float, rng: np.random.Generator) -> np.ndarray:
    """Negate exactly round(frac*K) distinct, uniformly chosen entries."""
    k = t.shape[0]
    count = int(round(float(frac) * k))
    out = t.copy()
    if count > 0:
        pos = rng.choice(k, size=count, replace=False)
        out[pos] = -out[pos]
    return out


def noise_sigma(snr_db: float, signal_power: float = 1.0) -> float:
    """Noise standard deviation for SNR = 10 log10(P_s / sigma^2)."""
    return math.sqrt(signal_power * 10.0 ** (-float(snr_db) / 10.0))


def add_noise(v: np.ndarray, snr_db: float, rng: np.random.Generator,
              signal_power: float = 1.0, dtype=np.float32) -> np.ndarray:
    s = noise_sigma(snr_db, signal_power)
    return (v.astype(np.float64) + s * rng.standard_normal(v.shape[0])).astype(dtype)


def log_uniform_int(lo_exp: float, hi_exp: float, rng: np.random.Generator) -> int:
    """round(2**U(lo_exp, hi_exp))."""
    return int(round(2.0 ** rng.uniform(lo_exp, hi_exp)))


@dataclasses.dataclass
class Instance:
    """One matching problem: signal x, template t and the planted shift."""
    x: np.ndarray
    t: np.ndarray
    shift: int
    config_id: int
    index: int
    fold_mult: int = 1
    exact: bool = True        # integer-valued inputs (exact arithmetic applies)
    note: str = ""

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def k(self) -> int:
        return int(self.t.shape[0])


def planted_pm1(n: int, k: int, config_id: int, index: int, flip_frac: float = 0.0,
                x_dtype=np.int8, shift: Optional[int] = None) -> Instance:
    """The paper's test procedure: +-1 signal, template = cyclic window at a
    uniform shift, optionally with an exact count of sign flips."""
    g = instance_streams(config_id, index)
    x = rademacher(n, g[_S_SIGNAL], dtype=np.int8)
    m = int(g[_S_SHIFT].integers(0, n)) if shift is None else int(shift) % n
    t = cyclic_window(x, m, k)
    if flip_frac > 0:
        t = flip_exact(t, flip_frac, g[_S_FLIPS])
    return Instance(x=x.astype(x_dtype), t=t.astype(x_dtype), shift=m,
                    config_id=config_id, index=index, exact=True)


def planted_pm1_noisy_x(n: int, k: int, snr_db: float, config_id: int, index: int) -> Instance:
    """Section 5 noise experiment: x_e = x + e with Gaussian e at the given
    SNR (unit signal power), template cut from the clean x."""
    g = instance_streams(config_id, index)
    x = rademacher(n, g[_S_SIGNAL], dtype=np.int8)
    m = int(g[_S_SHIFT].integers(0, n))
    t = cyclic_window(x, m, k).astype(np.float32)
    xe = add_noise(x, snr_db, g[_S_NOISE])
    return Instance(x=xe, t=t, shift=m, config_id=config_id, index=index, exact=False)


def planted_gauss(n: int, k: int, snr_db: Optional[float], config_id: int, index: int) -> Instance:
    """N(0,1) float signal; template = window plus Gaussian noise at snr_db on t."""
    g = instance_streams(config_id, index)
    x = gaussian(n, g[_S_SIGNAL])
    m = int(g[_S_SHIFT].integers(0, n))
    t = cyclic_window(x, m, k)
    if snr_db is not None:
        t = add_noise(t, snr_db, g[_S_NOISE])
    return Instance(x=x, t=t.astype(np.float32), shift=m, config_id=config_id, index=index,
                    exact=False)


# --- the five benchmark workloads -------------------------------------------

def config1(index: int = 0, fold_mult: int = 1) -> Instance:
    """N=65536 +-1 int8, K=1024, 5% flips; fold length c*K with c in {1,2}."""
    inst = planted_pm1(65536, 1024, 1, index, flip_frac=0.05)
    inst.fold_mult = fold_mult
    return inst


def config2(index: int = 0) -> Instance:
    """N=2^22 +-1 stored as fp32, K=4096, 10% flips."""
    inst = planted_pm1(1 << 22, 4096, 2, index, flip_frac=0.10, x_dtype=np.float32)
    return inst


def config3_sizes(index: int):
    g = instance_streams(3, index)
    n = log_uniform_int(16, 20, g[_S_SIZE])
    k = log_uniform_int(9, 12, g[_S_SIZE])
    f = float(g[_S_SIZE].uniform(0.05, 0.15))
    return n, k, f


def config3(index: int) -> Instance:
    """Uneven batch member: N ~ 2^U(16,20), K ~ 2^U(9,12), flips U[5%,15%]."""
    n, k, f = config3_sizes(index)
    return planted_pm1(n, k, 3, index, flip_frac=f)


def config3_batch(count: int = 4096, start: int = 0) -> List[Instance]:
    return [config3(start + i) for i in range(count)]


def config5a(index: int = 0, n: int = 1 << 24, k: int = 1 << 14, snr_db: float = -3.0) -> Instance:
    """fp32 N(0,1) signal, template at SNR -3 dB (noise on t)."""
    return planted_gauss(n, k, snr_db, 51, index)


def config5b_batch(count: int = 1024, n: int = 1 << 18, k: int = 1024,
                   flip_frac: float = 0.0) -> List[Instance]:
    """count +-1 signals sharing one Rademacher template planted in each."""
    g0 = instance_streams(52, 0)
    t = rademacher(k, g0[_S_SIGNAL])
    out = []
    for i in range(count):
        g = instance_streams(52, i + 1)
        x = rademacher(n, g[_S_SIGNAL])
        m = int(g[_S_SHIFT].integers(0, n))
        tt = flip_exact(t, flip_frac, g[_S_FLIPS]) if flip_frac > 0 else t
        out.append(Instance(x=plant(x, tt, m), t=t.copy(), shift=m, config_id=52, index=i))
    return out


@dataclasses.dataclass
class Request:
    arrival_s: float
    pool_id: int
    shift: int
    k: int
    t: np.ndarray
    exact: bool


def poisson_arrivals(rate_hz: float, duration_s: float, rng: np.random.Generator) -> np.ndarray:
    """Arrival times of a Poisson process on [0, duration)."""
    out = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        out.append(t)
    return np.asarray(out, dtype=np.float64)


def config4_pool(pool_size: int, n_lo: float = 14, n_hi: float = 24,
                 int_frac: float = 0.7) -> List[Instance]:
    """Device-pool signals for the serving workload: 70% +-1 int8, 30% fp32 N(0,1)."""
    pool = []
    for i in range(pool_size):
        g = instance_streams(4, i)
        n = log_uniform_int(n_lo, n_hi, g[_S_SIZE])
        is_int = bool(g[_S_DTYPE].uniform() < int_frac)
        x = rademacher(n, g[_S_SIGNAL]) if is_int else gaussian(n, g[_S_SIGNAL])
        pool.append(Instance(x=x, t=np.zeros(0, x.dtype), shift=-1, config_id=4, index=i,
                             exact=is_int))
    return pool


def config4_requests(pool: Sequence[Instance], count: int, rate_hz: float = 20000.0,
                     k_lo: float = 8, k_hi: float = 13, snr_db: float = 0.0,
                     seed_index: int = 1 << 20) -> List[Request]:
    """Requests against the pool: planted window of a pool signal plus noise at snr_db."""
    g = instance_streams(4, seed_index)
    times = np.cumsum(g[_S_SHIFT].exponential(1.0 / rate_hz, size=count))
    reqs = []
    for r in range(count):
        pid = int(g[_S_SIZE].integers(0, len(pool)))
        sig = pool[pid]
        k = min(log_uniform_int(k_lo, k_hi, g[_S_SIZE]), sig.n)
        m = int(g[_S_SHIFT].integers(0, sig.n))
        win = cyclic_window(sig.x, m, k)
        # window plus Gaussian noise: a real-valued template for both signal
        # kinds (an int8 signal is still folded exactly, the correlation is real)
        t = add_noise(win, snr_db, g[_S_NOISE])
        reqs.append(Request(arrival_s=float(times[r]), pool_id=pid, shift=m, k=k, t=t,
                            exact=False))
    return reqs
