// gfx950 kernels of the template matcher.
//
//   k_fold     Algorithm 1 step 3 (Eq. (2)): per-tile partial folds.  x is read
//              as rows of M1 elements; a tile of R rows x W columns yields the
//              column sums (fold M1) and, when M2 = M1 + 1, the diagonal sums
//              (element (i, c) has index i*M1 + c = i*M2 + (c - i), so it falls
//              in bucket (c - i) mod M2): both folds from one read of x.
//   k_reduce   sums the partials of each bucket in a fixed order and applies the
//              cyclic wrap of Algorithm 1's indices (Section 2: indices mod N),
//              giving the literal folds y[0 .. M+K-1).
//   k_finish   one workgroup per instance: packs y1 + i*y2, FFT, product with
//              the plan's spectrum conj(FFT(t))/P, inverse FFT (steps 4-6 as a
//              cross-correlation), argmax over [0, M) (step 7), candidate
//              intersection (steps 8-9, Theorem 4) and (Tx) scoring.
//   k_twiddles FP64 twiddles exp(-2 pi i e / P) (stored FP64 or FP32).
//   k_spectrum plan-time FP64 spectrum of the zero-padded template.

#include <hip/hip_fp16.h>

#include "tm_internal.h"

namespace tmi {

// --------------------------------------------------------------------------
// element types and conversions
// --------------------------------------------------------------------------

struct bf16_t { uint16_t b; };
struct f16_t { uint16_t b; };

__device__ __forceinline__ float to_float(int8_t v) { return (float)v; }
__device__ __forceinline__ float to_float(float v) { return v; }
__device__ __forceinline__ float to_float(bf16_t v) { return __uint_as_float((uint32_t)v.b << 16); }
__device__ __forceinline__ float to_float(f16_t v) { return __half2float(__ushort_as_half(v.b)); }

template <typename Acc> struct AccOf;
template <> struct AccOf<int> {
  __device__ __forceinline__ static int from(int8_t v) { return (int)v; }
  template <typename Tin> __device__ __forceinline__ static int from(Tin v) {
    return __float2int_rn(to_float(v));
  }
};
template <> struct AccOf<float> {
  template <typename Tin> __device__ __forceinline__ static float from(Tin v) { return to_float(v); }
};

// value of x[idx] as a double (for scores) for any storage type
__device__ __forceinline__ double load_as_double(const void* p, int dt, int64_t idx) {
  switch (dt) {
    case TM_I8: return (double)((const int8_t*)p)[idx];
    case TM_F32: return (double)((const float*)p)[idx];
    case TM_BF16: return (double)to_float(((const bf16_t*)p)[idx]);
    default: return (double)to_float(((const f16_t*)p)[idx]);
  }
}

// --------------------------------------------------------------------------
// fold tiles
// --------------------------------------------------------------------------

__host__ __device__ __forceinline__ int fold_slot_bytes(int cols, int eb) {
  return ((cols * eb + 15) & ~15) + 16;
}

size_t fold_lds_bytes(const View& v, int x_dtype) {
  const int eb = dtype_bytes(x_dtype);
  return (size_t)v.rows * fold_slot_bytes(v.cols, eb) + (size_t)v.rows * sizeof(int2);
}

template <typename Tin, typename Acc>
__device__ void fold_tile(const Inst& d, int lt, unsigned char* lds) {
  const int tid = threadIdx.x;
  const int NT = blockDim.x;
  const int nta = d.va.nrb * d.va.ncb;
  const bool in_a = lt < nta;
  const View v = in_a ? d.va : d.vb;
  if (!in_a) lt -= nta;
  const bool want_diag = in_a && d.dual;
  const int rb = lt / v.ncb;
  const int cb = lt - rb * v.ncb;
  const int R = v.rows, W = v.cols, M = v.m;
  const int64_t N = d.n;
  const int Reff = min(R, v.l - rb * R);
  const int c0 = cb * W;
  constexpr int EB = sizeof(Tin);
  const int SLOT = fold_slot_bytes(W, EB);
  const int CQ = SLOT >> 4;
  int2* rowinfo = reinterpret_cast<int2*>(lds + (size_t)R * SLOT);
  const uintptr_t xa = reinterpret_cast<uintptr_t>(d.x);
  const uintptr_t xend = xa + (uintptr_t)N * EB;

  // per row: byte offset of column c0 inside its 16-byte envelope, valid columns
  for (int r = tid; r < Reff; r += NT) {
    const int64_t n0 = (int64_t)(rb * R + r) * M + c0;
    int64_t nv = min((int64_t)min(M - c0, W), N - n0);
    if (nv < 0) nv = 0;
    const uintptr_t a0 = xa + (uintptr_t)n0 * EB;
    rowinfo[r] = make_int2((int)(a0 & 15), (int)nv);
  }
  __syncthreads();

  // stage the tile: aligned 16-byte loads, byte loads at the array's ends
  for (int idx = tid; idx < Reff * CQ; idx += NT) {
    const int r = idx / CQ;
    const int q = idx - r * CQ;
    const int2 ri = rowinfo[r];
    if (q * 16 >= ri.x + ri.y * EB) continue;
    const int64_t n0 = (int64_t)(rb * R + r) * M + c0;
    const uintptr_t A = ((xa + (uintptr_t)n0 * EB) & ~(uintptr_t)15) + (uintptr_t)q * 16;
    unsigned char* dst = lds + (size_t)r * SLOT + q * 16;
    if (A >= xa && A + 16 <= xend) {
      *reinterpret_cast<uint4*>(dst) = *reinterpret_cast<const uint4*>(A);
    } else {
      for (int b = 0; b < 16; ++b) {
        const uintptr_t ad = A + b;
        dst[b] = (ad >= xa && ad < xend) ? *reinterpret_cast<const unsigned char*>(ad) : 0;
      }
    }
  }
  __syncthreads();

  // column sums (fold over modulus M), rows in increasing order
  Acc* colp = reinterpret_cast<Acc*>(in_a ? d.col_a : d.col_b);
  for (int j = tid; j < W && c0 + j < M; j += NT) {
    Acc acc = 0;
    for (int r = 0; r < Reff; ++r) {
      const int2 ri = rowinfo[r];
      if (j < ri.y)
        acc += AccOf<Acc>::from(*reinterpret_cast<const Tin*>(lds + (size_t)r * SLOT + ri.x + j * EB));
    }
    colp[(int64_t)rb * M + c0 + j] = acc;
  }

  // diagonal sums (fold over M + 1): diagonal e holds elements (r, j) with
  // j - r = e - (R - 1); rows in increasing order
  if (want_diag) {
    const int E = W + R - 1;
    Acc* dp = reinterpret_cast<Acc*>(d.diag) + (int64_t)(rb * v.ncb + cb) * E;
    for (int e = tid; e < E; e += NT) {
      Acc acc = 0;
      const int rlo = max(0, R - 1 - e);
      const int rhi = min(Reff, R - 1 - e + W);
      for (int r = rlo; r < rhi; ++r) {
        const int j = e - (R - 1) + r;
        const int2 ri = rowinfo[r];
        if (j < ri.y)
          acc += AccOf<Acc>::from(*reinterpret_cast<const Tin*>(lds + (size_t)r * SLOT + ri.x + j * EB));
      }
      dp[e] = acc;
    }
  }
}

__device__ __forceinline__ int find_inst_by_tile(const InstTable& tab, int tile) {
  int lo = 0, hi = tab.count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab.get(mid).tile_base <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int find_inst_by_chunk(const InstTable& tab, int chunk) {
  int lo = 0, hi = tab.count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab.get(mid).red_base <= chunk) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ bool acc_is_int(const Inst& d) {
  return d.x_dtype == TM_I8 || d.mode == MODE_EXACT;
}

__global__ void __launch_bounds__(kFoldThreads) k_fold(InstTable tab, int total_tiles) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int tile = blockIdx.x;
  if (tile >= total_tiles) return;
  const Inst& d = tab.get(find_inst_by_tile(tab, tile));
  const int lt = tile - d.tile_base;
  if (acc_is_int(d)) {
    switch (d.x_dtype) {
      case TM_I8: fold_tile<int8_t, int>(d, lt, lds); break;
      case TM_F32: fold_tile<float, int>(d, lt, lds); break;
      case TM_BF16: fold_tile<bf16_t, int>(d, lt, lds); break;
      default: fold_tile<f16_t, int>(d, lt, lds); break;
    }
  } else {
    switch (d.x_dtype) {
      case TM_F32: fold_tile<float, float>(d, lt, lds); break;
      case TM_BF16: fold_tile<bf16_t, float>(d, lt, lds); break;
      default: fold_tile<f16_t, float>(d, lt, lds); break;
    }
  }
}

// --------------------------------------------------------------------------
// reduce partials to the literal folds
// --------------------------------------------------------------------------

// partition sum of bucket s: sum of x[n] over n < N with n = s (mod M)
template <typename Acc>
__device__ Acc bucket_sum(const Inst& d, int fold, int s) {
  Acc acc = 0;
  if (fold == 0) {
    const Acc* p = reinterpret_cast<const Acc*>(d.col_a);
    for (int rb = 0; rb < d.va.nrb; ++rb) acc += p[(int64_t)rb * d.va.m + s];
  } else if (!d.dual) {
    const Acc* p = reinterpret_cast<const Acc*>(d.col_b);
    for (int rb = 0; rb < d.vb.nrb; ++rb) acc += p[(int64_t)rb * d.vb.m + s];
  } else {
    // diagonal e of tile (rb, cb) covers bucket (e + cb*W - rb*R - (R-1)) mod mb
    const Acc* p = reinterpret_cast<const Acc*>(d.diag);
    const int R = d.va.rows, W = d.va.cols, E = W + R - 1, ncb = d.va.ncb;
    const int64_t mb = d.vb.m;
    const int64_t qmax = (int64_t)ncb * W + R - 1;
    for (int rb = 0; rb < d.va.nrb; ++rb) {
      const int64_t v0 = ((int64_t)s + (int64_t)rb * R + R - 1) % mb;
      for (int64_t q = v0; q < qmax; q += mb) {
        const int cb_hi = (int)min(q / W, (int64_t)ncb - 1);
        const int64_t lo_num = q - (E - 1);
        const int cb_lo = lo_num <= 0 ? 0 : (int)((lo_num + W - 1) / W);
        for (int cb = cb_lo; cb <= cb_hi; ++cb)
          acc += p[(int64_t)(rb * ncb + cb) * E + (q - (int64_t)cb * W)];
      }
    }
  }
  return acc;
}

template <typename Tin, typename Acc>
__device__ __forceinline__ Acc xval(const Inst& d, int64_t idx) {
  return AccOf<Acc>::from(reinterpret_cast<const Tin*>(d.x)[idx]);
}

// literal fold entry u of fold f (Algorithm 1 step 3): y[u] for u < M + K - 1
template <typename Tin, typename Acc>
__device__ Acc literal_fold(const Inst& d, int f, int u) {
  const int64_t M = f ? d.vb.m : d.va.m;
  const int64_t L = f ? d.vb.l : d.va.l;
  const int64_t N = d.n;
  const int s = u < M ? u : (int)(u - M);
  Acc acc = bucket_sum<Acc>(d, f, s);
  // the last of the L terms wraps past N-1 (cyclic index of Section 2)
  if ((int64_t)s + (L - 1) * M >= N) acc += xval<Tin, Acc>(d, ((int64_t)s + (L - 1) * M) % N);
  // y[M + s] = y[s] - x[s] + x[(s + L M) mod N]
  if (u >= M) acc += xval<Tin, Acc>(d, ((int64_t)s + L * M) % N) - xval<Tin, Acc>(d, s);
  return acc;
}

template <typename Tin, typename Acc>
__device__ void reduce_chunk(const Inst& d, int lc) {
  const int totA = d.va.m + d.k - 1;
  const int tot = totA + d.vb.m + d.k - 1;
  const int u0 = lc * kReduceChunk;
  const int u1 = min(u0 + kReduceChunk, tot);
  Acc* y = reinterpret_cast<Acc*>(d.y);
  for (int u = u0 + threadIdx.x; u < u1; u += blockDim.x) {
    const int f = u >= totA;
    y[u] = literal_fold<Tin, Acc>(d, f, f ? u - totA : u);
  }
}

__global__ void __launch_bounds__(kReduceThreads) k_reduce(InstTable tab, int total_chunks) {
  const int chunk = blockIdx.x;
  if (chunk >= total_chunks) return;
  const Inst& d = tab.get(find_inst_by_chunk(tab, chunk));
  const int lc = chunk - d.red_base;
  if (acc_is_int(d)) {
    switch (d.x_dtype) {
      case TM_I8: reduce_chunk<int8_t, int>(d, lc); break;
      case TM_F32: reduce_chunk<float, int>(d, lc); break;
      case TM_BF16: reduce_chunk<bf16_t, int>(d, lc); break;
      default: reduce_chunk<f16_t, int>(d, lc); break;
    }
  } else {
    switch (d.x_dtype) {
      case TM_F32: reduce_chunk<float, float>(d, lc); break;
      case TM_BF16: reduce_chunk<bf16_t, float>(d, lc); break;
      default: reduce_chunk<f16_t, float>(d, lc); break;
    }
  }
}

// --------------------------------------------------------------------------
// FFT correlation in LDS
// --------------------------------------------------------------------------

template <typename T> struct cplx { T x, y; };
template <typename T> __device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T> __device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

// one pad element per 16 keeps strided butterfly accesses off a single bank
__device__ __forceinline__ int padi(int j) { return j + (j >> 4); }

__host__ __device__ __forceinline__ int padded_len(int P) { return P + (P >> 4) + 1; }

int fft_lds_max_log2(int mode) { return mode == MODE_EXACT ? 13 : 14; }

size_t finish_lds_bytes(int p_log2, int mode) {
  const size_t el = mode == MODE_EXACT ? 16 : 8;
  return (size_t)padded_len(1 << p_log2) * el + (size_t)kFinishThreads * 16;
}

// A pass applies radix-2 stages s0 .. s0+KB-1 to groups of 2^KB elements
// spaced 2^(p - s0 - KB) apart.  DIR 0: forward decimation-in-frequency
// stages (natural order in, bit-reversed out).  DIR 1: inverse
// decimation-in-time stages in descending order (each undoes the forward
// stage up to a factor 2).  DIR 2: forward stages, product with the spectrum
// (stored at the bit-reversed positions), inverse stages.
template <int KB, int DIR, typename T>
__device__ void fft_pass(cplx<T>* buf, int p, int s0, const cplx<T>* __restrict__ tw,
                         const cplx<T>* __restrict__ spec) {
  constexpr int RR = 1 << KB;
  const int P = 1 << p;
  const int lh = p - s0 - KB;
  const int hl = 1 << lh;
  const int ng = P >> KB;
  for (int g = threadIdx.x; g < ng; g += blockDim.x) {
    const int blk = g >> lh;
    const int off = g & (hl - 1);
    const int base = (blk << (p - s0)) + off;
    cplx<T> v[RR];
#pragma unroll
    for (int m = 0; m < RR; ++m) v[m] = buf[padi(base + (m << lh))];
    if (DIR != 1) {
#pragma unroll
      for (int st = 0; st < KB; ++st) {
        const int s = s0 + st;
        const int hm = RR >> (st + 1);
        const int hmask = (P >> (s + 1)) - 1;
#pragma unroll
        for (int m = 0; m < RR; ++m) {
          if (m & hm) continue;
          const int e = ((off + (m << lh)) & hmask) << s;
          const cplx<T> a = v[m], b = v[m + hm];
          v[m] = a + b;
          v[m + hm] = cmul(a - b, tw[e]);
        }
      }
    }
    if (DIR == 2) {
#pragma unroll
      for (int m = 0; m < RR; ++m) v[m] = cmul(v[m], spec[base + (m << lh)]);
    }
    if (DIR != 0) {
#pragma unroll
      for (int st = KB - 1; st >= 0; --st) {
        const int s = s0 + st;
        const int hm = RR >> (st + 1);
        const int hmask = (P >> (s + 1)) - 1;
#pragma unroll
        for (int m = 0; m < RR; ++m) {
          if (m & hm) continue;
          const int e = ((off + (m << lh)) & hmask) << s;
          const cplx<T> a = v[m];
          const cplx<T> b = cmulc(v[m + hm], tw[e]);
          v[m] = a + b;
          v[m + hm] = a - b;
        }
      }
    }
#pragma unroll
    for (int m = 0; m < RR; ++m) buf[padi(base + (m << lh))] = v[m];
  }
}

template <int DIR, typename T>
__device__ __forceinline__ void fft_pass_kb(int kb, cplx<T>* buf, int p, int s0, const cplx<T>* tw,
                                            const cplx<T>* spec) {
  switch (kb) {
    case 1: fft_pass<1, DIR>(buf, p, s0, tw, spec); break;
    case 2: fft_pass<2, DIR>(buf, p, s0, tw, spec); break;
    case 3: fft_pass<3, DIR>(buf, p, s0, tw, spec); break;
    default: fft_pass<4, DIR>(buf, p, s0, tw, spec); break;
  }
}

// c[n] = sum_j t_j z[(n + j) mod P]: forward transform, product with the
// spectrum, inverse transform, all in LDS.
// Pass i of the plan for length 2^p: radix-2^kb stages starting at s0.
// p <= 4: one pass; otherwise an optional p mod 4 pass first, then radix 16.
__device__ __forceinline__ int fft_npasses(int p) { return p <= 4 ? 1 : ((p & 3) ? 1 : 0) + (p >> 2); }
__device__ __forceinline__ void fft_pass_of(int i, int p, int& s0, int& kb) {
  if (p <= 4) { s0 = 0; kb = p; return; }
  const int rem = p & 3;
  if (rem == 0) { s0 = 4 * i; kb = 4; return; }
  if (i == 0) { s0 = 0; kb = rem; return; }
  s0 = rem + 4 * (i - 1);
  kb = 4;
}

// c[n] = sum_j t_j z[(n + j) mod P]: forward transform, product with the
// spectrum, inverse transform, all in LDS.
template <typename T>
__device__ void fft_correlate(cplx<T>* buf, int p, const cplx<T>* tw, const cplx<T>* spec) {
  const int np = fft_npasses(p);
  int s0, kb;
  for (int i = 0; i + 1 < np; ++i) {
    fft_pass_of(i, p, s0, kb);
    fft_pass_kb<0>(kb, buf, p, s0, tw, spec);
    __syncthreads();
  }
  fft_pass_of(np - 1, p, s0, kb);
  fft_pass_kb<2>(kb, buf, p, s0, tw, spec);
  __syncthreads();
  for (int i = np - 2; i >= 0; --i) {
    fft_pass_of(i, p, s0, kb);
    fft_pass_kb<1>(kb, buf, p, s0, tw, spec);
    __syncthreads();
  }
}

// --------------------------------------------------------------------------
// workgroup reductions (fixed pairing: deterministic)
// --------------------------------------------------------------------------

struct VI { double v; int i; };

__device__ __forceinline__ bool vi_better(const VI& a, const VI& b) {
  return a.v > b.v || (a.v == b.v && a.i < b.i);
}

__device__ VI block_argmax(VI mine, VI* scratch) {
  const int tid = threadIdx.x;
  scratch[tid] = mine;
  __syncthreads();
  for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
    if (tid < s && vi_better(scratch[tid + s], scratch[tid])) scratch[tid] = scratch[tid + s];
    __syncthreads();
  }
  const VI r = scratch[0];
  __syncthreads();
  return r;
}

template <typename S>
__device__ S block_sum(S mine, S* scratch) {
  const int tid = threadIdx.x;
  scratch[tid] = mine;
  __syncthreads();
  for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
    if (tid < s) scratch[tid] = scratch[tid] + scratch[tid + s];
    __syncthreads();
  }
  const S r = scratch[0];
  __syncthreads();
  return r;
}

// --------------------------------------------------------------------------
// finish: FFT correlation, argmax, candidate intersection, scoring
// --------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T store_round(float v, int fold_store) {
  if (fold_store == TM_BF16) {
    const uint32_t u = __float_as_uint(v);
    const uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);      // round to nearest even
    return (T)__uint_as_float(r & 0xffff0000u);
  }
  if (fold_store == TM_F16) return (T)__half2float(__float2half_rn(v));
  return (T)v;
}

// Score (Tx)_c = sum_j t_j x[(c + j) mod N]: int64 on the exact path, FP64 otherwise.
__device__ double score_at(const Inst& d, int64_t c, void* scratch) {
  const int64_t N = d.n;
  if (d.mode == MODE_EXACT) {
    long long acc = 0;
    for (int j = threadIdx.x; j < d.k; j += blockDim.x) {
      const int64_t xi = (c + j) % N;
      acc += (long long)llrint(load_as_double(d.t, d.t_dtype, j)) *
             (long long)llrint(load_as_double(d.x, d.x_dtype, xi));
    }
    return (double)block_sum<long long>(acc, (long long*)scratch);
  }
  double acc = 0.0;
  for (int j = threadIdx.x; j < d.k; j += blockDim.x) {
    const int64_t xi = (c + j) % N;
    acc += load_as_double(d.t, d.t_dtype, j) * load_as_double(d.x, d.x_dtype, xi);
  }
  return block_sum<double>(acc, (double*)scratch);
}

template <typename T, typename Acc>
__device__ void finish_instance(const Inst& d, unsigned char* lds) {
  const int tid = threadIdx.x;
  const int NT = blockDim.x;
  const int p = d.p_log2;
  const int P = 1 << p;
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(lds);
  void* scratch = lds + (size_t)padded_len(P) * sizeof(cplx<T>);
  const int ma = d.va.m, mb = d.vb.m, K = d.k;
  const int na = ma + K - 1, nb = mb + K - 1;
  const Acc* y = reinterpret_cast<const Acc*>(d.y);
  const bool exact = d.mode == MODE_EXACT;
  double* dya = d.swapped ? d.dbg_y2 : d.dbg_y1;
  double* dyb = d.swapped ? d.dbg_y1 : d.dbg_y2;
  double* dra = d.swapped ? d.dbg_r2 : d.dbg_r1;
  double* drb = d.swapped ? d.dbg_r1 : d.dbg_r2;

  // pack z = yA + i yB, zero padded to P
  double ss = 0.0;
  for (int n = tid; n < P; n += NT) {
    T re = 0, im = 0;
    if (n < na) {
      re = exact ? (T)y[n] : store_round<T>((float)y[n], d.fold_store);
      if (dya) dya[n] = (double)re;
    }
    if (n < nb) {
      im = exact ? (T)y[na + n] : store_round<T>((float)y[na + n], d.fold_store);
      if (dyb) dyb[n] = (double)im;
    }
    ss += (double)re * (double)re + (double)im * (double)im;
    buf[padi(n)] = cplx<T>{re, im};
  }
  const double znorm2 = block_sum<double>(ss, (double*)scratch);   // includes a barrier

  fft_correlate<T>(buf, p, reinterpret_cast<const cplx<T>*>(d.tw), reinterpret_cast<const cplx<T>*>(d.spec));

  // step 7: argmax over [0, M) of each fold, lowest index on ties
  VI ba{-INFINITY, 0x7fffffff}, bb{-INFINITY, 0x7fffffff};
  for (int n = tid; n < ma; n += NT) {
    const double v = exact ? rint((double)buf[padi(n)].x) : (double)buf[padi(n)].x;
    if (dra) dra[n] = v;
    const VI c{v, n};
    if (vi_better(c, ba)) ba = c;
  }
  for (int n = tid; n < mb; n += NT) {
    const double v = exact ? rint((double)buf[padi(n)].y) : (double)buf[padi(n)].y;
    if (drb) drb[n] = v;
    const VI c{v, n};
    if (vi_better(c, bb)) bb = c;
  }
  VI* vs = reinterpret_cast<VI*>(scratch);
  const VI amax = block_argmax(ba, vs);
  const VI bmax = block_argmax(bb, vs);

  uint32_t flags = 0;
  if (!exact) {
    // near tie: second largest (excluding the argmax) within 1e-5 of the fold's peak scale
    VI sa{-INFINITY, 0x7fffffff}, sb{-INFINITY, 0x7fffffff};
    double absa = 0.0, absb = 0.0;
    for (int n = tid; n < ma; n += NT) {
      const double v = (double)buf[padi(n)].x;
      absa = fmax(absa, fabs(v));
      if (n != amax.i && vi_better(VI{v, n}, sa)) sa = VI{v, n};
    }
    for (int n = tid; n < mb; n += NT) {
      const double v = (double)buf[padi(n)].y;
      absb = fmax(absb, fabs(v));
      if (n != bmax.i && vi_better(VI{v, n}, sb)) sb = VI{v, n};
    }
    const VI sa2 = block_argmax(sa, vs);
    const VI sb2 = block_argmax(sb, vs);
    const VI ma2 = block_argmax(VI{absa, 0}, vs);
    const VI mb2 = block_argmax(VI{absb, 0}, vs);
    if (amax.v - sa2.v <= 1e-5 * ma2.v || bmax.v - sb2.v <= 1e-5 * mb2.v) flags |= TM_R_NEAR_TIE;
  } else {
    // FP64 FFT error bound: |dc| <= 20 p u ||t||_1 ||z||_2, u = 2^-53
    const double bound = 20.0 * p * 0x1p-53 * d.tnorm1 * sqrt(znorm2);
    if (bound < 0.5) flags |= TM_R_EXACT;
  }

  // steps 8-9: S_A(a) cap S_B(b) with the candidate sets taken mod N
  __shared__ long long cand[4];
  __shared__ int ncand;
  if (tid == 0) {
    const int64_t N = d.n;
    const int64_t A = ma, B = mb, La = d.va.l, Lb = d.vb.l;
    const int64_t a = amax.i, b = bmax.i;
    long long c0 = -1, c1 = -1, c2 = -1;   // ascending after insertion, -1 = unused
    auto insert = [&](long long v) {
      if (v == c0 || v == c1 || v == c2) return;
      if (c0 < 0 || v < c0) { c2 = c1; c1 = c0; c0 = v; }
      else if (c1 < 0 || v < c1) { c2 = c1; c1 = v; }
      else c2 = v;
    };
    // regular members {a + iA < N} and {b + jB < N}: Chinese remaindering
    if (a < N && b < N) {
      const int64_t t = ((((b - a) % B) + B) % B) * d.inv_a_mod_b % B;
      const int64_t v = a + A * t;
      if (v < N) insert(v);
    }
    // the wrapped members (a + (La-1) A) mod N and (b + (Lb-1) B) mod N
    const bool wa = a + (La - 1) * A >= N;
    const bool wb = b + (Lb - 1) * B >= N;
    const int64_t va = (a + (La - 1) * A) % N;
    const int64_t vb = (b + (Lb - 1) * B) % N;
    if (wa && ((b < N && va % B == b) || (wb && va == vb))) insert(va);
    if (wb && (a < N && vb % A == a)) insert(vb);
    int w = 0;
    if (c0 >= 0) cand[w++] = c0;
    if (c1 >= 0) cand[w++] = c1;
    if (c2 >= 0) cand[w++] = c2;
    ncand = w;
  }
  __syncthreads();
  const int nc = ncand;
  int64_t best = -1;
  double best_score = 0.0;
  for (int i = 0; i < nc; ++i) {
    const double sc = score_at(d, cand[i], scratch);
    if (i == 0 || sc > best_score) { best = cand[i]; best_score = sc; }
  }
  if (nc == 0) flags |= TM_R_NOMATCH;
  if (nc > 1) flags |= TM_R_RESCORED;
  if (tid == 0) {
    tm_result r;
    r.shift = best;
    r.m1_tilde = d.swapped ? bmax.i : amax.i;
    r.m2_tilde = d.swapped ? amax.i : bmax.i;
    r.n_candidates = nc;
    r.flags = flags;
    r.peak1 = d.swapped ? bmax.v : amax.v;
    r.peak2 = d.swapped ? amax.v : bmax.v;
    r.score = nc ? best_score : 0.0;
    *d.out = r;
  }
}

template <typename T>
__global__ void __launch_bounds__(kFinishThreads) k_finish(InstTable tab, const int32_t* list, int count) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int b = blockIdx.x;
  if (b >= count) return;
  const Inst& d = tab.get(list ? list[b] : b);
  if (acc_is_int(d)) finish_instance<T, int>(d, lds);
  else finish_instance<T, float>(d, lds);
}

// --------------------------------------------------------------------------
// plan-time kernels
// --------------------------------------------------------------------------

__global__ void k_twiddles(void* tw, int p, int as_double) {
  const int P = 1 << p;
  const int half = P >> 1;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < half; e += gridDim.x * blockDim.x) {
    double s, c;
    sincospi(-2.0 * (double)e / (double)P, &s, &c);
    if (as_double) reinterpret_cast<double2*>(tw)[e] = make_double2(c, s);
    else reinterpret_cast<float2*>(tw)[e] = make_float2((float)c, (float)s);
  }
}

// Radix-2 decimation-in-frequency transform of the zero-padded template in FP64
// (global scratch, one workgroup), then S = conj(Z) / P at the same positions.
__global__ void __launch_bounds__(1024) k_spectrum(const void* t, int t_dtype, int k, int p,
                                                   const double2* tw64, double2* z, void* spec,
                                                   int as_double) {
  const int P = 1 << p;
  const int tid = threadIdx.x, NT = blockDim.x;
  for (int n = tid; n < P; n += NT) z[n] = make_double2(n < k ? load_as_double(t, t_dtype, n) : 0.0, 0.0);
  __syncthreads();
  for (int s = 0; s < p; ++s) {
    const int h = P >> (s + 1);
    for (int idx = tid; idx < (P >> 1); idx += NT) {
      const int j = ((idx >> (p - s - 1)) << (p - s)) + (idx & (h - 1));
      const double2 a = z[j], b = z[j + h];
      const double2 w = tw64[(j & (h - 1)) << s];
      const double dx = a.x - b.x, dy = a.y - b.y;
      z[j] = make_double2(a.x + b.x, a.y + b.y);
      z[j + h] = make_double2(dx * w.x - dy * w.y, dx * w.y + dy * w.x);
    }
    __syncthreads();
  }
  const double inv = 1.0 / (double)P;
  for (int n = tid; n < P; n += NT) {
    const double2 v = z[n];
    if (as_double) reinterpret_cast<double2*>(spec)[n] = make_double2(v.x * inv, -v.y * inv);
    else reinterpret_cast<float2*>(spec)[n] = make_float2((float)(v.x * inv), (float)(-v.y * inv));
  }
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------

// Best effort: AMD devices accept dynamic LDS up to the per-workgroup limit
// without an opt-in, so a refused attribute is not an error.
hipError_t configure_kernels() {
  int dev = 0, lds = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  const void* fns[] = {reinterpret_cast<const void*>(k_fold), reinterpret_cast<const void*>(k_finish<double>),
                       reinterpret_cast<const void*>(k_finish<float>)};
  for (const void* f : fns) {
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
      (void)hipGetLastError();
  }
  return hipSuccess;
}

hipError_t launch_fold(const InstTable& tab, int total_tiles, size_t lds, hipStream_t s) {
  if (total_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fold, dim3(total_tiles), dim3(kFoldThreads), lds, s, tab, total_tiles);
  return hipGetLastError();
}

hipError_t launch_reduce(const InstTable& tab, int total_chunks, hipStream_t s) {
  if (total_chunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3(total_chunks), dim3(kReduceThreads), 0, s, tab, total_chunks);
  return hipGetLastError();
}

hipError_t launch_finish(const InstTable& tab, const int32_t* list, int count, int mode, size_t lds,
                         hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (mode == MODE_EXACT)
    hipLaunchKernelGGL(k_finish<double>, dim3(count), dim3(kFinishThreads), lds, s, tab, list, count);
  else
    hipLaunchKernelGGL(k_finish<float>, dim3(count), dim3(kFinishThreads), lds, s, tab, list, count);
  return hipGetLastError();
}

hipError_t launch_twiddles(void* tw, int p_log2, int as_double, hipStream_t s) {
  const int half = (1 << p_log2) >> 1;
  const int blocks = (half + 255) / 256;
  hipLaunchKernelGGL(k_twiddles, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, tw, p_log2, as_double);
  return hipGetLastError();
}

hipError_t launch_spectrum(const void* t, int t_dtype, int k, int p_log2, const double* tw64,
                           double* scratch, void* spec, int as_double, hipStream_t s) {
  hipLaunchKernelGGL(k_spectrum, dim3(1), dim3(1024), 0, s, t, t_dtype, k, p_log2,
                     reinterpret_cast<const double2*>(tw64), reinterpret_cast<double2*>(scratch), spec,
                     as_double);
  return hipGetLastError();
}

}  // namespace tmi
