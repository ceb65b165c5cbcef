// gfx950 kernels of the template matcher.
//
//   k_fold     Algorithm 1 step 3 (Eq. (2)).  x is read as rows of M1 elements;
//              a tile of R rows x W columns is staged in LDS and yields the
//              column sums (fold over M1) and, when M2 = M1 + 1, the diagonal
//              sums (element (i, c) has index i*M1 + c = i*M2 + (c - i), so it
//              belongs to bucket (c - i) mod M2): both folds from one read of x.
//              Integer folds are added straight into the partition-fold buckets
//              with int32 atomics (exact and order independent); real-valued
//              folds are written as per-tile partials.
//   k_reduce   real-valued folds only: sums each bucket's partials in a fixed
//              order and applies the cyclic wrap of Algorithm 1's indices
//              (indices mod N, Section 2), giving the literal folds y[0..M+K-1).
//   k_finish   one workgroup per instance: literal folds (wrapping the integer
//              buckets itself), z = y1 + i*y2, FFT, product with the plan's
//              spectrum conj(FFT(t))/P, inverse FFT (steps 4-6 read as a
//              cross-correlation), argmax over [0, M) (step 7), candidate
//              intersection (steps 8-9, Theorem 4) and (Tx) scoring.
//   k_fold_s8 / k_fold_band   streaming fold of int8 signals through an LDS
//              ring, band fold of 4-byte signals (both moduli in one pass).
//   k_gfft_*   the FFT correlation through global memory for P above LDS.
//   k_cgemm_prep / k_cgemm / k_cgemm_wave / k_cgemm_ring / k_cgemm_final
//              exact plans with an int8-valued template: the correlation of
//              steps 4-6 computed directly as an int8 MFMA product of the
//              literal folds' base-128 digits with the banded Toeplitz block
//              of t (row tiles per workgroup, per wave, or per wave with both
//              operands staged in LDS rings), argmax, resolve.
//   k_many_*   one template, many signals: one GEMM against the template.
//   k_combine3 three moduli: intersection of the three candidate sets.
//   k_twiddles FP64 twiddles exp(-2 pi i e / P) (stored FP64 or FP32).
//   k_spectrum plan-time FP64 spectrum of the zero-padded template.

#include <algorithm>
#include <cstdlib>

#include <hip/hip_ext.h>
#include <hip/hip_fp16.h>

#include "tm_internal.h"

namespace tmi {

thread_local LaunchEvents g_launch_events;

// every launch goes through here: a plain launch unless a timed region is open
#define TM_LAUNCH(K, GRID, BLOCK, LDS, S, ...)                                                  \
  do {                                                                                          \
    LaunchEvents& ev_ = g_launch_events;                                                        \
    if (ev_.stop) {                                                                             \
      hipExtLaunchKernelGGL(K, GRID, BLOCK, (uint32_t)(LDS), S, ev_.start, ev_.stop, 0u, __VA_ARGS__); \
      ev_.start = nullptr;                                                                      \
    } else {                                                                                    \
      hipLaunchKernelGGL(K, GRID, BLOCK, LDS, S, __VA_ARGS__);                                \
    }                                                                                           \
  } while (0)

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
  static constexpr bool kInt = true;
  __device__ __forceinline__ static int from(int8_t v) { return (int)v; }
  // integer-valued storage: truncation is exact (one instruction)
  template <typename Tin> __device__ __forceinline__ static int from(Tin v) {
    return __float2int_rz(to_float(v));
  }
};
template <> struct AccOf<float> {
  static constexpr bool kInt = false;
  template <typename Tin> __device__ __forceinline__ static float from(Tin v) { return to_float(v); }
};

// Global memory through explicit address-space-1 pointers: plain global
// instructions instead of FLAT ones (which would also tie LDS waits to
// outstanding memory traffic).
#define GAS __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ GAS T* G(T* p) { return (GAS T*)p; }
template <typename T> __device__ __forceinline__ GAS const T* G(const T* p) { return (GAS const T*)p; }

__device__ __forceinline__ double load_as_double(const void* p, int dt, int64_t idx) {
  switch (dt) {
    case TM_I8: return (double)G((const int8_t*)p)[idx];
    case TM_F32: return (double)G((const float*)p)[idx];
    case TM_BF16: return (double)to_float(bf16_t{G((const uint16_t*)p)[idx]});
    default: return (double)to_float(f16_t{G((const uint16_t*)p)[idx]});
  }
}

__device__ __forceinline__ int load_as_int(const void* p, int dt, int64_t idx) {
  switch (dt) {
    case TM_I8: return (int)G((const int8_t*)p)[idx];
    case TM_F32: return __float2int_rn(G((const float*)p)[idx]);
    case TM_BF16: return __float2int_rn(to_float(bf16_t{G((const uint16_t*)p)[idx]}));
    default: return __float2int_rn(to_float(f16_t{G((const uint16_t*)p)[idx]}));
  }
}

__device__ __forceinline__ float load_as_float(const void* p, int dt, int64_t idx) {
  switch (dt) {
    case TM_I8: return (float)G((const int8_t*)p)[idx];
    case TM_F32: return G((const float*)p)[idx];
    case TM_BF16: return to_float(bf16_t{G((const uint16_t*)p)[idx]});
    default: return to_float(f16_t{G((const uint16_t*)p)[idx]});
  }
}

__device__ __forceinline__ bool acc_is_int(const Inst& d) { return d.acc_int != 0; }

// typed loads of one element as int / double (storage type known at compile time)
template <typename Tin> __device__ __forceinline__ int ld_int(const void* p, int64_t i);
template <> __device__ __forceinline__ int ld_int<int8_t>(const void* p, int64_t i) { return G((const int8_t*)p)[i]; }
template <> __device__ __forceinline__ int ld_int<float>(const void* p, int64_t i) { return __float2int_rn(G((const float*)p)[i]); }
template <> __device__ __forceinline__ int ld_int<bf16_t>(const void* p, int64_t i) {
  return __float2int_rn(to_float(bf16_t{G((const uint16_t*)p)[i]}));
}
template <> __device__ __forceinline__ int ld_int<f16_t>(const void* p, int64_t i) {
  return __float2int_rn(to_float(f16_t{G((const uint16_t*)p)[i]}));
}
template <typename Tin> __device__ __forceinline__ double ld_dbl(const void* p, int64_t i);
template <> __device__ __forceinline__ double ld_dbl<int8_t>(const void* p, int64_t i) { return G((const int8_t*)p)[i]; }
template <> __device__ __forceinline__ double ld_dbl<float>(const void* p, int64_t i) { return G((const float*)p)[i]; }
template <> __device__ __forceinline__ double ld_dbl<bf16_t>(const void* p, int64_t i) {
  return to_float(bf16_t{G((const uint16_t*)p)[i]});
}
template <> __device__ __forceinline__ double ld_dbl<f16_t>(const void* p, int64_t i) {
  return to_float(f16_t{G((const uint16_t*)p)[i]});
}

// v mod n for 0 <= v: a few subtractions cover the common v < 4n, a division the rest
__device__ __forceinline__ int64_t mod_pos(int64_t v, int64_t n) {
  if (v >= 4 * n) return v % n;
  while (v >= n) v -= n;
  return v;
}

// --------------------------------------------------------------------------
// fold tiles
// --------------------------------------------------------------------------

// global-memory (address space 1) views: plain loads, never FLAT
typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 gload16(uintptr_t a) {
  const u32x4v v = *(__attribute__((address_space(1))) const u32x4v*)a;
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ unsigned char gload8(uintptr_t a) {
  return *(__attribute__((address_space(1))) const unsigned char*)a;
}

// Tile staging layout: row r of the tile sits in LDS shifted right by R-1-r
// elements inside a zero-filled row of S = W + R - 1 elements.  Column j of the
// tile is then the stride-(S-1) sequence starting at j + R - 1, and diagonal e
// (elements (r, j) with j - r = e - (R - 1)) the stride-S sequence starting at e.
__host__ __device__ __forceinline__ size_t fold_tile_bytes(int rows, int cols, int eb) {
  return (((size_t)rows * (cols + rows - 1) * eb) + 15) & ~(size_t)15;
}

size_t fold_lds_bytes(const View& v, int x_dtype) {
  return fold_tile_bytes(v.rows, v.cols, dtype_bytes(x_dtype));
}

template <typename Acc, typename Tin>
__device__ __forceinline__ Acc strided_sum(const Tin* p, int stride, int n) {
  Acc acc = 0;
  int r = 0;
  for (; r + 8 <= n; r += 8) {
    Tin v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = p[(r + i) * stride];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc += AccOf<Acc>::from(v[i]);
  }
  for (; r < n; ++r) acc += AccOf<Acc>::from(p[r * stride]);
  return acc;
}

template <typename Tin>
__device__ __forceinline__ Tin chunk_elem(const uint4& c, int e) {
  const uint32_t w = e * (int)sizeof(Tin) / 4 == 0 ? c.x : e * (int)sizeof(Tin) / 4 == 1 ? c.y
                   : e * (int)sizeof(Tin) / 4 == 2 ? c.z : c.w;
  const int sh = (e * (int)sizeof(Tin)) % 4 * 8;
  if constexpr (sizeof(Tin) == 4) { Tin v; __builtin_memcpy(&v, &w, 4); return v; }
  else if constexpr (sizeof(Tin) == 2) { const uint16_t h = (uint16_t)(w >> sh); Tin v; __builtin_memcpy(&v, &h, 2); return v; }
  else { const uint8_t b = (uint8_t)(w >> sh); Tin v; __builtin_memcpy(&v, &b, 1); return v; }
}

template <typename Tin, typename Acc>
__device__ __forceinline__ void fold_tile(const Inst& d, int lt, unsigned char* lds) {
  const int tid = threadIdx.x;
  constexpr int NT = kFoldThreads;
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
  const int S = W + R - 1;
  constexpr int EB = sizeof(Tin);
  constexpr int EPC = 16 / EB;                        // elements per 16-byte chunk
  const int CQ = fold_chunks(W, EB);
  const uintptr_t xa = reinterpret_cast<uintptr_t>(d.x);
  const uintptr_t xend = xa + (uintptr_t)N * EB;
  Tin* t = reinterpret_cast<Tin*>(lds);

  // valid columns: Wc in every row but the last row of x
  const int Wc = min(M - c0, W);
  const int64_t n_last = (int64_t)(rb * R + Reff - 1) * M + c0;
  const int nv_last = (int)max((int64_t)0, min((int64_t)Wc, N - n_last));
  const int Rfull = nv_last == Wc ? Reff : Reff - 1;

  // 1) issue every 16-byte load of the tile (global address space, no branch
  //    around the load: lanes without a chunk read a safe in-bounds chunk)
  const unsigned total = (unsigned)(Reff * CQ);
  const unsigned magic = 0xFFFFFFFFu / (unsigned)CQ + 1u;   // exact r = idx / CQ for idx < 2^16
  const uintptr_t safeA = (xa + 15) & ~(uintptr_t)15;
  const bool has_safe = safeA + 16 <= xend;
  uint4 vb[kFoldLoads];
  unsigned need = 0, slow = 0;
#pragma unroll
  for (int u = 0; u < kFoldLoads; ++u) {
    const unsigned idx = tid + u * NT;
    const unsigned r = __umulhi(idx, magic);
    const unsigned q = idx - r * (unsigned)CQ;
    const uintptr_t a0 = xa + (uintptr_t)(((int64_t)(rb * R + (int)r) * M + c0) * EB);
    const int off = (int)(a0 & 15);
    const int nv = (int)r < Rfull ? Wc : nv_last;
    const uintptr_t A = (a0 & ~(uintptr_t)15) + (uintptr_t)q * 16;
    const bool has = idx < total && (int)(q * 16) < off + nv * EB;
    const bool fast = has && A >= xa && A + 16 <= xend;
    if (has_safe) vb[u] = gload16(fast ? A : safeA);
    need |= (unsigned)has << u;
    slow |= (unsigned)(has && !fast) << u;
  }

  // 2) zero the skewed tile, then 3) scatter the valid elements into it
  {
    uint4* z = reinterpret_cast<uint4*>(lds);
    const int nz = (int)(fold_tile_bytes(R, W, EB) >> 4);
    for (int i = tid; i < nz; i += NT) z[i] = make_uint4(0, 0, 0, 0);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kFoldLoads; ++u) {
    if (!((need >> u) & 1)) continue;
    const unsigned idx = tid + u * NT;
    const int r = (int)__umulhi(idx, magic);
    const int q = (int)(idx - (unsigned)r * (unsigned)CQ);
    const uintptr_t a0 = xa + (uintptr_t)(((int64_t)(rb * R + r) * M + c0) * EB);
    const int off = (int)(a0 & 15);
    const int nv = r < Rfull ? Wc : nv_last;
    uint4 c = vb[u];
    if ((slow >> u) & 1) {
      const uintptr_t A = (a0 & ~(uintptr_t)15) + (uintptr_t)q * 16;
      unsigned char bytes[16];
      for (int b = 0; b < 16; ++b) {
        const uintptr_t ad = A + b;
        bytes[b] = (ad >= xa && ad < xend) ? gload8(ad) : 0;
      }
      __builtin_memcpy(&c, bytes, 16);
    }
    const int j0 = (q * 16 - off) / EB;                // column of the chunk's first element
    Tin* row = t + (size_t)r * S + (R - 1 - r);
#pragma unroll
    for (int e = 0; e < EPC; ++e) {
      const int j = j0 + e;
      if (j >= 0 && j < nv) row[j] = chunk_elem<Tin>(c, e);
    }
  }
  __syncthreads();

  // 4) column sums (fold over M) and diagonal sums (fold over M + 1), rows in
  //    increasing order, no bounds checks (invalid positions hold zeros)
  for (int j = tid; j < Wc; j += NT) {
    const Acc acc = strided_sum<Acc>(t + j + R - 1, S - 1, Reff);
    if constexpr (AccOf<Acc>::kInt) {   // integer: exact, order-independent atomics
      int* yp = d.yp + (in_a ? 0 : d.va.m);
      if (acc) __hip_atomic_fetch_add(G(yp + c0 + j), (int)acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      Acc* colp = reinterpret_cast<Acc*>(in_a ? d.col_a : d.col_b);
      G(colp)[(int64_t)rb * M + c0 + j] = acc;
    }
  }
  if (want_diag) {
    const int64_t mb = d.vb.m;
    for (int e = tid; e < S; e += NT) {
      const Acc acc = strided_sum<Acc>(t + e, S, Reff);
      if constexpr (AccOf<Acc>::kInt) {
        int64_t b = ((int64_t)c0 + e - (R - 1) - (int64_t)rb * R) % mb;
        if (b < 0) b += mb;
        if (acc) __hip_atomic_fetch_add(G(d.yp + d.va.m + b), (int)acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        G(reinterpret_cast<Acc*>(d.diag))[(int64_t)(rb * v.ncb + cb) * S + e] = acc;
      }
    }
  }
}

// The last instance whose first work unit (base_of) is <= w, over a table
// sorted by it.  Every wave searches on its own, 64 probes per round: lane l
// reads the base at lo + floor(l * span / 64), the ballot of "base <= w" is a
// prefix of the lanes, and its last lane narrows [lo, hi] 64-fold, so 4096
// instances take two rounds of one load each (a bisection takes twelve
// dependent loads).  base_of(lo) <= w holds throughout (base_of(0) = 0).
// The whole wave must be active.
template <typename W, typename BaseOf>
__device__ __forceinline__ int find_inst(int count, W w, BaseOf base_of) {
  int lo = 0, hi = count - 1;
  const int lane = (int)(threadIdx.x & 63);
  while (lo < hi) {
    const int span = hi - lo + 1;
    const int pos = lo + (int)(((int64_t)lane * span) >> 6);
    const uint64_t le = __ballot(base_of(pos) <= w);
    const int last = 63 - __clzll((long long)le);     // lane 0 probes lo: le != 0
    const int nlo = lo + (int)(((int64_t)last * span) >> 6);
    const int nhi = last == 63 ? hi : lo + (int)(((int64_t)(last + 1) * span) >> 6) - 1;
    lo = __builtin_amdgcn_readfirstlane(nlo);
    hi = __builtin_amdgcn_readfirstlane(nhi);
  }
  return lo;
}

__device__ __forceinline__ int find_inst_by_tile(const InstTable& tab, int tile) {
  return find_inst(tab.count, tile, [&](int i) { return tab.table[i].tile_base; });
}

__device__ __forceinline__ int find_inst_by_red(const InstTable& tab, int wg) {
  return find_inst(tab.count, wg, [&](int i) { return tab.table[i].red_base; });
}

__device__ __forceinline__ void fold_dispatch(const Inst& d, int lt, unsigned char* lds) {
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

// The table and the single instance take separate paths, each inlined on its
// own.  On the single path, thread 0 of the first workgroup stores the launch's
// signal and result slot into the instance's device copy for the later kernels.
__global__ void __launch_bounds__(kFoldThreads) k_fold(InstTable tab, int total_tiles) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int tile = blockIdx.x;
  if (tile >= total_tiles) return;
  if (tab.table) {
    const Inst& d = tab.table[find_inst_by_tile(tab, tile)];
    fold_dispatch(d, tile - d.tile_base, lds);
  } else {
    if (tile == 0 && threadIdx.x == 0) tab.publish();
    fold_dispatch(tab.single(), tile, lds);
  }
}

// --------------------------------------------------------------------------
// streaming int8 fold (int8 signals, both moduli in [kSegMinM, kSegMaxM])
// --------------------------------------------------------------------------
//
// One workgroup folds one segment of x: a run of 16-byte chunks, addressed
// from x rounded down to 16 bytes (d = x mod 16 bytes sit before x[0]).  A
// row belongs to the segment holding its first byte.
//
// Chunks pass through a two-piece LDS ring whose first kSegLook bytes are
// mirrored after it, so a row that starts in one piece is read whole.  Two
// register sets each hold a piece in flight: while piece j is folded, pieces
// j + 2 and j + 3 are loading.  Threads 0..127 fold with modulus ma, threads
// 128..255 with mb.  Lane u owns buckets 4u..4u+3 (plus 512 s for slot s):
// for each row it reads the two aligned words that hold the row's bytes
// 4u..4u+3 and one v_perm per parity both realigns them and spreads the even
// (odd) bytes into 16-bit lanes.  Bytes enter LDS as x + 128 (bit 7 flipped;
// zero outside x) so the lane sums are unsigned; the bias is removed when the
// literal folds are formed.  A segment holds at most 256 rows of either
// modulus, so a 16-bit lane stays below 256 * 255 < 2^16.

// bytes [lo, hi) of a 16-byte chunk kept, the rest cleared
__device__ __forceinline__ uint4 keep_bytes(uint4 v, int lo, int hi) {
  uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    uint32_t m = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) m |= (4 * q + b >= lo && 4 * q + b < hi) ? (0xFFu << (8 * b)) : 0u;
    w[q] &= m;
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// where a segment's loads read: chunks from xseg on, load_bytes of them in x
struct SegSrc {
  uintptr_t xseg;    // address of the segment's first chunk
  int load_bytes;    // bytes read from xseg on (staged chunks that hold x)
};

struct SegGeom {
  uintptr_t xc;      // x rounded down to 16 bytes
  int delta;         // x - xc
  int64_t nch;       // chunks that hold bytes of x
  int64_t c_begin;   // first chunk of the segment
  int64_t c_end;     // one past its last chunk
  int64_t c_stage;   // one past the last chunk staged (segment plus look-ahead)
  // the same bounds relative to c_begin, in 32 bits
  int stage_rel;     // chunks staged
  int x_rel;         // chunks of x from c_begin on (clamped)
  int first_rel;     // chunk 0 of x relative to c_begin (edge: bytes before x), or -1
  int last_rel;      // last chunk of x relative to c_begin (edge: bytes after x), or -1
  SegSrc src;
};

// segment seg of signal d (the last one takes the tail)
__device__ __forceinline__ void seg_geom(SegGeom& g, const Inst& d, int seg) {
  const uintptr_t xa = reinterpret_cast<uintptr_t>(d.x);
  const int64_t cb = (int64_t)seg * d.seg_chunks;
  g.xc = xa & ~(uintptr_t)15;
  g.delta = (int)(xa & 15);
  g.nch = (d.n + g.delta + 15) >> 4;
  g.c_begin = cb;
  g.c_end = seg == d.nseg - 1 ? g.nch : min(g.nch, cb + d.seg_chunks);
  const int64_t mmax = max(d.va.m, d.vb.m);
  g.c_stage = g.c_end + (mmax + 16 + 15) / 16;
  g.stage_rel = (int)(g.c_stage - cb);
  g.x_rel = (int)min(g.nch - cb, (int64_t)1 << 30);
  g.first_rel = cb == 0 ? 0 : -1;
  g.last_rel = g.nch - 1 - cb < g.stage_rel ? (int)(g.nch - 1 - cb) : -1;
  g.src.xseg = g.xc + (uintptr_t)cb * 16;
  g.src.load_bytes = 16 * max(0, min(g.stage_rel, g.x_rel));
}

// A piece's chunks through a buffer resource that starts at the piece and
// ends at the last chunk staged from x: chunks past it read as zero without a
// memory access, so every load is issued unconditionally.  The per-thread
// offsets stay fixed and the piece moves only the (scalar) base, so issuing
// the next loads writes no vector register that an earlier load still fills.
// x is read once, so the loads carry the non-temporal hint (aux bit 1): the
// streamed bytes do not displace what the caches hold for other work.
__device__ __forceinline__ void seg_load(uintptr_t xseg, int load_bytes, int piece, uint4 (&v)[kSegLoads]) {
  // the values are wave-uniform; readfirstlane keeps the resource in scalar
  // registers (no per-lane loop around each load)
  const int rel = piece * kSegPiece;
  const int lim = __builtin_amdgcn_readfirstlane(max(0, load_bytes - rel));
  const uintptr_t base = xseg + (uintptr_t)(unsigned)rel;
  const uintptr_t ub = (uintptr_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)base) |
                       ((uintptr_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(base >> 32)) << 32);
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(ub), 0, lim, kBufRsrcWord3);
#pragma unroll
  for (int u = 0; u < kSegLoads; ++u) {
    const auto w = __builtin_amdgcn_raw_buffer_load_b128(rs, ((int)threadIdx.x + u * kSegThreads) * 16, 0, 2);
    v[u] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

__device__ __forceinline__ void seg_store(const SegGeom& g, int64_t n, int piece, const uint4 (&v)[kSegLoads],
                                          unsigned char* lds) {
  const int half = piece & 1;
#pragma unroll
  for (int u = 0; u < kSegLoads; ++u) {
    const int cl = (int)threadIdx.x + u * kSegThreads;
    const int cr = piece * kSegPieceChunks + cl;
    if (cr >= g.stage_rel) continue;
    uint4 w = make_uint4(0, 0, 0, 0);
    if (cr < g.x_rel) {
      w = make_uint4(v[u].x ^ 0x80808080u, v[u].y ^ 0x80808080u, v[u].z ^ 0x80808080u, v[u].w ^ 0x80808080u);
      if (cr == g.first_rel || cr == g.last_rel) {
        const int64_t b0 = (g.c_begin + cr) * 16;
        w = keep_bytes(w, (int)max((int64_t)0, g.delta - b0), (int)min((int64_t)16, g.delta + n - b0));
      }
    }
    *reinterpret_cast<uint4*>(lds + half * kSegPiece + cl * 16) = w;
    if (half == 0 && cl * 16 < kSegLook) *reinterpret_cast<uint4*>(lds + 2 * kSegPiece + cl * 16) = w;
  }
}

// the two aligned words under bytes 4u..4u+3 of a row, for every slot
template <int NSL>
__device__ __forceinline__ void seg_read_row(const unsigned char* lds, int abase, int u0,
                                             uint32_t (&w0)[NSL], uint32_t (&w1)[NSL]) {
  const uint32_t* p = reinterpret_cast<const uint32_t*>(lds + abase) + u0;
#pragma unroll
  for (int s = 0; s < NSL; ++s) {
    w0[s] = p[kSegHalf * s];
    w1[s] = p[kSegHalf * s + 1];
  }
}

template <int NSL>
__device__ __forceinline__ void fold_segment(const Inst& d, int seg, int half, unsigned char* lds) {
  const int tid = threadIdx.x;
  SegGeom g;
  seg_geom(g, d, seg);
  const int u0 = tid & (kSegHalf - 1);
  const int64_t N = d.n;
  const int nproc = (int)((g.c_end - g.c_begin + kSegPieceChunks - 1) / kSegPieceChunks);   // >= 1

  // this half's modulus (wave-uniform); row k spans bytes [kM + d, (k+1)M + d) from xc
  const int64_t M = half ? d.vb.m : d.va.m;
  const int64_t L = (N + M - 1) / M;
  const int64_t B0 = g.c_begin * 16, B1 = g.c_end * 16;
  const int64_t k0 = B0 > g.delta ? (B0 - g.delta + M - 1) / M : 0;
  int64_t rb = k0 * M + g.delta;                // first byte of the segment's next row
  const int64_t last_start = (L - 1) * M + g.delta;   // first byte of row L - 1
  // the top slot also sums bytes past the row's end into lanes of buckets >= M:
  // those lanes stay below 2^16 like the others and are never flushed

  uint32_t lo[NSL], hi[NSL];
#pragma unroll
  for (int s = 0; s < NSL; ++s) { lo[s] = 0; hi[s] = 0; }

  // pieces past the staged end read nothing: every step issues the same
  // loads, so the loads in flight keep one order in every pass of the loop
  auto load_pos = [&](int p, uint4 (&v)[kSegLoads]) { seg_load(g.src.xseg, g.src.load_bytes, p, v); };

  uint4 va[kSegLoads], vb[kSegLoads];
  load_pos(0, va);
  load_pos(1, vb);
  seg_store(g, N, 0, va, lds);
  seg_store(g, N, 1, vb, lds);
  load_pos(2, va);
  load_pos(3, vb);
  __syncthreads();

  // the rows that start in piece j (ring slot j & 1)
  auto piece_rows = [&](int j) {
    const int64_t Bp = B0 + (int64_t)j * kSegPiece;
    const int64_t Bend = min(Bp + kSegPiece, B1);
    const int ring = (j & 1) * kSegPiece;              // LDS offset of byte b: ring + (b - Bp)
    // rows starting in this piece (first byte in [Bp, Bend), row < L), counted
    // once: row rb + r M for r M < span (no division).  Row i starts at LDS
    // offset rel + i M; its misalignment (rel + i M) mod 4 has period 4 in i,
    // so four byte selectors and four word-aligned bases, computed once per
    // piece, serve every group of four rows (no per-row scalar work beyond
    // the group's offset)
    const int64_t lim = min(Bend, last_start + 1);
    const int span = lim > rb ? (int)(lim - rb) : 0;
    const int M32 = (int)M;
    const int rel = ring + (int)(rb - Bp);
    uint32_t se[4], so[4];
    int base[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int off = rel + q * M32;
      const uint32_t a = (uint32_t)off & 3u;
      se[q] = 0x0C020C00u + a * 0x00010001u;      // bytes c, c + 2 of the row's four
      so[q] = se[q] + 0x00010001u;                // bytes c + 1, c + 3
      base[q] = off - (int)a;
    }
    auto row = [&](int q, int r) {                // row r + q, r a multiple of 4
      uint32_t w0[NSL], w1[NSL];
      seg_read_row<NSL>(lds, base[q] + r * M32, u0, w0, w1);
#pragma unroll
      for (int s = 0; s < NSL; ++s) {
        lo[s] += __builtin_amdgcn_perm(w1[s], w0[s], se[q]);
        hi[s] += __builtin_amdgcn_perm(w1[s], w0[s], so[q]);
      }
    };
    int full = 0;
    for (; (full + 3) * M32 < span; full += 4) {
#pragma unroll
      for (int q = 0; q < 4; ++q) row(q, full);
    }
    int nr = full;
    if (nr * M32 < span) { row(0, full); ++nr; }
    if (nr * M32 < span) { row(1, full); ++nr; }
    if (nr * M32 < span) { row(2, full); ++nr; }
    rb += (int64_t)nr * M;
  };
  // Pieces go in pairs with no exit between the halves, so set A's loads are
  // always older than set B's where the loop repeats, and waiting for set A
  // leaves set B in flight.  A piece past the last holds no row start, so an
  // odd count folds nothing in the last half; seg_store keeps only chunks
  // below the staged end.
  for (int j = 0; j < nproc; j += 2) {
    piece_rows(j);
    __syncthreads();
    seg_store(g, N, j + 2, va, lds);
    load_pos(j + 4, va);
    __syncthreads();
    piece_rows(j + 1);
    __syncthreads();
    seg_store(g, N, j + 3, vb, lds);
    load_pos(j + 5, vb);
    __syncthreads();
  }

  // flush: word u's lanes are buckets 4u..4u+3; transpose through LDS so the
  // global atomics are coalesced
  int* Z = reinterpret_cast<int*>(lds) + half * kSegZ;
#pragma unroll
  for (int s = 0; s < NSL; ++s) {
    const int u = u0 + kSegHalf * s;
    *reinterpret_cast<uint4*>(Z + 4 * u) =
        make_uint4(lo[s] & 0xFFFFu, hi[s] & 0xFFFFu, lo[s] >> 16, hi[s] >> 16);
  }
  __syncthreads();
  int* yp = d.yp + (half ? d.va.m : 0);
  for (int b = u0; b < M; b += kSegHalf) {
    const int val = Z[b];
    if (val) __hip_atomic_fetch_add(G(yp + b), val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__device__ __forceinline__ int find_inst_by_seg(const InstTable& tab, int seg) {
  return find_inst(tab.count, seg, [&](int i) { return tab.table[i].seg_base; });
}

// one instantiation per word count of a row (ceil(M / 512) slots per lane)
__device__ __forceinline__ void fold_segment_any(const Inst& d, int seg, unsigned char* lds) {
  const int half = __builtin_amdgcn_readfirstlane(threadIdx.x >> 7);
  const int m = half ? d.vb.m : d.va.m;
  switch ((m + 4 * kSegHalf - 1) / (4 * kSegHalf)) {
    case 1: fold_segment<1>(d, seg, half, lds); break;
    case 2: fold_segment<2>(d, seg, half, lds); break;
    case 3: fold_segment<3>(d, seg, half, lds); break;
    case 4: fold_segment<4>(d, seg, half, lds); break;
    case 5: fold_segment<5>(d, seg, half, lds); break;
    case 6: fold_segment<6>(d, seg, half, lds); break;
    case 7: fold_segment<7>(d, seg, half, lds); break;
    case 8: fold_segment<8>(d, seg, half, lds); break;
    default: fold_segment<9>(d, seg, half, lds); break;
  }
}

// The two halves of a workgroup may run different instantiations; each runs
// the same sequence of barriers.
__global__ void __launch_bounds__(kSegThreads) k_fold_s8(InstTable tab, int total_segs) {
  __shared__ __align__(16) unsigned char lds[kSegLds];
  const int seg = blockIdx.x;
  if (seg >= total_segs) return;
  if (tab.table) {
    const Inst& d = tab.table[find_inst_by_seg(tab, seg)];
    fold_segment_any(d, seg - d.seg_base, lds);
  } else {
    if (seg == 0 && threadIdx.x == 0) tab.publish();
    fold_segment_any(tab.single(), seg, lds);
  }
}

// --------------------------------------------------------------------------
// band fold (4-byte signals)
// --------------------------------------------------------------------------
//
// One wave folds a band of 64 columns over R rows of view A (of view B too when
// the moduli are not consecutive).  Lane j reads column c0 + j of every row (a
// coalesced 256-byte row), adds it to its column sum in a register and to
// diagonal e = j - r + R - 1 (row r of the band) of a per-wave LDS array with an
// LDS atomic.  Within a row the lanes hit distinct diagonals and a diagonal
// receives its rows in order, so float sums are deterministic.  Diagonal e
// holds the elements of bucket (c0 + e - (R-1) - r0) mod M2 (element (i, c) of
// view A is x[i M1 + c], which is c - i mod M2 when M2 = M1 + 1): the layout of
// the tiled fold's partials, which the real path reduces in a fixed order.

template <typename Acc>
__device__ __forceinline__ void band_task(const Inst& d, int task, Acc* dg) {
  const int lane = threadIdx.x & 63;
  const int nta = d.va.nrb * d.va.ncb;
  const bool in_a = task < nta;
  const View v = in_a ? d.va : d.vb;
  if (!in_a) task -= nta;
  const bool want_diag = in_a && d.dual;
  const int rb = task / v.ncb, cb = task - rb * v.ncb;
  const int R = v.rows;
  const int64_t M = v.m, N = d.n;
  const int64_t r0 = (int64_t)rb * R;
  const int Reff = (int)min((int64_t)R, (int64_t)v.l - r0);
  const int c0 = cb * kBandCols;
  const int c = c0 + lane;
  const bool colok = c < M;
  const int S = R + kBandCols - 1;
  if (want_diag)
    for (int e = lane; e < S; e += 64) dg[e] = (Acc)0;
  Acc ca = (Acc)0;
  const GAS float* x = G(reinterpret_cast<const float*>(d.x));
  const int64_t nbase = r0 * M + c;
  for (int r = 0; r < Reff; r += kBandUnroll) {
    float xv[kBandUnroll];
#pragma unroll
    for (int u = 0; u < kBandUnroll; ++u) {
      const int64_t n = nbase + (int64_t)(r + u) * M;
      const bool ok = r + u < Reff && colok && n < N;
      xv[u] = x[ok ? n : 0];
      if (!ok) xv[u] = 0.f;
    }
#pragma unroll
    for (int u = 0; u < kBandUnroll; ++u) {
      if (r + u < Reff) {
        const Acc a = AccOf<Acc>::from(xv[u]);
        ca += a;
        if (want_diag)
          __hip_atomic_fetch_add(dg + (lane - (r + u) + R - 1), a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
      }
    }
  }
  if constexpr (AccOf<Acc>::kInt) {   // integer: exact, order-independent atomics
    int* yp = d.yp + (in_a ? 0 : d.va.m);
    if (colok && ca) __hip_atomic_fetch_add(G(yp + c), (int)ca, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (want_diag) {
      const int64_t mb = d.vb.m;
      for (int e = lane; e < S; e += 64) {
        const int val = (int)dg[e];
        if (!val) continue;
        int64_t b = ((int64_t)c0 + e - (R - 1) - r0) % mb;
        if (b < 0) b += mb;
        __hip_atomic_fetch_add(G(d.yp + d.va.m + b), val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  } else {
    Acc* colp = reinterpret_cast<Acc*>(in_a ? d.col_a : d.col_b);
    if (colok) G(colp)[(int64_t)rb * M + c] = ca;
    if (want_diag) {
      Acc* dp = reinterpret_cast<Acc*>(d.diag) + (int64_t)(rb * v.ncb + cb) * S;
      for (int e = lane; e < S; e += 64) G(dp)[e] = dg[e];
    }
  }
}

__device__ __forceinline__ int find_inst_by_band(const InstTable& tab, int wg) {
  return find_inst(tab.count, wg, [&](int i) { return tab.table[i].band_base; });
}

__device__ __forceinline__ void band_dispatch(const Inst& d, int wg, unsigned char* lds) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: scalar task indices
  const int task = wg * kBandWaves + wave;
  const int ntasks = d.va.nrb * d.va.ncb + (d.dual ? 0 : d.vb.nrb * d.vb.ncb);
  if (task >= ntasks) return;
  const size_t per = (size_t)(kBandRowsMax + kBandCols) * 4;
  if (d.acc_int) band_task<int>(d, task, reinterpret_cast<int*>(lds + wave * per));
  else band_task<float>(d, task, reinterpret_cast<float*>(lds + wave * per));
}

__global__ void __launch_bounds__(64 * kBandWaves) k_fold_band(InstTable tab, int total_wgs) {
  __shared__ __align__(16) unsigned char lds[kBandWaves * (kBandRowsMax + kBandCols) * 4];
  const int wg = blockIdx.x;
  if (wg >= total_wgs) return;
  if (tab.table) {
    const Inst& d = tab.table[find_inst_by_band(tab, wg)];
    band_dispatch(d, wg - d.band_base, lds);
  } else {
    if (wg == 0 && threadIdx.x == 0) tab.publish();
    band_dispatch(tab.single(), wg, lds);
  }
}

// --------------------------------------------------------------------------
// real-valued folds: fixed-order reduction of the partials
// --------------------------------------------------------------------------

// contribution of row block rb to bucket s of fold f (partition fold)
__device__ __forceinline__ float bucket_part(const Inst& d, int f, int s, int rb) {
  if (f == 0) return G(reinterpret_cast<const float*>(d.col_a))[(int64_t)rb * d.va.m + s];
  if (!d.dual) return G(reinterpret_cast<const float*>(d.col_b))[(int64_t)rb * d.vb.m + s];
  // diagonal e of tile (rb, cb) covers bucket (e + cb*W - rb*R - (R-1)) mod mb
  const float* p = reinterpret_cast<const float*>(d.diag);
  const int R = d.va.rows, W = d.va.cols, E = W + R - 1, ncb = d.va.ncb;
  const int64_t mb = d.vb.m;
  const int64_t qmax = (int64_t)ncb * W + R - 1;
  float acc = 0.f;
  const int64_t v0 = ((int64_t)s + (int64_t)rb * R + R - 1) % mb;
  for (int64_t q = v0; q < qmax; q += mb) {
    const int cb_hi = (int)min(q / W, (int64_t)ncb - 1);
    const int64_t lo_num = q - (E - 1);
    const int cb_lo = lo_num <= 0 ? 0 : (int)((lo_num + W - 1) / W);
    for (int cb = cb_lo; cb <= cb_hi; ++cb) acc += G(p)[(int64_t)(rb * ncb + cb) * E + (q - (int64_t)cb * W)];
  }
  return acc;
}

// Threads of a workgroup are split into groups of red_tpe lanes, one group per
// fold entry; lane t sums row blocks t, t + tpe, ... and lane 0 adds the lanes
// in order, then the cyclic wrap terms.  (SINGLE only keeps the table and the
// single-instance call sites apart, so that they are not merged into one call
// through a pointer that could point at either.)
template <bool SINGLE>
__device__ __forceinline__ void reduce_wg(const Inst& d, int lc, float* part) {
  const int tpe = d.red_tpe;
  const int epw = kReduceThreads / tpe;
  const int tid = threadIdx.x;
  const int e = tid / tpe, t = tid - e * tpe;
  const int totA = d.va.m + d.k - 1;
  const int tot = totA + d.vb.m + d.k - 1;
  const int u = lc * epw + e;
  const int f = u >= totA;
  const int uu = f ? u - totA : u;
  const int64_t M = f ? d.vb.m : d.va.m;
  const int s = uu < M ? uu : (int)(uu - M);
  const int nrb = f ? (d.dual ? d.va.nrb : d.vb.nrb) : d.va.nrb;
  float acc = 0.f;
  if (u < tot)
    for (int rb = t; rb < nrb; rb += tpe) acc += bucket_part(d, f, s, rb);
  part[tid] = acc;
  __syncthreads();
  if (t == 0 && u < tot) {
    float sum = 0.f;
    for (int i = 0; i < tpe; ++i) sum += part[e * tpe + i];
    const int64_t L = f ? d.vb.l : d.va.l;
    const int64_t N = d.n;
    // the zero-padded variant keeps the bucket sums: y[M + s] = y[s]
    if (!d.zpad && (int64_t)s + (L - 1) * M >= N)
      sum += load_as_float(d.x, d.x_dtype, mod_pos((int64_t)s + (L - 1) * M, N));
    if (!d.zpad && uu >= M)
      sum += load_as_float(d.x, d.x_dtype, mod_pos((int64_t)s + L * M, N)) - load_as_float(d.x, d.x_dtype, s);
    G(reinterpret_cast<float*>(d.y))[u] = sum;
  }
}

// Literal real-valued folds for every real instance of a launch (integer
// folds are formed by the finish kernel from their buckets): the threads of a
// workgroup are split into groups of red_tpe lanes, one group per fold entry
// (lane t sums row blocks t, t + tpe, ...; lane 0 adds the lanes in order,
// then the cyclic wrap terms).
__global__ void __launch_bounds__(kReduceThreads) k_reduce(InstTable tab, int total_wgs) {
  __shared__ float part[kReduceThreads];
  const int wg = blockIdx.x;
  if (wg >= total_wgs) return;
  if (tab.table) {
    const Inst& d = tab.table[find_inst_by_red(tab, wg)];
    reduce_wg<false>(d, wg - d.red_base, part);
  } else {
    reduce_wg<true>(tab.resident(), wg, part);
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

// cos(pi j / 16), j = 0..8
__device__ __forceinline__ constexpr double cos_pi16(int j) {
  return j == 0 ? 1.0
       : j == 1 ? 0.98078528040323044913
       : j == 2 ? 0.92387953251128675613
       : j == 3 ? 0.83146961230254523708
       : j == 4 ? 0.70710678118654752440
       : j == 5 ? 0.55557023301960222474
       : j == 6 ? 0.38268343236508977173
       : j == 7 ? 0.19509032201612826785
       : 0.0;
}
// omega_32^J = exp(-2 pi i J / 32) for J in [0, 16)
__device__ __forceinline__ constexpr double root_re(int J) { return J <= 8 ? cos_pi16(J) : -cos_pi16(16 - J); }
__device__ __forceinline__ constexpr double root_im(int J) { return -(J <= 8 ? cos_pi16(8 - J) : cos_pi16(J - 8)); }

// x * omega_32^J (J fixed at compile time after unrolling)
template <typename T>
__device__ __forceinline__ cplx<T> mul_root(cplx<T> x, int J) {
  const T c = (T)0.70710678118654752440;
  if (J == 0) return x;
  if (J == 8) return {x.y, -x.x};
  if (J == 4) return {(x.x + x.y) * c, (x.y - x.x) * c};
  if (J == 12) return {(x.y - x.x) * c, -(x.x + x.y) * c};
  const T wr = (T)root_re(J), wi = (T)root_im(J);
  return {x.x * wr - x.y * wi, x.x * wi + x.y * wr};
}
// x * conj(omega_32^J)
template <typename T>
__device__ __forceinline__ cplx<T> mul_root_conj(cplx<T> x, int J) {
  const T c = (T)0.70710678118654752440;
  if (J == 0) return x;
  if (J == 8) return {-x.y, x.x};
  if (J == 4) return {(x.x - x.y) * c, (x.x + x.y) * c};
  if (J == 12) return {-(x.x + x.y) * c, (x.x - x.y) * c};
  const T wr = (T)root_re(J), wi = (T)root_im(J);
  return {x.x * wr + x.y * wi, x.y * wr - x.x * wi};
}

// Radix-2 decimation-in-frequency stages over 2^KB points with constant
// twiddles: natural order in, DFT at bit-reversed positions out.
template <int KB, typename T>
__device__ __forceinline__ void dft_dif(cplx<T>* v) {
  constexpr int RR = 1 << KB;
#pragma unroll
  for (int st = 0; st < KB; ++st) {
    const int hm = RR >> (st + 1);
#pragma unroll
    for (int m = 0; m < RR; ++m) {
      if (m & hm) continue;
      const cplx<T> a = v[m], b = v[m + hm];
      v[m] = a + b;
      v[m + hm] = mul_root(a - b, (m & (hm - 1)) * (16 / hm));
    }
  }
}

// Exact inverse of dft_dif up to the factor 2^KB.
template <int KB, typename T>
__device__ __forceinline__ void dft_dit(cplx<T>* v) {
  constexpr int RR = 1 << KB;
#pragma unroll
  for (int st = KB - 1; st >= 0; --st) {
    const int hm = RR >> (st + 1);
#pragma unroll
    for (int m = 0; m < RR; ++m) {
      if (m & hm) continue;
      const cplx<T> a = v[m];
      const cplx<T> b = mul_root_conj(v[m + hm], (m & (hm - 1)) * (16 / hm));
      v[m] = a + b;
      v[m + hm] = a - b;
    }
  }
}

__device__ __forceinline__ constexpr int bitrev(int m, int kb) {
  int r = 0;
  for (int i = 0; i < kb; ++i) r |= ((m >> i) & 1) << (kb - 1 - i);
  return r;
}

// one pad element per 16 keeps strided butterfly accesses off a single bank
__device__ __forceinline__ int padi(int j) { return j + (j >> 4); }
__host__ __device__ __forceinline__ int padded_len(int P) { return P + (P >> 4) + 1; }

int fft_lds_max_log2(int mode) { return mode == MODE_EXACT ? 13 : 14; }

// Threads of a finish workgroup: one radix-16 group of every pass per thread.
int finish_threads(int p_log2) {
  const int t = (1 << p_log2) >> 4;
  return t < 64 ? 64 : (t > kFinishThreads ? kFinishThreads : t);
}

// The middle pass takes contiguous groups of 2^mid elements, mid = min(p,
// kFftMid); element m of group g of the spectrum is stored at m * (P >> mid) + g
// so that the pass's spectrum loads are coalesced across threads.
__host__ __device__ __forceinline__ int spec_slot(int i, int p) {
  const int mid = p < kFftMid ? p : kFftMid;
  const int g = i >> mid, m = i & ((1 << mid) - 1);
  return (m << (p - mid)) + g;
}

size_t finish_lds_bytes(int p_log2, int mode) {
  const size_t el = mode == MODE_EXACT ? 16 : 8;
  return (size_t)padded_len(1 << p_log2) * el + (size_t)kFinishThreads * 16;
}

template <typename T>
__device__ __forceinline__ cplx<T> ldc(const cplx<T>* p, int i) {
  const GAS T* q = G(reinterpret_cast<const T*>(p));
  return cplx<T>{q[2 * i], q[2 * i + 1]};
}

// Output twiddles of a pass: w = W^(off 2^s0); position m gets w^br(m).  The
// pass loads w^(2^j) from the table and forms w^q = w^(q & 3) * (w^4)^(q >> 2).
template <int KB, typename T>
struct PassTwiddles {
  cplx<T> lo[4];     // w^0 .. w^3
  cplx<T> hi[8];     // (w^4)^0 .. (w^4)^7
  __device__ __forceinline__ void init(const cplx<T>* __restrict__ tw, int off, int s0) {
    lo[0] = {(T)1, (T)0};
    hi[0] = {(T)1, (T)0};
    if (KB >= 1) lo[1] = ldc(tw, off << s0);
    if (KB >= 2) { lo[2] = ldc(tw, (off << 1) << s0); lo[3] = cmul(lo[2], lo[1]); }
    if (KB >= 3) hi[1] = ldc(tw, (off << 2) << s0);
    if (KB >= 4) { hi[2] = ldc(tw, (off << 3) << s0); hi[3] = cmul(hi[2], hi[1]); }
    if (KB >= 5) {
      hi[4] = ldc(tw, (off << 4) << s0);
      hi[5] = cmul(hi[4], hi[1]);
      hi[6] = cmul(hi[4], hi[2]);
      hi[7] = cmul(hi[6], hi[1]);
    }
  }
  __device__ __forceinline__ cplx<T> pow(int q) const {
    const int a = q & 3, b = q >> 2;
    if (b == 0) return lo[a];
    if (a == 0) return hi[b];
    return cmul(lo[a], hi[b]);
  }
};

// DIR 0: forward pass (constant DFT, then output twiddles).  DIR 1: inverse
// pass (conjugate twiddles, then the inverse constant DFT).  DIR 2: the last
// forward pass, the product with the spectrum and the first inverse pass; its
// groups are contiguous (offset 0), so it has no output twiddles.
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
    if (DIR == 0) {
      dft_dif<KB>(v);
      if (off) {
        PassTwiddles<KB, T> w;
        w.init(tw, off, s0);
#pragma unroll
        for (int m = 1; m < RR; ++m) v[m] = cmul(v[m], w.pow(bitrev(m, KB)));
      }
    } else if (DIR == 1) {
      if (off) {
        PassTwiddles<KB, T> w;
        w.init(tw, off, s0);
#pragma unroll
        for (int m = 1; m < RR; ++m) v[m] = cmulc(v[m], w.pow(bitrev(m, KB)));
      }
      dft_dit<KB>(v);
    } else {
      // spectrum loads first: their latency overlaps the LDS reads and the DFT
      cplx<T> sp[RR];
#pragma unroll
      for (int m = 0; m < RR; ++m) sp[m] = ldc(spec, (m << (p - KB)) + g);
      dft_dif<KB>(v);
#pragma unroll
      for (int m = 0; m < RR; ++m) v[m] = cmul(v[m], sp[m]);
      dft_dit<KB>(v);
    }
#pragma unroll
    for (int m = 0; m < RR; ++m) buf[padi(base + (m << lh))] = v[m];
  }
}

// Twiddled passes stop at radix 16 (a twiddled radix-32 pass with its twiddle
// table would not fit the register file); the twiddle-free middle pass may be
// radix 32.
template <typename T> struct FftLimits { static constexpr int kTw = 4; static constexpr int kMid = kFftMid; };

template <int DIR, typename T>
__device__ __forceinline__ void fft_pass_kb(int kb, cplx<T>* buf, int p, int s0, const cplx<T>* tw,
                                            const cplx<T>* spec) {
  switch (kb) {
    case 1: fft_pass<1, DIR>(buf, p, s0, tw, spec); break;
    case 2: fft_pass<2, DIR>(buf, p, s0, tw, spec); break;
    case 3: fft_pass<3, DIR>(buf, p, s0, tw, spec); break;
    case 4: fft_pass<4, DIR>(buf, p, s0, tw, spec); break;
    default:
      if constexpr (DIR == 2 || FftLimits<T>::kTw >= 5) fft_pass<5, DIR>(buf, p, s0, tw, spec);
      break;
  }
}

// Pass plan for length 2^p: the middle pass takes min(p, 5) stages, the
// twiddled passes before it split the rest as evenly as possible.
template <typename T>
__device__ __forceinline__ int fft_npasses(int p) {
  const int rest = p - min(p, FftLimits<T>::kMid);
  return 1 + (rest + FftLimits<T>::kTw - 1) / FftLimits<T>::kTw;
}
template <typename T>
__device__ __forceinline__ void fft_pass_of(int i, int p, int& s0, int& kb) {
  const int mid = min(p, FftLimits<T>::kMid);
  const int rest = p - mid;
  const int ntw = fft_npasses<T>(p) - 1;
  if (i == ntw) { s0 = rest; kb = mid; return; }
  const int small = rest / ntw, nbig = rest - small * ntw;   // the last nbig get small + 1
  const int nsmall = ntw - nbig;
  if (i < nsmall) { s0 = i * small; kb = small; }
  else { s0 = nsmall * small + (i - nsmall) * (small + 1); kb = small + 1; }
}

// c[n] = sum_j t_j z[(n + j) mod P]: forward transform, product with the
// spectrum, inverse transform, all in LDS.
template <typename T>
__device__ __forceinline__ void fft_correlate(cplx<T>* buf, int p, const cplx<T>* tw, const cplx<T>* spec) {
  const int np = fft_npasses<T>(p);
  int s0, kb;
  for (int i = 0; i + 1 < np; ++i) {
    fft_pass_of<T>(i, p, s0, kb);
    fft_pass_kb<0>(kb, buf, p, s0, tw, spec);
    __syncthreads();
  }
  fft_pass_of<T>(np - 1, p, s0, kb);
  fft_pass_kb<2>(kb, buf, p, s0, tw, spec);
  __syncthreads();
  for (int i = np - 2; i >= 0; --i) {
    fft_pass_of<T>(i, p, s0, kb);
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

// wave reduction with xor shuffles, then one value per wave through LDS
__device__ __forceinline__ VI block_argmax(VI mine, VI* scratch) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    const VI o{__shfl_xor(mine.v, m), __shfl_xor(mine.i, m)};
    if (vi_better(o, mine)) mine = o;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) scratch[wave] = mine;
  __syncthreads();
  VI r = scratch[0];
  for (int w = 1; w < nw; ++w)
    if (vi_better(scratch[w], r)) r = scratch[w];
  __syncthreads();
  return r;
}

// fixed pairing (xor butterflies inside a wave, waves in index order): the
// same inputs always give the same sum
template <typename S>
__device__ __forceinline__ S block_sum(S mine, S* scratch) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) mine = mine + __shfl_xor(mine, m);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) scratch[wave] = mine;
  __syncthreads();
  S r = scratch[0];
  for (int w = 1; w < nw; ++w) r = r + scratch[w];
  __syncthreads();
  return r;
}

// --------------------------------------------------------------------------
// finish: literal folds, FFT correlation, argmax, intersection, scoring
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
template <typename Tin, typename Tt>
__device__ __forceinline__ double score_at(const Inst& d, int64_t c, void* scratch) {
  const int64_t N = d.n;
  if (d.mode == MODE_EXACT) {
    long long acc = 0;
    // 16 pairs of loads in flight per thread: K <= 4096 in one round trip
#pragma unroll 16
    for (int j = threadIdx.x; j < d.k; j += blockDim.x) {
      const int64_t xi = c + j < N ? c + j : c + j - N;   // c < N, j < K <= N
      acc += (long long)ld_int<Tt>(d.t, j) * (long long)ld_int<Tin>(d.x, xi);
    }
    return (double)block_sum<long long>(acc, (long long*)scratch);
  }
  double acc = 0.0;
#pragma unroll 4
  for (int j = threadIdx.x; j < d.k; j += blockDim.x) {
    const int64_t xi = c + j < N ? c + j : c + j - N;
    acc += ld_dbl<Tt>(d.t, j) * ld_dbl<Tin>(d.x, xi);
  }
  return block_sum<double>(acc, (double*)scratch);
}

template <typename Tin>
__device__ __forceinline__ double score_any_t(const Inst& d, int64_t c, void* scratch) {
  switch (d.t_dtype) {
    case TM_I8: return score_at<Tin, int8_t>(d, c, scratch);
    case TM_F32: return score_at<Tin, float>(d, c, scratch);
    case TM_BF16: return score_at<Tin, bf16_t>(d, c, scratch);
    default: return score_at<Tin, f16_t>(d, c, scratch);
  }
}

// Literal folds from the partition buckets (Algorithm 1 step 3 with Section 2's
// indices mod N), with rho = N - (L-1) M the length of the last row:
//   y[s]     = yP[s] + [s >= rho] x[s - rho]                  (s < M)
//   y[M + s] = y[s] - x[s] + x[(s + L M) mod N]              (s < K - 1)
// Pass 1 copies the buckets (less 128 per counted element for the streaming
// int8 fold, whose buckets hold sums of x + 128); pass 2 adds the x terms, one
// thread per s, so no entry is written twice.
__device__ __forceinline__ int64_t mod_small(int64_t v, int64_t n, bool general) {
  if (general) return v % n;                  // only when N < M (single-row folds)
  return v >= n ? v - n : v;                  // v < 2N whenever N >= M
}

// Pass 2 for both folds at once (fold A writes the real parts, fold B the
// imaginary parts, so no element half is written by two threads).
template <typename Tin, typename T>
__device__ __forceinline__ void lit_fix(const Inst& d, cplx<T>* buf, int ma, int rhoA, int mb, int rhoB, int K,
                                        bool general) {
  constexpr int U = 8;                 // work items whose loads are in flight together
  const int64_t N = d.n;
  const int loA = max(rhoA, K - 1), loB = max(rhoB, K - 1);   // [0, K-1) extension, [lo, M) wrap only
  const int nA = (K - 1) + max(0, ma - loA), nB = (K - 1) + max(0, mb - loB);
  const int NT = blockDim.x;
  for (int t0 = threadIdx.x; t0 < nA + nB; t0 += U * NT) {
    int s[U], xw[U], e1[U], e0[U];
    bool fb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int t = t0 + u * NT;
      const bool ok = t < nA + nB;
      fb[u] = t >= nA;
      if (fb[u]) t -= nA;
      const int M = fb[u] ? mb : ma, rho = fb[u] ? rhoB : rhoA, lo = fb[u] ? loB : loA;
      s[u] = t < K - 1 ? t : lo + (t - (K - 1));
      const bool wrap = ok && s[u] >= rho && s[u] < M;
      const bool ext = ok && s[u] < K - 1;
      xw[u] = ld_int<Tin>(d.x, wrap ? mod_small((int64_t)(s[u] - rho), N, general) : 0);
      e1[u] = ld_int<Tin>(d.x, ext ? mod_small((int64_t)s[u] + M - rho, N, general) : 0);
      e0[u] = ld_int<Tin>(d.x, ext ? s[u] : 0);
      if (!wrap) xw[u] = 0;
      if (!ext) { e1[u] = 0; e0[u] = 0; }
      if (!ok) s[u] = -1;
    }
    // the targets of different items never coincide: read them all, then write
    T* ze[U];
    T* zw[U];
    T ve[U], vw[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int M = fb[u] ? mb : ma;
      const int half = fb[u] ? 1 : 0;
      const bool ext = s[u] >= 0 && s[u] < K - 1, wrap = s[u] >= 0 && xw[u] != 0;
      ze[u] = ext ? reinterpret_cast<T*>(&buf[padi(M + s[u])]) + half : nullptr;
      zw[u] = wrap ? reinterpret_cast<T*>(&buf[padi(s[u])]) + half : nullptr;
      ve[u] = ext ? *ze[u] : (T)0;
      vw[u] = wrap ? *zw[u] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (ze[u]) *ze[u] = ve[u] + (T)(xw[u] + e1[u] - e0[u]);
      if (zw[u]) *zw[u] = vw[u] + (T)xw[u];
    }
  }
}

// argmax of both folds (lowest index on ties) and the sum of |z|^2, one pass
struct FinRed { double va; double vb; double ss; int ia; int ib; };

__device__ __forceinline__ void finred_merge(FinRed& a, const FinRed& o) {
  if (vi_better(VI{o.va, o.ia}, VI{a.va, a.ia})) { a.va = o.va; a.ia = o.ia; }
  if (vi_better(VI{o.vb, o.ib}, VI{a.vb, a.ib})) { a.vb = o.vb; a.ib = o.ib; }
  a.ss += o.ss;
}

// One DPP step of the wave reduction: lanes in the enabled rows merge the
// value DPP brings them; lanes of disabled rows receive the identity.
template <int CTRL, int ROWS>
__device__ __forceinline__ void finred_dpp(FinRed& r) {
  auto mv = [](int ident, int v) { return __builtin_amdgcn_update_dpp(ident, v, CTRL, ROWS, 0xF, false); };
  auto mvd = [&](double ident, double v) {
    const int lo = mv(__double2loint(ident), __double2loint(v));
    const int hi = mv(__double2hiint(ident), __double2hiint(v));
    return __hiloint2double(hi, lo);
  };
  FinRed o;
  o.va = mvd(-INFINITY, r.va);
  o.vb = mvd(-INFINITY, r.vb);
  o.ss = mvd(0.0, r.ss);
  o.ia = mv(0x7fffffff, r.ia);
  o.ib = mv(0x7fffffff, r.ib);
  finred_merge(r, o);
}

// wave reduction by DPP (the full result lands in lane 63), then the waves'
// results in wave order through LDS
__device__ __forceinline__ FinRed block_finred(FinRed mine, FinRed* scratch) {
  finred_dpp<0xB1, 0xF>(mine);    // quad_perm [1,0,3,2]
  finred_dpp<0x4E, 0xF>(mine);    // quad_perm [2,3,0,1]
  finred_dpp<0x141, 0xF>(mine);   // row_half_mirror
  finred_dpp<0x140, 0xF>(mine);   // row_mirror: every lane holds its row's result
  finred_dpp<0x142, 0xA>(mine);   // row_bcast:15 into rows 1 and 3
  finred_dpp<0x143, 0xC>(mine);   // row_bcast:31 into rows 2 and 3: lane 63 holds the wave
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 63) scratch[wave] = mine;
  __syncthreads();
  FinRed r = scratch[0];
  for (int w = 1; w < nw; ++w) finred_merge(r, scratch[w]);
  __syncthreads();
  return r;
}

// Steps 8-9 (Theorem 4): S_A(a) cap S_B(b) with the candidate sets taken mod
// N (or cut at N for the zero-padded variant of Theorem 2), for every pair of
// the given residues of fold A and fold B (one each for step 9 itself; the
// runners-up for top-T re-scoring), the union re-scored by (Tx)_c, and the
// result record.
template <typename Tin, bool T8 = false>
__device__ __forceinline__ void resolve_lists(const Inst& d, const VI* A, int na, const VI* B, int nb, uint32_t flags,
                              void* scratch, double err_bound = 0.0) {
  const int tid = threadIdx.x;
  const int ma = d.va.m, mb = d.vb.m;
  __shared__ long long cand[3 * kTopTMax * kTopTMax];
  __shared__ int ncand;
  if (tid == 0) {
    const int64_t N = d.n;
    const int64_t Am = ma, Bm = mb, La = d.va.l, Lb = d.vb.l;
    int w = 0;
    auto insert = [&](long long v) {          // ascending, no repeats
      int p = 0;
      while (p < w && cand[p] < v) ++p;
      if (p < w && cand[p] == v) return;
      for (int q = w; q > p; --q) cand[q] = cand[q - 1];
      cand[p] = v;
      ++w;
    };
    for (int ia = 0; ia < na; ++ia)
      for (int ib = 0; ib < nb; ++ib) {
        const int64_t a = A[ia].i, b = B[ib].i;
        // regular members {a + i A < N} and {b + j B < N}: Chinese remaindering
        if (a < N && b < N) {
          const int64_t t = ((((b - a) % Bm) + Bm) % Bm) * d.inv_a_mod_b % Bm;
          const int64_t v = a + Am * t;
          if (v < N) insert(v);
        }
        // the wrapped members (a + (La-1) A) mod N and (b + (Lb-1) B) mod N; the
        // zero-padded variant's sets stop at N
        const bool wa = !d.zpad && a + (La - 1) * Am >= N;
        const bool wb = !d.zpad && b + (Lb - 1) * Bm >= N;
        const int64_t va = (a + (La - 1) * Am) % N;
        const int64_t vb = (b + (Lb - 1) * Bm) % N;
        if (wa && ((b < N && va % Bm == b) || (wb && va == vb))) insert(va);
        if (wb && (a < N && vb % Am == a)) insert(vb);
      }
    ncand = w;
  }
  __syncthreads();
  const int nc = ncand;
  int64_t best = -1;
  double best_score = 0.0;
  for (int i = 0; i < nc; ++i) {
    double sc;
    if constexpr (T8) sc = score_at<Tin, int8_t>(d, cand[i], scratch);
    else sc = score_any_t<Tin>(d, cand[i], scratch);
    if (i == 0 || sc > best_score) { best = cand[i]; best_score = sc; }
  }
  if (nc == 0) flags |= TM_R_NOMATCH;
  if (nc > 1) flags |= TM_R_RESCORED;
  const VI amax = A[0], bmax = B[0];
  if (tid == 0) {
    GAS tm_result* r = G(d.out);
    r->shift = best;
    r->m1_tilde = d.swapped ? bmax.i : amax.i;
    r->m2_tilde = d.swapped ? amax.i : bmax.i;
    r->n_candidates = nc;
    r->flags = flags;
    r->peak1 = d.swapped ? bmax.v : amax.v;
    r->peak2 = d.swapped ? amax.v : bmax.v;
    r->score = nc ? best_score : 0.0;
    r->err_bound = err_bound;
    r->reserved = 0;
  }
}

template <typename Tin, bool T8 = false>
__device__ __forceinline__ void resolve_and_report(const Inst& d, VI amax, VI bmax, uint32_t flags, void* scratch,
                                                   double err_bound = 0.0) {
  resolve_lists<Tin, T8>(d, &amax, 1, &bmax, 1, flags, scratch, err_bound);
}

// Error bound of a real plan's correlations (FP32 transform of 2^stages
// points, the BF16/FP16 storage of the fold) given ||z||_2 of the stored
// folds: the rounding of a radix-2^k FFT of 2^p points is at most
// p (mu + gamma_4 (sqrt 2 + mu)) of ||FFT z||_2 with mu <= 2u the twiddles'
// error, about 7 p u; the forward transform, the product with the stored
// spectrum and the inverse transform give (14 p + 8) u ||FFT(t)||_inf ||z||_2
// (u = 2^-24); stored fold values off by u_s |y| move each r[k] by at most
// u_s sum_j |t_j| |y_{k+j}| <= u_s ||t||_2 ||z||_2 (Cauchy-Schwarz).
__device__ __forceinline__ double real_err_bound(const Inst& d, int stages, double znorm2) {
  const double us = d.fold_store == TM_BF16 ? 0x1p-8 : (d.fold_store == TM_F16 ? 0x1p-11 : 0.0);
  return ((14.0 * stages + 8.0) * 0x1p-24 * d.tspec_max + d.tnorm2 * us) * sqrt(znorm2);
}

// Runners-up of one fold for top-T (reading of the option: value descending,
// lowest index first among equal values): top[0] holds the argmax; passes
// p = 1..T-1 take the best entry not yet taken.  Returns how many exist
// (fewer than T when M < T).  value_of(n) gives r[n] for n < m.
template <typename F>
__device__ __forceinline__ int block_top_t(F value_of, int m, int T, VI (&top)[kTopTMax], VI* scratch) {
  int got = 1;
#pragma unroll
  for (int p = 1; p < kTopTMax; ++p) {
    if (p >= T) break;                       // uniform over the block
    VI mine{-INFINITY, 0x7fffffff};
    for (int n = threadIdx.x; n < m; n += blockDim.x) {
      bool taken = false;
#pragma unroll
      for (int q = 0; q < kTopTMax; ++q)
        if (q < p && top[q].i == n) taken = true;
      if (taken) continue;
      const VI v{value_of(n), n};
      if (vi_better(v, mine)) mine = v;
    }
    const VI r = block_argmax(mine, scratch);
    if (r.i == 0x7fffffff) break;            // uniform: every thread sees the same r
    top[p] = r;
    got = p + 1;
  }
  return got;
}

// top-T re-scoring from the whole correlations in `rtop` (fold A at 0, fold B
// at ma), given both argmaxes
template <typename Tin>
__device__ __forceinline__ void resolve_top_t(const Inst& d, VI amax, VI bmax, uint32_t flags, void* scratch,
                                              double err_bound = 0.0) {
  const int ma = d.va.m, mb = d.vb.m;
  const GAS double* r = G(d.rtop);
  VI A[kTopTMax], B[kTopTMax];
  A[0] = amax;
  B[0] = bmax;
  const int na = block_top_t([&](int n) { return r[n]; }, ma, d.top_t, A, reinterpret_cast<VI*>(scratch));
  const int nb = block_top_t([&](int n) { return r[ma + n]; }, mb, d.top_t, B, reinterpret_cast<VI*>(scratch));
  resolve_lists<Tin>(d, A, na, B, nb, flags, scratch, err_bound);
}

template <typename T, typename Tin>
__device__ __forceinline__ void finish_instance(const Inst& d, unsigned char* lds) {
  const int tid = threadIdx.x;
  const int NT = blockDim.x;
  const int p = d.p_log2;
  const int P = 1 << p;
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(lds);
  void* scratch = lds + (size_t)padded_len(P) * sizeof(cplx<T>);
  const int ma = d.va.m, mb = d.vb.m, K = d.k;
  const int na = ma + K - 1, nb = mb + K - 1;
  const bool exact = d.mode == MODE_EXACT;
  const bool ints = acc_is_int(d);
  double* dya = d.swapped ? d.dbg_y2 : d.dbg_y1;
  double* dyb = d.swapped ? d.dbg_y1 : d.dbg_y2;
  double* dra = d.swapped ? d.dbg_r2 : d.dbg_r1;
  double* drb = d.swapped ? d.dbg_r1 : d.dbg_r2;
  double ss = 0.0;

  // Touch one word of every 128-byte line of the twiddle and spectrum tables
  // now, so that the FFT passes find them in L2; the words are consumed (as
  // an empty asm operand) only after the FFT.
  uint32_t touch[5] = {0, 0, 0, 0, 0};
  {
    const int tw_lines = (int)(((size_t)(P / 2) * sizeof(cplx<T>) + 127) / 128);
    const int sp_lines = (int)(((size_t)P * sizeof(cplx<T>) + 127) / 128);
    const GAS uint32_t* tw32 = G(reinterpret_cast<const uint32_t*>(d.tw));
    const GAS uint32_t* sp32 = G(reinterpret_cast<const uint32_t*>(d.spec));
#pragma unroll
    for (int u = 0; u < 4; ++u) {     // 3 lines per thread when NT = P / 16
      const int i = tid + u * NT;
      const int j = i < tw_lines + sp_lines ? i : 0;
      touch[u] = j < tw_lines ? tw32[j * 32] : sp32[(j - tw_lines) * 32];
    }
    // and the head of x, which the literal folds' wrap and extension terms read
    if (ints) {
      const int64_t head = min(d.n * (int64_t)sizeof(Tin), (int64_t)(max(d.va.m, d.vb.m) + d.k) * (int64_t)sizeof(Tin));
      const GAS unsigned char* xb = G(reinterpret_cast<const unsigned char*>(d.x));
      const int hl = (int)((head + 127) / 128);
      const int i = tid < hl ? tid : 0;
      touch[4] = xb[min((int64_t)i * 128, head - 1)];
    }
  }

  // literal folds (Algorithm 1 step 3) packed as z = yA + i yB, zero padded
  // to P; thread tid owns n = tid + v NT, 16 entries' loads in flight at once
  {
    constexpr int CH = 16;
    const int V = (P + NT - 1) / NT;
    const int64_t N = d.n;
    const int64_t La = d.va.l, Lb = d.vb.l;
    const int rhoA = (int)(N - (La - 1) * ma), rhoB = (int)(N - (Lb - 1) * mb);
    const GAS float* yf = G(reinterpret_cast<const float*>(d.y));
    const GAS int* yp = G(d.yp);
    const int biasA = d.sfold ? 128 * (int)(La - 1) : 0, biasB = d.sfold ? 128 * (int)(Lb - 1) : 0;
    const int bias1 = d.sfold ? 128 : 0;
    for (int v0 = 0; v0 < V; v0 += CH) {
      T re[CH], im[CH];
      if (ints) {
        int ia[CH], ib[CH];
#pragma unroll
        for (int v = 0; v < CH; ++v) {
          const int n = tid + (v0 + v) * NT;
          const int sa = n < ma ? n : n - ma, sb = n < mb ? n : n - mb;
          ia[v] = yp[n < na ? sa : 0];
          ib[v] = yp[ma + (n < nb ? sb : 0)];
        }
#pragma unroll
        for (int v = 0; v < CH; ++v) {
          const int n = tid + (v0 + v) * NT;
          const int sa = n < ma ? n : n - ma, sb = n < mb ? n : n - mb;
          re[v] = n < na && n < P ? (T)(ia[v] - biasA - (sa < rhoA ? bias1 : 0)) : (T)0;
          im[v] = n < nb && n < P ? (T)(ib[v] - biasB - (sb < rhoB ? bias1 : 0)) : (T)0;
        }
      } else {
        float fa[CH], fb[CH];
#pragma unroll
        for (int v = 0; v < CH; ++v) {
          const int n = tid + (v0 + v) * NT;
          fa[v] = yf[n < na && n < P ? n : 0];
          fb[v] = yf[n < nb && n < P ? na + n : 0];
        }
#pragma unroll
        for (int v = 0; v < CH; ++v) {
          const int n = tid + (v0 + v) * NT;
          re[v] = n < na ? store_round<T>(fa[v], d.fold_store) : (T)0;
          im[v] = n < nb ? store_round<T>(fb[v], d.fold_store) : (T)0;
        }
      }
#pragma unroll
      for (int v = 0; v < CH; ++v) {
        const int n = tid + (v0 + v) * NT;
        if (v0 + v < V && n < P) buf[padi(n)] = cplx<T>{re[v], im[v]};
      }
    }
    __syncthreads();
    if (ints) {
      // every bucket has been read: back to zero for the next launch
      for (int s = tid; s < ma + mb; s += NT) G(d.yp)[s] = 0;
      const bool general = N < (int64_t)max(ma, mb);
      // zero-padded variant: the periodic bucket copy of pass 1 is the fold
      if (!d.zpad) lit_fix<Tin, T>(d, buf, ma, rhoA, mb, rhoB, K, general);
      __syncthreads();
    }
    // storage rounding (real path), |z|^2 and the optional intermediates
    for (int n = tid; n < P; n += NT) {
      cplx<T> z = buf[padi(n)];
      if (ints && !exact) {
        z.x = store_round<T>((float)z.x, d.fold_store);
        z.y = store_round<T>((float)z.y, d.fold_store);
        buf[padi(n)] = z;
      }
      if (dya && n < na) G(dya)[n] = (double)z.x;
      if (dyb && n < nb) G(dyb)[n] = (double)z.y;
      ss += (double)z.x * (double)z.x + (double)z.y * (double)z.y;
    }
    __syncthreads();
  }

  fft_correlate<T>(buf, p, reinterpret_cast<const cplx<T>*>(d.tw), reinterpret_cast<const cplx<T>*>(d.spec));
  asm volatile("" : : "v"(touch[0]), "v"(touch[1]), "v"(touch[2]), "v"(touch[3]), "v"(touch[4]));

  // step 7: argmax over [0, M) of each fold, lowest index on ties
  FinRed fr{-INFINITY, -INFINITY, ss, 0x7fffffff, 0x7fffffff};
#pragma unroll 4
  for (int n = tid; n < ma; n += NT) {
    const double v = exact ? rint((double)buf[padi(n)].x) : (double)buf[padi(n)].x;
    if (dra) G(dra)[n] = v;
    if (vi_better(VI{v, n}, VI{fr.va, fr.ia})) { fr.va = v; fr.ia = n; }
  }
#pragma unroll 4
  for (int n = tid; n < mb; n += NT) {
    const double v = exact ? rint((double)buf[padi(n)].y) : (double)buf[padi(n)].y;
    if (drb) G(drb)[n] = v;
    if (vi_better(VI{v, n}, VI{fr.vb, fr.ib})) { fr.vb = v; fr.ib = n; }
  }
  const FinRed red = block_finred(fr, reinterpret_cast<FinRed*>(scratch));
  const VI amax{red.va, red.ia}, bmax{red.vb, red.ib};
  const double znorm2 = red.ss;
  VI* vs = reinterpret_cast<VI*>(scratch);

  uint32_t flags = 0;
  const double err = exact ? 0.0 : real_err_bound(d, p, znorm2);
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

  if (d.top_t > 1) {
    VI A[kTopTMax], B[kTopTMax];
    A[0] = amax;
    B[0] = bmax;
    const int na = block_top_t([&](int n) {
      return exact ? rint((double)buf[padi(n)].x) : (double)buf[padi(n)].x; }, ma, d.top_t, A, vs);
    const int nb = block_top_t([&](int n) {
      return exact ? rint((double)buf[padi(n)].y) : (double)buf[padi(n)].y; }, mb, d.top_t, B, vs);
    resolve_lists<Tin>(d, A, na, B, nb, flags, scratch, err);
    return;
  }
  resolve_and_report<Tin>(d, amax, bmax, flags, scratch, err);
}

template <typename T>
__device__ __forceinline__ void finish_dispatch(const Inst& d, unsigned char* lds) {
  switch (d.x_dtype) {
    case TM_I8: finish_instance<T, int8_t>(d, lds); break;
    case TM_F32: finish_instance<T, float>(d, lds); break;
    case TM_BF16: finish_instance<T, bf16_t>(d, lds); break;
    default: finish_instance<T, f16_t>(d, lds); break;
  }
}

template <typename T>
__global__ void __launch_bounds__(kFinishThreads) k_finish(InstTable tab, const int32_t* list, int count) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int b = blockIdx.x;
  if (b >= count) return;
  if (tab.table) finish_dispatch<T>(tab.table[list ? list[b] : b], lds);
  else finish_dispatch<T>(tab.resident(), lds);
}

// --------------------------------------------------------------------------
// FFT correlation through global memory (P above one workgroup's LDS)
// --------------------------------------------------------------------------
//
// Four-step transform, P = P1 P2, n = n1 P2 + n2, k = k1 + P1 k2:
//   cols:  length-P1 DIF transforms of the columns (in blocks of B adjacent
//          columns, so rows are read as coalesced segments), times W_P^(n2 k1);
//          position j of a column holds k1 = bitrev(j), written to row j
//   rows:  each row j: the LDS correlation of fft_correlate (DIF, product with
//          the spectrum stored per row, DIT), times conj W_P^(n2 k1)
//   icols: length-P1 DIT transforms of the column blocks back to n1, argmax
//          partials per block (best, second best, largest magnitude)
// plus the literal folds into the working buffer before and the final
// reduction, intersection and scoring after.  The spectrum of row j at
// position i is S[bitrev(j) + P1 bitrev(i)], which is the plan's bit-reversed
// spectrum at j P2 + i.

template <typename T>
__device__ __forceinline__ void stc(cplx<T>* p, int64_t i, cplx<T> v) {
  GAS T* q = G(reinterpret_cast<T*>(p));
  q[2 * i] = v.x;
  q[2 * i + 1] = v.y;
}

template <typename T>
__device__ __forceinline__ cplx<T> w_pow(const cplx<T>* tw, int64_t e, int p) {
  const int64_t P = (int64_t)1 << p;
  e &= P - 1;
  const cplx<T> w = ldc(tw, (int)(e & ((P >> 1) - 1)));
  return e >= (P >> 1) ? cplx<T>{-w.x, -w.y} : w;
}

// DIF passes over stages [lb, lb + q) of a length-2^(lb + q) transform: B
// independent length-2^q transforms stored one after another.  The last pass
// has contiguous groups and no output twiddles.  DIT inverse in reverse order.
__device__ __forceinline__ int batch_npasses(int q) { return (q + 3) / 4; }
__device__ __forceinline__ void batch_pass_of(int i, int q, int lb, int& s0, int& kb) {
  const int np = batch_npasses(q);
  const int small = q / np, nbig = q - small * np;    // the last nbig passes get one more stage
  const int nsmall = np - nbig;
  if (i < nsmall) { s0 = lb + i * small; kb = small; }
  else { s0 = lb + nsmall * small + (i - nsmall) * (small + 1); kb = small + 1; }
}

template <typename T>
__device__ void fft_batch_forward(cplx<T>* buf, int lb, int q, const cplx<T>* tw) {
  for (int i = 0; i < batch_npasses(q); ++i) {
    int s0, kb;
    batch_pass_of(i, q, lb, s0, kb);
    fft_pass_kb<0>(kb, buf, lb + q, s0, tw, (const cplx<T>*)nullptr);
    __syncthreads();
  }
}

template <typename T>
__device__ void fft_batch_inverse(cplx<T>* buf, int lb, int q, const cplx<T>* tw) {
  for (int i = batch_npasses(q) - 1; i >= 0; --i) {
    int s0, kb;
    batch_pass_of(i, q, lb, s0, kb);
    fft_pass_kb<1>(kb, buf, lb + q, s0, tw, (const cplx<T>*)nullptr);
    __syncthreads();
  }
}

template <typename T, typename Tin>
__global__ void __launch_bounds__(kGfftThreads) k_gfft_literal(InstTable tab) {
  const Inst& d = tab.resident();
  __shared__ double red[kGfftThreads / 64];
  const int n = blockIdx.x * kGfftThreads + threadIdx.x;
  const int P = 1 << d.p_log2;
  const int ma = d.va.m, mb = d.vb.m, K = d.k;
  const int na = ma + K - 1, nb = mb + K - 1;
  const bool exact = d.mode == MODE_EXACT;
  T re = 0, im = 0;
  if (n < P) {
    if (d.acc_int) {
      const int64_t N = d.n;
      const bool general = N < (int64_t)max(ma, mb);
      int val[2];
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const int M = f ? mb : ma, nn = f ? nb : na;
        const int64_t L = f ? d.vb.l : d.va.l;
        const int rho = (int)(N - (L - 1) * M);
        const bool ok = n < nn;
        const int s = n < M ? n : n - M;
        const bool wrap = ok && !d.zpad && s >= rho, ext = ok && !d.zpad && n >= M;
        const int yb = G(d.yp)[(f ? ma : 0) + (ok ? s : 0)];
        const int xw = ld_int<Tin>(d.x, wrap ? mod_small((int64_t)(s - rho), N, general) : 0);
        const int x1 = ld_int<Tin>(d.x, ext ? mod_small((int64_t)s + M - rho, N, general) : 0);
        const int x0 = ld_int<Tin>(d.x, ext ? s : 0);
        const int bias = d.sfold ? 128 * ((int)L - 1 + (s < rho ? 1 : 0)) : 0;
        val[f] = ok ? yb - bias + (wrap ? xw : 0) + (ext ? x1 - x0 : 0) : 0;
      }
      re = exact ? (T)val[0] : store_round<T>((float)val[0], d.fold_store);
      im = exact ? (T)val[1] : store_round<T>((float)val[1], d.fold_store);
    } else {
      const GAS float* yf = G(reinterpret_cast<const float*>(d.y));
      re = n < na ? store_round<T>(yf[n], d.fold_store) : (T)0;
      im = n < nb ? store_round<T>(yf[na + n], d.fold_store) : (T)0;
    }
    double* dya = d.swapped ? d.dbg_y2 : d.dbg_y1;
    double* dyb = d.swapped ? d.dbg_y1 : d.dbg_y2;
    if (dya && n < na) G(dya)[n] = (double)re;
    if (dyb && n < nb) G(dyb)[n] = (double)im;
    stc(reinterpret_cast<cplx<T>*>(d.gz), n, cplx<T>{re, im});
  }
  const double ss = block_sum<double>((double)re * (double)re + (double)im * (double)im, red);
  if (threadIdx.x == 0) G(d.gss)[blockIdx.x] = ss;
}

template <typename T>
__global__ void __launch_bounds__(kFinishThreads) k_gfft_cols(InstTable tab) {
  extern __shared__ __align__(16) unsigned char lds[];
  const Inst& d = tab.resident();
  const int p = d.p_log2, q = d.g_q, lb = d.g_logb, bb = p - q;
  const int P1 = 1 << q, P2 = 1 << bb, B = 1 << lb;
  const int c0 = blockIdx.x * B;
  const int NT = blockDim.x, tid = threadIdx.x;
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(lds);
  cplx<T>* z = reinterpret_cast<cplx<T>*>(d.gz);
  if (d.acc_int)   // every literal entry has been formed: buckets back to zero
    for (int s = blockIdx.x * NT + tid; s < d.va.m + d.vb.m; s += gridDim.x * NT) G(d.yp)[s] = 0;
  for (int idx = tid; idx < B * P1; idx += NT) {
    const int b = idx & (B - 1), n1 = idx >> lb;
    buf[padi(b * P1 + n1)] = ldc(z, n1 * P2 + c0 + b);
  }
  __syncthreads();
  fft_batch_forward<T>(buf, lb, q, reinterpret_cast<const cplx<T>*>(d.tw_cols));
  const cplx<T>* tw = reinterpret_cast<const cplx<T>*>(d.tw);
  for (int idx = tid; idx < B * P1; idx += NT) {
    const int b = idx & (B - 1), i = idx >> lb;
    const cplx<T> v = buf[padi(b * P1 + i)];
    stc(z, i * P2 + c0 + b, cmul(v, w_pow(tw, (int64_t)(c0 + b) * bitrev(i, q), p)));
  }
}

template <typename T>
__global__ void __launch_bounds__(kFinishThreads) k_gfft_rows(InstTable tab) {
  extern __shared__ __align__(16) unsigned char lds[];
  const Inst& d = tab.resident();
  const int p = d.p_log2, q = d.g_q, bb = p - q;
  const int P2 = 1 << bb;
  const int j = blockIdx.x;
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(lds);
  cplx<T>* z = reinterpret_cast<cplx<T>*>(d.gz) + (size_t)j * P2;
  for (int n = threadIdx.x; n < P2; n += blockDim.x) buf[padi(n)] = ldc(z, n);
  __syncthreads();
  fft_correlate<T>(buf, bb, reinterpret_cast<const cplx<T>*>(d.tw_rows),
                   reinterpret_cast<const cplx<T>*>(d.spec) + (size_t)j * P2);
  const cplx<T>* tw = reinterpret_cast<const cplx<T>*>(d.tw);
  const int k1 = bitrev(j, q);
  for (int n = threadIdx.x; n < P2; n += blockDim.x)
    stc(z, n, cmulc(buf[padi(n)], w_pow(tw, (int64_t)n * k1, p)));
}

// best, second best (lowest index on ties) and largest magnitude of one fold
struct Top2 { double v1, v2, mag; int i1, i2; };

__device__ __forceinline__ void top2_add(Top2& t, double v, int i) {
  t.mag = fmax(t.mag, fabs(v));
  if (vi_better(VI{v, i}, VI{t.v1, t.i1})) { t.v2 = t.v1; t.i2 = t.i1; t.v1 = v; t.i1 = i; }
  else if (vi_better(VI{v, i}, VI{t.v2, t.i2})) { t.v2 = v; t.i2 = i; }
}

__device__ __forceinline__ void top2_merge(Top2& t, const Top2& o) {
  const double mag = fmax(t.mag, o.mag);
  top2_add(t, o.v1, o.i1);
  top2_add(t, o.v2, o.i2);
  t.mag = mag;
}

struct GPart { Top2 a, b; };

size_t gfft_part_bytes() { return sizeof(GPart); }

__device__ Top2 block_top2(Top2 mine, Top2* scratch) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    const Top2 o{__shfl_xor(mine.v1, m), __shfl_xor(mine.v2, m), __shfl_xor(mine.mag, m),
                 __shfl_xor(mine.i1, m), __shfl_xor(mine.i2, m)};
    top2_merge(mine, o);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) scratch[wave] = mine;
  __syncthreads();
  Top2 r = scratch[0];
  for (int w = 1; w < nw; ++w) top2_merge(r, scratch[w]);
  __syncthreads();
  return r;
}

template <typename T>
__global__ void __launch_bounds__(kFinishThreads) k_gfft_icols(InstTable tab) {
  extern __shared__ __align__(16) unsigned char lds[];
  const Inst& d = tab.resident();
  const int p = d.p_log2, q = d.g_q, lb = d.g_logb, bb = p - q;
  const int P1 = 1 << q, P2 = 1 << bb, B = 1 << lb;
  const int c0 = blockIdx.x * B;
  const int NT = blockDim.x, tid = threadIdx.x;
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(lds);
  Top2* scratch = reinterpret_cast<Top2*>(lds + (size_t)padded_len(B * P1) * sizeof(cplx<T>));
  const cplx<T>* z = reinterpret_cast<const cplx<T>*>(d.gz);
  for (int idx = tid; idx < B * P1; idx += NT) {
    const int b = idx & (B - 1), j = idx >> lb;
    buf[padi(b * P1 + j)] = ldc(z, j * P2 + c0 + b);
  }
  __syncthreads();
  fft_batch_inverse<T>(buf, lb, q, reinterpret_cast<const cplx<T>*>(d.tw_cols));
  const bool exact = d.mode == MODE_EXACT;
  const int ma = d.va.m, mb = d.vb.m;
  double* dra = d.swapped ? d.dbg_r2 : d.dbg_r1;
  double* drb = d.swapped ? d.dbg_r1 : d.dbg_r2;
  Top2 ta{-INFINITY, -INFINITY, 0.0, 0x7fffffff, 0x7fffffff}, tb = ta;
  for (int idx = tid; idx < B * P1; idx += NT) {
    const int b = idx & (B - 1), n1 = idx >> lb;
    const int n = n1 * P2 + c0 + b;
    const cplx<T> v = buf[padi(b * P1 + n1)];
    if (n < ma) {
      const double r = exact ? rint((double)v.x) : (double)v.x;
      if (dra) G(dra)[n] = r;
      if (d.rtop) G(d.rtop)[n] = r;
      top2_add(ta, r, n);
    }
    if (n < mb) {
      const double r = exact ? rint((double)v.y) : (double)v.y;
      if (drb) G(drb)[n] = r;
      if (d.rtop) G(d.rtop)[ma + n] = r;
      top2_add(tb, r, n);
    }
  }
  const Top2 ra = block_top2(ta, scratch);
  const Top2 rb = block_top2(tb, scratch);
  if (tid == 0) {
    GPart* part = reinterpret_cast<GPart*>(d.gpart) + blockIdx.x;
    part->a = ra;
    part->b = rb;
  }
}

template <typename Tin>
__global__ void __launch_bounds__(kGfftThreads) k_gfft_final(InstTable tab) {
  const Inst& d = tab.resident();
  __shared__ __align__(16) unsigned char scratch[kGfftThreads * 16];
  __shared__ Top2 fa, fb;
  __shared__ double zn2;
  const int nparts = (1 << (d.p_log2 - d.g_q)) >> d.g_logb;
  const int nss = (1 << d.p_log2) / kGfftThreads;
  if (threadIdx.x == 0) {   // fixed order: deterministic
    const GPart* parts = reinterpret_cast<const GPart*>(d.gpart);
    Top2 a = parts[0].a, b = parts[0].b;
    for (int i = 1; i < nparts; ++i) { top2_merge(a, parts[i].a); top2_merge(b, parts[i].b); }
    double s2 = 0.0;
    for (int i = 0; i < nss; ++i) s2 += G(d.gss)[i];
    fa = a;
    fb = b;
    zn2 = s2;
  }
  __syncthreads();
  const Top2 a = fa, b = fb;
  uint32_t flags = 0;
  if (d.mode == MODE_EXACT) {
    // the two twiddle products of the four-step transform count as two more stages
    const double bound = 20.0 * (d.p_log2 + 2) * 0x1p-53 * d.tnorm1 * sqrt(zn2);
    if (bound < 0.5) flags |= TM_R_EXACT;
  } else if (a.v1 - a.v2 <= 1e-5 * a.mag || b.v1 - b.v2 <= 1e-5 * b.mag) {
    flags |= TM_R_NEAR_TIE;
  }
  // the two twiddle products of the four-step transform count as two more stages
  const double err = d.mode == MODE_EXACT ? 0.0 : real_err_bound(d, d.p_log2 + 2, zn2);
  if (d.top_t > 1) resolve_top_t<Tin>(d, VI{a.v1, a.i1}, VI{b.v1, b.i1}, flags, scratch, err);
  else resolve_and_report<Tin>(d, VI{a.v1, a.i1}, VI{b.v1, b.i1}, flags, scratch, err);
}

template <typename T, typename Tin>
hipError_t launch_gfft_t(const Inst& one, const Inst* dev, hipStream_t s) {
  InstTable tab{};
  tab.table = nullptr;
  tab.count = 1;
  tab.one = dev;
  tab.x = one.x;
  tab.out = one.out;
  const int p = one.p_log2, q = one.g_q, lb = one.g_logb, bb = p - q;
  const int P = 1 << p, P2 = 1 << bb, B = 1 << lb;
  const int cols_threads = std::min(kFinishThreads, std::max(64, (B << q) >> 4));
  const size_t cols_lds = (size_t)padded_len(B << q) * sizeof(cplx<T>) + (size_t)(kFinishThreads / 64) * sizeof(Top2);
  const int mode = one.mode;
  TM_LAUNCH((k_gfft_literal<T, Tin>), dim3(P / kGfftThreads), dim3(kGfftThreads), 0, s, tab);
  TM_LAUNCH(k_gfft_cols<T>, dim3(P2 / B), dim3(cols_threads), cols_lds, s, tab);
  TM_LAUNCH(k_gfft_rows<T>, dim3(1 << q), dim3(finish_threads(bb)), finish_lds_bytes(bb, mode), s, tab);
  TM_LAUNCH(k_gfft_icols<T>, dim3(P2 / B), dim3(cols_threads), cols_lds, s, tab);
  TM_LAUNCH(k_gfft_final<Tin>, dim3(1), dim3(kGfftThreads), 0, s, tab);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gfft_x(const Inst& one, const Inst* dev, hipStream_t s) {
  switch (one.x_dtype) {
    case TM_I8: return launch_gfft_t<T, int8_t>(one, dev, s);
    case TM_F32: return launch_gfft_t<T, float>(one, dev, s);
    case TM_BF16: return launch_gfft_t<T, bf16_t>(one, dev, s);
    default: return launch_gfft_t<T, f16_t>(one, dev, s);
  }
}

// `host` is the instance as the host built it (grid sizes, signal, result
// slot), `dev` its copy in device memory
hipError_t launch_gfft(const Inst& host, const Inst* dev, hipStream_t s) {
  return host.mode == MODE_EXACT ? launch_gfft_x<double>(host, dev, s) : launch_gfft_x<float>(host, dev, s);
}

// --------------------------------------------------------------------------
// many signals, one template: correlation as an int8 MFMA GEMM
// --------------------------------------------------------------------------
//
// For signals y_i sharing the template t, r_i[k] = sum_l y_i[l] t[l - k] is a
// matrix product R = Y T with Y[i][l] the literal folds and T[l][k] = t[l - k]
// (a banded Toeplitz matrix).  The folds are split into balanced base-128 digits
// (int8 limbs; |y| <= 128 L), each limb product runs on v_mfma_i32_16x16x64_i8
// with exact int32 sums, and the limbs are recombined in int64.  The B operand
// (16 consecutive l of column k) is t[l - k .. l - k + 15]: read aligned from one
// of 16 byte-shifted copies of the zero-padded template in LDS, so the band's
// edges come out as zeros.  Each wave produces a 16-signal x 64-shift tile and
// keeps only its per-signal best (value, lowest shift); a last kernel reduces
// the blocks in shift order and resolves each signal (steps 7-9).

typedef int v4i_t __attribute__((ext_vector_type(4)));

// a raw buffer resource over [base, base + bytes) in scalar registers (base is
// wave-uniform)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t uniform_rsrc(const void* base, uint32_t bytes) {
  const uintptr_t b = reinterpret_cast<uintptr_t>(base);
  const uintptr_t ub = (uintptr_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b) |
                       ((uintptr_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32)) << 32);
  return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(ub), 0,
                                           (int)__builtin_amdgcn_readfirstlane((int)bytes), kBufRsrcWord3);
}

__device__ __forceinline__ v4i_t buf_v4i(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  const auto w = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
  return v4i_t{(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
}


__global__ void __launch_bounds__(256) k_many_prep(ManyArgs a) {
  const Inst& b = a.base;
  const int u = blockIdx.x * 256 + threadIdx.x;
  const int i = blockIdx.y, f = blockIdx.z;
  const int ma = b.va.m, mb = b.vb.m, K = b.k;
  const int M = f ? mb : ma;
  const int64_t L = f ? b.vb.l : b.va.l, N = b.n;
  const int rho = (int)(N - (L - 1) * M);
  const bool general = N < (int64_t)max(ma, mb);
  const int8_t* x = reinterpret_cast<const int8_t*>(a.xs[i]);
  const GAS int* yp = G(a.yp) + (int64_t)i * a.yp_stride + (f ? ma : 0);
  int val = 0;
  if (u < M + K - 1) {
    const int s = u < M ? u : u - M;
    const bool wrap = !b.zpad && s >= rho, ext = !b.zpad && u >= M;
    const int yb = yp[s];
    const int xw = G(x)[wrap ? mod_small((int64_t)(s - rho), N, general) : 0];
    const int x1 = G(x)[ext ? mod_small((int64_t)s + M - rho, N, general) : 0];
    const int x0 = G(x)[ext ? s : 0];
    const int bias = b.sfold ? 128 * ((int)L - 1 + (s < rho ? 1 : 0)) : 0;
    val = yb - bias + (wrap ? xw : 0) + (ext ? x1 - x0 : 0);
  }
  if (u < a.lp) {
    int rest = val;
#pragma unroll
    for (int l = 0; l < kGemmMaxLimbs; ++l) {
      const int digit = l + 1 < kGemmMaxLimbs ? ((rest + 64) & 127) - 64 : rest;
      rest = (rest - digit) >> 7;
      G(a.ylimb)[(((int64_t)f * kGemmMaxLimbs + l) * a.rows + i) * a.lp + u] = (int8_t)digit;
    }
  }
  // largest |y| of this fold and signal: wave, then workgroup, then one atomic
  __shared__ int wmax[4];
  int m = val < 0 ? -val : val;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
    if (m) __hip_atomic_fetch_max(G(a.maxabs) + (int64_t)f * a.count + i, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Wave `wave` of the workgroup: signals sg .. sg + 15 (rows) against shifts
// k0 .. k0 + 63 of fold f.  The B operand comes from the plan's 16 interleaved
// template copies (as in cgw_tile: step st, column tile nt at 1024 st +
// boff[nt]), the digit rows of A through buffer loads at a fixed per-lane
// offset plus a per-step scalar offset; two steps in flight over two register
// sets (a load past the band reads the last step again, unused).
template <int NL>
__device__ __forceinline__ void many_gemm_tile(const ManyArgs& a) {
  const Inst& b = a.base;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int f = blockIdx.z;
  const int M = f ? b.vb.m : b.va.m, K = b.k;
  const int k0 = blockIdx.y * kGemmTile;
  const int sg = blockIdx.x * kGemmTile + wave * 16;
  const int nst = (kGemmTile - 1 + K + 63) / 64;               // 64-deep steps of the band
  const int64_t fold_bytes = (int64_t)kGemmMaxLimbs * a.rows * a.lp;
  const __amdgpu_buffer_rsrc_t ra = uniform_rsrc(a.ylimb + (int64_t)f * fold_bytes, (uint32_t)fold_bytes);
  const __amdgpu_buffer_rsrc_t rb = uniform_rsrc(b.tsh, (uint32_t)(16 * b.c_lt));
  const int aoff = (sg + c) * a.lp + 16 * g + k0;
  const int limb_bytes = (int)(a.rows * a.lp);
  int boff[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int j0 = 16 * g - (16 * nt + c) + kCgPad;
    boff[nt] = (j0 + 2 * ((-j0) & 15)) * 16;
  }
  auto load = [&](int st, v4i_t (&bt)[4], v4i_t (&av)[NL]) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) bt[nt] = buf_v4i(rb, boff[nt], 1024 * st);
#pragma unroll
    for (int l = 0; l < NL; ++l) av[l] = buf_v4i(ra, aoff, l * limb_bytes + 64 * st);
  };
  v4i_t acc[NL][4];
#pragma unroll
  for (int l = 0; l < NL; ++l)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[l][nt] = v4i_t{0, 0, 0, 0};
  auto mfma = [&](const v4i_t (&bt)[4], const v4i_t (&av)[NL]) {
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[l][nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(av[l], bt[nt], acc[l][nt], 0, 0, 0);
  };
  v4i_t b0[4], a0[NL], b1[4], a1[NL];
  load(0, b0, a0);
  for (int st = 0; st < nst; st += 2) {
    load(min(st + 1, nst - 1), b1, a1);
    mfma(b0, a0);
    load(min(st + 2, nst - 1), b0, a0);
    if (st + 1 < nst) mfma(b1, a1);               // uniform
  }
  // lane holds rows (signals) 4g + j and column (shift) c of each 16 x 16 tile
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    VI best{-INFINITY, 0x7fffffff};
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      int64_t r = 0, w = 1;
#pragma unroll
      for (int l = 0; l < NL; ++l) { r += w * (int64_t)acc[l][nt][j]; w *= 128; }
      const int k = k0 + 16 * nt + c;
      if (k < M && vi_better(VI{(double)r, k}, best)) best = VI{(double)r, k};
    }
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      const VI other{__shfl_xor(best.v, o), __shfl_xor(best.i, o)};
      if (vi_better(other, best)) best = other;
    }
    const int sig = sg + 4 * g + j;
    if (c == 0 && sig < a.count) {
      double* pp = a.part + (((int64_t)f * a.count + sig) * a.nkb + blockIdx.y) * 2;
      G(pp)[0] = best.v;
      G(pp)[1] = (double)best.i;
    }
  }
}

__global__ void __launch_bounds__(256) k_many_gemm(ManyArgs a) {
  // limbs needed by this workgroup's 64 signals
  __shared__ int tmax;
  if (threadIdx.x == 0) tmax = 0;
  __syncthreads();
  if (threadIdx.x < kGemmTile) {
    const int sig = blockIdx.x * kGemmTile + threadIdx.x;
    if (sig < a.count) atomicMax(&tmax, G(a.maxabs)[(int64_t)blockIdx.z * a.count + sig]);
  }
  __syncthreads();
  const Inst& b = a.base;
  const int M = blockIdx.z ? b.vb.m : b.va.m;
  if ((int)blockIdx.y * kGemmTile >= M) return;
  const int mx = tmax;
  const int nl = mx < 64 ? 1 : (mx < 64 + 128 * 63 ? 2 : 3);
  if (nl == 1) many_gemm_tile<1>(a);
  else if (nl == 2) many_gemm_tile<2>(a);
  else many_gemm_tile<3>(a);
}

// One workgroup of four waves per signal: wave 0 reduces the block bests, all
// clear the buckets and take part in the resolve and its re-score
__global__ void __launch_bounds__(256) k_many_finish(ManyArgs a) {
  __shared__ __align__(16) unsigned char scratch[64 * 16];
  __shared__ VI fin[2];
  const int i = blockIdx.x;
  Inst d = a.base;
  d.x = a.xs[i];
  d.out = a.out + i;
  const int ma = d.va.m, mb = d.vb.m;
  // each fold's block bests: lane b of wave 0 takes blocks b, b + 64, ...,
  // then a wave argmax (the lowest shift on ties, as in one scan)
#pragma unroll
  for (int f = 0; f < 2 && threadIdx.x < 64; ++f) {
    const int nb = ((f ? mb : ma) + kGemmTile - 1) / kGemmTile;
    const double* pp = a.part + ((int64_t)f * a.count + i) * a.nkb * 2;
    VI best{-INFINITY, 0x7fffffff};
    for (int blk = threadIdx.x; blk < nb; blk += 64) {
      const VI v{G(pp)[2 * blk], (int)G(pp)[2 * blk + 1]};
      if (vi_better(v, best)) best = v;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const VI other{__shfl_xor(best.v, o), __shfl_xor(best.i, o)};
      if (vi_better(other, best)) best = other;
    }
    if (threadIdx.x == 0) fin[f] = best;
  }
  int* yp = a.yp + (int64_t)i * a.yp_stride;
  for (int s = threadIdx.x; s < ma + mb; s += blockDim.x) G(yp)[s] = 0;   // buckets consumed
  __syncthreads();
  resolve_and_report<int8_t, true>(d, fin[0], fin[1], TM_R_EXACT, scratch);
}

hipError_t launch_many(const ManyArgs& a, hipStream_t s) {
  TM_LAUNCH(k_many_prep, dim3((a.lp + 255) / 256, a.count, 2), dim3(256), 0, s, a);
  TM_LAUNCH(k_many_gemm, dim3((unsigned)(a.rows / kGemmTile), a.nkb, 2), dim3(256), 0, s, a);
  TM_LAUNCH(k_many_finish, dim3(a.count), dim3(256), 0, s, a);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// exact instances: the correlation as an int8 MFMA GEMM
// --------------------------------------------------------------------------
//
// For one fold, r[k] = sum_{j<K} t_j y[k + j] (k < M) is the product R = Y T
// with the shift written k = 64 a + b: Y[a][l] = y[64 a + l] (the literal fold
// read as rows of stride 64) and T[l][b] = t[l - b] (the banded Toeplitz block
// of t, l < K + 63, b < 64).  The folds are split into balanced base-128
// digits so that every digit row is an int8 A operand; the B operand of column
// b, t[l - b .. l - b + 15], is read 16-byte aligned from one of 16 copies of
// the zero-padded template shifted by 0..15 bytes (built once per plan and
// interleaved by 16-byte chunk, so neighbouring columns read neighbouring
// chunks).  A
// wave computes a 16 x 16 tile of shifts (rows 16 rt + 0..15, columns
// 16 nt + 0..15) over the whole band with exact int32 sums per digit, combines
// the digits in int64 and keeps its best (value, lowest shift); the last
// kernel reduces the waves of each fold and resolves (steps 7-9).  Every r[k]
// is the exact integer, so the result always carries TM_R_EXACT.

// |y| < T_n is held by n balanced digits, each in [-64, 63], with T_1 = 64
// and T_{n+1} = 64 + 128 (T_n - 1)
__host__ __device__ inline int cg_limbs(int64_t maxabs) {
  int n = 1;
  int64_t th = 64;
  while (n < kCgMaxLimbs && maxabs >= th) {
    th = 64 + 128 * (th - 1);
    ++n;
  }
  return n;
}

int cgemm_limbs_for(int64_t maxabs) { return cg_limbs(maxabs); }

// literal fold entries [e0, e0 + chunk) of the pair (fold A entries u < c_lp,
// then fold B): Algorithm 1 step 3 with Section 2's indices (the zero-padded
// variant keeps the periodic bucket sums), their digits, the intermediates and
// each fold's largest |y|
template <typename Tin, bool GENERAL>
__device__ void cg_prep_chunk(const Inst& d, int f, int e0, int chunk) {
  __shared__ int wmax[kCgPrepThreads / 64];
  // everything the loop needs in registers (its global stores could alias
  // the instance table as far as the compiler knows), the fold's values
  // uniform over the workgroup
  const int lp = d.c_lp, nlc = d.c_nlcap, K = d.k;
  const int M = f ? d.vb.m : d.va.m;
  const int64_t N = d.n, L = f ? d.vb.l : d.va.l;
  const bool sfold = d.sfold != 0, zpad = d.zpad != 0;
  const int rho = (int)(N - (L - 1) * M);
  const int bias = sfold ? 128 * ((int)L - 1) : 0;
  const GAS int* yp = G(d.yp) + (f ? d.va.m : 0);
  const void* x = d.x;
  double* dy = (f != d.swapped) ? d.dbg_y2 : d.dbg_y1;
  GAS int8_t* limb = G(d.ylimb) + (int64_t)f * nlc * lp;
  int mx = 0;
  const int e1 = min(e0 + chunk, lp);
  // a trip: four entries per thread, kCgPrepThreads apart, so that every load
  // and store instruction of a wave covers consecutive entries (one or two
  // cache lines).  Every load of a trip is issued first, at valid addresses
  // (index 0 where an entry does not use one), so one wait covers them all:
  // the debug and digit stores could alias the loads as far as the compiler
  // knows and would otherwise order later loads after them.  Without GENERAL
  // (N >= M) the x indices stay below 2 M and use int32.
  constexpr int U = 4;
  const int n32 = (int)min<int64_t>(N, 0x7fffffff);
  for (int eb = e0 + (int)threadIdx.x; eb < e1; eb += U * kCgPrepThreads) {
    int val[U], xw[U], xe[U], xs[U];
    bool in[U], wrap[U], ext[U];
#pragma unroll
    for (int i = 0; i < U; ++i) {
      const int u = eb + i * kCgPrepThreads;
      in[i] = u < e1 && u < M + K - 1;
      const int s = !in[i] ? 0 : (u < M ? u : u - M);
      wrap[i] = !zpad && in[i] && s >= rho;
      ext[i] = !zpad && in[i] && u >= M;
      val[i] = yp[s];
      int64_t iw, ie;
      if constexpr (GENERAL) {
        iw = mod_small((int64_t)(s - rho), N, true);
        ie = mod_small((int64_t)s + M - rho, N, true);
      } else {
        const int t = s + M - rho;                  // < 2 M
        iw = s - rho;                               // < M <= N
        ie = t >= n32 ? t - n32 : t;
      }
      xw[i] = ld_int<Tin>(x, wrap[i] ? iw : 0);
      xe[i] = ld_int<Tin>(x, ext[i] ? ie : 0);
      xs[i] = ld_int<Tin>(x, ext[i] ? s : 0);
      if (sfold) val[i] -= bias + (s < rho ? 128 : 0);
    }
#pragma unroll
    for (int i = 0; i < U; ++i) {
      int v = in[i] ? val[i] : 0;
      v += (wrap[i] ? xw[i] : 0) + (ext[i] ? xe[i] - xs[i] : 0);
      val[i] = v;
      mx = max(mx, v < 0 ? -v : v);
    }
#pragma unroll
    for (int i = 0; i < U; ++i) {
      const int u = eb + i * kCgPrepThreads;
      if (u >= e1) break;
      if (dy && in[i]) G(dy)[u] = (double)val[i];
      int v = val[i];
      for (int l = 0; l < nlc; ++l) {
        const int t = v + 64;                       // balanced base-128 digit
        limb[(int64_t)l * lp + u] = (int8_t)((t & 127) - 64);
        v = t >> 7;
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    int m = wmax[0];
    for (int w = 1; w < kCgPrepThreads / 64; ++w) m = max(m, wmax[w]);
    if (m) __hip_atomic_fetch_max(G(d.cmax) + f, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// the loop without int64 remainders (no branches between an entry's loads)
// unless N < M, where a fold's indices can wrap more than once
__device__ __forceinline__ void cg_prep_dispatch(const Inst& d, int f, int e0, int chunk) {
  if (e0 >= d.c_lp) return;
  if (d.n < (int64_t)max(d.va.m, d.vb.m)) {
    switch (d.x_dtype) {
      case TM_I8: cg_prep_chunk<int8_t, true>(d, f, e0, chunk); break;
      case TM_F32: cg_prep_chunk<float, true>(d, f, e0, chunk); break;
      case TM_BF16: cg_prep_chunk<bf16_t, true>(d, f, e0, chunk); break;
      default: cg_prep_chunk<f16_t, true>(d, f, e0, chunk); break;
    }
    return;
  }
  switch (d.x_dtype) {
    case TM_I8: cg_prep_chunk<int8_t, false>(d, f, e0, chunk); break;
    case TM_F32: cg_prep_chunk<float, false>(d, f, e0, chunk); break;
    case TM_BF16: cg_prep_chunk<bf16_t, false>(d, f, e0, chunk); break;
    default: cg_prep_chunk<f16_t, false>(d, f, e0, chunk); break;
  }
}

// grid (instances, 2 x chunks per fold): blockIdx.x picks the instance from
// the list; the first half of blockIdx.y covers fold A, the second fold B,
// `chunk` entries each
__global__ void __launch_bounds__(kCgPrepThreads) k_cgemm_prep(InstTable tab, const int32_t* list, int chunk) {
  const int cpf = gridDim.y >> 1;
  const int f = (int)blockIdx.y >= cpf ? 1 : 0;
  const int e0 = ((int)blockIdx.y - f * cpf) * chunk;
  if (list) cg_prep_dispatch(tab.table[list[blockIdx.x]], f, e0, chunk);
  else cg_prep_dispatch(tab.resident(), f, e0, chunk);
}

// The W parts of a workgroup's 16 x 64 tile summed in LDS (int64; with 8
// waves, waves 4..7 first hand their parts to waves 0..3 through the same
// 32 KiB), then the intermediates and wave nt's best shift of column tile nt;
// or, when several workgroups share the band, the sum added into the fold's
// accumulators for the final kernel.
template <int NL, int W>
__device__ __forceinline__ void cg_finish_rows(const Inst& d, int f, int rt, int M, const v4i_t (&acc)[NL][4],
                                               long long* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = lane & 15, g = lane >> 4;
  // digits to int64
  long long part[4][4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      long long r = 0, wt = 1;
#pragma unroll
      for (int l = 0; l < NL; ++l) { r += wt * (long long)acc[l][nt][jj]; wt *= 128; }
      part[nt][jj] = r;
    }
  if constexpr (W == 8) {
    if (w >= 4)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) red[(((w - 4) * 4 + nt) * 4 + jj) * 64 + lane] = part[nt][jj];
    __syncthreads();
    if (w < 4)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) part[nt][jj] += red[((w * 4 + nt) * 4 + jj) * 64 + lane];
    __syncthreads();
  }
  // waves 0..3: their parts into LDS, red[w][nt][jj][lane]
  if (w < 4)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) red[((w * 4 + nt) * 4 + jj) * 64 + lane] = part[nt][jj];
  __syncthreads();
  if (w >= 4) return;
  // wave w owns column tile nt = w: lane holds rows 4 g + jj, column c
  const int nt = w;
  if (d.c_split > 1) {   // this workgroup's share of the band, added into r (exact int64)
    long long* ca = d.cacc + (f ? d.va.m : 0);
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      long long r = 0;
#pragma unroll
      for (int ww = 0; ww < 4; ++ww) r += red[((ww * 4 + nt) * 4 + jj) * 64 + lane];
      const int k = 64 * (kCgRows * rt + 4 * g + jj) + 16 * nt + c;
      if (k < M && r != 0)
        __hip_atomic_fetch_add(G(ca + k), r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  double* dr = (f != d.swapped) ? d.dbg_r2 : d.dbg_r1;
  VI best{-INFINITY, 0x7fffffff};
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) {
    long long r = 0;
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) r += red[((ww * 4 + nt) * 4 + jj) * 64 + lane];
    const int k = 64 * (kCgRows * rt + 4 * g + jj) + 16 * nt + c;
    if (k < M) {
      if (dr) G(dr)[k] = (double)r;
      if (d.rtop) G(d.rtop)[(f ? d.va.m : 0) + k] = (double)r;
      if (vi_better(VI{(double)r, k}, best)) best = VI{(double)r, k};
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const VI other{__shfl_xor(best.v, o), __shfl_xor(best.i, o)};
    if (vi_better(other, best)) best = other;
  }
  if (lane == 0) {
    const int rtm = max(d.c_rta, d.c_rtb);
    double* pp = reinterpret_cast<double*>(d.cpart) + ((int64_t)(f * rtm + rt) * 4 + nt) * 2;
    G(pp)[0] = best.v;
    G(pp)[1] = (double)best.i;
  }
}

// One workgroup: rows 16 rt .. 16 rt + 15 (64 shifts each) of fold f.  Wave w
// of W takes a contiguous share of the band's steps for all four 16-column
// tiles; the shares are summed in LDS (int64) and wave nt then keeps the best
// of column tile nt.  8 waves halve each wave's chain of dependent steps for
// launches of few instances.
template <int NL, int W>
__device__ __forceinline__ void cg_gemm_rows(const Inst& d, int f, int rt, int part, long long* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int M = f ? d.vb.m : d.va.m;
  const int lp = d.c_lp, KS = d.c_ks;
  // this workgroup's share [lo, hi) of the band's steps, then the wave's
  const int split = max(d.c_split, 1);
  const int lo = (int)((int64_t)KS * part / split), hi = (int)((int64_t)KS * (part + 1) / split);
  const int qw = (hi - lo + W - 1) / W;
  const int st0 = lo + min(w * qw, hi - lo);
  const int q = max(0, min(qw, hi - st0));   // this wave's steps (may be 0)
  // operands as in cgw_tile: buffer loads at fixed per-lane offsets (the
  // template copies interleaved by 16-byte chunk, chunk m of copy sh at
  // (16 m + sh) * 16, so the 16 lanes of a column tile read neighbouring
  // chunks) with per-step scalar offsets, steps in pairs over two register
  // sets; loads past the wave's share read the last step again, unused
  const __amdgpu_buffer_rsrc_t ra =
      uniform_rsrc(d.ylimb + (int64_t)f * d.c_nlcap * lp, (uint32_t)(d.c_nlcap * lp));
  const __amdgpu_buffer_rsrc_t rb = uniform_rsrc(d.tsh, (uint32_t)(16 * d.c_lt));
  const int aoff = 64 * (kCgRows * rt + c) + 16 * g;
  int boff[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int j0 = 16 * g - (16 * nt + c) + kCgPad;
    boff[nt] = (j0 + 2 * ((-j0) & 15)) * 16;
  }
  auto load = [&](int st, v4i_t (&b)[4], v4i_t (&a)[NL]) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) b[nt] = buf_v4i(rb, boff[nt], 1024 * st);
#pragma unroll
    for (int l = 0; l < NL; ++l) a[l] = buf_v4i(ra, aoff, l * lp + 64 * st);
  };
  v4i_t acc[NL][4];
#pragma unroll
  for (int l = 0; l < NL; ++l)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[l][nt] = v4i_t{0, 0, 0, 0};
  auto mfma = [&](const v4i_t (&b)[4], const v4i_t (&a)[NL]) {
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[l][nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[l], b[nt], acc[l][nt], 0, 0, 0);
  };
  v4i_t b0[4], a0[NL], b1[4], a1[NL];
  load(min(st0, KS - 1), b0, a0);
  for (int i = 0; i < q; i += 2) {
    load(min(st0 + i + 1, KS - 1), b1, a1);
    mfma(b0, a0);
    load(min(st0 + i + 2, KS - 1), b0, a0);
    if (i + 1 < q) mfma(b1, a1);             // uniform over the wave
  }
  cg_finish_rows<NL, W>(d, f, rt, M, acc, red);
}

// MAXNL: largest digit count this variant is built for (register budget:
// the int8 signals need at most 3 digits and run on the narrow variant with
// more waves per SIMD)
template <int MAXNL, int W>
__device__ __forceinline__ void cg_gemm_dispatch(const Inst& d, int task, long long* red) {
  const int ntask = d.c_rta + d.c_rtb;
  if (task >= ntask * max(d.c_split, 1)) return;
  const int part = task / ntask;
  task -= part * ntask;
  const int f = task >= d.c_rta ? 1 : 0;
  const int rt = task - f * d.c_rta;
  const int nl = min(min(cg_limbs(G(d.cmax)[f]), d.c_nlcap), MAXNL);
  switch (nl) {
    case 1: cg_gemm_rows<1, W>(d, f, rt, part, red); break;
    case 2: cg_gemm_rows<2, W>(d, f, rt, part, red); break;
    case 3: cg_gemm_rows<3, W>(d, f, rt, part, red); break;
    case 4: if constexpr (MAXNL >= 4) cg_gemm_rows<4, W>(d, f, rt, part, red); break;
    default: if constexpr (MAXNL >= 5) cg_gemm_rows<5, W>(d, f, rt, part, red); break;
  }
}

// grid (instances, row-tile tasks of both folds), W waves per workgroup
template <int MAXNL, int W>
__global__ void __launch_bounds__(64 * W) k_cgemm(InstTable tab, const int32_t* list) {
  __shared__ long long red[4 * 4 * 4 * 64];
  if (list) cg_gemm_dispatch<MAXNL, W>(tab.table[list[blockIdx.x]], blockIdx.y, red);
  else cg_gemm_dispatch<MAXNL, W>(tab.resident(), blockIdx.y, red);
}

// LEAN: int8 signal and template, one workgroup per band, no top-T (the
// common batch; fewer registers, so more workgroups resident).  YP_DONE: the
// product kernel has already returned the bucket zone to zero.
template <typename Tin, bool LEAN = false, bool YP_DONE = false>
__device__ __forceinline__ void cg_final(const Inst& d) {
  __shared__ __align__(16) unsigned char scratch[16 * 16];
  __shared__ VI fin[2];
  __shared__ VI wbest[4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (!LEAN && d.c_split > 1) {
    // split band: r of each fold from the accumulators (cleared as read)
    for (int f = 0; f < 2; ++f) {
      const int M = f ? d.vb.m : d.va.m;
      long long* ca = d.cacc + (f ? d.va.m : 0);
      double* dr = (f != d.swapped) ? d.dbg_r2 : d.dbg_r1;
      VI best{-INFINITY, 0x7fffffff};
      // 16 loads per thread in flight before any is used
      constexpr int kB = 16;
      for (int base = 0; base < M; base += kB * (int)blockDim.x) {
        long long v[kB];
#pragma unroll
        for (int b = 0; b < kB; ++b) {
          const int k = base + b * (int)blockDim.x + (int)threadIdx.x;
          v[b] = k < M ? G(ca)[k] : 0;
        }
#pragma unroll
        for (int b = 0; b < kB; ++b) {
          const int k = base + b * (int)blockDim.x + (int)threadIdx.x;
          if (k < M) {
            G(ca)[k] = 0;
            if (dr) G(dr)[k] = (double)v[b];
            if (d.rtop) G(d.rtop)[(f ? d.va.m : 0) + k] = (double)v[b];
            if (vi_better(VI{(double)v[b], k}, best)) best = VI{(double)v[b], k};
          }
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const VI other{__shfl_xor(best.v, o), __shfl_xor(best.i, o)};
        if (vi_better(other, best)) best = other;
      }
      if (lane == 0) wbest[wave] = best;
      __syncthreads();
      if (threadIdx.x == 0) {
        VI b = wbest[0];
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i)
          if (vi_better(wbest[i], b)) b = wbest[i];
        fin[f] = b;
      }
      __syncthreads();
    }
  } else if (wave < 2) {
    const int f = wave;
    const int n = (f ? d.c_rtb : d.c_rta) * 4;
    const int rtm = max(d.c_rta, d.c_rtb);
    const double* pp = reinterpret_cast<const double*>(d.cpart) + (int64_t)f * rtm * 4 * 2;
    VI best{-INFINITY, 0x7fffffff};
    for (int i = lane; i < n; i += 64) {
      const VI v{G(pp)[2 * i], (int)G(pp)[2 * i + 1]};
      if (vi_better(v, best)) best = v;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const VI other{__shfl_xor(best.v, o), __shfl_xor(best.i, o)};
      if (vi_better(other, best)) best = other;
    }
    if (lane == 0) fin[f] = best;
  }
  // the buckets and the fold maxima have been consumed: back to zero
  if constexpr (!YP_DONE) {
    const int nz = d.va.m + d.vb.m;
    for (int s = threadIdx.x; s < nz; s += blockDim.x) G(d.yp)[s] = 0;
  }
  if (threadIdx.x < 2) G(d.cmax)[threadIdx.x] = 0;
  __syncthreads();
  if (!LEAN && d.top_t > 1) resolve_top_t<Tin>(d, fin[0], fin[1], TM_R_EXACT, scratch);
  else resolve_and_report<Tin, LEAN>(d, fin[0], fin[1], TM_R_EXACT, scratch);
}

__device__ __forceinline__ void cg_final_dispatch(const Inst& d) {
  switch (d.x_dtype) {
    case TM_I8: cg_final<int8_t>(d); break;
    case TM_F32: cg_final<float>(d); break;
    case TM_BF16: cg_final<bf16_t>(d); break;
    default: cg_final<f16_t>(d); break;
  }
}

template <bool LEAN, bool YP_DONE>
__global__ void __launch_bounds__(256) k_cgemm_final(InstTable tab, const int32_t* list) {
  const Inst& d = list ? tab.table[list[blockIdx.x]] : tab.resident();
  if constexpr (LEAN) cg_final<int8_t, true, YP_DONE>(d);
  else cg_final_dispatch(d);
}

// --------------------------------------------------------------------------
// the same product for batches: one wave per row tile
// --------------------------------------------------------------------------
//
// Each wave computes one 16 x 64 row tile of one fold over the whole band
// (all steps, every digit, the four column tiles) and writes the best of each
// column tile to cpart, so no partial sums meet across waves; the four waves
// of a workgroup take consecutive row tiles of one instance, which read the
// same template copies through the compute unit's cache.  For batches, whose
// many row tiles fill the machine without splitting a band over waves.

template <int NL>
__device__ __forceinline__ void cg2_report(const Inst& d, int f, int rt, const int* red, const v4i_t (&acc)[NL][4],
                                           VI* tbest);

// One wave: row tile rt of fold f over the whole band.  Every operand load is
// a buffer load at a fixed per-lane offset plus a per-step scalar offset: B
// chunk (step st, column tile nt) sits at 1024 st + boff[nt] in the template
// copies (the copy shift of 64 st + j0 is the one of j0, since 64 st is a
// multiple of 16), and digit l of A at l lp + 64 st + aoff.  The steps go in
// pairs through two register sets (c_ks is a multiple of 4), so no register
// moves separate the loads from the products.
template <int NL>
__device__ __forceinline__ void cgw_tile(const Inst& d, int f, int rt) {
  const int lane = threadIdx.x & 63;
  const int c = lane & 15, g = lane >> 4;
  const int M = f ? d.vb.m : d.va.m;
  const int ntc = min(4, (M - 1024 * rt + 15) >> 4);
  const int lp = d.c_lp, KS = d.c_ks;
  const __amdgpu_buffer_rsrc_t ra =
      uniform_rsrc(d.ylimb + (int64_t)f * d.c_nlcap * lp, (uint32_t)(d.c_nlcap * lp));
  const __amdgpu_buffer_rsrc_t rb = uniform_rsrc(d.tsh, (uint32_t)(16 * d.c_lt));
  const int aoff = 64 * (kCgRows * rt + c) + 16 * g;
  int boff[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int j0 = 16 * g - (16 * nt + c) + kCgPad;
    boff[nt] = (j0 + 2 * ((-j0) & 15)) * 16;
  }
  auto load = [&](int st, v4i_t (&b)[4], v4i_t (&a)[NL]) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) b[nt] = buf_v4i(rb, boff[nt], 1024 * st);
#pragma unroll
    for (int l = 0; l < NL; ++l) a[l] = buf_v4i(ra, aoff, l * lp + 64 * st);
  };
  v4i_t acc[NL][4];
#pragma unroll
  for (int l = 0; l < NL; ++l)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[l][nt] = v4i_t{0, 0, 0, 0};
  auto mfma = [&](const v4i_t (&b)[4], const v4i_t (&a)[NL]) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      if (nt < ntc) {                         // uniform over the wave
#pragma unroll
        for (int l = 0; l < NL; ++l)
          acc[l][nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[l], b[nt], acc[l][nt], 0, 0, 0);
      }
    }
  };
  v4i_t b0[4], a0[NL], b1[4], a1[NL];
  load(0, b0, a0);
  for (int st = 0; st < KS; st += 2) {
    // the other set's step is in flight during each set's products; the last
    // pass reloads the final step into set 0 (unused)
    load(st + 1, b1, a1);
    mfma(b0, a0);
    load(min(st + 2, KS - 1), b0, a0);
    mfma(b1, a1);
  }
  cg2_report<NL>(d, f, rt, nullptr, acc, nullptr);
}

// grid (instances, groups of four row tiles), one row tile per wave
template <int MAXNL>
__global__ void __launch_bounds__(256) k_cgemm_wave(InstTable tab, const int32_t* list) {
  const Inst& d = list ? tab.table[list[blockIdx.x]] : tab.resident();
  const int task = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (task >= d.c_rta + d.c_rtb) return;          // no barriers in this kernel
  const int f = task >= d.c_rta ? 1 : 0;
  const int rt = task - f * d.c_rta;
  const int nl = min(min(cg_limbs(G(d.cmax)[f]), d.c_nlcap), MAXNL);
  switch (nl) {
    case 1: cgw_tile<1>(d, f, rt); break;
    case 2: cgw_tile<2>(d, f, rt); break;
    case 3: cgw_tile<3>(d, f, rt); break;
    case 4: if constexpr (MAXNL >= 4) cgw_tile<4>(d, f, rt); break;
    default: if constexpr (MAXNL >= 5) cgw_tile<5>(d, f, rt); break;
  }
}

// The same product with both operands staged in LDS rings a phase ahead of
// their use.  The template copies (B) are read alike by the four waves of a
// workgroup (row tiles of one instance) and are staged once per workgroup;
// each wave's digit rows (A) slide by one row per step, so a wave stages
// only the 4 new rows of each digit per phase.  Fetching both straight from
// memory every step left each wave waiting on its loads (the matrix cores
// ran at about a quarter of their rate).
//
// B: step st reads bytes 1024 st + boff (boff in [1040, 3312)) of the
// copies, i.e. 1 KiB blocks st+1 .. st+3; block b sits in slot b mod 16.
// The prologue stages blocks 0 .. 11; phase p (steps 4p .. 4p+3, plus the
// early read of step 4p+4) reads blocks up to 4p+7 while the workgroup
// fetches blocks 4p+12 .. 4p+15, writes them at the end of the phase (their
// slots last held blocks up to 4p-1) and meets at one barrier.
// A: lane (c, g) of step st reads row R0 + c + st (R0 = 16 rt), bytes 16 g ..
// 16 g + 15, of each digit row; row r sits in slot r mod 32 of the wave's
// ring for that digit.  The prologue stages rows R0 .. R0+31; phase p reads
// rows up to R0+4p+19 while the wave fetches rows R0+4p+32 .. R0+4p+35 and
// writes them at the end of the phase over rows R0+4p .. R0+4p+3.
// Every wave reads one contiguous KiB per operand tile, so the LDS reads are
// free of bank conflicts.  Waves past the instance's row tiles take part in
// the staging of B and the barriers only.
constexpr int kRingB = 16;             // B slots of 1 KiB
constexpr int kRingA = 32;             // A slots of one 64-byte row per digit
constexpr int kRingPhase = 4;          // steps per phase (c_ks is a multiple of 4)
constexpr int kRingMaxNL = 3;
constexpr int kRingLds = kRingB * 1024 + 4 * kRingMaxNL * kRingA * 64;

template <int NL>
__device__ __forceinline__ void cgr_tile(const Inst& d, int task, int ntask, unsigned char* lds) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const bool active = task < ntask;                // uniform over the wave
  const int f = task >= d.c_rta ? 1 : 0;
  const int rt = task - f * d.c_rta;
  const int M = f ? d.vb.m : d.va.m;
  const int ntc = active ? min(4, (M - 1024 * rt + 15) >> 4) : 0;
  const int lp = d.c_lp, KS = d.c_ks;
  const int R0 = kCgRows * rt;
  const __amdgpu_buffer_rsrc_t ra =
      uniform_rsrc(d.ylimb + (int64_t)f * d.c_nlcap * lp, (uint32_t)(d.c_nlcap * lp));
  const __amdgpu_buffer_rsrc_t rb = uniform_rsrc(d.tsh, (uint32_t)(16 * d.c_lt));
  unsigned char* ringb = lds;
  unsigned char* ringa = lds + kRingB * 1024 + w * (kRingMaxNL * kRingA * 64);
  int boff[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int j0 = 16 * g - (16 * nt + c) + kCgPad;
    boff[nt] = (j0 + 2 * ((-j0) & 15)) * 16;
  }
  // prologue: B blocks 0 .. 11 (three 4 KiB rounds of the workgroup), A rows
  // R0 .. R0+31 of each digit (two 1 KiB rounds of the wave)
  {
    v4i_t vb[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) vb[r] = buf_v4i(rb, 16 * tid, 4096 * r);
    v4i_t va[NL][2];
    if (active)
#pragma unroll
      for (int l = 0; l < NL; ++l)
#pragma unroll
        for (int q = 0; q < 2; ++q) va[l][q] = buf_v4i(ra, 16 * lane, l * lp + 64 * R0 + 1024 * q);
#pragma unroll
    for (int r = 0; r < 3; ++r) *reinterpret_cast<v4i_t*>(ringb + 4096 * r + 16 * tid) = vb[r];
    if (active)
#pragma unroll
      for (int l = 0; l < NL; ++l)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int row = R0 + 16 * q + (lane >> 2);
          *reinterpret_cast<v4i_t*>(ringa + l * (kRingA * 64) + ((row & (kRingA - 1)) << 6) + 16 * (lane & 3)) =
              va[l][q];
        }
  }
  __syncthreads();
  v4i_t acc[NL][4];
#pragma unroll
  for (int l = 0; l < NL; ++l)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[l][nt] = v4i_t{0, 0, 0, 0};
  auto read_a = [&](int st, v4i_t (&a)[NL]) {
    const int off = (((R0 + c + st) & (kRingA - 1)) << 6) + 16 * g;
#pragma unroll
    for (int l = 0; l < NL; ++l) a[l] = *reinterpret_cast<const v4i_t*>(ringa + l * (kRingA * 64) + off);
  };
  auto read_b = [&](int st, v4i_t (&b)[4]) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
      b[nt] = *reinterpret_cast<const v4i_t*>(ringb + ((1024 * st + boff[nt]) & (kRingB * 1024 - 1)));
  };
  auto step = [&](const v4i_t (&a)[NL], const v4i_t (&b)[4]) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      if (nt < ntc) {                              // uniform over the wave
#pragma unroll
        for (int l = 0; l < NL; ++l)
          acc[l][nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[l], b[nt], acc[l][nt], 0, 0, 0);
      }
    }
  };
  // the operands of the next step are read while the products of the
  // current one run: two register sets, steps in pairs
  v4i_t a0[NL], a1[NL], b0[4], b1[4];
  if (active) {
    read_a(0, a0);
    read_b(0, b0);
  }
  for (int p0 = 0; p0 < KS; p0 += kRingPhase) {
    // B blocks p0+12 .. p0+15 (one 4 KiB round); A rows R0+p0+32 .. +35
    const v4i_t nb = buf_v4i(rb, 16 * tid, 1024 * (p0 + 12));
    int na[NL];
    if (active)
#pragma unroll
      for (int l = 0; l < NL; ++l)
        na[l] = (int)__builtin_amdgcn_raw_buffer_load_b32(ra, 4 * lane, l * lp + 64 * (R0 + p0 + 32), 0);
    if (active) {
#pragma unroll
      for (int st = p0; st < p0 + kRingPhase; st += 2) {
        read_a(st + 1, a1);
        read_b(st + 1, b1);
        step(a0, b0);
        const int sn = min(st + 2, KS - 1);
        read_a(sn, a0);
        read_b(sn, b0);
        step(a1, b1);
      }
    }
    *reinterpret_cast<v4i_t*>(ringb + (((p0 + 12) & (kRingB - 1)) << 10) + 16 * tid) = nb;
    if (active) {
      const int row = R0 + p0 + 32 + (lane >> 4);
#pragma unroll
      for (int l = 0; l < NL; ++l)
        *reinterpret_cast<int*>(ringa + l * (kRingA * 64) + ((row & (kRingA - 1)) << 6) + 4 * (lane & 15)) = na[l];
    }
    __syncthreads();
  }
  if (active) cg2_report<NL>(d, f, rt, nullptr, acc, nullptr);
}

// grid (instances, groups of four row tiles); one row tile per wave, the
// digit count of the group's folds taken for all four waves (the extra
// digits of a fold that needs fewer are zero rows).  Four waves per SIMD
// (128 registers; the LDS allows four workgroups per compute unit): the
// kernel waits on latency, and the fourth wave is worth more than the few
// spilled registers of the three-digit variant.
template <int MAXNL>
__global__ void __launch_bounds__(256, 4) k_cgemm_ring(InstTable tab, const int32_t* list) {
  static_assert(MAXNL <= kRingMaxNL, "ring sized for three digits");
  __shared__ __align__(16) unsigned char lds[kRingLds];
  const Inst& d = list ? tab.table[list[blockIdx.x]] : tab.resident();
  const int ntask = d.c_rta + d.c_rtb;
  const int t0 = blockIdx.y * 4;
  if (t0 >= ntask) return;                         // the whole workgroup
  const int t1 = min(t0 + 3, ntask - 1);
  const int f0 = t0 >= d.c_rta ? 1 : 0, f1 = t1 >= d.c_rta ? 1 : 0;
  const int mx = max(G(d.cmax)[f0], G(d.cmax)[f1]);
  const int nl = min(min(cg_limbs(mx), d.c_nlcap), MAXNL);
  const int task = __builtin_amdgcn_readfirstlane(t0 + (int)(threadIdx.x >> 6));
  switch (nl) {
    case 1: cgr_tile<1>(d, task, ntask, lds); break;
    case 2: cgr_tile<2>(d, task, ntask, lds); break;
    default: cgr_tile<3>(d, task, ntask, lds); break;
  }
  // the instance's bucket zone has been consumed (by the prep kernel): the
  // first workgroup returns it to zero here, where the stores overlap the
  // other workgroups' products, instead of in the final kernel
  if (blockIdx.y == 0) {
    const int nz = d.va.m + d.vb.m;
    for (int s = threadIdx.x; s < nz; s += blockDim.x) G(d.yp)[s] = 0;
  }
}

hipError_t launch_cgemm_ring(const InstTable& tab, const int32_t* list, int count, int gemm_y, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  TM_LAUNCH(k_cgemm_ring<3>, dim3(count, (gemm_y + 3) / 4), dim3(256), 0, s, tab, list);
  return hipGetLastError();
}

hipError_t launch_cgemm_wave(const InstTable& tab, const int32_t* list, int count, int gemm_y, int max_limbs,
                             hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const dim3 grid(count, (gemm_y + 3) / 4);
  if (max_limbs <= 3) TM_LAUNCH(k_cgemm_wave<3>, grid, dim3(256), 0, s, tab, list);
  else TM_LAUNCH(k_cgemm_wave<5>, grid, dim3(256), 0, s, tab, list);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// the same product for batches: one workgroup per instance, operands in LDS
// --------------------------------------------------------------------------
//
// A workgroup of kCg2Waves waves owns one instance: it stages the 16 shifted
// template copies (the interleaved layout above) and the digit rows the prep
// kernel wrote in LDS once, then every wave computes whole 16 x 64 row tiles
// (all four column tiles, every digit, the whole band) from LDS, so the
// template is read from memory once per instance rather than once per row
// tile and the B operand of each step serves all digits of its row tile; the
// same workgroup then takes both argmaxes and resolves (no final kernel, no
// partials in memory).  When an
// instance has fewer row tiles than waves, the band's steps are split over
// P = kCg2Waves / tiles waves per tile and their digit sums meet in an LDS
// int32 buffer (each digit's full sum fits int32: |d| <= 64, |t| <= 128,
// K <= 2^17).  The digit rows sit in LDS with 16 pad bytes after every 256,
// so the 16 rows of an A operand (64 bytes apart) fall in distinct banks.
// Each (fold, row tile) keeps the best (value, lowest shift) of each column
// tile in LDS.

__host__ __device__ __forceinline__ int cg2_pad(int b) { return b + ((b >> 8) << 4); }   // padded LDS offset

// digit sums of a finished tile (registers, or the split band's LDS
// accumulators) to r (int64), the intermediates, and the best of each column
// tile into `tbest` (LDS), or into cpart when tbest is null (lane layout of
// the MFMA result: rows 4 g + jj, column c)
template <int NL>
__device__ __forceinline__ void cg2_report(const Inst& d, int f, int rt, const int* red,
                                           const v4i_t (&acc)[NL][4], VI* tbest) {
  const int lane = threadIdx.x & 63;
  const int c = lane & 15, g = lane >> 4;
  const int M = f ? d.vb.m : d.va.m;
  double* dr = (f != d.swapped) ? d.dbg_r2 : d.dbg_r1;
  const int rtm = max(d.c_rta, d.c_rtb);
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    VI best{-INFINITY, 0x7fffffff};
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      long long r = 0, wt = 1;
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        const int v = red ? red[((l * 4 + nt) * 4 + jj) * 64 + lane] : acc[l][nt][jj];
        r += wt * (long long)v;
        wt *= 128;
      }
      const int k = 64 * (kCgRows * rt + 4 * g + jj) + 16 * nt + c;
      if (k < M) {
        if (dr) G(dr)[k] = (double)r;
        if (d.rtop) G(d.rtop)[(f ? d.va.m : 0) + k] = (double)r;
        if (vi_better(VI{(double)r, k}, best)) best = VI{(double)r, k};
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const VI other{__shfl_xor(best.v, o), __shfl_xor(best.i, o)};
      if (vi_better(other, best)) best = other;
    }
    if (lane == 0) {
      if (tbest) {
        tbest[(f * rtm + rt) * 4 + nt] = best;
      } else {
        double* pp = reinterpret_cast<double*>(d.cpart) + ((int64_t)(f * rtm + rt) * 4 + nt) * 2;
        G(pp)[0] = best.v;
        G(pp)[1] = (double)best.i;
      }
    }
  }
}

// One wave: row tile rt of fold f over the band's steps [s0, s1), every
// digit and column tile, operands from LDS (`lb`: template copies; `la`: the
// padded digit rows, this fold's digit l at row row0 + l).  With `red` (the
// tile's own block of accumulators, 1024 ints per digit) the sums go there,
// else straight to the report.
template <int NL>
__device__ __forceinline__ void cg2_tile(const Inst& d, const unsigned char* lb, const unsigned char* la, int row0,
                                         int f, int rt, int s0, int s1, int* red, VI* tbest) {
  const int lane = threadIdx.x & 63;
  const int c = lane & 15, g = lane >> 4;
  const int M = f ? d.vb.m : d.va.m;
  // column tiles that hold a shift below M (the last row tile of a fold may need fewer)
  const int ntc = min(4, (M - 1024 * rt + 15) >> 4);
  const int lp = d.c_lp;
  const int abase = row0 * lp + 64 * (kCgRows * rt + c) + 16 * g;   // this lane's A bytes at step 0, digit 0
  v4i_t acc[NL][4];
#pragma unroll
  for (int l = 0; l < NL; ++l)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[l][nt] = v4i_t{0, 0, 0, 0};
  auto ld_b = [&](int st, int nt) {
    const int j = 64 * st + 16 * g - (16 * nt + c) + kCgPad;
    const int sh = (-j) & 15;
    return *reinterpret_cast<const v4i_t*>(lb + (((j + sh) >> 4) * 16 + sh) * 16);
  };
  auto ld_a = [&](int st, int l) {
    return *reinterpret_cast<const v4i_t*>(la + cg2_pad(abase + l * lp + 64 * st));
  };
  if (s1 > s0) {
    v4i_t bc[4], ac[NL];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) bc[nt] = ld_b(s0, nt);
#pragma unroll
    for (int l = 0; l < NL; ++l) ac[l] = ld_a(s0, l);
    for (int st = s0; st < s1; ++st) {
      // the next step's operands are read while this step's products run
      v4i_t bn[4], an[NL];
      const int sn = min(st + 1, s1 - 1);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) bn[nt] = ld_b(sn, nt);
#pragma unroll
      for (int l = 0; l < NL; ++l) an[l] = ld_a(sn, l);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        if (nt < ntc) {                       // uniform over the wave
#pragma unroll
          for (int l = 0; l < NL; ++l)
            acc[l][nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ac[l], bc[nt], acc[l][nt], 0, 0, 0);
        }
      }
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) bc[nt] = bn[nt];
#pragma unroll
      for (int l = 0; l < NL; ++l) ac[l] = an[l];
    }
  }
  if (red) {   // a share of the band: digit sums into the tile's LDS accumulators
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          atomicAdd(red + ((l * 4 + nt) * 4 + jj) * 64 + lane, acc[l][nt][jj]);
  } else {
    cg2_report<NL>(d, f, rt, nullptr, acc, tbest);
  }
}

__device__ __forceinline__ void cg2_dispatch_task(int nl, const Inst& d, const unsigned char* lb,
                                                  const unsigned char* la, int row0, int f, int rt, int s0, int s1,
                                                  int* red, VI* tbest) {
  switch (nl) {
    case 1: cg2_tile<1>(d, lb, la, row0, f, rt, s0, s1, red, tbest); break;
    case 2: cg2_tile<2>(d, lb, la, row0, f, rt, s0, s1, red, tbest); break;
    case 3: cg2_tile<3>(d, lb, la, row0, f, rt, s0, s1, red, tbest); break;
    case 4: cg2_tile<4>(d, lb, la, row0, f, rt, s0, s1, red, tbest); break;
    default: cg2_tile<5>(d, lb, la, row0, f, rt, s0, s1, red, tbest); break;
  }
}

__device__ __forceinline__ void cg2_dispatch_report(int nl, const Inst& d, int f, int rt, const int* red, VI* tbest) {
  switch (nl) {
    case 1: { v4i_t a[1][4]; cg2_report<1>(d, f, rt, red, a, tbest); break; }
    case 2: { v4i_t a[2][4]; cg2_report<2>(d, f, rt, red, a, tbest); break; }
    case 3: { v4i_t a[3][4]; cg2_report<3>(d, f, rt, red, a, tbest); break; }
    case 4: { v4i_t a[4][4]; cg2_report<4>(d, f, rt, red, a, tbest); break; }
    default: { v4i_t a[5][4]; cg2_report<5>(d, f, rt, red, a, tbest); break; }
  }
}

// LDS of one instance: template copies, both folds' padded digit rows (nlcap
// each), the split-band accumulators, and the best entry of every column tile
__host__ __device__ inline size_t cg2_lds_bytes(int c_lt, int c_lp, int nlcap, int tasks, int rtm) {
  const size_t b = (size_t)16 * c_lt;
  const size_t a = ((size_t)cg2_pad(2 * nlcap * c_lp) + 15) & ~(size_t)15;
  const size_t red = kCg2Waves / tasks > 1 ? (size_t)tasks * nlcap * 4 * 4 * 64 * 4 : 0;
  return b + a + red + (size_t)2 * rtm * 4 * sizeof(VI);
}

// Global -> LDS copy of `n` 16-byte chunks, eight loads in flight per thread
// before their stores (the workgroup's copies overlap their latencies)
template <typename Dst>
__device__ __forceinline__ void cg2_stage(uintptr_t src, int n, Dst dst_of) {
  constexpr int U = 8;
  const int tid = threadIdx.x, NT = blockDim.x;
  for (int base = 0; base < n; base += U * NT) {
    uint4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * NT + tid;
      if (i < n) v[u] = gload16(src + (uintptr_t)i * 16);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * NT + tid;
      if (i < n) *reinterpret_cast<uint4*>(dst_of(i)) = v[u];
    }
  }
}

// One workgroup does the product, both argmaxes and the resolve of one
// instance (Algorithm 1 steps 4-9) from the digit rows the prep kernel wrote:
// template copies and digit rows into LDS, the row tiles, the argmaxes from
// the per-column-tile bests in LDS, the buckets and fold maxima back to zero,
// and the resolve with its re-score.
template <typename Tin>
__device__ __forceinline__ void cg2_instance(const Inst& d, unsigned char* lds) {
  __shared__ VI fin[2];
  __shared__ __align__(16) unsigned char scratch[16 * 16];
  const int tid = threadIdx.x, NT = blockDim.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int lt = d.c_lt, lp = d.c_lp, nlcap = d.c_nlcap;
  const int ma = d.va.m, mb = d.vb.m;
  const int rtm = max(d.c_rta, d.c_rtb);
  const int ntask = d.c_rta + d.c_rtb;
  const int parts = ntask < kCg2Waves ? kCg2Waves / ntask : 1;
  unsigned char* lb = lds;
  unsigned char* la = lds + (size_t)16 * lt;
  const size_t a_bytes = ((size_t)cg2_pad(2 * nlcap * lp) + 15) & ~(size_t)15;
  int* red = parts > 1 ? reinterpret_cast<int*>(la + a_bytes) : nullptr;
  VI* tbest = reinterpret_cast<VI*>(la + a_bytes + (parts > 1 ? (size_t)ntask * nlcap * 4 * 4 * 64 * 4 : 0));
  int nl[2];
  nl[0] = min(cg_limbs(G(d.cmax)[0]), nlcap);
  nl[1] = min(cg_limbs(G(d.cmax)[1]), nlcap);
  // the 16 template copies (contiguous), then the digit rows in use: fold f's
  // digit l at padded LDS row f nlcap + l
  cg2_stage(reinterpret_cast<uintptr_t>(d.tsh), lt, [&](int i) { return lb + (size_t)i * 16; });
  const int cpr = lp >> 4;
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    const uintptr_t src = reinterpret_cast<uintptr_t>(d.ylimb + (int64_t)f * nlcap * lp);
    cg2_stage(src, nl[f] * cpr, [&](int i) {
      const int l = i / cpr, q = i - l * cpr;
      return la + cg2_pad((f * nlcap + l) * lp + 16 * q);
    });
  }
  if (red) {
    const int nred = ntask * nlcap * 4 * 4 * 64;
    for (int i = tid; i < nred; i += NT) red[i] = 0;
  }
  __syncthreads();
  // the buckets and fold maxima have been consumed (the fold maxima by every
  // thread above): back to zero for the next launch
  for (int i = tid; i < ma + mb; i += NT) G(d.yp)[i] = 0;
  if (tid < 2) G(d.cmax)[tid] = 0;
  const int KS = d.c_ks;
  for (int w = wave; w < ntask * parts; w += kCg2Waves) {
    const int task = w % ntask, part = w / ntask;
    const int f = task >= d.c_rta ? 1 : 0;
    const int rt = task - f * d.c_rta;
    const int s0 = (int)((int64_t)KS * part / parts), s1 = (int)((int64_t)KS * (part + 1) / parts);
    cg2_dispatch_task(nl[f], d, lb, la, f * nlcap, f, rt, s0, s1, red ? red + task * nlcap * 1024 : nullptr, tbest);
  }
  if (red) {
    __syncthreads();
    for (int task = wave; task < ntask; task += kCg2Waves) {
      const int f = task >= d.c_rta ? 1 : 0;
      cg2_dispatch_report(nl[f], d, f, task - f * d.c_rta, red + task * nlcap * 1024, tbest);
    }
  }
  // the correlations (global memory, read by top-T) and the per-column-tile
  // bests of every tile are written: the two argmaxes, lowest shift first
  __threadfence_block();
  __syncthreads();
  if (wave < 2) {
    const int f = wave;
    const int n = (f ? d.c_rtb : d.c_rta) * 4;
    VI best{-INFINITY, 0x7fffffff};
    for (int i = lane; i < n; i += 64) {
      const VI v = tbest[f * rtm * 4 + i];
      if (vi_better(v, best)) best = v;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const VI other{__shfl_xor(best.v, o), __shfl_xor(best.i, o)};
      if (vi_better(other, best)) best = other;
    }
    if (lane == 0) fin[f] = best;
  }
  __syncthreads();
  if (d.top_t > 1) resolve_top_t<Tin>(d, fin[0], fin[1], TM_R_EXACT, scratch);
  else resolve_and_report<Tin>(d, fin[0], fin[1], TM_R_EXACT, scratch);
}

__global__ void __launch_bounds__(64 * kCg2Waves) k_cgemm_inst(InstTable tab, const int32_t* list) {
  extern __shared__ __align__(16) unsigned char lds2[];
  const Inst& d = list ? tab.table[list[blockIdx.x]] : tab.resident();
  switch (d.x_dtype) {
    case TM_I8: cg2_instance<int8_t>(d, lds2); break;
    case TM_F32: cg2_instance<float>(d, lds2); break;
    case TM_BF16: cg2_instance<bf16_t>(d, lds2); break;
    default: cg2_instance<f16_t>(d, lds2); break;
  }
}

size_t cgemm_inst_lds_bytes(int c_lt, int c_lp, int nlcap, int tasks, int rtm) {
  return cg2_lds_bytes(c_lt, c_lp, nlcap, tasks, rtm);
}

hipError_t launch_cgemm_inst(const InstTable& tab, const int32_t* list, int count, size_t lds, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  TM_LAUNCH(k_cgemm_inst, dim3(count), dim3(64 * kCg2Waves), lds, s, tab, list);
  return hipGetLastError();
}

hipError_t launch_cgemm_prep(const InstTable& tab, const int32_t* list, int count, int chunk, int prep_y,
                             hipStream_t s) {
  if (count <= 0) return hipSuccess;
  TM_LAUNCH(k_cgemm_prep, dim3(count, prep_y), dim3(kCgPrepThreads), 0, s, tab, list, chunk);
  return hipGetLastError();
}

// TM_CGEMM_WAVES=4 keeps 4 waves per workgroup for every launch
static int env_int_dev(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v && *v ? std::atoi(v) : dflt;
}

hipError_t launch_cgemm_gemm(const InstTable& tab, const int32_t* list, int count, int gemm_y, int max_limbs,
                             hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const dim3 grid(count, gemm_y);
  // few instances: 8 waves per workgroup, half the dependent steps per wave
  const bool wide = count * gemm_y < 512 && env_int_dev("TM_CGEMM_WAVES", 8) == 8;
  if (wide) {
    if (max_limbs <= 3) TM_LAUNCH((k_cgemm<3, 8>), grid, dim3(512), 0, s, tab, list);
    else TM_LAUNCH((k_cgemm<5, 8>), grid, dim3(512), 0, s, tab, list);
  } else {
    if (max_limbs <= 3) TM_LAUNCH((k_cgemm<3, 4>), grid, dim3(256), 0, s, tab, list);
    else TM_LAUNCH((k_cgemm<5, 4>), grid, dim3(256), 0, s, tab, list);
  }
  return hipGetLastError();
}

hipError_t launch_cgemm_final(const InstTable& tab, const int32_t* list, int count, hipStream_t s, bool lean,
                              bool yp_done) {
  if (count <= 0) return hipSuccess;
  if (lean && yp_done) TM_LAUNCH((k_cgemm_final<true, true>), dim3(count), dim3(256), 0, s, tab, list);
  else if (lean) TM_LAUNCH((k_cgemm_final<true, false>), dim3(count), dim3(256), 0, s, tab, list);
  else if (yp_done) TM_LAUNCH((k_cgemm_final<false, true>), dim3(count), dim3(256), 0, s, tab, list);
  else TM_LAUNCH((k_cgemm_final<false, false>), dim3(count), dim3(256), 0, s, tab, list);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// three moduli (Theorem 4 with alpha = 3): combine the two pairs' residues
// --------------------------------------------------------------------------
//
// c belongs to S(a, M) = {(a + i M) mod N : i < L} iff c = a mod M (the
// regular members a + i M < N) or c is the wrapped member (a + (L-1) M) mod N
// when a + (L-1) M >= N.  The regular classes of the three moduli meet at most
// once below N (M1 M2 M3 >= N); candidates are the members of the (a1, a2)
// class below N, found by Chinese remaindering and checked against S3 in
// parallel, and the three wrapped members checked against all three sets.

struct ResSet { int64_t a, m, w; bool wrap; };

__device__ __forceinline__ ResSet res_set(int64_t a, int64_t m, int64_t n) {
  const int64_t l = (n + m - 1) / m;
  const int64_t last = a + (l - 1) * m;
  return ResSet{a, m, last % n, last >= n};
}

__device__ __forceinline__ bool in_set(int64_t c, const ResSet& s) {
  return (c % s.m == s.a) || (s.wrap && c == s.w);
}

template <typename Tin>
__device__ __forceinline__ void combine3(const Inst& d, const Combine3& cb, const tm_result& r1, const tm_result& r2,
                         tm_result* out, void* scratch) {
  constexpr int kMaxCand = 16;
  __shared__ long long cand[kMaxCand];
  __shared__ int ncand;
  const int64_t N = d.n;
  const ResSet s1 = res_set(r1.m1_tilde, cb.m1, N), s2 = res_set(r1.m2_tilde, cb.m2, N),
               s3 = res_set(r2.m1_tilde, cb.m3, N);
  if (threadIdx.x == 0) ncand = 0;
  __syncthreads();
  auto push = [&](long long v) {
    const int slot = atomicAdd(&ncand, 1);
    if (slot < kMaxCand) cand[slot] = v;
  };
  if (s1.a < N && s2.a < N) {
    const int64_t m12 = (int64_t)cb.m1 * cb.m2;
    const int64_t t = ((((s2.a - s1.a) % cb.m2) + cb.m2) % cb.m2) * cb.inv12 % cb.m2;
    const int64_t v0 = s1.a + (int64_t)cb.m1 * t;
    for (int64_t v = v0 + (int64_t)threadIdx.x * m12; v < N; v += (int64_t)blockDim.x * m12)
      if (in_set(v, s3)) push(v);
  }
  if (threadIdx.x == 0) {
    const ResSet* sets[3] = {&s1, &s2, &s3};
    for (int i = 0; i < 3; ++i)
      if (sets[i]->wrap && in_set(sets[i]->w, s1) && in_set(sets[i]->w, s2) && in_set(sets[i]->w, s3))
        push(sets[i]->w);
  }
  __syncthreads();
  if (threadIdx.x == 0) {   // ascending, no repeats
    int w = min(ncand, kMaxCand);
    for (int i = 1; i < w; ++i)
      for (int j = i; j > 0 && cand[j - 1] > cand[j]; --j) {
        const long long tmp = cand[j];
        cand[j] = cand[j - 1];
        cand[j - 1] = tmp;
      }
    int u = 0;
    for (int i = 0; i < w; ++i)
      if (u == 0 || cand[u - 1] != cand[i]) cand[u++] = cand[i];
    ncand = u;
  }
  __syncthreads();
  const int nc = ncand;
  int64_t best = -1;
  double best_score = 0.0;
  for (int i = 0; i < nc; ++i) {
    const double sc = score_any_t<Tin>(d, cand[i], scratch);
    if (i == 0 || sc > best_score) { best = cand[i]; best_score = sc; }
  }
  if (threadIdx.x == 0) {
    uint32_t flags = (r1.flags & r2.flags & TM_R_EXACT) | ((r1.flags | r2.flags) & TM_R_NEAR_TIE);
    if (nc == 0) flags |= TM_R_NOMATCH;
    if (nc > 1) flags |= TM_R_RESCORED;
    tm_result r;
    r.shift = best;
    r.m1_tilde = r1.m1_tilde;
    r.m2_tilde = r1.m2_tilde;
    r.n_candidates = nc;
    r.flags = flags;
    r.peak1 = r1.peak1;
    r.peak2 = r1.peak2;
    r.score = nc ? best_score : 0.0;
    r.err_bound = fmax(r1.err_bound, r2.err_bound);
    r.reserved = 0;
    *out = r;
  }
}

__global__ void __launch_bounds__(256) k_combine3(const Inst* tab, const Combine3* cmb, const tm_result* res,
                                                  tm_result* out) {
  __shared__ __align__(16) unsigned char scratch[16 * 16];
  const Combine3 cb = cmb[blockIdx.x];
  const tm_result r1 = res[cb.i1];
  if (cb.i2 < 0) {
    if (threadIdx.x == 0) out[blockIdx.x] = r1;
    return;
  }
  const tm_result r2 = res[cb.i2];
  const Inst& d = tab[cb.i1];
  tm_result* o = out + blockIdx.x;
  switch (d.x_dtype) {
    case TM_I8: combine3<int8_t>(d, cb, r1, r2, o, scratch); break;
    case TM_F32: combine3<float>(d, cb, r1, r2, o, scratch); break;
    case TM_BF16: combine3<bf16_t>(d, cb, r1, r2, o, scratch); break;
    default: combine3<f16_t>(d, cb, r1, r2, o, scratch); break;
  }
}

hipError_t launch_combine3(const Inst* tab, const Combine3* cmb, const tm_result* res, tm_result* out, int count,
                           hipStream_t s) {
  if (count <= 0) return hipSuccess;
  TM_LAUNCH(k_combine3, dim3(count), dim3(256), 0, s, tab, cmb, res, out);
  return hipGetLastError();
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
                                                   int as_double, int row_log2) {
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
    // one length-P correlation in LDS, or rows of 2^row_log2 (global-memory FFT)
    const int slot = row_log2 ? ((n >> row_log2) << row_log2) + spec_slot(n & ((1 << row_log2) - 1), row_log2)
                              : spec_slot(n, p);
    if (as_double) reinterpret_cast<double2*>(spec)[slot] = make_double2(v.x * inv, -v.y * inv);
    else reinterpret_cast<float2*>(spec)[slot] = make_float2((float)(v.x * inv), (float)(-v.y * inv));
  }
}

// --------------------------------------------------------------------------
// device scratch of the allocation-free single match
// --------------------------------------------------------------------------
//
// One array per device, allocated when the code object loads and kept until
// the process ends.  Host code never passes `scratch` itself to a kernel (in
// host code the name is a stand-in, not a device address): the address that
// hipGetSymbolAddress returns for the current device is kept per device when
// the kernels are configured and handed to the kernels as an argument.

static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static void* g_scratch_ptr[kMaxDevices] = {};

// the instance record into scratch (one thread) and the bucket zone cleared
// (a fill kernel rather than a memset, so a captured sequence holds no memset)
__global__ void __launch_bounds__(256) k_noalloc_setup(Inst rec, Inst* dst, int* zero, int64_t nzero) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *dst = rec;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nzero; i += (int64_t)gridDim.x * blockDim.x)
    G(zero)[i] = 0;
}

void* scratch_device_ptr(int dev) { return dev >= 0 && dev < kMaxDevices ? g_scratch_ptr[dev] : nullptr; }

hipError_t launch_noalloc_setup(const Inst& rec, Inst* dst, int* zero, int64_t nzero, hipStream_t s) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (nzero + 255) / 256));
  TM_LAUNCH(k_noalloc_setup, dim3(grid), dim3(256), 0, s, rec, dst, zero, nzero);
  return hipGetLastError();
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
                       reinterpret_cast<const void*>(k_finish<float>),
                       reinterpret_cast<const void*>(k_gfft_cols<double>), reinterpret_cast<const void*>(k_gfft_cols<float>),
                       reinterpret_cast<const void*>(k_gfft_rows<double>), reinterpret_cast<const void*>(k_gfft_rows<float>),
                       reinterpret_cast<const void*>(k_gfft_icols<double>),
                       reinterpret_cast<const void*>(k_gfft_icols<float>), reinterpret_cast<const void*>(k_cgemm_inst)};
  for (const void* f : fns) {
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
      (void)hipGetLastError();
  }
  // this device's copy of the scratch array (the device is current here)
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = ptr;
  return hipSuccess;
}

hipError_t launch_fold(const InstTable& tab, int total_tiles, size_t lds, hipStream_t s) {
  if (total_tiles <= 0) return hipSuccess;
  TM_LAUNCH(k_fold, dim3(total_tiles), dim3(kFoldThreads), lds, s, tab, total_tiles);
  return hipGetLastError();
}

hipError_t launch_fold_band(const InstTable& tab, int total_wgs, hipStream_t s) {
  if (total_wgs <= 0) return hipSuccess;
  TM_LAUNCH(k_fold_band, dim3(total_wgs), dim3(64 * kBandWaves), 0, s, tab, total_wgs);
  return hipGetLastError();
}

hipError_t launch_fold_s8(const InstTable& tab, int total_segs, hipStream_t s) {
  if (total_segs <= 0) return hipSuccess;
  TM_LAUNCH(k_fold_s8, dim3(total_segs), dim3(kSegThreads), 0, s, tab, total_segs);
  return hipGetLastError();
}

hipError_t launch_reduce(const InstTable& tab, int total_wgs, hipStream_t s) {
  if (total_wgs <= 0) return hipSuccess;
  TM_LAUNCH(k_reduce, dim3(total_wgs), dim3(kReduceThreads), 0, s, tab, total_wgs);
  return hipGetLastError();
}

hipError_t launch_finish(const InstTable& tab, const int32_t* list, int count, int mode, int p_log2,
                         size_t lds, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int nt = finish_threads(p_log2);
  if (mode == MODE_EXACT)
    TM_LAUNCH(k_finish<double>, dim3(count), dim3(nt), lds, s, tab, list, count);
  else
    TM_LAUNCH(k_finish<float>, dim3(count), dim3(nt), lds, s, tab, list, count);
  return hipGetLastError();
}

hipError_t launch_twiddles(void* tw, int p_log2, int as_double, hipStream_t s) {
  const int half = (1 << p_log2) >> 1;
  const int blocks = (half + 255) / 256;
  TM_LAUNCH(k_twiddles, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, tw, p_log2, as_double);
  return hipGetLastError();
}

hipError_t launch_spectrum(const void* t, int t_dtype, int k, int p_log2, const double* tw64,
                           double* scratch, void* spec, int as_double, int row_log2, hipStream_t s) {
  TM_LAUNCH(k_spectrum, dim3(1), dim3(1024), 0, s, t, t_dtype, k, p_log2,
                     reinterpret_cast<const double2*>(tw64), reinterpret_cast<double2*>(scratch), spec,
                     as_double, row_log2);
  return hipGetLastError();
}

}  // namespace tmi
