// Internal declarations shared by the host runtime and the gfx950 kernels.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "tm.h"

namespace tmi {

enum : int32_t { MODE_EXACT = 0, MODE_REAL = 1 };

// Tiles of one row view of x: x read as rows of `m` elements (row i holds
// x[i*m .. i*m+m)), cut into tiles of `rows` x `cols` elements.
struct View {
  int32_t m;      // row length (a fold modulus)
  int32_t l;      // number of rows, ceil(N / m)
  int32_t rows;   // tile rows R
  int32_t cols;   // tile columns W
  int32_t nrb;    // row blocks, ceil(l / R)
  int32_t ncb;    // column blocks, ceil(m / W)
};

// Everything a launch needs about one matching instance.  Built on the host,
// read by every kernel; 16-byte aligned so a table of them can be copied as is.
struct alignas(16) Inst {
  const void* x;          // signal (device)
  int64_t n;              // N
  int32_t k;              // K
  int32_t x_dtype;        // tm_dtype
  int32_t t_dtype;        // tm_dtype
  int32_t mode;           // MODE_EXACT / MODE_REAL
  int32_t fold_store;     // tm_dtype used to store the fold on the real path
  int32_t dual;           // 1: mb == ma + 1, fold B comes from view A's diagonals
  int32_t swapped;        // 1: the user's M1 is mb (results are mapped back)
  int32_t zpad;           // 1: zero-padded variant (partition folds, circular correlation,
                          //    no wrapped candidates)
  int32_t top_t;          // runners-up per fold whose residue pairs are re-scored (1: step 9)
  int32_t top_pad;
  int32_t p_log2;         // FFT length P = 2^p_log2
  View va;                // view with modulus ma (always tiled)
  View vb;                // view with modulus mb (tiled only when !dual)
  int32_t tile_base;      // first fold tile of this instance in the launch
  int32_t ntiles;         // fold tiles of this instance
  int32_t red_base;       // first reduce workgroup of this instance in the launch
  int32_t nred;           // reduce workgroups (real folds; 0 for integer folds)
  int32_t red_tpe;        // reduce threads per fold entry (a power of two <= 256)
  int32_t acc_int;        // 1: integer fold accumulated with atomics into `yp`
  int32_t sfold;          // 1: int8 signal folded by k_fold_s8 (biased bucket sums)
  int32_t seg_base;       // first k_fold_s8 segment of this instance in the launch
  int32_t nseg;           // k_fold_s8 segments of this instance
  int32_t seg_chunks;     // 16-byte chunks per segment
  int32_t band;           // 1: 4-byte signal folded by k_fold_band (views of 64-column bands)
  int32_t band_base;      // first k_fold_band workgroup of this instance in the launch
  int32_t nband;          // k_fold_band workgroups of this instance
  int32_t gfft;           // 1: FFT correlation through global memory (P above one workgroup's LDS)
  int32_t g_q;            // P = P1 x P2 with P1 = 2^g_q (column transforms), P2 = 2^(p_log2 - g_q)
  int32_t g_logb;         // columns per column workgroup: 2^g_logb
  void* gz;               // P complex working values (T of the mode)
  double* gss;            // |z|^2 partials, one per literal-fold workgroup
  void* gpart;            // argmax partials, one per column workgroup
  const void* tw_cols;    // twiddles for 2^(g_logb + g_q)
  const void* tw_rows;    // twiddles for P2
  int32_t cgemm;          // 1: correlation as an int8 MFMA GEMM (exact path, int8-valued t)
  int32_t c_nlcap;        // limbs the literal folds are split into (upper bound of the need)
  int32_t c_lp;           // bytes per limb row of one fold (multiple of 64)
  int32_t c_ks;           // 64-deep steps over the template band: ceil((K + 63) / 64) rounded up to 4
  int32_t c_rta, c_rtb;   // GEMM workgroups (16 rows of 64 shifts) of fold A and fold B
  int32_t c_lt;           // bytes per shifted template copy in tsh
  int32_t c_split;        // workgroups sharing each row tile's band (1: one; above 1, the shares
                          // are added into `cacc` and the final kernel takes the argmax)
  int8_t* ylimb;          // [2 folds][c_nlcap][c_lp] balanced base-128 digits of the folds
  void* cpart;            // [2 folds][max(c_rta, c_rtb) * 4] best (value, shift) per wave
  int* cmax;              // [2] largest |y| per fold (in the zeroed bucket zone)
  long long* cacc;        // split band: r of fold A [ma], then B [mb]; zero between launches
  const int8_t* tsh;      // 16 copies of the zero-padded template, copy c shifted by c bytes
  double* rtop;           // top-T on the GEMM and four-step routes: r of fold A [ma], then B [mb]
  int64_t inv_a_mod_b;    // ma^{-1} mod mb
  // workspace (device)
  void* col_a;            // [va.nrb][ma] column partials
  void* diag;             // [va.nrb][va.ncb][va.cols + va.rows - 1] diagonal partials (dual)
  void* col_b;            // [vb.nrb][mb] column partials (!dual)
  void* y;                // literal folds (real path): [ma + k - 1] then [mb + k - 1]
  int* yp;                // partition folds (integer path): [ma] then [mb]; all zero
                          // between launches (the finish kernel clears what it read)
  // plan (device)
  const void* t;          // template, t_dtype
  const void* spec;       // P complex values: conj(FFT_P(t)) / P at bit-reversed positions
  const void* tw;         // P/2 complex values W^e = exp(-2 pi i e / P)
  double tnorm1;          // sum |t_j|
  double tspec_max;       // max_k |FFT_P(t)[k]| (real plans; for the results' error bound)
  double tnorm2;          // ||t||_2
  tm_result* out;         // device result slot
  double* dbg_y1;         // optional intermediates (user order), may be null
  double* dbg_y2;
  double* dbg_r1;
  double* dbg_r2;
};

// A launch's view of its instances: a device table (batches), or one
// device-resident instance (single matches: the kernel arguments stay within
// 64 bytes, which keeps the host's cost per launch low).  A single match's
// signal and result slot travel with the launch of its fold kernel, which
// stores them into the device copy for the kernels that follow on the stream.
struct InstTable {
  const Inst* table;      // device table, or nullptr for the single instance at `one`
  const Inst* one;        // device copy of the single instance
  const void* x;          // the single instance's signal (fold kernels)
  tm_result* out;         // its result slot (fold kernels)
  int32_t count;
  // fold kernels: the instance with this launch's signal and result slot
  __device__ __forceinline__ Inst single() const {
    Inst d = *one;
    d.x = x;
    d.out = out;
    return d;
  }
  // kernels after the fold: the device copy, signal and result slot included
  __device__ __forceinline__ const Inst& resident() const { return *one; }
  // fold kernels, one thread of the launch: store the signal and result slot
  // into the device copy (ordinary vector stores; the next kernel on the
  // stream sees them)
  __device__ __forceinline__ void publish() const {
    Inst* w = const_cast<Inst*>(one);
    w->x = x;
    w->out = out;
  }
};
static_assert(sizeof(InstTable) <= 40, "single-match kernel arguments stay small");

constexpr int kFoldThreads = 256;
constexpr int kFoldLoads = 16;          // 16-byte chunks each fold thread stages per tile
constexpr int kFoldMaxCols = 512;       // tile columns W <= 512 (elements)
constexpr int kFoldMaxRows = 256;       // tile rows R <= 256
constexpr size_t kFoldLdsBudget = 60 * 1024;   // skewed tile bytes (two workgroups per CU)
// streaming int8 fold (k_fold_s8)
constexpr int kSegThreads = 256;
// word 3 of a raw buffer resource on gfx950: 32-bit data format, untyped loads
constexpr int kBufRsrcWord3 = 0x00020000;
constexpr int kSegHalf = 128;                       // threads per modulus
constexpr int kSegPiece = 16384;                    // bytes per LDS ring piece
constexpr int kSegPieceChunks = kSegPiece / 16;
constexpr int kSegLoads = kSegPieceChunks / kSegThreads;
constexpr int kSegSlots = 9;                        // words per lane per row
constexpr int kSegMaxM = 4 * kSegHalf * kSegSlots;  // 4608
constexpr int kSegMinM = 16;
constexpr int kSegLook = 4640;                      // mirrored bytes: a row of kSegMaxM + 16
constexpr int kSegLds = 2 * kSegPiece + kSegLook;
constexpr int kSegZ = 4 * kSegHalf * kSegSlots;     // flush buckets per modulus
constexpr int kSegMaxRows = 256;                    // rows of the shorter modulus per segment
static_assert(2 * kSegZ * 4 <= kSegLds, "flush area must fit the ring");
static_assert(kSegLook >= kSegMaxM + 16 && kSegLook % 16 == 0, "mirror must hold a row");

// band fold of 4-byte signals (k_fold_band)
constexpr int kBandCols = 64;                       // columns per band: one per lane
constexpr int kBandWaves = 4;                       // bands (tasks) per workgroup
constexpr int kBandRowsMax = 256;                   // rows per task
constexpr int kBandUnroll = 16;                     // rows whose loads are in flight together

// FFT through global memory (k_gfft_*)
constexpr int kGfftThreads = 256;                   // literal-fold and final workgroups
constexpr int kGfftMaxLog2 = 21;                    // P up to 2^21 (rows of <= 4096)
constexpr int kGfftMaxQ = 9;                        // column transforms of <= 512

// shared-template correlation as an int8 MFMA GEMM (k_many_*)
constexpr int kGemmTile = 64;                       // signals and shifts per workgroup
constexpr int kGemmMaxLimbs = 3;                    // balanced base-128 digits of the folds

// correlation of exact instances as an int8 MFMA GEMM (k_cgemm_*)
constexpr int kCgPad = 128;                         // zero bytes around the template copies
constexpr int kCgRows = 16;                         // rows (64-shift blocks) per GEMM workgroup
constexpr int kCgMaxLimbs = 5;                      // balanced base-128 digits of int32 folds
constexpr int kCgMaxK = 1 << 17;                    // int32 limb sums stay exact below this K
constexpr int kCgPrepThreads = 256;
constexpr int kTopTMax = 4;                         // runners-up per fold for top-T re-scoring
constexpr int kCg2Waves = 4;                        // waves of the per-instance product kernel (batches)
constexpr size_t kCg2MaxLds = 156 * 1024;           // its largest LDS footprint (template copies, digit rows)
constexpr int kCgClasses = 5;                       // LDS classes of its launches

// One user instance of a batch that holds three-moduli plans: the indices of
// its results in the expanded instance list (i2 < 0: a two-moduli plan whose
// result is copied) and, for three moduli, the user's moduli with
// m1^{-1} mod m2.  The first pair (m1, m2) is instance i1, the second pair
// (m3, m1) instance i2.
struct alignas(8) Combine3 {
  int32_t i1, i2;
  int32_t m1, m2, m3, pad;
  int64_t inv12;
};

// Arguments of the shared-template kernels (one plan, `count` signals).
struct ManyArgs {
  Inst base;              // the plan's instance record (x, out, workspace unset)
  const void* const* xs;  // device array of count signal pointers
  tm_result* out;         // count results (device)
  int* yp;                // bucket sums, yp_stride ints per signal, zero between launches
  int64_t yp_stride;
  int8_t* ylimb;          // [2 folds][kGemmMaxLimbs][rows][lp] limbs of the literal folds
  int64_t rows;           // count rounded up to kGemmTile
  int32_t lp;             // padded fold length (multiple of 64)
  int32_t count;
  int32_t nkb;            // shift blocks per fold: ceil(mb / 64)
  int32_t pad0;
  int* maxabs;            // [2][count] largest |y| per fold and signal (limb counts)
  double* part;           // [2][count][nkb][2]: best value and its shift per block
};

constexpr int kReduceThreads = 256;
constexpr int kFinishThreads = 512;     // largest finish workgroup (P / 16 threads)
constexpr int kFftMid = 5;              // stages of the FFT's twiddle-free middle pass

// 16-byte chunks that cover one tile row of `cols` elements at any alignment
inline __host__ __device__ int fold_chunks(int cols, int eb) { return (cols * eb + 15) / 16 + 1; }

// Element sizes of tm_dtype values.
inline int dtype_bytes(int dt) { return dt == TM_I8 ? 1 : (dt == TM_F32 ? 4 : 2); }

// Dynamic LDS bytes the kernels need.
size_t fold_lds_bytes(const View& v, int x_dtype);
size_t finish_lds_bytes(int p_log2, int mode);
int fft_lds_max_log2(int mode);         // largest P (log2) whose FFT fits one workgroup
int finish_threads(int p_log2);         // finish workgroup size for FFT length 2^p_log2

// Kernel timing: while `stop` is set, every kernel launched on this thread
// carries the two events on its own dispatch (hipExtLaunchKernel), so their
// elapsed time covers the kernels' execution only, not the host's launch
// gaps. The first launch takes `start` and clears it; every launch re-takes
// `stop`, so a region of several kernels spans first start to last end.
struct LaunchEvents {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};
extern thread_local LaunchEvents g_launch_events;

// Kernel launchers (tm_kernels.hip).
hipError_t configure_kernels();        // raise dynamic LDS limits on the current device
hipError_t launch_fold(const InstTable& tab, int total_tiles, size_t lds, hipStream_t s);
hipError_t launch_fold_s8(const InstTable& tab, int total_segs, hipStream_t s);
hipError_t launch_fold_band(const InstTable& tab, int total_wgs, hipStream_t s);
hipError_t launch_reduce(const InstTable& tab, int total_chunks, hipStream_t s);
hipError_t launch_finish(const InstTable& tab, const int32_t* list, int count, int mode, int p_log2,
                         size_t lds, hipStream_t s);
hipError_t launch_twiddles(void* tw, int p_log2, int as_double, hipStream_t s);
hipError_t launch_spectrum(const void* t, int t_dtype, int k, int p_log2, const double* tw64,
                           double* scratch, void* spec, int as_double, int row_log2, hipStream_t s);
size_t gfft_part_bytes();
hipError_t launch_many(const ManyArgs& a, hipStream_t s);   // literal folds .. results
// exact instances with the GEMM correlation (list: `count` instance indices
// of the table, or nullptr for tab.one): literal-fold digits in chunks of
// `chunk` entries; the GEMM with per-wave argmax over gemm_y row-tile tasks
// per instance (variant by the largest digit count); per instance the argmax
// reduction and the resolve
hipError_t launch_cgemm_prep(const InstTable& tab, const int32_t* list, int count, int chunk, int prep_y,
                             hipStream_t s);
hipError_t launch_cgemm_gemm(const InstTable& tab, const int32_t* list, int count, int gemm_y, int max_limbs,
                             hipStream_t s);
// int8 batches: the per-wave product with the template copies staged in an
// LDS ring per workgroup (digit counts up to 3); it also returns the
// instances' bucket zones to zero (the final kernel then takes yp_done)
hipError_t launch_cgemm_ring(const InstTable& tab, const int32_t* list, int count, int gemm_y, hipStream_t s);
// lean: every listed instance has an int8 signal and template, top_t 1 and
// an unsplit band; yp_done: the product kernel (k_cgemm_ring) has already
// cleared the instances' bucket zones
hipError_t launch_cgemm_final(const InstTable& tab, const int32_t* list, int count, hipStream_t s,
                              bool lean = false, bool yp_done = false);
// batches: one wave per row tile over the whole band (gemm_y row tiles per
// instance at most, four per workgroup), per-column-tile bests to cpart
hipError_t launch_cgemm_wave(const InstTable& tab, const int32_t* list, int count, int gemm_y, int max_limbs,
                             hipStream_t s);
// batches: the correlation stage with one workgroup per instance (literal
// folds, product with its operands in LDS, argmaxes, resolve; no prep or
// final kernel); `lds` bytes: the largest cgemm_inst_lds_bytes of the listed
// instances (tasks = c_rta + c_rtb, rtm = max(c_rta, c_rtb))
size_t cgemm_inst_lds_bytes(int c_lt, int c_lp, int nlcap, int tasks, int rtm);
hipError_t launch_cgemm_inst(const InstTable& tab, const int32_t* list, int count, size_t lds, hipStream_t s);
int cgemm_limbs_for(int64_t maxabs);                   // limbs that hold |y| <= maxabs
// Theorem 4 with three moduli: per user instance, S1 cap S2 cap S3 from the two
// pairs' argmaxes, re-scored by (Tx)_c (one workgroup each)
hipError_t launch_combine3(const Inst* tab, const Combine3* cmb, const tm_result* res, tm_result* out, int count,
                           hipStream_t s);
hipError_t launch_gfft(const Inst& host, const Inst* dev, hipStream_t s);   // literal folds .. result, one instance

// Per-stream workspace pools (tm_runtime.cpp), for the request server's own
// streams: grow to exactly what a launch needs, report the device bytes a
// stream's pool holds, and free them (after the stream drains; keep_entry
// keeps the stream's settings for later launches).
void stream_pool_set_exact(int dev, hipStream_t s);
size_t stream_pool_device_bytes(int dev, hipStream_t s);
hipError_t stream_pool_release(int dev, hipStream_t s, bool keep_entry);

// Allocation-free single match: a device array of kScratchBytes per device
// (tm_kernels.hip), its address on device `dev` (looked up by
// configure_kernels), and the kernel that stores an instance record into it
// and clears `nzero` ints of its bucket zone.
constexpr size_t kScratchBytes = size_t(16) << 20;
constexpr int kMaxDevices = 64;
void* scratch_device_ptr(int dev);
hipError_t launch_noalloc_setup(const Inst& rec, Inst* dst, int* zero, int64_t nzero, hipStream_t s);

}  // namespace tmi
