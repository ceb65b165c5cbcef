// Host runtime and C ABI of the template matcher: plan construction
// (Algorithm 1 steps 2 and 4), per-stream workspace pools and the launch
// sequence fold -> reduce -> finish for single and batched matches.

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <utility>
#include <vector>

#include "tm_internal.h"

using namespace tmi;

namespace {

thread_local std::string g_err;

tm_status fail(tm_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define TM_HIP(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(e_ == hipErrorOutOfMemory ? TM_ERR_NOMEM : TM_ERR_DEVICE,            \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                  \
  } while (0)

int64_t env_int(const char* name, int64_t dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  return std::strtoll(v, nullptr, 10);
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

static_assert(sizeof(tm_plan_desc) == 48, "tm_plan_desc layout is part of the ABI");
static_assert(sizeof(tm_result) == 64, "tm_result layout is part of the ABI");

int64_t gcd64(int64_t a, int64_t b) {
  while (b) { const int64_t t = a % b; a = b; b = t; }
  return a;
}

// a^{-1} mod m for gcd(a, m) = 1 (extended Euclid); 0 when m == 1
int64_t mod_inverse(int64_t a, int64_t m) {
  if (m == 1) return 0;
  int64_t g = m, x = 0, x1 = 1, a1 = a % m;
  while (a1) {
    const int64_t q = g / a1;
    int64_t t = g - q * a1; g = a1; a1 = t;
    t = x - q * x1; x = x1; x1 = t;
  }
  return ((x % m) + m) % m;
}

// least m >= 1 with m (m + 1) > n
int64_t least_m0(int64_t n) {
  int64_t m = (int64_t)std::sqrt((double)n);
  if (m < 1) m = 1;
  while (m > 1 && (m - 1) * m > n) --m;
  while (m * (m + 1) <= n) ++m;
  return m;
}

bool valid_dtype(int32_t dt) { return dt >= TM_I8 && dt <= TM_F16; }

// Tile shape of one row view: TM_TILE_WBYTES-wide rows (1 KiB for 4-byte
// elements, 512 elements otherwise), as many rows as the skewed LDS tile
// budget, the staging loads and TM_TILE_BYTES allow.
View make_view(int64_t n, int64_t m, int eb) {
  View v{};
  v.m = (int32_t)m;
  v.l = (int32_t)ceil_div(n, m);
  const int64_t wdef = eb == 4 ? 256 : 512;
  const int64_t tile_bytes = std::max<int64_t>(256, env_int("TM_TILE_BYTES", 1 << 20));
  const int64_t wbytes = std::max<int64_t>(eb, env_int("TM_TILE_WBYTES", wdef * eb));
  const int64_t w = std::min<int64_t>({m, std::max<int64_t>(1, wbytes / eb), (int64_t)kFoldMaxCols});
  const int64_t rmax_stage = (int64_t)kFoldThreads * kFoldLoads / fold_chunks((int)w, eb);
  int64_t r = std::max<int64_t>(1, std::min<int64_t>({(int64_t)v.l, tile_bytes / (w * eb), rmax_stage,
                                                       (int64_t)kFoldMaxRows}));
  while (r > 1 && (size_t)r * (w + r - 1) * eb > kFoldLdsBudget) --r;
  v.cols = (int32_t)w;
  v.rows = (int32_t)r;
  v.nrb = (int32_t)ceil_div(v.l, r);
  v.ncb = (int32_t)ceil_div(m, w);
  return v;
}

// Segments of the streaming int8 fold: x spans at most N/16 + 1 chunks at any
// alignment; the last segment also takes the one chunk a misaligned x adds
// (so it holds at most seg_chunks + 1 chunks, within the row limit's margin).
int32_t segments_of(int64_t n, int64_t sc) { return (int32_t)std::max<int64_t>(1, ceil_div((n + 15) / 16, sc)); }

// Band view of a 4-byte signal: 64-column bands of R rows, R a multiple of
// kBandUnroll chosen for about 2048 tasks (TM_BAND_ROWS overrides).
View make_band_view(int64_t n, int64_t m) {
  View v{};
  v.m = (int32_t)m;
  v.l = (int32_t)ceil_div(n, m);
  v.cols = kBandCols;
  v.ncb = (int32_t)ceil_div(m, kBandCols);
  int64_t r = env_int("TM_BAND_ROWS", 0);
  if (r <= 0) r = ceil_div((int64_t)v.l * v.ncb, 2048);
  r = ceil_div(std::max<int64_t>(r, 1), kBandUnroll) * kBandUnroll;
  r = std::min<int64_t>(r, kBandRowsMax);
  v.rows = (int32_t)r;
  v.nrb = (int32_t)ceil_div(v.l, r);
  return v;
}

// Plan parameters derived from the descriptor; pure host arithmetic.
struct Core {
  int64_t n = 0;
  int32_t k = 0, m1 = 0, m2 = 0, ma = 0, mb = 0;
  int32_t swapped = 0, dual = 0, mode = MODE_EXACT, p_log2 = 1, zpad = 0, top_t = 1;
  int32_t three = 0, m3 = 0;   // three moduli: (m1, m2) here, (m3, m1) in the plan's second core
  int32_t x_dtype = 0, t_dtype = 0, fold_store = TM_F32;
  int64_t inv = 0;
  View va{}, vb{};
  // workspace offsets (bytes) of one instance
  size_t off_col_a = 0, off_diag = 0, off_col_b = 0, off_y = 0, off_res = 0, ws_bytes = 0;
  int32_t ntiles = 0, nred = 0, red_tpe = 1, acc_int = 0;
  int32_t sfold = 0, nseg = 0, seg_chunks = 0;   // streaming int8 fold
  int32_t band = 0, nband = 0;                    // band fold of 4-byte signals
  int32_t gfft = 0, g_q = 0, g_logb = 0;          // FFT through global memory
  size_t off_gz = 0, off_gss = 0, off_gpart = 0;
  size_t acc_bytes = 0;     // integer bucket zone (int32 [ma + mb], then the GEMM path's two
                            // fold maxima); lives in the zeroed pool
  // correlation as an int8 MFMA GEMM (exact path, int8-valued template)
  int32_t cgemm = 0, c_nlcap = 0, c_lp = 0, c_ks = 0, c_rta = 0, c_rtb = 0, c_lt = 0;
  size_t off_ylimb = 0, off_cpart = 0, off_rtop = 0;
  size_t fold_lds = 0, finish_lds = 0;
  int fft_in_lds = 1;
};

// Segment length for a launch: about 2048 segments (a few per resident
// workgroup amortise each segment's prologue and flush) but at most 192 KiB,
// so that the last segments to start leave no long tail when the signals
// differ in size; never above the row limit.
// the product route's final kernel without the dtype and top-T branches
static bool cg_lean_core(const Core& c) {
  return c.x_dtype == TM_I8 && c.t_dtype == TM_I8 && c.top_t == 1;
}

int64_t launch_seg_chunks(const Core& c, int64_t launch_bytes) {
  const int64_t cap = std::max<int64_t>(1, (int64_t)kSegMaxRows * std::min(c.ma, c.mb) / 16 - 1);
  const int64_t cap_kib = std::max<int64_t>(1, env_int("TM_SEG_LAUNCH_KIB", 192));
  const int64_t want = std::min<int64_t>(launch_bytes / 16 / 2048, (cap_kib << 10) / 16);
  return std::min(cap, std::max<int64_t>(c.seg_chunks, want));
}

// Literal-fold entries per prep workgroup: about 4096 workgroups over the
// launch's entries (TM_CG_PREP_WGS), at least 1024 (four per thread) and at
// most one fold; grid rows = 2 x the chunks of the largest instance's fold
// (fold A's chunks, then fold B's).  max_entries: the largest 2 c_lp.
struct CgLaunch { int chunk; int prep_y; };
CgLaunch cgemm_launch(int64_t total_entries, int64_t max_entries, int64_t count) {
  (void)count;
  const int64_t wgs = std::max<int64_t>(1, env_int("TM_CG_PREP_WGS", 4096));
  const int64_t fold_max = ceil_div(max_entries, 2);
  int64_t chunk = std::max<int64_t>(1024, align_up(ceil_div(total_entries, wgs), 1024));
  chunk = std::min(chunk, align_up(fold_max, 1024));
  return CgLaunch{(int)chunk, (int)(2 * ceil_div(fold_max, chunk))};
}

// t_i8: every template value is an integer in [-128, 127] (known for int8
// templates without looking at them; checked on the values at plan creation)
tm_status compute_core(const tm_plan_desc* d, Core* c, bool t_i8, bool pair_of_three = false) {
  if (!d) return fail(TM_ERR_INVALID, "null plan descriptor");
  if (d->n < 1) return fail(TM_ERR_INVALID, "N must be >= 1");
  if (d->k < 1 || (int64_t)d->k > d->n) return fail(TM_ERR_INVALID, "need 1 <= K <= N");
  if (!valid_dtype(d->x_dtype) || !valid_dtype(d->t_dtype)) return fail(TM_ERR_INVALID, "unknown dtype");
  // TM_I8 (0, the zero-initialised value) selects the default TM_F32
  const int32_t fs = d->fold_store == TM_I8 ? TM_F32 : d->fold_store;
  if (fs != TM_F32 && fs != TM_BF16 && fs != TM_F16)
    return fail(TM_ERR_INVALID, "fold_store must be TM_F32, TM_BF16 or TM_F16");
  if (d->fold_mult < 0 || d->fold_mult > 2) return fail(TM_ERR_INVALID, "fold_mult must be 0, 1 or 2");
  if (d->flags & ~(TM_F_EXACT | TM_F_REAL | TM_F_ZERO_PAD | TM_F_FFT))
    return fail(TM_ERR_INVALID, "unknown plan flags");
  if ((d->flags & TM_F_EXACT) && (d->flags & TM_F_REAL))
    return fail(TM_ERR_INVALID, "TM_F_EXACT and TM_F_REAL are exclusive");
  if (d->n > (int64_t(1) << 40)) return fail(TM_ERR_INVALID, "N above 2^40 is not supported");

  c->n = d->n;
  c->k = d->k;
  c->x_dtype = d->x_dtype;
  c->t_dtype = d->t_dtype;
  c->fold_store = fs;
  c->zpad = (d->flags & TM_F_ZERO_PAD) ? 1 : 0;
  if (d->top_t < 0 || d->top_t > kTopTMax) return fail(TM_ERR_INVALID, "top_t must be in 0..4");
  c->top_t = d->top_t == 0 ? 1 : d->top_t;
  int64_t m1 = d->m1, m2 = d->m2;
  // three pairwise co-prime moduli (Theorem 4): this core folds (M1, M2) and
  // the plan's second core (M3, M1); neither pair alone needs to cover N
  const bool three = d->m3 != 0 && !pair_of_three;
  if (three) {
    if (c->top_t > 1) return fail(TM_ERR_INVALID, "three moduli are not combined with top_t > 1");
    if (c->zpad) return fail(TM_ERR_INVALID, "three moduli are not combined with TM_F_ZERO_PAD");
    int64_t m3 = d->m3;
    if (m3 == -1 && m1 == 0 && m2 == 0) {
      const int64_t mult = d->fold_mult == 0 ? 1 : d->fold_mult;
      int64_t m = std::max<int64_t>(mult * d->k, 1);
      if (m % 2 == 0) ++m;
      while ((double)m * (double)(m + 1) * (double)(m + 2) <= (double)d->n) m += 2;
      m1 = m;
      m2 = m + 1;
      m3 = m + 2;
    } else if (m3 > 0 && m1 > 0 && m2 > 0) {
      if (m1 < d->k || m2 < d->k || m3 < d->k) return fail(TM_ERR_INVALID, "need M1, M2, M3 >= K");
      if (gcd64(m1, m2) != 1 || gcd64(m1, m3) != 1 || gcd64(m2, m3) != 1)
        return fail(TM_ERR_INVALID, "M1, M2 and M3 must be pairwise co-prime");
      if ((double)m1 * (double)m2 * (double)m3 < (double)d->n) return fail(TM_ERR_INVALID, "need M1 M2 M3 >= N");
    } else {
      return fail(TM_ERR_INVALID, "m3 must be -1 (automatic, with m1 = m2 = 0) or > 0 (with explicit m1, m2)");
    }
    if (m3 >= (int64_t(1) << 30)) return fail(TM_ERR_INVALID, "fold lengths above 2^30 are not supported");
    c->three = 1;
    c->m3 = (int32_t)m3;
  } else if (d->m3 != 0 && !pair_of_three) {
    return fail(TM_ERR_INVALID, "bad m3");
  } else if (m1 == 0 && m2 == 0) {
    const int64_t mult = d->fold_mult == 0 ? 1 : d->fold_mult;
    m1 = std::max<int64_t>(mult * d->k, least_m0(d->n));
    m2 = m1 + 1;
  } else {
    if (m1 < 1 || m2 < 1) return fail(TM_ERR_INVALID, "explicit M1 and M2 must both be >= 1");
    if (m1 < d->k || m2 < d->k) return fail(TM_ERR_INVALID, "need M1 >= K and M2 >= K");
    if (gcd64(m1, m2) != 1) return fail(TM_ERR_INVALID, "M1 and M2 must be co-prime");
    if (m1 * m2 < d->n && !pair_of_three) return fail(TM_ERR_INVALID, "need M1 * M2 >= N");
  }
  if (m1 >= (int64_t(1) << 30) || m2 >= (int64_t(1) << 30))
    return fail(TM_ERR_INVALID, "fold lengths above 2^30 are not supported");
  c->m1 = (int32_t)m1;
  c->m2 = (int32_t)m2;
  if (m2 == m1 + 1) { c->ma = (int32_t)m1; c->mb = (int32_t)m2; c->dual = 1; }
  else if (m1 == m2 + 1) { c->ma = (int32_t)m2; c->mb = (int32_t)m1; c->dual = 1; c->swapped = 1; }
  else { c->ma = (int32_t)m1; c->mb = (int32_t)m2; }
  c->inv = mod_inverse(c->ma, c->mb);

  const bool both_int = d->x_dtype == TM_I8 && d->t_dtype == TM_I8;
  c->mode = (d->flags & TM_F_REAL) ? MODE_REAL
            : ((d->flags & TM_F_EXACT) || both_int) ? MODE_EXACT : MODE_REAL;

  const int64_t need = std::max<int64_t>(c->ma, c->mb) + d->k - 1;
  int p = 1;
  while ((int64_t(1) << p) < need) ++p;
  c->p_log2 = p;
  c->fft_in_lds = p <= fft_lds_max_log2(c->mode);
  // exact folds with an int8-valued template: correlation by the int8 GEMM
  // unless the FFT is asked for (TM_F_FFT, or TM_CORR_GEMM=0 for the process)
  c->cgemm = c->mode == MODE_EXACT && t_i8 && d->k <= kCgMaxK && !(d->flags & TM_F_FFT) &&
             (int64_t)(c->ma + c->mb) * (d->k + 63) <= (int64_t(1) << 32) && std::max(c->ma, c->mb) <= (1 << 25) &&
             env_int("TM_CORR_GEMM", 1) != 0;
  // TM_FFT_GLOBAL=1 also sends in-LDS lengths of 2^10 and more through global memory
  if (c->fft_in_lds && p >= 10 && env_int("TM_FFT_GLOBAL", 0) != 0) c->fft_in_lds = 0;
  if (!c->cgemm && !c->fft_in_lds && p <= kGfftMaxLog2) {
    // P = P1 x P2: blocks of B columns of P1 with B P1 = 4096 at most, rows of P2
    c->gfft = 1;
    c->g_logb = c->mode == MODE_EXACT ? 3 : 4;          // 128-byte row segments
    c->g_q = std::min(12 - c->g_logb, std::max(p - 7, (p + 1) / 2));
  }

  const int eb = dtype_bytes(d->x_dtype);
  // 4-byte signals: band fold (views of 64-column bands, R rows per task);
  // everything else that the streaming int8 fold below does not take: tiles
  c->band = d->x_dtype == TM_F32 && env_int("TM_FOLD_BAND", 1) != 0;
  // The band fold takes fold B of a consecutive pair as plain column sums of
  // its own view (a second pass over x, mostly from cache): the diagonal sums
  // of view A through LDS atomics took 3.4 times as long as both passes
  if (c->band && env_int("TM_BAND_DIAG", 0) == 0) c->dual = 0;
  auto view_of = [&](int64_t m) { return c->band ? make_band_view(d->n, m) : make_view(d->n, m, eb); };
  c->va = view_of(c->ma);
  if (c->dual) {
    c->vb = View{};
    c->vb.m = c->mb;
    c->vb.l = (int32_t)ceil_div(d->n, c->mb);
  } else {
    c->vb = view_of(c->mb);
  }
  const int64_t nviews = (int64_t)c->va.nrb * c->va.ncb + (c->dual ? 0 : (int64_t)c->vb.nrb * c->vb.ncb);
  if (nviews > (int64_t(1) << 30)) return fail(TM_ERR_UNSUPPORTED, "signal too large for one launch");
  if (c->band) {
    c->nband = (int32_t)ceil_div(nviews, kBandWaves);
    c->ntiles = 0;
  } else {
    c->ntiles = (int32_t)nviews;
  }
  c->acc_int = d->x_dtype == TM_I8 || c->mode == MODE_EXACT;
  // int8 signals with both moduli in [kSegMinM, kSegMaxM]: streaming fold over
  // segments of x.  A segment holds at most kSegMaxRows rows of the shorter
  // modulus (16-bit lane sums; a row straddling the end adds one) and, by
  // default, about N/512 bytes but at least 64 KiB (4 KiB for signals below
  // 1 MiB), so a batch of many instances gets long segments (the launch
  // lengthens them further) and one instance still spreads over many
  // workgroups.
  const int64_t mmin = std::min(c->ma, c->mb), mmax = std::max(c->ma, c->mb);
  if (d->x_dtype == TM_I8 && mmin >= kSegMinM && mmax <= kSegMaxM && ceil_div(d->n, mmin) < (1 << 23) &&
      env_int("TM_FOLD_STREAM", 1) != 0) {
    const int64_t cap = std::max<int64_t>(1, kSegMaxRows * mmin / 16 - 1);
    int64_t sc = env_int("TM_SEG_BYTES", 0) / 16;
    // about N/512 bytes, at least 64 KiB, except that a small signal still
    // spreads over 16 segments (of at least 4 KiB) when it is matched alone
    if (sc <= 0)
      sc = std::max<int64_t>(ceil_div(d->n, 512 * 16),
                             std::min<int64_t>(4096, std::max<int64_t>(256, ceil_div(d->n, 16 * 16))));
    sc = std::max<int64_t>(1, std::min(sc, cap));
    c->sfold = 1;
    c->seg_chunks = (int32_t)sc;
    c->nseg = segments_of(d->n, sc);
    c->ntiles = 0;
  }
  if (d->x_dtype == TM_I8 && ceil_div(d->n, std::min(c->ma, c->mb)) > (int64_t(1) << 24))
    return fail(TM_ERR_UNSUPPORTED, "int8 folds of more than 2^24 rows would overflow int32 buckets");
  const int64_t ytot = (int64_t)c->ma + c->k - 1 + c->mb + c->k - 1;
  size_t off = 0;
  if (c->acc_int) {
    // integer folds go straight to the bucket zone; the finish kernel forms
    // the literal folds from it
    c->acc_bytes = align256((size_t)(c->ma + c->mb + 2) * 4);
    c->nred = 0;
  } else {
    const int nrb = std::max(c->va.nrb, c->dual ? 0 : c->vb.nrb);
    int tpe = 1;
    while (tpe < nrb && tpe < kReduceThreads) tpe *= 2;
    c->red_tpe = tpe;
    c->nred = (int32_t)ceil_div(ytot, kReduceThreads / tpe);
    c->off_col_a = off; off = align256(off + (size_t)c->va.nrb * c->ma * 4);
    c->off_diag = off;
    if (c->dual) off = align256(off + (size_t)c->va.nrb * c->va.ncb * (c->va.cols + c->va.rows - 1) * 4);
    c->off_col_b = off;
    if (!c->dual) off = align256(off + (size_t)c->vb.nrb * c->mb * 4);
    c->off_y = off; off = align256(off + (size_t)ytot * 4);
  }
  if (c->gfft) {
    const size_t P = size_t(1) << p;
    c->off_gz = off; off = align256(off + P * (c->mode == MODE_EXACT ? 16 : 8));
    c->off_gss = off; off = align256(off + (P / kGfftThreads) * sizeof(double));
    c->off_gpart = off;
    off = align256(off + ((P >> c->g_q) >> c->g_logb) * gfft_part_bytes());
  }
  if (c->cgemm) {
    // rows of 64 shifts, 16 rows per GEMM workgroup; digit rows long enough
    // for the last row's band, in whole prep workgroups
    c->c_ks = (int32_t)align_up(ceil_div(d->k + 63, 64), 4);
    c->c_rta = (int32_t)ceil_div(ceil_div(c->ma, 64), kCgRows);
    c->c_rtb = (int32_t)ceil_div(ceil_div(c->mb, 64), kCgRows);
    const int64_t rtm = std::max(c->c_rta, c->c_rtb);
    c->c_lp = (int32_t)(ceil_div(64 * kCgRows * rtm + 64 * (int64_t)c->c_ks, kCgPrepThreads) * kCgPrepThreads);
    // digits needed by the largest possible |y|: L |x| for int8 and half
    // signals, the int32 range otherwise
    const int64_t lmax = std::max(ceil_div(d->n, c->ma), ceil_div(d->n, c->mb));
    int64_t ymax = int64_t(1) << 31;
    if (d->x_dtype == TM_I8) ymax = 128 * lmax;
    if (d->x_dtype == TM_F16) ymax = std::min<int64_t>(ymax, 65504 * lmax);
    c->c_nlcap = cgemm_limbs_for(ymax);
    c->c_lt = (int32_t)align_up(std::max<int64_t>(d->k + kCgPad + 16, 64 * (int64_t)c->c_ks + kCgPad + 32), 16);
    c->off_ylimb = off; off = align256(off + (size_t)2 * c->c_nlcap * c->c_lp);
    c->off_cpart = off; off = align256(off + (size_t)2 * rtm * 4 * 2 * sizeof(double));
  }
  if (c->top_t > 1 && (c->cgemm || c->gfft)) {
    // routes without the whole correlation in LDS keep it for the runner-up scan
    c->off_rtop = off;
    off = align256(off + (size_t)(c->ma + c->mb) * sizeof(double));
  }
  c->off_res = off; off = align256(off + sizeof(tm_result));
  c->ws_bytes = off;
  c->fold_lds = std::max(fold_lds_bytes(c->va, d->x_dtype), c->dual ? 0 : fold_lds_bytes(c->vb, d->x_dtype));
  c->finish_lds = finish_lds_bytes(p, c->mode);
  return TM_OK;
}

void fill_info(const Core& c, tm_plan_info* info) {
  info->m1 = c.m1;
  info->m2 = c.m2;
  info->l1 = (int32_t)ceil_div(c.n, c.m1);
  info->l2 = (int32_t)ceil_div(c.n, c.m2);
  info->fft_log2 = c.p_log2;
  info->exact = c.mode == MODE_EXACT;
  info->dual = c.dual;
  info->fft_in_lds = c.fft_in_lds;
  info->fft_global = c.gfft;
  info->corr_gemm = c.cgemm;
  info->m3 = c.m3;
  info->fold_tiles = c.ntiles;
  info->fold_segments = c.nseg;
  info->fold_bands = c.nband;
  info->workspace_bytes = (int64_t)(c.ws_bytes + c.acc_bytes);
  info->x_bytes = c.n * dtype_bytes(c.x_dtype);
}

// ---------------------------------------------------------------- pools

struct StreamPool {
  void* dev = nullptr;
  size_t cap = 0;
  void* acc = nullptr;           // integer bucket zone: all zero between launches
  size_t acc_cap = 0;
  bool acc_dirty = false;        // a launch sequence broke off after its fold
  bool exact_growth = false;     // grow to exactly what a launch needs (request server streams)
  // two pinned staging buffers for descriptor tables, used in turn: the host
  // fills one while the copy out of the other may still be in flight
  void* host[2] = {nullptr, nullptr};
  size_t hcap[2] = {0, 0};
  hipEvent_t staged[2] = {nullptr, nullptr};   // completes when that buffer's copy is done
  bool staged_pending[2] = {false, false};
  int next = 0;
  // the instance table the last batch left in `dev`, with what it was built
  // from: a batch of the same plans, signals and results on the same memory
  // finds it there and uploads nothing (any other use of `dev` clears it)
  bool tab_valid = false;
  std::vector<tm_plan> tab_plans;
  std::vector<const void*> tab_xs;
  const void* tab_out = nullptr;
  const void* tab_dev = nullptr;
  const void* tab_acc = nullptr;
  std::vector<Inst> tab_host;
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, StreamPool> g_pools;

// fold kernel timing (tm_profile_*), guarded by g_mu
bool g_prof_on = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_live;   // recorded, not yet read
std::vector<hipEvent_t> g_prof_free;
double g_prof_ms = 0.0;
int64_t g_prof_n = 0;
// the correlation kernel (k_cgemm, or k_finish on the FFT path), same scheme
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_corr_live;
double g_prof_corr_ms = 0.0;
int64_t g_prof_corr_n = 0;

hipError_t prof_event(hipEvent_t* e) {
  if (!g_prof_free.empty()) { *e = g_prof_free.back(); g_prof_free.pop_back(); return hipSuccess; }
  return hipEventCreate(e);
}

// the fold kernels of one launch (tiles, int8 segments, 4-byte bands), wrapped
// with the optional timing events
struct FoldWork { int tiles = 0; size_t lds = 0; int segs = 0; int bands = 0; };

hipError_t folds(const InstTable& tab, const FoldWork& w, hipStream_t s) {
  hipError_t e = launch_fold(tab, w.tiles, w.lds, s);
  if (e != hipSuccess) return e;
  if ((e = launch_fold_s8(tab, w.segs, s)) != hipSuccess) return e;
  return launch_fold_band(tab, w.bands, s);
}

// When profiling, the region's kernels carry a pair of events on their own
// dispatches: the elapsed time is first kernel start to last kernel end.
template <typename F>
hipError_t timed_region(std::vector<std::pair<hipEvent_t, hipEvent_t>>& live, F&& launch) {
  if (!g_prof_on) return launch();
  hipEvent_t a, b;
  hipError_t e = prof_event(&a);
  if (e != hipSuccess) return e;
  if ((e = prof_event(&b)) != hipSuccess) return e;
  g_launch_events.start = a;
  g_launch_events.stop = b;
  e = launch();
  const bool launched = g_launch_events.start == nullptr;
  g_launch_events = LaunchEvents{};
  if (e == hipSuccess && launched) {
    live.emplace_back(a, b);
  } else {
    g_prof_free.push_back(a);
    g_prof_free.push_back(b);
  }
  return e;
}

template <typename F>
hipError_t timed_corr(hipStream_t, F&& launch) {
  return timed_region(g_prof_corr_live, launch);
}

hipError_t timed_fold(const InstTable& tab, const FoldWork& w, hipStream_t s) {
  return timed_region(g_prof_live, [&] { return folds(tab, w, s); });
}
bool g_configured[64] = {};

// FP64 twiddles exp(-2 pi i e / P), e < P/2, stored FP64 or FP32: one table per
// (device, P, storage), shared by every plan and kept until the process ends.
std::mutex g_tw_mu;
std::map<std::tuple<int, int, int>, void*> g_twiddles;

tm_status shared_twiddles(int dev, int p_log2, int as_double, hipStream_t s, void** out) {
  std::lock_guard<std::mutex> lock(g_tw_mu);
  auto it = g_twiddles.find({dev, p_log2, as_double});
  if (it != g_twiddles.end()) { *out = it->second; return TM_OK; }
  void* tw = nullptr;
  const size_t half = std::max<size_t>((size_t(1) << p_log2) / 2, 1);
  TM_HIP(hipMalloc(&tw, half * (as_double ? 16 : 8)));
  hipError_t e = launch_twiddles(tw, p_log2, as_double, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipFree(tw);
    return fail(TM_ERR_DEVICE, std::string("twiddles: ") + hipGetErrorString(e));
  }
  g_twiddles[{dev, p_log2, as_double}] = tw;
  *out = tw;
  return TM_OK;
}

tm_status ensure_device(StreamPool& p, size_t need, hipStream_t s) {
  if (p.cap >= need) return TM_OK;
  if (p.dev) {
    TM_HIP(hipStreamSynchronize(s));   // in-flight work may still use the old buffer
    TM_HIP(hipFree(p.dev));
    p.dev = nullptr;
    p.cap = 0;
  }
  const size_t cap = align256(p.exact_growth ? need : need + need / 4);
  TM_HIP(hipMalloc(&p.dev, cap));
  p.cap = cap;
  return TM_OK;
}

tm_status ensure_acc(StreamPool& p, size_t need, hipStream_t s) {
  if (p.acc_cap < need) {
    if (p.acc) {
      TM_HIP(hipStreamSynchronize(s));
      TM_HIP(hipFree(p.acc));
      p.acc = nullptr;
      p.acc_cap = 0;
    }
    const size_t cap = align256(std::max<size_t>(p.exact_growth ? need : need + need / 4, 4096));
    TM_HIP(hipMalloc(&p.acc, cap));
    p.acc_cap = cap;
    p.acc_dirty = true;
  }
  if (p.acc_dirty) {
    TM_HIP(hipMemsetAsync(p.acc, 0, p.acc_cap, s));
    p.acc_dirty = false;
  }
  return TM_OK;
}

// Pick the next staging buffer, wait until its previous copy has been read,
// grow it if needed.  Returns its index in *slot.
tm_status ensure_host(StreamPool& p, size_t need, int* slot) {
  const int i = p.next;
  p.next ^= 1;
  *slot = i;
  if (p.staged_pending[i]) {
    TM_HIP(hipEventSynchronize(p.staged[i]));
    p.staged_pending[i] = false;
  }
  if (!p.staged[i]) TM_HIP(hipEventCreateWithFlags(&p.staged[i], hipEventDisableTiming));
  if (p.hcap[i] >= need) return TM_OK;
  if (p.host[i]) TM_HIP(hipHostFree(p.host[i]));
  p.host[i] = nullptr;
  p.hcap[i] = 0;
  const size_t cap = align256(need + need / 4);
  TM_HIP(hipHostMalloc(&p.host[i], cap, hipHostMallocDefault));
  p.hcap[i] = cap;
  return TM_OK;
}

bool is_device_pointer(const void* ptr) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

}  // namespace

// ---------------------------------------------------------------- pool control (request server)

namespace tmi {

void stream_pool_set_exact(int dev, hipStream_t s) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_pools[{dev, s}].exact_growth = true;
}

size_t stream_pool_device_bytes(int dev, hipStream_t s) {
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_pools.find({dev, s});
  return it == g_pools.end() ? 0 : it->second.cap + it->second.acc_cap;
}

hipError_t stream_pool_release(int dev, hipStream_t s, bool keep_entry) {
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_pools.find({dev, s});
  if (it == g_pools.end()) return hipSuccess;
  StreamPool& p = it->second;
  hipError_t err = hipStreamSynchronize(s);     // nothing on the stream may still use the pool
  auto note = [&](hipError_t e) { if (err == hipSuccess) err = e; };
  p.tab_valid = false;
  if (p.dev) note(hipFree(p.dev));
  if (p.acc) note(hipFree(p.acc));
  p.dev = p.acc = nullptr;
  p.cap = p.acc_cap = 0;
  p.acc_dirty = false;
  for (int i = 0; i < 2; ++i) {
    if (p.host[i]) note(hipHostFree(p.host[i]));
    if (p.staged[i]) note(hipEventDestroy(p.staged[i]));
    p.host[i] = nullptr;
    p.hcap[i] = 0;
    p.staged[i] = nullptr;
    p.staged_pending[i] = false;
  }
  if (!keep_entry) g_pools.erase(it);
  return err;
}

}  // namespace tmi

// ---------------------------------------------------------------- plan

constexpr int kResidentSlots = 8;   // stream pools per plan served from the plan's slabs

struct tm_plan_s {
  tm_plan_desc desc{};
  Core core;
  int device = 0;
  void* t_dev = nullptr;
  void* tw64 = nullptr;      // shared twiddle tables (not owned)
  void* tw32 = nullptr;
  void* tw_cols = nullptr;   // global-memory FFT: column blocks and rows
  void* tw_rows = nullptr;
  void* spec = nullptr;
  int8_t* tsh = nullptr;     // GEMM path: 16 shifted copies of the zero-padded template
  double tnorm1 = 0.0;
  double tnorm2 = 0.0;          // ||t||_2
  double tspec_max = 0.0;       // ||FFT_P(t)||_inf (real plans)
  tm_plan_s* pair2 = nullptr;   // three moduli: the plan of the pair (M3, M1) (owned)
  // single matches: the instance in device memory, one copy per stream pool
  // (the first kResidentSlots in slabs made at the plan's first single
  // match), each with a pinned staging copy and the host's image of it
  // (signal and result slot null)
  struct Resident {
    const StreamPool* pool = nullptr;
    Inst* dev = nullptr;
    Inst* staging = nullptr;
    hipEvent_t copied = nullptr;   // the last upload from `staging` is done
    bool pending = false;
    bool own = false;              // dev / staging allocated for this entry
    Inst shadow{};
  };
  Inst* res_dev = nullptr;
  Inst* res_host = nullptr;
  std::vector<Resident> resident;
};

namespace {

tm_status configure_device(int dev) {
  if (dev >= 0 && dev < 64 && !g_configured[dev]) {
    hipError_t e = configure_kernels();
    if (e != hipSuccess) return fail(TM_ERR_DEVICE, std::string("configure kernels: ") + hipGetErrorString(e));
    g_configured[dev] = true;
  }
  return TM_OK;
}

void fill_inst(const tm_plan_s* p, const void* x, Inst* in) {
  const Core& c = p->core;
  std::memset(in, 0, sizeof(*in));
  in->x = x;
  in->n = c.n;
  in->k = c.k;
  in->x_dtype = c.x_dtype;
  in->t_dtype = c.t_dtype;
  in->mode = c.mode;
  in->fold_store = c.fold_store;
  in->dual = c.dual;
  in->swapped = c.swapped;
  in->zpad = c.zpad;
  in->top_t = c.top_t;
  in->p_log2 = c.p_log2;
  in->va = c.va;
  in->vb = c.vb;
  in->ntiles = c.ntiles;
  in->nred = c.nred;
  in->red_tpe = c.red_tpe;
  in->acc_int = c.acc_int;
  in->sfold = c.sfold;
  in->nseg = c.nseg;
  in->seg_chunks = c.seg_chunks;
  in->band = c.band;
  in->nband = c.nband;
  in->inv_a_mod_b = c.inv;
  in->t = p->t_dev;
  in->spec = p->spec;
  in->tw = c.mode == MODE_EXACT ? p->tw64 : p->tw32;
  in->gfft = c.gfft;
  in->g_q = c.g_q;
  in->g_logb = c.g_logb;
  in->tw_cols = p->tw_cols;
  in->tw_rows = p->tw_rows;
  in->tnorm1 = p->tnorm1;
  in->tspec_max = p->tspec_max;
  in->tnorm2 = p->tnorm2;
  in->cgemm = c.cgemm;
  in->c_nlcap = c.c_nlcap;
  in->c_lp = c.c_lp;
  in->c_ks = c.c_ks;
  in->c_rta = c.c_rta;
  in->c_rtb = c.c_rtb;
  in->c_lt = c.c_lt;
  in->c_split = 1;
  in->tsh = p->tsh;
}

void place_workspace(const Core& c, char* base, char* acc, Inst* in) {
  if (c.gfft) {
    in->gz = base + c.off_gz;
    in->gss = reinterpret_cast<double*>(base + c.off_gss);
    in->gpart = base + c.off_gpart;
  }
  if (c.top_t > 1 && (c.cgemm || c.gfft)) in->rtop = reinterpret_cast<double*>(base + c.off_rtop);
  if (c.cgemm) {
    in->ylimb = reinterpret_cast<int8_t*>(base + c.off_ylimb);
    in->cpart = base + c.off_cpart;
    in->cmax = reinterpret_cast<int*>(acc) + c.ma + c.mb;
  }
  if (c.acc_int) {
    in->yp = reinterpret_cast<int*>(acc);
    in->y = base + c.off_y;
    return;
  }
  in->col_a = base + c.off_col_a;
  in->diag = c.dual ? base + c.off_diag : nullptr;
  in->col_b = c.dual ? nullptr : base + c.off_col_b;
  in->y = base + c.off_y;
}

tm_status check_plan_for_match(tm_plan p) {
  if (!p) return fail(TM_ERR_INVALID, "null plan");
  if (!p->core.cgemm && !p->core.fft_in_lds && !p->core.gfft)
    return fail(TM_ERR_UNSUPPORTED, "FFT length 2^" + std::to_string(p->core.p_log2) +
                                        " exceeds one workgroup's LDS on this build");
  return TM_OK;
}

tm_status check_x(const tm_plan_s* p, const void* x) {
  if (!x) return fail(TM_ERR_INVALID, "null signal pointer");
  const uintptr_t a = reinterpret_cast<uintptr_t>(x);
  if (a % (uintptr_t)dtype_bytes(p->core.x_dtype)) return fail(TM_ERR_INVALID, "signal is not aligned to its element size");
  return TM_OK;
}

double host_value(const void* t, int dt, int64_t i) {
  switch (dt) {
    case TM_I8: return (double)static_cast<const int8_t*>(t)[i];
    case TM_F32: return (double)static_cast<const float*>(t)[i];
    case TM_BF16: {
      uint32_t u = (uint32_t)static_cast<const uint16_t*>(t)[i] << 16;
      float f;
      std::memcpy(&f, &u, 4);
      return f;
    }
    default: {
      const uint16_t h = static_cast<const uint16_t*>(t)[i];
      const int sgn = h >> 15, ex = (h >> 10) & 31, man = h & 1023;
      double v = ex == 0 ? std::ldexp((double)man, -24) : (ex == 31 ? INFINITY : std::ldexp((double)(man | 1024), ex - 25));
      return sgn ? -v : v;
    }
  }
}

// the descriptor of a three-moduli plan's second pair (M3, M1)
tm_plan_desc pair2_desc(const tm_plan_desc& d, const Core& c) {
  tm_plan_desc d2 = d;
  d2.m1 = c.m3;
  d2.m2 = c.m1;
  d2.m3 = 0;
  d2.top_t = 1;
  return d2;
}

}  // namespace

extern "C" {

const char* tm_version(void) { return "0.1.0"; }

const char* tm_status_string(tm_status s) {
  switch (s) {
    case TM_OK: return "ok";
    case TM_ERR_INVALID: return "invalid argument";
    case TM_ERR_NOMEM: return "out of memory";
    case TM_ERR_DEVICE: return "device error";
    case TM_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* tm_last_error(void) { return g_err.c_str(); }

tm_status tm_plan_params(const tm_plan_desc* desc, tm_plan_info* info) {
  if (!info) return fail(TM_ERR_INVALID, "null info");
  Core c;
  const bool t_i8 = desc && desc->t_dtype == TM_I8;
  tm_status s = compute_core(desc, &c, t_i8);
  if (s != TM_OK) return s;
  fill_info(c, info);
  if (c.three) {
    Core c2;
    const tm_plan_desc d2 = pair2_desc(*desc, c);
    s = compute_core(&d2, &c2, t_i8, true);
    if (s != TM_OK) return s;
    info->workspace_bytes += (int64_t)(c2.ws_bytes + c2.acc_bytes);
  }
  return TM_OK;
}

static tm_status plan_create_impl(const tm_plan_desc* desc, const void* t, int t_is_device, void* stream,
                                  tm_plan* out, bool pair_of_three);

tm_status tm_plan_create(const tm_plan_desc* desc, const void* t, int t_is_device, void* stream,
                         tm_plan* out) {
  tm_status st = plan_create_impl(desc, t, t_is_device, stream, out, false);
  if (st != TM_OK || !(*out)->core.three) return st;
  // three moduli: the second pair (M3, M1) as a plan of its own
  const tm_plan_desc d2 = pair2_desc(*desc, (*out)->core);
  tm_plan p2 = nullptr;
  st = plan_create_impl(&d2, t, t_is_device, stream, &p2, true);
  if (st != TM_OK) {
    const std::string msg = g_err;
    (void)tm_plan_destroy(*out);
    *out = nullptr;
    return fail(st, msg);
  }
  (*out)->pair2 = p2;
  return TM_OK;
}

static tm_status plan_create_impl(const tm_plan_desc* desc, const void* t, int t_is_device, void* stream,
                                  tm_plan* out, bool pair_of_three) {
  if (!out) return fail(TM_ERR_INVALID, "null plan output");
  *out = nullptr;
  if (!t) return fail(TM_ERR_INVALID, "null template pointer");
  Core c;
  tm_status st = compute_core(desc, &c, false, pair_of_three);
  if (st != TM_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0;
  TM_HIP(hipGetDevice(&dev));
  st = configure_device(dev);
  if (st != TM_OK) return st;

  const size_t tb = (size_t)c.k * dtype_bytes(c.t_dtype);
  std::vector<unsigned char> th(tb);
  if (t_is_device) {
    TM_HIP(hipMemcpy(th.data(), t, tb, hipMemcpyDeviceToHost));
  } else {
    std::memcpy(th.data(), t, tb);
  }
  double norm1 = 0.0, sumsq = 0.0;
  bool t_i8 = true;
  for (int64_t i = 0; i < c.k; ++i) {
    const double v = host_value(th.data(), c.t_dtype, i);
    if (!std::isfinite(v)) return fail(TM_ERR_INVALID, "template holds a non-finite value");
    if (c.mode == MODE_EXACT && v != std::nearbyint(v))
      return fail(TM_ERR_INVALID, "exact path needs an integer-valued template");
    t_i8 = t_i8 && v == std::nearbyint(v) && v >= -128.0 && v <= 127.0;
    norm1 += std::fabs(v);
    sumsq += v * v;
  }
  st = compute_core(desc, &c, t_i8, pair_of_three);
  if (st != TM_OK) return st;
  if (!c.cgemm && !c.fft_in_lds && !c.gfft)
    return fail(TM_ERR_UNSUPPORTED, "FFT length 2^" + std::to_string(c.p_log2) + " is above 2^" +
                                        std::to_string(kGfftMaxLog2));

  tm_plan_s* p = new tm_plan_s();
  p->desc = *desc;
  p->core = c;
  p->device = dev;
  p->tnorm1 = norm1;
  p->tnorm2 = std::sqrt(sumsq);
  const size_t P = size_t(1) << c.p_log2;
  void* z = nullptr;
  auto cleanup = [&]() {
    if (z) (void)hipFree(z);
    if (p->t_dev) (void)hipFree(p->t_dev);
    if (p->spec) (void)hipFree(p->spec);
    if (p->tsh) (void)hipFree(p->tsh);
    if (p->res_dev) (void)hipFree(p->res_dev);
    if (p->res_host) (void)hipHostFree(p->res_host);
    delete p;
  };
#define TM_HIP_PLAN(expr)                                                              \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      cleanup();                                                                       \
      return fail(e_ == hipErrorOutOfMemory ? TM_ERR_NOMEM : TM_ERR_DEVICE,            \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                  \
    }                                                                                  \
  } while (0)
  TM_HIP_PLAN(hipMalloc(&p->t_dev, std::max<size_t>(tb, 16)));
  TM_HIP_PLAN(hipMemcpyAsync(p->t_dev, th.data(), tb, hipMemcpyHostToDevice, s));
  if (c.cgemm) {
    // the GEMM path needs no spectrum: 16 copies of [0 (pad + sh), t, 0 ...],
    // byte q of copy sh stored at ((q / 16) * 16 + sh) * 16 + q % 16
    const size_t lt = (size_t)c.c_lt;
    std::vector<int8_t> h(16 * lt, 0);
    for (size_t sh = 0; sh < 16; ++sh)
      for (int64_t i = 0; i < c.k; ++i) {
        const size_t q = kCgPad + sh + (size_t)i;
        h[((q / 16) * 16 + sh) * 16 + q % 16] = (int8_t)host_value(th.data(), c.t_dtype, i);
      }
    TM_HIP_PLAN(hipMalloc(&p->tsh, h.size()));
    TM_HIP_PLAN(hipMemcpyAsync(p->tsh, h.data(), h.size(), hipMemcpyHostToDevice, s));
    TM_HIP_PLAN(hipStreamSynchronize(s));
    *out = p;
    return TM_OK;
  }
  st = shared_twiddles(dev, c.p_log2, 1, s, &p->tw64);
  if (st == TM_OK && c.mode == MODE_REAL) st = shared_twiddles(dev, c.p_log2, 0, s, &p->tw32);
  if (st == TM_OK && c.gfft) st = shared_twiddles(dev, c.g_logb + c.g_q, c.mode == MODE_EXACT, s, &p->tw_cols);
  if (st == TM_OK && c.gfft) st = shared_twiddles(dev, c.p_log2 - c.g_q, c.mode == MODE_EXACT, s, &p->tw_rows);
  if (st != TM_OK) {
    cleanup();
    return st;
  }
  TM_HIP_PLAN(hipMalloc(&p->spec, P * (c.mode == MODE_EXACT ? 16 : 8)));
  TM_HIP_PLAN(hipMalloc(&z, P * 16));
  TM_HIP_PLAN(launch_spectrum(p->t_dev, c.t_dtype, c.k, c.p_log2, static_cast<const double*>(p->tw64),
                              static_cast<double*>(z), p->spec, c.mode == MODE_EXACT,
                              c.gfft ? c.p_log2 - c.g_q : 0, s));
  TM_HIP_PLAN(hipStreamSynchronize(s));
  if (c.mode == MODE_REAL) {
    // ||FFT_P(t)||_inf in FP64 (z holds the unscaled transform) for the
    // results' error bound
    std::vector<double> zh((size_t)2 * P);
    TM_HIP_PLAN(hipMemcpy(zh.data(), z, (size_t)P * 16, hipMemcpyDeviceToHost));
    double mx = 0.0;
    for (size_t i = 0; i < (size_t)P; ++i) mx = std::max(mx, std::hypot(zh[2 * i], zh[2 * i + 1]));
    p->tspec_max = mx;
  }
  TM_HIP_PLAN(hipFree(z));
  z = nullptr;
#undef TM_HIP_PLAN
  *out = p;
  return TM_OK;
}

tm_status tm_plan_destroy(tm_plan p) {
  if (!p) return TM_OK;
  if (p->pair2) {
    const tm_status st = tm_plan_destroy(p->pair2);
    p->pair2 = nullptr;
    if (st != TM_OK) return st;
  }
  TM_HIP(hipDeviceSynchronize());
  for (auto& r : p->resident) {
    if (r.copied) TM_HIP(hipEventDestroy(r.copied));
    if (r.own) {
      TM_HIP(hipFree(r.dev));
      TM_HIP(hipHostFree(r.staging));
    }
  }
  p->resident.clear();
  if (p->res_dev) TM_HIP(hipFree(p->res_dev));
  if (p->res_host) TM_HIP(hipHostFree(p->res_host));
  if (p->t_dev) TM_HIP(hipFree(p->t_dev));
  if (p->spec) TM_HIP(hipFree(p->spec));
  if (p->tsh) TM_HIP(hipFree(p->tsh));
  delete p;
  return TM_OK;
}

tm_status tm_plan_get_info(tm_plan p, tm_plan_info* info) {
  if (!p || !info) return fail(TM_ERR_INVALID, "null argument");
  fill_info(p->core, info);
  if (p->pair2) info->workspace_bytes += (int64_t)(p->pair2->core.ws_bytes + p->pair2->core.acc_bytes);
  return TM_OK;
}

tm_status tm_match_batch(int32_t count, const tm_plan* plans, const void* const* xs, tm_result* out,
                         void* stream);

// The single-match instance in device memory for a stream's pool.  The copy
// is rewritten only when the host's instance differs from it, signal and
// result slot aside (the fold kernel of each match stores those two): through
// the entry's pinned staging copy, ordered on the stream after the kernels
// that may still read the old one.  The first match of a plan on a stream, or
// one after the pool's workspace moved, pays for one small upload.
static tm_status resident_inst(tm_plan p, StreamPool& pool, const Inst& host, hipStream_t s,
                               const Inst** dev) {
  Inst key;
  std::memcpy(&key, &host, sizeof(Inst));
  key.x = nullptr;
  key.out = nullptr;
  tm_plan_s::Resident* r = nullptr;
  for (auto& e : p->resident)
    if (e.pool == &pool) r = &e;
  if (r && std::memcmp(&r->shadow, &key, sizeof(Inst)) == 0) {
    *dev = r->dev;
    return TM_OK;
  }
  if (!r) {
    if (!p->res_dev) {   // the plan's first single match: its slabs
      void* dv = nullptr;
      void* hs = nullptr;
      TM_HIP(hipMalloc(&dv, kResidentSlots * sizeof(Inst)));
      const hipError_t he = hipHostMalloc(&hs, kResidentSlots * sizeof(Inst), hipHostMallocDefault);
      if (he != hipSuccess) {
        (void)hipFree(dv);
        TM_HIP(he);
      }
      p->res_dev = static_cast<Inst*>(dv);
      p->res_host = static_cast<Inst*>(hs);
    }
    tm_plan_s::Resident e;
    e.pool = &pool;
    const size_t i = p->resident.size();
    if (i < (size_t)kResidentSlots) {
      e.dev = p->res_dev + i;
      e.staging = p->res_host + i;
    } else {
      TM_HIP(hipMalloc(reinterpret_cast<void**>(&e.dev), sizeof(Inst)));
      hipError_t he = hipHostMalloc(reinterpret_cast<void**>(&e.staging), sizeof(Inst), hipHostMallocDefault);
      if (he != hipSuccess) {
        (void)hipFree(e.dev);
        TM_HIP(he);
      }
      e.own = true;
    }
    p->resident.push_back(e);
    r = &p->resident.back();
    TM_HIP(hipEventCreateWithFlags(&r->copied, hipEventDisableTiming));
  } else if (r->pending) {
    TM_HIP(hipEventSynchronize(r->copied));   // the staging copy is about to change
    r->pending = false;
  }
  std::memcpy(r->staging, &key, sizeof(Inst));
  std::memset(&r->shadow, 0, sizeof(Inst));     // no match until the upload is enqueued
  TM_HIP(hipMemcpyAsync(r->dev, r->staging, sizeof(Inst), hipMemcpyHostToDevice, s));
  const hipError_t er = hipEventRecord(r->copied, s);
  if (er != hipSuccess) {
    (void)hipStreamSynchronize(s);   // the staging copy must not change under the upload
    TM_HIP(er);
  }
  r->pending = true;
  std::memcpy(&r->shadow, &key, sizeof(Inst));
  *dev = r->dev;
  return TM_OK;
}

// Workgroups sharing each row tile's band in a single match's product kernel
// (TM_CGEMM_SPLIT, default 1).  With a split, the shares are added into int64
// accumulators and the final kernel takes the argmax from them.  Measured on
// a 16 MiB fp32 instance (M = 4096, K = 4096): the product kernel falls from
// about 11 to 5 us at a split of 14, but the final kernel's pass over the
// accumulators raises it from about 7 to 22 us, so the split stays off.
static int cgemm_split(const Core& c) {
  const int64_t env = env_int("TM_CGEMM_SPLIT", 1);
  return (int)std::max<int64_t>(1, std::min<int64_t>(env, std::max(1, c.c_ks)));
}

// Product kernel choice (TM_CGEMM_KIND): 0 automatic (batches of at least
// 2048 row tiles one wave per row tile, else each row tile's band split over
// a workgroup's waves), 1 always the split band, 2 per instance wherever its
// LDS holds the operands (single matches included), 3 one wave per row tile
// for every batch.  Measured on 4096 uneven int8 instances (N up to 2^20,
// K up to 4096), the per-instance kernel's correlation stage took about
// 600 us per batch against 390 us for prep, row-tile product and final
// kernel: with up to 133 KB of LDS per instance a compute unit holds one or
// two of its workgroups, and their staging loads leave the matrix cores idle
// (3% busy).
static int cgemm_kind() { return (int)env_int("TM_CGEMM_KIND", 0); }

// LDS classes of the per-instance product kernel: footprints that let 8, 5,
// 3, 2 and 1 workgroups share a compute unit; kCgClasses: too large for it
static int cg_class(const Core& c) {
  static const size_t lim[kCgClasses] = {20u << 10, 32u << 10, 53u << 10, 80u << 10, kCg2MaxLds};
  const size_t b = cgemm_inst_lds_bytes(c.c_lt, c.c_lp, c.c_nlcap, c.c_rta + c.c_rtb, std::max(c.c_rta, c.c_rtb));
  for (int i = 0; i < kCgClasses; ++i)
    if (b <= lim[i]) return i;
  return kCgClasses;
}

static tm_status match_one(tm_plan p, const void* x, tm_result* out, double* y1, double* y2,
                           double* r1, double* r2, void* stream) {
  tm_status st = check_plan_for_match(p);
  if (st != TM_OK) return st;
  if (p->core.three) {
    if (y1 || y2 || r1 || r2) return fail(TM_ERR_UNSUPPORTED, "no intermediates for three-moduli plans");
    return tm_match_batch(1, &p, &x, out, stream);
  }
  st = check_x(p, x);
  if (st != TM_OK) return st;
  if (!out) return fail(TM_ERR_INVALID, "null result pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool dev_out = is_device_pointer(out);
  std::lock_guard<std::mutex> lock(g_mu);
  StreamPool& pool = g_pools[{p->device, s}];
  pool.tab_valid = false;                // the workspace is reused below
  st = ensure_device(pool, p->core.ws_bytes, s);
  if (st != TM_OK) return st;
  const int split = p->core.cgemm ? cgemm_split(p->core) : 1;
  const size_t cacc_bytes = split > 1 ? align256((size_t)(p->core.ma + p->core.mb) * sizeof(long long)) : 0;
  st = ensure_acc(pool, p->core.acc_bytes + cacc_bytes, s);
  if (st != TM_OK) return st;
  Inst one;
  fill_inst(p, x, &one);
  char* base = static_cast<char*>(pool.dev);
  place_workspace(p->core, base, static_cast<char*>(pool.acc), &one);
  if (split > 1) {
    one.c_split = split;
    one.cacc = reinterpret_cast<long long*>(static_cast<char*>(pool.acc) + p->core.acc_bytes);
  }
  one.tile_base = 0;
  one.seg_base = 0;
  one.band_base = 0;
  one.red_base = 0;
  one.out = dev_out ? out : reinterpret_cast<tm_result*>(base + p->core.off_res);
  one.dbg_y1 = y1;
  one.dbg_y2 = y2;
  one.dbg_r1 = r1;
  one.dbg_r2 = r2;
  const Inst* dev_one = nullptr;
  st = resident_inst(p, pool, one, s, &dev_one);
  if (st != TM_OK) return st;
  InstTable tab{};
  tab.table = nullptr;
  tab.count = 1;
  tab.one = dev_one;
  tab.x = one.x;
  tab.out = one.out;
  FoldWork fw;
  fw.tiles = p->core.ntiles;
  fw.lds = p->core.fold_lds;
  fw.segs = p->core.nseg;
  fw.bands = p->core.nband;
  // the fold kernel stores the signal and result slot for the kernels after it
  if (fw.tiles + fw.segs + fw.bands <= 0) return fail(TM_ERR_INVALID, "plan without fold work");
  TM_HIP(timed_fold(tab, fw, s));
  pool.acc_dirty = true;                 // until the finish kernel is enqueued
  TM_HIP(launch_reduce(tab, p->core.nred, s));
  const Core& cc = p->core;
  if (cc.cgemm && split == 1 && cgemm_kind() == 2 && cg_class(cc) < kCgClasses) {
    // digit rows, then product .. resolve in one workgroup
    const CgLaunch cl = cgemm_launch(2 * (int64_t)cc.c_lp, 2 * (int64_t)cc.c_lp, 1);
    TM_HIP(launch_cgemm_prep(tab, nullptr, 1, cl.chunk, cl.prep_y, s));
    TM_HIP(timed_corr(s, [&] {
      return launch_cgemm_inst(tab, nullptr, 1,
                               cgemm_inst_lds_bytes(cc.c_lt, cc.c_lp, cc.c_nlcap, cc.c_rta + cc.c_rtb,
                                                    std::max(cc.c_rta, cc.c_rtb)), s);
    }));
  } else if (cc.cgemm) {
    const CgLaunch cl = cgemm_launch(2 * (int64_t)cc.c_lp, 2 * (int64_t)cc.c_lp, 1);
    TM_HIP(launch_cgemm_prep(tab, nullptr, 1, cl.chunk, cl.prep_y, s));
    const bool ring = split == 1 && cgemm_kind() == 4 && cc.c_nlcap <= 3;
    if (ring)
      TM_HIP(timed_corr(s, [&] { return launch_cgemm_ring(tab, nullptr, 1, cc.c_rta + cc.c_rtb, s); }));
    else if (split == 1 && (cgemm_kind() == 3 || cgemm_kind() == 4))
      TM_HIP(timed_corr(s, [&] { return launch_cgemm_wave(tab, nullptr, 1, cc.c_rta + cc.c_rtb, cc.c_nlcap, s); }));
    else
      TM_HIP(timed_corr(s, [&] { return launch_cgemm_gemm(tab, nullptr, 1, (cc.c_rta + cc.c_rtb) * split,
                                                          cc.c_nlcap, s); }));
    TM_HIP(launch_cgemm_final(tab, nullptr, 1, s, split == 1 && cg_lean_core(cc), ring));
  }
  else if (p->core.gfft) TM_HIP(launch_gfft(one, dev_one, s));
  else TM_HIP(timed_corr(s, [&] { return launch_finish(tab, nullptr, 1, p->core.mode, p->core.p_log2,
                                                        p->core.finish_lds, s); }));
  pool.acc_dirty = false;
  if (!dev_out) {
    TM_HIP(hipMemcpyAsync(out, one.out, sizeof(tm_result), hipMemcpyDeviceToHost, s));
    TM_HIP(hipStreamSynchronize(s));
  }
  return TM_OK;
}

tm_status tm_match(tm_plan p, const void* x, tm_result* out, void* stream) {
  return match_one(p, x, out, nullptr, nullptr, nullptr, nullptr, stream);
}

tm_status tm_match_intermediates(tm_plan p, const void* x, tm_result* out, double* y1, double* y2,
                                 double* r1, double* r2, void* stream) {
  return match_one(p, x, out, y1, y2, r1, r2, stream);
}

// tm_match without the per-stream pool: the instance record, the bucket zone
// and the workspace live in the device's scratch array (layout: record, then
// buckets, then workspace, each 256-byte aligned).  Host code uses only the
// address configure_kernels looked up for the plan's device.
tm_status tm_match_noalloc(tm_plan p, const void* x, tm_result* out, void* stream) {
  tm_status st = check_plan_for_match(p);
  if (st != TM_OK) return st;
  if (p->core.three) return fail(TM_ERR_UNSUPPORTED, "tm_match_noalloc: three-moduli plans are not supported");
  st = check_x(p, x);
  if (st != TM_OK) return st;
  if (!out) return fail(TM_ERR_INVALID, "null result pointer");
  if (!is_device_pointer(out)) return fail(TM_ERR_INVALID, "tm_match_noalloc: out must be device memory");
  int cur = -1;
  TM_HIP(hipGetDevice(&cur));
  if (cur != p->device) return fail(TM_ERR_INVALID, "tm_match_noalloc: the plan's device is not current");
  char* scr = static_cast<char*>(scratch_device_ptr(p->device));
  if (!scr) return fail(TM_ERR_DEVICE, "tm_match_noalloc: no scratch address for this device");
  const Core& c = p->core;
  const size_t off_acc = align256(sizeof(Inst));
  const size_t off_ws = off_acc + align256(c.acc_bytes);
  if (off_ws + c.ws_bytes > kScratchBytes)
    return fail(TM_ERR_UNSUPPORTED, "tm_match_noalloc: the plan needs " + std::to_string(off_ws + c.ws_bytes) +
                                        " bytes of scratch, above the " + std::to_string(kScratchBytes) +
                                        "-byte maximum");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Inst one;
  fill_inst(p, x, &one);
  place_workspace(c, scr + off_ws, scr + off_acc, &one);
  one.out = out;
  Inst* dev_one = reinterpret_cast<Inst*>(scr);
  // record and zeroed buckets (the previous call's contents are not trusted)
  TM_HIP(launch_noalloc_setup(one, dev_one, reinterpret_cast<int*>(scr + off_acc), (int64_t)(c.acc_bytes / 4), s));
  InstTable tab{};
  tab.table = nullptr;
  tab.count = 1;
  tab.one = dev_one;
  tab.x = one.x;
  tab.out = one.out;
  FoldWork fw;
  fw.tiles = c.ntiles;
  fw.lds = c.fold_lds;
  fw.segs = c.nseg;
  fw.bands = c.nband;
  if (fw.tiles + fw.segs + fw.bands <= 0) return fail(TM_ERR_INVALID, "plan without fold work");
  TM_HIP(folds(tab, fw, s));
  TM_HIP(launch_reduce(tab, c.nred, s));
  if (c.cgemm) {
    const CgLaunch cl = cgemm_launch(2 * (int64_t)c.c_lp, 2 * (int64_t)c.c_lp, 1);
    TM_HIP(launch_cgemm_prep(tab, nullptr, 1, cl.chunk, cl.prep_y, s));
    TM_HIP(launch_cgemm_gemm(tab, nullptr, 1, c.c_rta + c.c_rtb, c.c_nlcap, s));
    TM_HIP(launch_cgemm_final(tab, nullptr, 1, s, cg_lean_core(c)));
  } else if (c.gfft) {
    TM_HIP(launch_gfft(one, dev_one, s));
  } else {
    TM_HIP(launch_finish(tab, nullptr, 1, c.mode, c.p_log2, c.finish_lds, s));
  }
  return TM_OK;
}

// One launch sequence for `count` instances.  Without `cmb` the results go
// to out[0..count); with it the instances are the expanded list of a batch
// with three-moduli plans: their results stay in device scratch and one
// combine kernel writes out[0..cmb->size()).
// Host-side layout and launch parameters of one batch.
struct BatchPlan {
  int32_t count = 0, n_user = 0;
  bool dev_out = false, scratch_res = false, use_inst = false;
  std::vector<size_t> ws_off, acc_off;
  std::vector<int32_t> seg_chunks, nseg, order;
  size_t ws = 0, accb = 0, fold_lds = 0;
  int64_t tiles = 0, chunks = 0, segs = 0, bands = 0, cps = 0, cp_max = 0, cgs = 0, cg_limbs_max = 0, cg_tasks = 0;
  int32_t ncg_inst = 0;
  bool cg_lean = true;   // every product instance: int8 signal and template, top_t 1
  // device layout: [instance workspaces][results][user results][table][lists][combine records]
  size_t off_res = 0, off_ures = 0, off_tab = 0, tab_bytes = 0, off_lists = 0, list_bytes = 0, cmb_bytes = 0,
         total = 0;
};

static tm_status plan_batch(int32_t count, const tm_plan* plans, bool dev_out, const std::vector<Combine3>* cmb,
                            BatchPlan& b) {
  b.count = count;
  b.dev_out = dev_out;
  b.scratch_res = !dev_out || cmb;           // instance results in the workspace
  b.n_user = cmb ? (int32_t)cmb->size() : count;
  b.ws_off.resize(count);
  b.acc_off.resize(count);
  b.seg_chunks.resize(count);
  b.nseg.resize(count);
  int64_t launch_bytes = 0;
  for (int32_t i = 0; i < count; ++i) launch_bytes += plans[i]->core.n * dtype_bytes(plans[i]->core.x_dtype);
  for (int32_t i = 0; i < count; ++i) {
    const Core& c = plans[i]->core;
    b.ws_off[i] = b.ws;
    b.ws += c.ws_bytes;
    b.acc_off[i] = b.accb;
    b.accb += c.acc_bytes;
    b.tiles += c.ntiles;
    b.seg_chunks[i] = c.seg_chunks;
    b.nseg[i] = c.nseg;
    if (c.sfold) {
      b.seg_chunks[i] = (int32_t)launch_seg_chunks(c, launch_bytes);
      b.nseg[i] = segments_of(c.n, b.seg_chunks[i]);
    }
    b.segs += b.nseg[i];
    b.bands += c.nband;
    b.chunks += c.nred;
    if (c.cgemm) {
      b.cps += 2 * (int64_t)c.c_lp;
      b.cp_max = std::max<int64_t>(b.cp_max, 2 * (int64_t)c.c_lp);
      b.cgs = std::max<int64_t>(b.cgs, c.c_rta + c.c_rtb);
      b.cg_limbs_max = std::max<int64_t>(b.cg_limbs_max, c.c_nlcap);
    }
    b.fold_lds = std::max(b.fold_lds, c.fold_lds);
  }
  if (b.tiles > 0x7fffffff || b.chunks > 0x7fffffff || b.segs > 0x7fffffff || b.bands > 0x7fffffff ||
      b.cps > 0x7fffffff || b.cgs > 0x7fffffff)
    return fail(TM_ERR_UNSUPPORTED, "batch too large");
  // product kernel of the GEMM-correlation instances: per row tile, or per
  // instance with its operands in LDS when asked for
  for (int32_t i = 0; i < count; ++i) {
    const Core& c = plans[i]->core;
    if (!c.cgemm) continue;
    b.cg_tasks += c.c_rta + c.c_rtb;
    b.cg_lean = b.cg_lean && c.x_dtype == TM_I8 && c.t_dtype == TM_I8 && c.top_t == 1;
  }
  b.use_inst = cgemm_kind() == 2 && b.cg_tasks > 0;
  // the GEMM-correlation instances first: by product-kernel LDS class, the
  // largest first within a class (they start first); then the finish
  // launches grouped by (mode, FFT length) so each gets its own LDS size
  b.order.resize(count);
  const bool use_inst = b.use_inst;
  if (!use_inst) {
    // a stable counting sort on a small key (product route first, then the
    // finish launches by mode and FFT length): one pass over the plans
    // instead of a comparison sort that revisits every plan log(count) times
    constexpr int kKeys = 2 + 2 * 32;
    std::vector<int32_t> key((size_t)count);
    int32_t start[kKeys + 1] = {};
    for (int32_t i = 0; i < count; ++i) {
      const Core& c = plans[i]->core;
      key[i] = c.cgemm ? 0 : 1 + (c.mode != 0 ? 32 : 0) + std::min(c.p_log2, 31);
      ++start[key[i] + 1];
    }
    for (int k = 0; k < kKeys; ++k) start[k + 1] += start[k];
    for (int32_t i = 0; i < count; ++i) b.order[start[key[i]]++] = i;
  } else {
    for (int32_t i = 0; i < count; ++i) b.order[i] = i;
    std::stable_sort(b.order.begin(), b.order.end(), [&](int32_t x, int32_t y) {
      const Core& ca = plans[x]->core;
      const Core& cb = plans[y]->core;
      if (ca.cgemm != cb.cgemm) return ca.cgemm > cb.cgemm;
      if (ca.cgemm) {
        const int ka = cg_class(ca), kb = cg_class(cb);
        if (ka != kb) return ka < kb;
        return (int64_t)ca.k * (ca.ma + ca.mb) > (int64_t)cb.k * (cb.ma + cb.mb);
      }
      return ca.mode != cb.mode ? ca.mode < cb.mode : ca.p_log2 < cb.p_log2;
    });
  }
  while (b.ncg_inst < count && plans[b.order[b.ncg_inst]]->core.cgemm) ++b.ncg_inst;
  b.off_res = align256(b.ws);
  // combined user results staged on the device when out is host memory
  b.off_ures = align256(b.off_res + (b.scratch_res ? sizeof(tm_result) * (size_t)count : 0));
  b.off_tab = align256(b.off_ures + (cmb && !dev_out ? sizeof(tm_result) * (size_t)b.n_user : 0));
  b.tab_bytes = sizeof(Inst) * (size_t)count;
  b.off_lists = b.off_tab + b.tab_bytes;   // sizeof(Inst) keeps the list 16-byte aligned
  b.list_bytes = align_up(sizeof(int32_t) * (size_t)count, 16);
  b.cmb_bytes = cmb ? sizeof(Combine3) * cmb->size() : 0;
  b.total = b.off_lists + b.list_bytes + b.cmb_bytes;
  return TM_OK;
}

// The instance table (host image) and the launch list for workspace `base`
// and bucket zone `acc`.
static void fill_batch(const BatchPlan& b, const tm_plan* plans, const void* const* xs, tm_result* out, char* base,
                       char* acc, Inst* host_tab, int32_t* host_list) {
  int32_t tile_base = 0, red_base = 0, seg_base = 0, band_base = 0;
  for (int32_t i = 0; i < b.count; ++i) {
    const tm_plan_s* p = plans[i];
    Inst& in = host_tab[i];
    fill_inst(p, xs[i], &in);
    place_workspace(p->core, base + b.ws_off[i], acc + b.acc_off[i], &in);
    in.tile_base = tile_base;
    in.red_base = red_base;
    in.seg_base = seg_base;
    in.seg_chunks = b.seg_chunks[i];
    in.nseg = b.nseg[i];
    in.band_base = band_base;
    tile_base += p->core.ntiles;
    seg_base += b.nseg[i];
    band_base += p->core.nband;
    red_base += p->core.nred;
    in.out = b.scratch_res ? reinterpret_cast<tm_result*>(base + b.off_res) + i : out + i;
    host_list[i] = b.order[i];
  }
}

// The kernels of one batch, in stream order, on the device table at
// base + off_tab (host image host_tab): folds, the real path's reduction,
// the correlation stage of the GEMM-correlation instances, the finish
// launches, and the three-moduli combine.  `timed`: the fold and correlation
// kernels carry the profiling events.
static hipError_t launch_batch(const BatchPlan& b, const tm_plan* plans, const Inst* host_tab, char* base,
                               tm_result* out, const std::vector<Combine3>* cmb, hipStream_t s, bool timed) {
  InstTable tab{};
  tab.table = reinterpret_cast<const Inst*>(base + b.off_tab);
  tab.count = b.count;
  const int32_t* dlist = reinterpret_cast<const int32_t*>(base + b.off_lists);
  const std::vector<int32_t>& order = b.order;
  const int32_t ncg_inst = b.ncg_inst;
  auto corr = [&](auto&& launch) { return timed ? timed_corr(s, launch) : launch(); };
  FoldWork fw;
  fw.tiles = (int)b.tiles;
  fw.lds = b.fold_lds;
  fw.segs = (int)b.segs;
  fw.bands = (int)b.bands;
  hipError_t e = timed ? timed_fold(tab, fw, s) : folds(tab, fw, s);
  if (e != hipSuccess) return e;
  if ((e = launch_reduce(tab, (int)b.chunks, s)) != hipSuccess) return e;
  if (ncg_inst > 0 && b.use_inst) {
    // the digit rows of every instance, then per LDS class one launch of the
    // per-instance kernel (product .. resolve, each launch with its class's
    // largest footprint); the instances too large for its LDS, last in the
    // order, by row tile with the final kernel
    const CgLaunch cl = cgemm_launch(b.cps, b.cp_max, ncg_inst);
    if ((e = launch_cgemm_prep(tab, dlist, ncg_inst, cl.chunk, cl.prep_y, s)) != hipSuccess) return e;
    int32_t g0 = 0;
    std::vector<std::pair<int32_t, int32_t>> groups;
    while (g0 < ncg_inst && cg_class(plans[order[g0]]->core) < kCgClasses) {
      const int k0 = cg_class(plans[order[g0]]->core);
      int32_t g1 = g0;
      while (g1 < ncg_inst && cg_class(plans[order[g1]]->core) == k0) ++g1;
      groups.emplace_back(g0, g1);
      g0 = g1;
    }
    const int32_t n_inst = g0;
    e = corr([&] {
      for (const auto& gr : groups) {
        size_t lds = 0;
        for (int32_t g = gr.first; g < gr.second; ++g) {
          const Core& c = plans[order[g]]->core;
          lds = std::max(lds, cgemm_inst_lds_bytes(c.c_lt, c.c_lp, c.c_nlcap, c.c_rta + c.c_rtb,
                                                   std::max(c.c_rta, c.c_rtb)));
        }
        const hipError_t el = launch_cgemm_inst(tab, dlist + gr.first, gr.second - gr.first, lds, s);
        if (el != hipSuccess) return el;
      }
      return hipSuccess;
    });
    if (e != hipSuccess) return e;
    if (n_inst < ncg_inst) {
      int64_t gy = 0, nl = 0;
      for (int32_t g = n_inst; g < ncg_inst; ++g) {
        const Core& c = plans[order[g]]->core;
        gy = std::max<int64_t>(gy, c.c_rta + c.c_rtb);
        nl = std::max<int64_t>(nl, c.c_nlcap);
      }
      const int32_t n_rest = ncg_inst - n_inst;
      if ((e = launch_cgemm_gemm(tab, dlist + n_inst, n_rest, (int)gy, (int)nl, s)) != hipSuccess) return e;
      if ((e = launch_cgemm_final(tab, dlist + n_inst, n_rest, s, b.cg_lean)) != hipSuccess) return e;
    }
  } else if (ncg_inst > 0) {
    const CgLaunch cl = cgemm_launch(b.cps, b.cp_max, ncg_inst);
    if ((e = launch_cgemm_prep(tab, dlist, ncg_inst, cl.chunk, cl.prep_y, s)) != hipSuccess) return e;
    // launches of many row tiles: one wave per row tile; else the band of
    // each row tile split over the waves of a workgroup
    const bool per_wave = cgemm_kind() == 3 || cgemm_kind() == 4 || (cgemm_kind() == 0 && b.cg_tasks >= 2048);
    // the LDS-ring variant of the per-wave kernel for digit counts up to 3
    const bool ring = per_wave && b.cg_limbs_max <= 3 && cgemm_kind() != 3;
    e = corr([&] {
      if (ring) return launch_cgemm_ring(tab, dlist, ncg_inst, (int)b.cgs, s);
      return per_wave ? launch_cgemm_wave(tab, dlist, ncg_inst, (int)b.cgs, (int)b.cg_limbs_max, s)
                      : launch_cgemm_gemm(tab, dlist, ncg_inst, (int)b.cgs, (int)b.cg_limbs_max, s);
    });
    if (e != hipSuccess) return e;
    if ((e = launch_cgemm_final(tab, dlist, ncg_inst, s, b.cg_lean, ring)) != hipSuccess) return e;
  }
  for (int32_t g0 = ncg_inst; g0 < b.count;) {
    const Core& c0 = plans[order[g0]]->core;
    int32_t g1 = g0 + 1;
    while (g1 < b.count && plans[order[g1]]->core.mode == c0.mode && plans[order[g1]]->core.p_log2 == c0.p_log2)
      ++g1;
    if (c0.gfft) {   // one launch sequence per instance
      for (int32_t g = g0; g < g1; ++g)
        if ((e = launch_gfft(host_tab[order[g]], tab.table + order[g], s)) != hipSuccess) return e;
    } else {
      e = launch_finish(tab, dlist + g0, g1 - g0, c0.mode, c0.p_log2, c0.finish_lds, s);
      if (e != hipSuccess) return e;
    }
    g0 = g1;
  }
  if (cmb) {
    tm_result* user_dev = b.dev_out ? out : reinterpret_cast<tm_result*>(base + b.off_ures);
    e = launch_combine3(reinterpret_cast<const Inst*>(base + b.off_tab),
                        reinterpret_cast<const Combine3*>(base + b.off_lists + b.list_bytes),
                        reinterpret_cast<const tm_result*>(base + b.off_res), user_dev, b.n_user, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static tm_status run_batch(int32_t count, const tm_plan* plans, const void* const* xs, tm_result* out,
                           void* stream, const std::vector<Combine3>* cmb) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  BatchPlan b;
  tm_status st = plan_batch(count, plans, is_device_pointer(out), cmb, b);
  if (st != TM_OK) return st;
  std::lock_guard<std::mutex> lock(g_mu);
  StreamPool& pool = g_pools[{plans[0]->device, s}];
  st = ensure_device(pool, b.total, s);
  if (st != TM_OK) return st;
  st = ensure_acc(pool, b.accb, s);
  if (st != TM_OK) return st;
  char* base = static_cast<char*>(pool.dev);
  const bool reuse = !cmb && pool.tab_valid && pool.tab_dev == pool.dev && pool.tab_acc == pool.acc &&
                     pool.tab_out == out && pool.tab_plans.size() == (size_t)count &&
                     std::equal(plans, plans + count, pool.tab_plans.begin()) &&
                     std::equal(xs, xs + count, pool.tab_xs.begin());
  const Inst* host_tab = nullptr;
  if (reuse) {
    host_tab = pool.tab_host.data();
  } else {
    pool.tab_valid = false;
    int slot = 0;
    st = ensure_host(pool, b.tab_bytes + b.list_bytes + b.cmb_bytes, &slot);
    if (st != TM_OK) return st;
    Inst* tab = static_cast<Inst*>(pool.host[slot]);
    int32_t* host_list = reinterpret_cast<int32_t*>(static_cast<char*>(pool.host[slot]) + b.tab_bytes);
    if (cmb) std::memcpy(static_cast<char*>(pool.host[slot]) + b.tab_bytes + b.list_bytes, cmb->data(), b.cmb_bytes);
    fill_batch(b, plans, xs, out, base, static_cast<char*>(pool.acc), tab, host_list);
    TM_HIP(hipMemcpyAsync(base + b.off_tab, pool.host[slot], b.tab_bytes + b.list_bytes + b.cmb_bytes,
                          hipMemcpyHostToDevice, s));
    TM_HIP(hipEventRecord(pool.staged[slot], s));
    pool.staged_pending[slot] = true;
    host_tab = tab;
    if (!cmb) {
      pool.tab_host.assign(tab, tab + count);
      pool.tab_plans.assign(plans, plans + count);
      pool.tab_xs.assign(xs, xs + count);
      pool.tab_out = out;
      pool.tab_dev = pool.dev;
      pool.tab_acc = pool.acc;
      pool.tab_valid = true;
    }
  }
  pool.acc_dirty = true;                 // until every kernel that restores the buckets is enqueued
  TM_HIP(launch_batch(b, plans, host_tab, base, out, cmb, s, true));
  pool.acc_dirty = false;
  if (!b.dev_out) {
    tm_result* user_dev = reinterpret_cast<tm_result*>(base + (cmb ? b.off_ures : b.off_res));
    TM_HIP(hipMemcpyAsync(out, user_dev, sizeof(tm_result) * (size_t)b.n_user, hipMemcpyDeviceToHost, s));
    TM_HIP(hipStreamSynchronize(s));
  }
  return TM_OK;
}

// ---------------------------------------------------------------- reusable batches

struct tm_batch_s {
  int device = 0;
  BatchPlan plan;
  void* dev = nullptr;           // workspace, results, table and list
  void* acc = nullptr;           // bucket zone (zero between launches)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void batch_free(tm_batch_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->dev) (void)hipFree(b->dev);
  if (b->acc) (void)hipFree(b->acc);
  delete b;
}

tm_status tm_batch_create(int32_t count, const tm_plan* plans, const void* const* xs, tm_result* out, void* stream,
                          tm_batch* res) {
  if (!res) return fail(TM_ERR_INVALID, "null batch output");
  *res = nullptr;
  if (count < 1) return fail(TM_ERR_INVALID, "count must be >= 1");
  if (!plans || !xs || !out) return fail(TM_ERR_INVALID, "null argument");
  for (int32_t i = 0; i < count; ++i) {
    tm_status st = check_plan_for_match(plans[i]);
    if (st != TM_OK) return fail(st, "instance " + std::to_string(i) + ": " + g_err);
    st = check_x(plans[i], xs[i]);
    if (st != TM_OK) return fail(st, "instance " + std::to_string(i) + ": " + g_err);
    if (plans[i]->core.three) return fail(TM_ERR_UNSUPPORTED, "tm_batch_create: three-moduli plans are not supported");
    if (plans[i]->device != plans[0]->device) return fail(TM_ERR_INVALID, "plans on different devices");
  }
  if (!is_device_pointer(out)) return fail(TM_ERR_INVALID, "tm_batch_create: out must be device memory");
  hipStream_t s = static_cast<hipStream_t>(stream);
  tm_batch_s* b = new tm_batch_s();
  b->device = plans[0]->device;
  tm_status st = plan_batch(count, plans, true, nullptr, b->plan);
  if (st != TM_OK) { delete b; return st; }
  const BatchPlan& bp = b->plan;
  std::vector<Inst> tab((size_t)count);
  std::vector<int32_t> list((size_t)count);
  hipStream_t cs = nullptr;
  auto bail = [&](tm_status code, const std::string& msg) {
    if (cs) {
      hipGraph_t g = nullptr;
      hipStreamCaptureStatus cst;
      if (hipStreamIsCapturing(cs, &cst) == hipSuccess && cst == hipStreamCaptureStatusActive)
        (void)hipStreamEndCapture(cs, &g);
      if (g) (void)hipGraphDestroy(g);
      (void)hipStreamDestroy(cs);
    }
    batch_free(b);
    return fail(code, msg);
  };
#define TM_HIP_B(expr)                                                                  \
  do {                                                                                  \
    const hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) return bail(TM_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)
  TM_HIP_B(hipMalloc(&b->dev, std::max<size_t>(bp.total, 256)));
  TM_HIP_B(hipMalloc(&b->acc, std::max<size_t>(bp.accb, 256)));
  fill_batch(bp, plans, xs, out, static_cast<char*>(b->dev), static_cast<char*>(b->acc), tab.data(), list.data());
  char* base = static_cast<char*>(b->dev);
  TM_HIP_B(hipMemcpyAsync(base + bp.off_tab, tab.data(), bp.tab_bytes, hipMemcpyHostToDevice, s));
  TM_HIP_B(hipMemcpyAsync(base + bp.off_lists, list.data(), sizeof(int32_t) * (size_t)count, hipMemcpyHostToDevice, s));
  // the buckets start at zero; every replay leaves them at zero again (no
  // memset inside the graph)
  TM_HIP_B(hipMemsetAsync(b->acc, 0, std::max<size_t>(bp.accb, 256), s));
  TM_HIP_B(hipStreamSynchronize(s));
  // capture the kernels on a private stream, untimed
  TM_HIP_B(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  TM_HIP_B(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  TM_HIP_B(launch_batch(bp, plans, tab.data(), base, out, nullptr, cs, false));
  {
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (e != hipSuccess) return bail(TM_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    b->graph = g;
  }
  TM_HIP_B(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  (void)hipStreamDestroy(cs);
  cs = nullptr;
#undef TM_HIP_B
  *res = b;
  return TM_OK;
}

tm_status tm_batch_launch(tm_batch b, void* stream) {
  if (!b || !b->exec) return fail(TM_ERR_INVALID, "null batch");
  TM_HIP(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)));
  return TM_OK;
}

tm_status tm_batch_destroy(tm_batch b) {
  if (!b) return TM_OK;
  TM_HIP(hipDeviceSynchronize());
  batch_free(b);
  return TM_OK;
}

tm_status tm_match_batch(int32_t count, const tm_plan* plans, const void* const* xs, tm_result* out,
                         void* stream) {
  if (count < 0) return fail(TM_ERR_INVALID, "negative count");
  if (count == 0) return TM_OK;
  if (!plans || !xs || !out) return fail(TM_ERR_INVALID, "null argument");
  bool any3 = false;
  for (int32_t i = 0; i < count; ++i) {
    tm_status st = check_plan_for_match(plans[i]);
    if (st != TM_OK) return fail(st, "instance " + std::to_string(i) + ": " + g_err);
    st = check_x(plans[i], xs[i]);
    if (st != TM_OK) return fail(st, "instance " + std::to_string(i) + ": " + g_err);
    any3 = any3 || plans[i]->core.three;
  }
  if (!any3) return run_batch(count, plans, xs, out, stream, nullptr);
  // three moduli: each such plan runs as its two pairs, then the combine
  std::vector<tm_plan> ep;
  std::vector<const void*> ex;
  std::vector<Combine3> cmb((size_t)count);
  for (int32_t i = 0; i < count; ++i) {
    Combine3& cb = cmb[(size_t)i];
    cb.i1 = (int32_t)ep.size();
    cb.i2 = -1;
    ep.push_back(plans[i]);
    ex.push_back(xs[i]);
    const Core& c = plans[i]->core;
    if (c.three) {
      cb.i2 = (int32_t)ep.size();
      ep.push_back(plans[i]->pair2);
      ex.push_back(xs[i]);
      cb.m1 = c.m1;
      cb.m2 = c.m2;
      cb.m3 = c.m3;
      cb.inv12 = mod_inverse(c.m1, c.m2);
    }
  }
  if (ep.size() > 0x7fffffff) return fail(TM_ERR_UNSUPPORTED, "batch too large");
  return run_batch((int32_t)ep.size(), ep.data(), ex.data(), out, stream, &cmb);
}

// One template, many signals of the plan's N: tm_match_batch with the plan
// repeated (independent matches); with TM_MANY_GEMM=1 the signals' folds form
// the rows of one int8 MFMA GEMM against the shared template instead (exact
// int8 plans with K <= 2^14 and folds of at most 2^13 rows, not TM_F_FFT).
tm_status tm_match_many(tm_plan p, int32_t count, const void* const* xs, tm_result* out, void* stream) {
  if (!p || count < 0) return fail(TM_ERR_INVALID, "null plan or negative count");
  if (count == 0) return TM_OK;
  if (!xs || !out) return fail(TM_ERR_INVALID, "null argument");
  tm_status st = check_plan_for_match(p);
  if (st != TM_OK) return st;
  for (int32_t i = 0; i < count; ++i) {
    st = check_x(p, xs[i]);
    if (st != TM_OK) return fail(st, "signal " + std::to_string(i) + ": " + g_err);
  }
  const Core& c = p->core;
  // the shared GEMM reads the plan's template copies (exact plans of the
  // int8 product route), when asked for: the batch of per-signal products
  // is the faster route at the shapes measured
  const bool gemm = c.cgemm && c.x_dtype == TM_I8 && c.t_dtype == TM_I8 && c.mode == MODE_EXACT && c.k <= (1 << 14) &&
                    std::max(c.va.l, c.vb.l) <= (1 << 13) && !(p->desc.flags & TM_F_FFT) && c.top_t == 1 &&
                    !c.three &&
                    env_int("TM_MANY_GEMM", 0) == 1;
  if (!gemm) {
    std::vector<tm_plan> plans((size_t)count, p);
    return tm_match_batch(count, plans.data(), xs, out, stream);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool dev_out = is_device_pointer(out);
  const int64_t rows = ceil_div(count, kGemmTile) * kGemmTile;
  const int32_t lp = (int32_t)(ceil_div((int64_t)std::max(c.ma, c.mb) + c.k + 128, 64) * 64);
  const int32_t nkb = (int32_t)ceil_div(std::max(c.ma, c.mb), kGemmTile);
  // layout: [workspaces][limbs][partials][maxabs][results][table][signal pointers]
  const size_t ws = c.ws_bytes * (size_t)count;
  const size_t off_limb = align256(ws);
  const size_t off_part = align256(off_limb + (size_t)2 * kGemmMaxLimbs * rows * lp);
  const size_t off_max = align256(off_part + (size_t)2 * count * nkb * 2 * sizeof(double));
  const size_t off_res = align256(off_max + sizeof(int) * 2 * (size_t)count);
  const size_t off_tab = align256(off_res + (dev_out ? 0 : sizeof(tm_result) * (size_t)count));
  const size_t tab_bytes = sizeof(Inst) * (size_t)count;
  const size_t off_xs = off_tab + tab_bytes;
  const size_t xs_bytes = sizeof(void*) * (size_t)count;
  const size_t total = off_xs + xs_bytes;

  std::lock_guard<std::mutex> lock(g_mu);
  StreamPool& pool = g_pools[{p->device, s}];
  pool.tab_valid = false;                // the workspace is reused below
  st = ensure_device(pool, total, s);
  if (st != TM_OK) return st;
  st = ensure_acc(pool, c.acc_bytes * (size_t)count, s);
  if (st != TM_OK) return st;
  int slot = 0;
  st = ensure_host(pool, tab_bytes + xs_bytes, &slot);
  if (st != TM_OK) return st;
  char* base = static_cast<char*>(pool.dev);
  Inst* host_tab = static_cast<Inst*>(pool.host[slot]);
  const void** host_xs = reinterpret_cast<const void**>(static_cast<char*>(pool.host[slot]) + tab_bytes);
  tm_result* dout = dev_out ? out : reinterpret_cast<tm_result*>(base + off_res);
  const int32_t sc = c.sfold ? (int32_t)launch_seg_chunks(c, c.n * dtype_bytes(c.x_dtype) * count) : c.seg_chunks;
  const int32_t ns = c.sfold ? segments_of(c.n, sc) : c.nseg;
  for (int32_t i = 0; i < count; ++i) {
    Inst& in = host_tab[i];
    fill_inst(p, xs[i], &in);
    place_workspace(c, base + c.ws_bytes * (size_t)i, static_cast<char*>(pool.acc) + c.acc_bytes * (size_t)i, &in);
    in.tile_base = c.ntiles * i;
    in.seg_chunks = sc;
    in.nseg = ns;
    in.seg_base = ns * i;
    in.band_base = c.nband * i;
    in.red_base = 0;
    in.out = dout + i;
    host_xs[i] = xs[i];
  }
  TM_HIP(hipMemcpyAsync(base + off_tab, pool.host[slot], tab_bytes + xs_bytes, hipMemcpyHostToDevice, s));
  TM_HIP(hipEventRecord(pool.staged[slot], s));
  pool.staged_pending[slot] = true;

  InstTable tab{};
  tab.table = reinterpret_cast<const Inst*>(base + off_tab);
  tab.count = count;
  FoldWork fw;
  fw.tiles = c.ntiles * count;
  fw.lds = c.fold_lds;
  fw.segs = ns * count;
  fw.bands = c.nband * count;
  TM_HIP(timed_fold(tab, fw, s));
  pool.acc_dirty = true;
  ManyArgs a{};
  fill_inst(p, nullptr, &a.base);
  a.xs = reinterpret_cast<const void* const*>(base + off_xs);
  a.out = dout;
  a.yp = static_cast<int*>(pool.acc);
  a.yp_stride = (int64_t)(c.acc_bytes / sizeof(int));
  a.ylimb = reinterpret_cast<int8_t*>(base + off_limb);
  a.rows = rows;
  a.lp = lp;
  a.count = count;
  a.nkb = nkb;
  a.maxabs = reinterpret_cast<int*>(base + off_max);
  a.part = reinterpret_cast<double*>(base + off_part);
  TM_HIP(hipMemsetAsync(a.maxabs, 0, sizeof(int) * 2 * (size_t)count, s));
  TM_HIP(launch_many(a, s));
  pool.acc_dirty = false;
  if (!dev_out) {
    TM_HIP(hipMemcpyAsync(out, dout, sizeof(tm_result) * (size_t)count, hipMemcpyDeviceToHost, s));
    TM_HIP(hipStreamSynchronize(s));
  }
  return TM_OK;
}

tm_status tm_profile_enable(int on) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_prof_on = on != 0;
  return TM_OK;
}

tm_status tm_profile_read(double* fold_ms_total, int64_t* fold_launches, int reset) {
  std::lock_guard<std::mutex> lock(g_mu);
  for (auto& pr : g_prof_live) {
    TM_HIP(hipEventSynchronize(pr.second));
    float ms = 0.f;
    TM_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
    g_prof_ms += ms;
    ++g_prof_n;
    g_prof_free.push_back(pr.first);
    g_prof_free.push_back(pr.second);
  }
  g_prof_live.clear();
  if (fold_ms_total) *fold_ms_total = g_prof_ms;
  if (fold_launches) *fold_launches = g_prof_n;
  if (reset) { g_prof_ms = 0.0; g_prof_n = 0; }
  return TM_OK;
}

tm_status tm_profile_read_corr(double* ms_total, int64_t* launches, int reset) {
  std::lock_guard<std::mutex> lock(g_mu);
  for (auto& pr : g_prof_corr_live) {
    TM_HIP(hipEventSynchronize(pr.second));
    float ms = 0.f;
    TM_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
    g_prof_corr_ms += ms;
    ++g_prof_corr_n;
    g_prof_free.push_back(pr.first);
    g_prof_free.push_back(pr.second);
  }
  g_prof_corr_live.clear();
  if (ms_total) *ms_total = g_prof_corr_ms;
  if (launches) *launches = g_prof_corr_n;
  if (reset) { g_prof_corr_ms = 0.0; g_prof_corr_n = 0; }
  return TM_OK;
}

}  // extern "C"
