/*
 * tm.h -- C ABI of the MI355X (gfx950) template matcher.
 *
 * The library implements the fast template matching scheme of
 * "Fast Template Matching by Subsampled Circulant Matrix" (Hsieh, Lu, Pei,
 * arXiv 1509.04863): given a signal x of length N and a template t of length
 * K it returns the cyclic shift m^ that the paper's Algorithm 1 selects as
 * the maximiser of the cross-correlation (Tx)_k = sum_{j<K} t_j x_{(k+j) mod N}
 * (Eq. (1) with the similarity of Section 3).
 *
 * Every step runs on the GPU: the fold of Algorithm 1 step 3 (Eq. (2)), the
 * correlation of steps 4-6 (by FFT, or for exact plans with an int8-valued
 * template directly as an int8 matrix product on the matrix cores, which gives
 * the same integers), the argmax of step 7 and the candidate intersection of
 * steps 8-9 (Theorem 4, Chinese remaindering).
 *
 * Conventions for every entry point
 *   - Sizes are element counts.  Device pointers are HIP device addresses
 *     (memory from hipMalloc or any allocator on the same device).
 *   - Streams are hipStream_t values passed as void*; NULL is the null stream.
 *   - Nothing throws across the ABI.  Every call returns a tm_status.  On an
 *     error nothing has been launched and no output has been written;
 *     tm_last_error() returns a message for the calling thread.
 *   - Arguments are validated on the host before any launch.
 *
 * Readings of the paper that fix behaviour visible here:
 *   - shifts range over [0, N) (Eq. (1) prints 0 < k < N);
 *   - steps 4-6 compute a cross-correlation (step 6 prints a product of
 *     spectra, which would be a convolution);
 *   - the fold keeps Algorithm 1's cyclic indices when M does not divide N;
 *   - each argmax runs over [0, M) and ties go to the lowest index;
 *   - candidate sets are taken mod N; several common candidates are re-scored
 *     by (Tx)_c (largest wins, lowest index on ties); none gives shift = -1.
 */
#ifndef TM_H
#define TM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TM_OK = 0,
  TM_ERR_INVALID = 1,      /* bad argument: sizes, moduli, dtypes, null pointers, alignment */
  TM_ERR_NOMEM = 2,        /* device or pinned host allocation failed */
  TM_ERR_DEVICE = 3,       /* a HIP call failed; tm_last_error() has the HIP message */
  TM_ERR_UNSUPPORTED = 4   /* valid request this build cannot run (e.g. FFT length too large) */
} tm_status;

typedef enum {
  TM_I8 = 0,               /* int8_t */
  TM_F32 = 1,              /* float */
  TM_BF16 = 2,             /* bfloat16 (storage only; arithmetic in float) */
  TM_F16 = 3               /* IEEE half (storage only; arithmetic in float) */
} tm_dtype;

/* plan flags */
#define TM_F_EXACT      0x1u /* x and t hold integer values: fold in int32, FFT in FP64,
                                correlations rounded to integers.  Implied when both
                                dtypes are TM_I8.  Precondition: every partial sum of x
                                fits in int32 (e.g. |x_i| * ceil(N/M) < 2^31). */
#define TM_F_REAL       0x2u /* force the real (FP32 FFT) path even for int8 inputs */
#define TM_F_ZERO_PAD   0x4u /* Theorem 2 variant (Section 3.2): for each modulus M, x is
                                padded with zeros to L*M (L = ceil(N/M)); the fold is the
                                length-M partition fold y[s] = sum_i x[s + i*M] over the
                                padded signal, the correlation is circular of length M
                                (r[k] = sum_j t_j y[(k + j) mod M]), and the candidate set
                                of m~ is {m~ + i*M < N}, so at most one candidate remains.
                                Identical to the default when M divides N; a template that
                                wraps past the end of x is not matched by this variant.
                                The FFT length is not shortened: the two folds share one
                                transform of length >= max(M1, M2) + K - 1. */
#define TM_F_FFT        0x8u /* exact path: always compute the correlation by the FFT of
                                steps 4-6, never by the direct int8 matrix product */

/* result flags */
#define TM_R_NOMATCH    0x1u /* S_M1 and S_M2 share no element: shift = -1 */
#define TM_R_RESCORED   0x2u /* more than one common candidate; chosen by (Tx)_c */
#define TM_R_NEAR_TIE   0x4u /* real path: an argmax's top-2 gap is below 1e-5 of its fold's peak */
#define TM_R_EXACT      0x8u /* exact path and either the int8 matrix product computed the
                                correlation or the FP64 FFT error bound is below 1/2, so
                                every correlation value is the exact integer */

typedef struct {
  int64_t n;          /* signal length N >= 1 */
  int32_t k;          /* template length, 1 <= K <= N */
  int32_t m1, m2;     /* fold lengths; both 0 = automatic rule M1 = max(c*K, m0(N)),
                         M2 = M1 + 1 where m0(N) is the least m with m(m+1) > N
                         (Algorithm 1 step 2, with M1 = K, M2 = K + 1 of Section 4
                         raised when K(K+1) <= N).  Explicit values must satisfy
                         gcd(M1, M2) = 1, M1 >= K, M2 >= K, M1*M2 >= N (Theorem 4). */
  int32_t fold_mult;  /* c in {1, 2} for the automatic rule; 0 means 1 */
  int32_t x_dtype;    /* tm_dtype of x */
  int32_t t_dtype;    /* tm_dtype of t */
  int32_t fold_store; /* real path only: storage format of the folded signal fed to
                         the FFT: TM_F32 (default), TM_BF16 or TM_F16 */
  uint32_t flags;     /* TM_F_* */
  int32_t top_t;      /* 0 or 1: steps 8-9 as printed.  2..4: top-T re-scoring, a
                         robustness option beyond the paper: the T largest entries of
                         each correlation (lowest index first among equal values)
                         give T x T residue pairs, and the union of their candidate
                         sets is re-scored by (Tx)_c (exact on the exact path, FP64
                         otherwise).  m1_tilde / m2_tilde and the peaks stay the
                         argmaxes of step 7; n_candidates counts the union. */
  int32_t m3;         /* 0: two moduli (Algorithm 1).  Three pairwise co-prime moduli
                         (Theorem 4 with three moduli, for K(K+1) <= N where two
                         moduli near K cannot cover N): > 0 is an explicit third
                         modulus (m1, m2 explicit too; each >= K, pairwise co-prime,
                         M1*M2*M3 >= N); -1 chooses (m, m+1, m+2) with m the least
                         odd number >= c*K whose product exceeds N.  The third fold is
                         folded, correlated and maximised like the others and the
                         candidate set is the intersection of the three sets; the
                         result reports the first two folds' residues and peaks.
                         Not combined with top_t > 1 or TM_F_ZERO_PAD, and not
                         available to tm_match_intermediates. */
} tm_plan_desc;

typedef struct tm_plan_s* tm_plan;

typedef struct {
  int64_t  shift;        /* m^ in [0, N), or -1 with TM_R_NOMATCH */
  int32_t  m1_tilde;     /* argmax over [0, M1) of the M1-fold correlation (step 7) */
  int32_t  m2_tilde;     /* argmax over [0, M2) of the M2-fold correlation */
  int32_t  n_candidates; /* |S_M1 cap S_M2| before re-scoring, 0..3 (0..1 with
                            TM_F_ZERO_PAD; up to 3 T^2 with top-T) */
  uint32_t flags;        /* TM_R_* */
  double   peak1;        /* r_M1[m1_tilde] (an integer on the exact path) */
  double   peak2;        /* r_M2[m2_tilde] */
  double   score;        /* (Tx)_shift: exact integer on the exact path, FP64 sum
                            otherwise; 0 when shift = -1 */
  double   err_bound;    /* real path: a bound on max_k |r_i[k] - r*_i[k]| over both
                            folds, where r* is the correlation in exact arithmetic of
                            the FP32 fold sums: the FP32 transform's rounding
                            ((14 p + 8) 2^-24 ||FFT(t)||_inf ||z||_2 for a transform of
                            2^p points, p + 2 on the four-step route) plus the fold's
                            BF16/FP16 storage rounding (||t||_2 u_s ||z||_2, u_s =
                            2^-8 or 2^-11), with z = y1 + i y2 the stored folds.  The
                            rounding of the FP32 fold sums themselves (L terms each) is
                            not included.  0 on the exact path. */
  int64_t  reserved;     /* 0 */
} tm_result;             /* 64 bytes */

/* Host-side plan parameters (no GPU needed). */
typedef struct {
  int32_t m1, m2;        /* chosen fold lengths (user order) */
  int32_t l1, l2;        /* ceil(N / M1), ceil(N / M2) */
  int32_t fft_log2;      /* P = 2^fft_log2 >= max(M1, M2) + K - 1 */
  int32_t exact;         /* 1 = exact (integer) path, 0 = real path */
  int32_t dual;          /* 1 = |M1 - M2| = 1: both folds from one read of x */
  int32_t fft_in_lds;    /* 1 = the whole FFT fits one workgroup's LDS (P <= 2^13
                            on the exact path, 2^14 on the real path) */
  int32_t fold_tiles;    /* workgroups of the tiled fold (0 when streamed) */
  int32_t fold_segments; /* workgroups of the streaming int8 fold (0 when tiled) */
  int32_t fold_bands;    /* workgroups of the band fold of 4-byte signals */
  int32_t fft_global;    /* 1 = P above one workgroup's LDS: four-step FFT through
                            global memory (P up to 2^21) */
  int32_t corr_gemm;     /* 1 = the correlation of steps 4-6 may be computed directly
                            as an int8 MFMA matrix product (exact plans whose template
                            holds integers in [-128, 127], K <= 2^17, unless
                            TM_F_FFT); every correlation value is then exact */
  int32_t m3;            /* third modulus, or 0 for two */
  int64_t workspace_bytes; /* device workspace one match of this plan uses */
  int64_t x_bytes;       /* bytes of x read per match */
} tm_plan_info;

/*
 * tm_plan_params -- validate desc and compute the plan parameters on the host.
 * Pure host code: needs no GPU and touches no device.
 * Errors: TM_ERR_INVALID for K < 1, K > N, bad explicit moduli (see
 * tm_plan_desc.m1), fold_mult outside {0,1,2}, unknown dtypes or flags.
 */
tm_status tm_plan_params(const tm_plan_desc* desc, tm_plan_info* info);

/*
 * tm_plan_create -- Algorithm 1 steps 2 and 4 for a fixed template.
 * Chooses (M1, M2) and the FFT length P, copies t (K elements of desc->t_dtype,
 * host memory when t_is_device = 0, device memory otherwise) to the device,
 * generates the length-P twiddles in FP64 on the GPU and stores the scaled
 * template spectrum conj(FFT_P([t 0])) / P the correlation uses.
 * The plan owns its device memory, is immutable after creation and may be used
 * from several streams at once.  Work is enqueued on `stream` and the call
 * waits for it before returning.  Besides t and the spectrum (or the shifted
 * template copies of the int8 product), the plan's first single match adds
 * room for 8 device copies of its per-stream instance record (see tm_match).
 */
tm_status tm_plan_create(const tm_plan_desc* desc, const void* t, int t_is_device,
                         void* stream, tm_plan* out);

/* tm_plan_destroy -- waits for the device, frees the plan.  NULL is allowed. */
tm_status tm_plan_destroy(tm_plan plan);

/* tm_plan_get_info -- parameters of an existing plan. */
tm_status tm_plan_get_info(tm_plan plan, tm_plan_info* info);

/*
 * tm_match -- one signal, Algorithm 1 steps 3 and 5-9.
 * x: device pointer to N elements of the plan's x_dtype, aligned to the
 *    element size (any byte offset for int8).  Read only; the fold kernels
 *    read the whole 16-byte aligned chunks that overlap x.
 * out: one tm_result in host or device memory.  With host memory the call
 *    waits for the stream; with device memory it only enqueues work and `out`
 *    is valid once the stream reaches this point.
 * The caller keeps x (and a device `out`) alive until then.
 * The first match of a plan on a stream copies the plan's instance record
 * (about 400 bytes: sizes, workspace addresses) to device memory, ordered on
 * the stream; later matches on that stream reuse it and pass the kernels
 * only its address, x and out.  A plan used on more than 8 streams allocates
 * one more small device and pinned host block per further stream, kept until
 * tm_plan_destroy.
 */
tm_status tm_match(tm_plan plan, const void* x, tm_result* out, void* stream);

/*
 * tm_match_noalloc -- tm_match for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops and harnesses that forbid
 * allocation): the same kernels and the same result, bit for bit, with every
 * intermediate in a device array of 16 MiB that the library holds on each
 * GPU from the moment it is loaded until the process ends.  The call
 * allocates nothing: no hipMalloc, no hipFree, no pool growth, no per-stream
 * instance copy.
 * plan: created beforehand on the current device (plan creation allocates);
 *    its workspace (tm_plan_info.workspace_bytes) plus about 1 KiB must fit in
 *    16 MiB, else TM_ERR_UNSUPPORTED.  Three-moduli plans: TM_ERR_UNSUPPORTED.
 * x: as tm_match.  out: one tm_result in DEVICE memory (TM_ERR_INVALID for
 *    host memory); valid once `stream` reaches this point.  Nothing waits.
 * Every call on a GPU uses that GPU's one array, which keeps the previous
 * call's contents (each call clears what must start at zero): calls that
 * overlap on one GPU (on different streams or threads) race and give
 * undefined results; calls in one stream's order do not.
 */
tm_status tm_match_noalloc(tm_plan plan, const void* x, tm_result* out, void* stream);

/*
 * tm_match_batch -- Algorithm 1 steps 3 and 5-9 applied per instance to
 * `count` independent matches in one launch sequence
 * (uneven N and K allowed; plans may repeat).  plans[i] with xs[i] gives
 * out[i].  `out` points to count results in host or device memory (same rule
 * as tm_match).  The arrays plans and xs are host arrays read during the call.
 * Each result equals the one tm_match returns for the same plan and signal,
 * bit for bit.
 */
tm_status tm_match_batch(int32_t count, const tm_plan* plans, const void* const* xs,
                         tm_result* out, void* stream);

/*
 * Reusable batches -- Algorithm 1 steps 3 and 5-9 per instance, as
 * tm_match_batch, for a fixed list of plans and signals matched again and
 * again (the signals' contents may change between launches, their addresses
 * may not).  tm_batch_create builds the instance table once in device memory
 * of its own (workspace, buckets, table) and captures the batch's whole
 * kernel sequence in a HIP graph; tm_batch_launch replays it on `stream`
 * with one graph launch, so the host builds and uploads nothing per launch.
 * out: `count` results in DEVICE memory (TM_ERR_INVALID otherwise), written
 * by every launch.  plans, xs: host arrays read during the call; the plans
 * and signals must stay valid until tm_batch_destroy.  Launches of one batch
 * on several streams at once race (they share its workspace).  Three-moduli
 * plans: TM_ERR_UNSUPPORTED.  The creating call waits for `stream`.
 */
typedef struct tm_batch_s* tm_batch;
tm_status tm_batch_create(int32_t count, const tm_plan* plans, const void* const* xs, tm_result* out,
                          void* stream, tm_batch* batch);
tm_status tm_batch_launch(tm_batch batch, void* stream);
/* Waits for the device, then frees the batch's memory and graph.  NULL is allowed. */
tm_status tm_batch_destroy(tm_batch batch);

/*
 * tm_match_many -- one template, `count` signals of the plan's N (Algorithm 1
 * per signal).  xs is a host array of count device pointers; out holds count
 * results (host or device, as tm_match); every result equals tm_match's bit
 * for bit.  By default it runs as tm_match_batch with the plan repeated (for
 * exact int8 plans: one int8 MFMA product per signal, its template copies
 * staged once per workgroup).  With the environment variable TM_MANY_GEMM=1,
 * exact int8 plans (K <= 2^14, folds of at most 2^13 rows) instead take one
 * banded Toeplitz product over all signals (the folds split into base-128
 * int8 digits, exact int32/int64 sums), which reads the template once per
 * signal tile; at N = 2^18, K = 1024 it is the slower of the two.
 */
tm_status tm_match_many(tm_plan plan, int32_t count, const void* const* xs, tm_result* out, void* stream);

/*
 * tm_match_intermediates -- tm_match that also writes the intermediate vectors
 * (for parity checks): y1[0..M1+K-1) and y2[0..M2+K-1) are the literal folds of
 * Algorithm 1 step 3 (after the fold_store rounding on the real path),
 * r1[0..M1) and r2[0..M2) the correlations of step 6 (rounded to integers on the
 * exact path).  All four are device arrays of double; any may be NULL.
 */
tm_status tm_match_intermediates(tm_plan plan, const void* x, tm_result* out,
                                 double* y1, double* y2, double* r1, double* r2,
                                 void* stream);

/*
 * Kernel timing for benchmarks.  While enabled, every match call records a pair
 * of HIP events around its fold kernel launch on the call's stream.
 * tm_profile_read waits for the recorded events and returns the summed fold
 * kernel time in milliseconds and the number of fold launches since the last
 * reset (reset != 0 clears the record).
 */
tm_status tm_profile_enable(int on);
tm_status tm_profile_read(double* fold_ms_total, int64_t* fold_launches, int reset);
/* The same for the correlation kernel of tm_match and tm_match_batch: the
 * int8 matrix-product kernel on that route, the in-LDS FFT finish kernel on
 * the FFT route (the four-step global FFT is not timed). */
tm_status tm_profile_read_corr(double* ms_total, int64_t* launches, int reset);

/*
 * Request server (continuous batching).  Matches of uneven N and K submitted
 * from any thread are grouped first in, first out into batches of at most
 * max_batch requests; up to max_inflight batches run on the device at once,
 * each on its own stream, so requests that arrive while others run are
 * launched as soon as a slot is free.  A request is admitted while the device
 * workspace (tm_plan_info.workspace_bytes plus about 0.5 KiB of result slot and
 * instance record) of all batches in flight stays within budget_bytes, and a
 * batch is launched only while the device memory all the server's streams
 * hold (each grows to exactly what its batches need; idle ones give theirs
 * back first) stays within it too; a single request above the budget runs
 * alone.  tm_server_destroy frees all of it.
 * Every result equals the one tm_match returns for the same plan and signal.
 * Plans (templates, spectra and twiddles) stay on the device; the caller keeps
 * each plan and signal valid until its result has been taken.
 */
typedef struct tm_server_s* tm_server;

typedef struct {
  int64_t budget_bytes;  /* 0 = 1 GiB */
  int32_t max_batch;     /* 0 = 1024 */
  int32_t max_inflight;  /* 0 = 2; at most 8 */
} tm_server_desc;

typedef struct {
  int64_t submitted, completed, failed, batches;
  int64_t peak_inflight_bytes;   /* largest admitted workspace in flight */
  int64_t peak_held_bytes;       /* largest device memory the server's streams held at a
                                    launch: at most max(budget_bytes, the largest request) */
} tm_server_stats;

/* Creates the streams, pinned result buffers and worker thread on the current
 * device.  Errors: TM_ERR_INVALID for negative fields or max_inflight > 8,
 * TM_ERR_DEVICE when no device or allocation is available. */
tm_status tm_server_create(const tm_server_desc* desc, tm_server* out);

/* Queues one match (Algorithm 1 for plan and the device signal x) and returns
 * its ticket; does not wait.  Errors: TM_ERR_INVALID for null arguments or a
 * server being destroyed, TM_ERR_UNSUPPORTED for plans without an FFT path. */
tm_status tm_server_submit(tm_server server, tm_plan plan, const void* x, uint64_t* ticket);

/* *done = 0 while the request runs; once done, *done = 1, *out holds the
 * result, *latency_ns (optional) the time from submission to completion, and
 * the ticket is consumed.  The returned status is the request's own (a batch
 * that failed on the device reports TM_ERR_DEVICE).  TM_ERR_INVALID for an
 * unknown or consumed ticket. */
tm_status tm_server_poll(tm_server server, uint64_t ticket, tm_result* out, int64_t* latency_ns, int* done);

/* tm_server_poll that blocks until the request is done. */
tm_status tm_server_wait(tm_server server, uint64_t ticket, tm_result* out, int64_t* latency_ns);

tm_status tm_server_get_stats(tm_server server, tm_server_stats* out);

/* Runs every queued request to completion, then frees the server. */
tm_status tm_server_destroy(tm_server server);

/*
 * tm_admit_batches -- the server's admission rule on the host alone: with no
 * batch in flight, footprints[0..count) are cut first in, first out into
 * batches of at most max_batch requests whose summed footprint stays within
 * budget_bytes (a request above the budget forms a batch of its own);
 * batch_of[i] receives the batch index of request i.
 */
tm_status tm_admit_batches(int32_t count, const int64_t* footprints, int64_t budget_bytes, int32_t max_batch,
                           int32_t* batch_of);

/* Message strings. tm_last_error is per calling thread. */
const char* tm_status_string(tm_status status);
const char* tm_last_error(void);

/* Library version "major.minor.patch". */
const char* tm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TM_H */
