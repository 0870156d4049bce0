/*
 * idbf.h -- C ABI of the MI355X (gfx950) interpolative decomposition butterfly
 * factorization (IDBF) of Pang, Ho and Yang, arXiv:1809.10573.
 *
 * The library builds K ~= U^L ... U^h S^h V^h ... V^L (Section 2.4, eq. finishIDBF)
 * for K(x, xi) = exp(2 pi i Phi(x, xi)) or J_0(x xi) sampled entry by entry
 * (Introduction; Examples 1-3), and applies it or its adjoint to blocks of
 * vectors in O(N log N) per vector.
 *
 * Conventions shared by every entry point:
 *  - Pointers documented as "device" are HIP device pointers on the current
 *    device; "host" pointers are ordinary process memory.  The caller owns
 *    every buffer it passes; the library never retains one past the call,
 *    except that a handle owns the factor memory it allocates.
 *  - Complex arrays are interleaved (re, im): complex128 = 2 doubles,
 *    complex64 = 2 floats.  Multi-vector arrays are (rows, nrhs) row-major,
 *    right-hand sides fastest.
 *  - Index arrays are int32 positions into X / Omega (0-based).
 *  - No entry point aborts or throws.  Each returns an idbf_status; on failure
 *    idbf_last_error() returns a thread-local message describing it, and
 *    outputs are left unspecified (a failed idbf_construct sets *out = NULL
 *    and frees everything it allocated).
 *  - "stream" arguments are hipStream_t values (NULL: the null stream).
 *    idbf_construct synchronizes that stream; the other compute calls are
 *    asynchronous on it.
 */
#ifndef IDBF_H
#define IDBF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum idbf_status {
  IDBF_OK = 0,
  IDBF_EINVAL = 1,        /* invalid argument (sizes, pointers, tolerances) */
  IDBF_ENOMEM = 2,        /* device allocation failed or exceeded opts.mem_cap_bytes */
  IDBF_EHIP = 3,          /* a HIP runtime call failed */
  IDBF_ERANK = 4,         /* an ID needed a rank above the supported maximum (64) */
  IDBF_EUNSUPPORTED = 5   /* a candidate set above 128 or a sample set above 256 */
} idbf_status;

/* Kernels K(x, xi) = exp(2 pi i Phi(x, xi)) (Example 1 and the DFT kernel,
 * which on random points is Example 3's non-uniform transform):
 *   IDBF_PHASE_DFT: Phi(x, xi) = -x * xi
 *   IDBF_PHASE_FIO: Phi(x, xi) = x * xi + c(x) |xi|,
 *                   c(x) = (c0 + a * sin(2 pi freq x)) / cdiv
 * and the Schloemilch kernel of Example 2 (eq. S, nu = 0):
 *   IDBF_PHASE_J0:  K(x, xi) = J_0(x xi), real, at the FP64 product x xi
 *                   (Miller's recurrence below 25, Hankel's expansion above;
 *                   |x xi| < 2^24 pi/2)                                    */
enum { IDBF_PHASE_DFT = 0, IDBF_PHASE_FIO = 1, IDBF_PHASE_J0 = 2 };

/* Element types / arithmetic of the apply: complex128 on the FP64 factors,
 * complex64 on FP32 copies of the same FP64-constructed factors.
 * IDBF_C64_BF16X3 keeps complex64 input and output but forms the products of
 * the many-RHS stages from BF16 hi/lo splits (a = a_hi + a_lo;
 * a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi) on the matrix cores with FP32
 * accumulation. */
enum { IDBF_C128 = 0, IDBF_C64 = 1, IDBF_C64_BF16X3 = 2 };

/* The two ID families of a level: U (row IDs) and V (column IDs). */
enum { IDBF_SIDE_U = 0, IDBF_SIDE_V = 1 };

typedef struct idbf_phase {
  int32_t kind;   /* IDBF_PHASE_DFT, IDBF_PHASE_FIO or IDBF_PHASE_J0 */
  int32_t reserved;
  double c0, a, freq, cdiv;  /* c(x) parameters (FIO only; cdiv != 0 there) */
} idbf_phase;

/* opts.flags bits:
 *   IDBF_FLAG_PROFILE: record per-launch device times (idbf_profile_read).
 *   IDBF_FLAG_PROPOSER_FORCE_REJECT: the residual test rejects every proposal
 *     of opts.proposer, so every ID falls back to the plain ID (the factors
 *     then equal those of a construction without a proposer, bit for bit).
 *   IDBF_FLAG_ALLOW_TRUNCATE: an ID whose eps-rank exceeds the supported 64
 *     keeps 64 skeletons (a rank-64 truncated ID) instead of failing with
 *     IDBF_ERANK. */
enum { IDBF_FLAG_PROFILE = 1, IDBF_FLAG_PROPOSER_FORCE_REJECT = 2, IDBF_FLAG_ALLOW_TRUNCATE = 4 };

enum { IDBF_SAMPLER_MOCKCHEB = 0, IDBF_SAMPLER_RANDOM = 1 };

/* Default acceptance factor of the learned proposal's residual test. */
#define IDBF_DEFAULT_ACCEPT 1.0f

typedef struct idbf_opts {
  int32_t kmax;        /* rank parameter k of the (eps, k)-ID (Section 2.1); 0: k = min(s, c) */
  int32_t oversample;  /* oversampling parameter t >= 1: s = min(t |cand|, |allowed|) samples (<= 256) */
  int32_t flags;       /* IDBF_FLAG_* */
  int32_t sampler;     /* IDBF_SAMPLER_MOCKCHEB (Section 2.1, default) or IDBF_SAMPLER_RANDOM:
                          uniform distinct positions (Floyd's algorithm on SplitMix64 draws from
                          seed, level, side, ID), the comparison sampler of Section 3 */
  uint64_t mem_cap_bytes; /* cap on device memory a handle may allocate; 0: none */
  void* stream;        /* hipStream_t used by idbf_construct */
  /* Learned rank proposal (not in the paper), or NULL: every ID first samples
   * s' = min(s, t (ceil(k^) + proposal_margin)) points, k^ the network's rank
   * estimate; a randomized residual test on 8 fresh allowed points accepts it
   * (||A(r,red) - A(r,skel) T||_F <= f tol ||A(r,cand)||_F, f =
   * proposal_accept) or the plain ID of s samples replaces it.  seed drives
   * the test points and the random sampler (SplitMix64). */
  struct idbf_mlp_s* proposer;
  int32_t proposal_margin;
  float proposal_accept; /* acceptance factor f > 0 of the residual test; 0: IDBF_DEFAULT_ACCEPT */
  uint64_t seed;
  /* Skeleton proposal (not in the paper), or NULL; needs opts.proposer.  A
   * second network of the same form scores every candidate of every ID
   * (features: level, side, node centres, a, m, the candidate's position in
   * its set and its relative coordinate); the k_p = min(c, 64, ceil(k^) +
   * 2 proposal_margin) best form the ID's proposed set, and the pivot search
   * of the column-pivoted QR on the s' samples runs over that set only (the
   * eps-rank threshold still taken against the block's largest column norm;
   * T = R11^{-1} R12 for every other candidate).  Every such ID goes through
   * the residual test, and is rejected if no proposed column is above the
   * threshold; the plain pivoted ID replaces the rejected ones. */
  struct idbf_mlp_s* skeleton_proposer;
  /* The handle's device memory (factors, apply workspace, level scratch)
   * from the caller's allocator, e.g. a framework's caching allocator; both
   * NULL (the default) for the library's own: hipMalloc, with the chunks of
   * destroyed handles kept for later constructions (see idbf_destroy).
   * dev_alloc(bytes, user) returns device memory of at least `bytes` on the
   * current device, 256-byte aligned, or NULL (the call then fails with
   * IDBF_ENOMEM); dev_free(ptr, bytes, user) takes back what dev_alloc
   * returned, once the device has finished with it (the library
   * synchronizes first).  Both run on the thread of the library call that
   * needs them: construction, an apply with more right-hand sides than any
   * before it, destruction.  Give both or neither (IDBF_EINVAL). */
  void* (*dev_alloc)(size_t bytes, void* user);
  void (*dev_free)(void* ptr, size_t bytes, void* user);
  void* alloc_user;
} idbf_opts;

typedef struct idbf_handle_s* idbf_handle;
typedef struct idbf_mlp_s* idbf_mlp;

/* Fill *o with the defaults: kmax 0, oversample 1 (the paper's t = 1),
 * no flags, no memory cap, null stream.  NULL-safe. */
void idbf_opts_default(idbf_opts* o);

/*
 * idbf_construct -- build the IDBF of K(X, Omega) (Sections 2.1-2.4).
 *   phase  host; the phase function.
 *   X      device, N doubles, ascending: row points x_i.
 *   Omega  device, N doubles, ascending: column points xi_j.
 *   N      power of two >= leaf; leaf power of two in [1, 128].
 *   tol    ID tolerance eps of eq. acc, 0 <= tol < 1.
 *   opts   host, nullable (defaults).
 *   out    host; receives the handle (NULL on failure).
 * Every interpolative decomposition runs in FP64 on the GPU: Mock-Chebyshev
 * sample selection, entry sampling, column-pivoted Householder QR stopped at
 * the eps-rank, and the interpolation solve T = R11^{-1} R12 (eq. R2).
 * Levels run U_1, V_1, ..., U_H, V_H with H = floor(L/2), L = log2(N/leaf);
 * then the middle factor's blocks are sampled.  Each ID samples
 * s = min(oversample * |cand|, |allowed|) points (the t k rows of eq.
 * pivotedQR2 with k = |cand|).  A sample block of more than 128 rows is first
 * reduced to its |cand| x |cand| triangular factor by unpivoted Householder QR
 * (same pivots and T in exact arithmetic).  Candidate sets must stay <= 128
 * points and sample sets <= 256 (else IDBF_EUNSUPPORTED); ranks <= 64 (else
 * IDBF_ERANK).  Synchronizes opts->stream.  The handle owns all factor
 * memory (FP64 factors and an FP32 copy) until idbf_destroy.
 */
idbf_status idbf_construct(const idbf_phase* phase, const double* X, const double* Omega,
                           int64_t N, double tol, int32_t leaf, const idbf_opts* opts,
                           idbf_handle* out);

/*
 * idbf_apply -- y = U^L ... U^h S^h V^h ... V^L x (eq. finishIDBF).
 *   x      device, (N, nrhs) complex of the given dtype; read only.
 *   y      device, (N, nrhs) complex of the given dtype; fully overwritten;
 *          must not overlap x.
 *   nrhs   >= 0 (0 is a no-op).
 *   dtype  IDBF_C128 (FP64 factors and arithmetic), IDBF_C64 (FP32: VALU
 *          for nrhs = 1, FP32 MFMA for nrhs > 1) or IDBF_C64_BF16X3 (complex64
 *          data, BF16 hi/lo split MFMA products, FP32 accumulation).
 * Asynchronous on stream.  Intermediate vectors live in a workspace owned by
 * the handle, grown (hipMalloc, which synchronizes) when nrhs exceeds what
 * was used before; calls on one handle must not overlap in time.  With
 * IDBF_FLAG_PROFILE the stage launches are recorded as apply1_ (complex64,
 * 1 RHS), applyn_ (FP32 MFMA), applyb_ (BF16 split), apply1d_ (complex128,
 * 1 RHS) or applynd_ (complex128, several RHS), + v, s, u.
 */
idbf_status idbf_apply(idbf_handle h, const void* x, void* y, int64_t nrhs, int32_t dtype,
                       void* stream);

/*
 * idbf_apply_adjoint -- y = K~^H x = (V^L)^H ... (V^h)^H (S^h)^H (U^h)^H ...
 * (U^L)^H x, the conjugate transpose of the factorization idbf_apply applies
 * (the same factors, the stages in reverse order, each conjugate transposed;
 * the Conclusion's use in iterative solvers).  x is indexed like idbf_apply's
 * y (rows of K, the points X) and y like its x (columns, the points Omega).
 * Arguments, dtypes, workspace and error behaviour as idbf_apply; profile
 * records are named as idbf_apply's with adj in place of apply.
 */
idbf_status idbf_apply_adjoint(idbf_handle h, const void* x, void* y, int64_t nrhs, int32_t dtype,
                               void* stream);

/*
 * idbf_construct_batched -- build `count` independent IDBFs (uneven N, phase,
 * tol and leaf) in one lockstep level sweep: every phase of every level is
 * issued for all instances, spread over up to 4 device-lifetime streams of
 * the library, and the host waits once per phase for all of them.
 *   phases, X, Omega, N, tol, leaf: host arrays of `count` entries, each entry
 *          as in idbf_construct (X[i], Omega[i] device pointers).
 *   opts   host, nullable; applies to every instance.  opts->stream is the
 *          stream the inputs were produced on (waited for) and the stream the
 *          handles keep.
 *   out    host array of `count` handles; all NULL on failure.
 * Same per-instance results (bit for bit) as idbf_construct.  On failure
 * every instance is freed and idbf_last_error() names the failing instance.
 */
idbf_status idbf_construct_batched(int32_t count, const idbf_phase* phases, const double* const* X,
                                   const double* const* Omega, const int64_t* N, const double* tol,
                                   const int32_t* leaf, const idbf_opts* opts, idbf_handle* out);

/*
 * idbf_apply_batched -- y[i] = K~_i x[i] for `count` distinct handles, each as
 * in idbf_apply with nrhs[i] right-hand sides of one dtype.  The instances run
 * concurrently on the library's streams, ordered after prior work on `stream`;
 * `stream` waits for all of them.  Workspaces are grown first (synchronizing
 * `stream` when one grows); a batch whose workspaces were reserved allocates
 * nothing.
 */
idbf_status idbf_apply_batched(int32_t count, const idbf_handle* hs, const void* const* x, void* const* y,
                               const int64_t* nrhs, int32_t dtype, void* stream);

/*
 * Captured batched apply: idbf_apply_batched_plan records the launches of one
 * idbf_apply_batched call (same arguments; `stream` must be a created,
 * non-null stream) into a HIP graph instead of running them; idbf_plan_launch
 * replays that graph on any stream, with no host work per kernel.  The plan
 * keeps the device pointers it was built with: x, y and every handle must
 * stay alive until idbf_plan_destroy.  Workspaces are grown before the
 * capture; profiling is suspended while capturing.  The graph writes each
 * handle's apply workspace, so while a plan lives that workspace stays where
 * it is: idbf_apply, idbf_apply_adjoint or idbf_reserve on such a handle that
 * would need a larger workspace fails with IDBF_EINVAL (smaller applies reuse
 * it and must not overlap a replay in time), and idbf_destroy of the handle
 * fails with IDBF_EINVAL until every plan that holds it is destroyed.
 */
typedef struct idbf_plan_s* idbf_plan;
idbf_status idbf_apply_batched_plan(int32_t count, const idbf_handle* hs, const void* const* x, void* const* y,
                                    const int64_t* nrhs, int32_t dtype, void* stream, idbf_plan* out);
idbf_status idbf_plan_launch(idbf_plan p, void* stream);
idbf_status idbf_plan_destroy(idbf_plan p);

/*
 * idbf_apply_noalloc -- idbf_apply for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, kernels and results (bit for bit) as
 * idbf_apply, but the stage vectors live in one fixed device array of the
 * library (128 MiB per device, held until the process ends) instead of the
 * handle's workspace; the call allocates nothing and records no profile
 * events.  The array holds 2 * (largest skeleton count of a level) * nrhs
 * complex values: nrhs beyond that gives IDBF_EINVAL with the size in the
 * message (at N = 2^20, leaf 16, tol 1e-6 one complex128 or complex64 vector
 * fits).  Every call on a device shares that device's array, so calls that
 * overlap in time on one device race; the array keeps the last call's
 * contents, which no call reads before writing.
 */
idbf_status idbf_apply_noalloc(idbf_handle h, const void* x, void* y, int64_t nrhs, int32_t dtype,
                               void* stream);

/* Grow the handle's apply workspace (device memory, a kept chunk when one
 * fits) so that idbf_apply with up to nrhs right-hand sides of dtype
 * allocates nothing.  Synchronizes the device if it allocates. */
idbf_status idbf_reserve(idbf_handle h, int64_t nrhs, int32_t dtype);

/* Free a handle and everything it owns.  NULL-safe.  Synchronizes the device.
 * IDBF_EINVAL (nothing freed) while a captured plan still holds the handle.
 * Its device chunks (factor arena, apply workspace) and pinned staging block
 * are kept by the library for later constructions on the same device, up to
 * IDBF_CACHE_BYTES bytes (environment, read once; default 32 GiB, 0 keeps
 * nothing), the oldest freed first. */
idbf_status idbf_destroy(idbf_handle h);

/* Free the device and pinned memory kept from destroyed handles (see
 * idbf_destroy).  Live handles are not affected.  Thread-safe: a
 * construction running meanwhile on another thread only finds less memory to
 * reuse. */
idbf_status idbf_release_cached_memory(void);

/* Launch configuration of the many-right-hand-side apply (a schedule of the
 * product of eq. finishIDBF, not a change to it):
 *   fuse: 1 runs each pair of consecutive V stages, and of U stages, of the
 *     complex64 forward apply (FP32 MFMA or BF16 split) as one launch over
 *     closed groups (two level-t units and the two neighbouring-level units
 *     they feed), the intermediate kept in registers, where every ID of both
 *     levels has rank <= 32; 0 (the default) runs one launch per stage.
 *     Results agree to the precision's rounding.
 *   rhs_iter: right-hand-side blocks (32 complex64 or 16 complex128 columns
 *     per wavefront) each workgroup walks through with one LDS-staged
 *     factor block: 0 (the kernels' default, 8) or a power of two <= 64.
 * The setting belongs to the handle; idbf_tune_apply picks one by timing. */
typedef struct idbf_apply_config {
  int32_t fuse;
  int32_t rhs_iter;
  int32_t from_cache; /* idbf_tune_apply's answer: 1 if read from its cache file */
  float ms;           /* idbf_tune_apply's answer: the chosen configuration's time per apply */
  int32_t reserved[4];
} idbf_apply_config;
/* Read or replace a handle's apply configuration (IDBF_EINVAL on NULL
 * arguments or values outside the ranges above; nothing changes then). */
idbf_status idbf_get_apply_config(idbf_handle h, idbf_apply_config* cfg);
idbf_status idbf_set_apply_config(idbf_handle h, const idbf_apply_config* cfg);

/* Autotuner of the many-RHS apply (not in the paper): times every
 * configuration (fuse 1 and 0 for complex64 and the BF16 split, the
 * handle's current fuse for complex128, which has no fused path; rhs_iter
 * 1, 2, 4, ... up to 16 or the number of right-hand-side blocks) on this
 * handle's factors for (nrhs, dtype) -- one warm-up and three forward
 * applies each, HIP events on `stream` -- and sets the fastest on the
 * handle (*chosen, nullable, gets it with its time).  cache_path (nullable): a text file, one line per tuned
 * problem, "<key>\t<fuse> <rhs_iter> <ms>", the key naming the device's
 * architecture, N, L, H, nrhs, dtype and every level's rank and candidate
 * bounds; a problem found there is set without timing (from_cache = 1), and
 * a newly tuned one is appended.  The library allocates two N x nrhs
 * operands for the timing (IDBF_ENOMEM if it cannot) and frees them before
 * returning.  Synchronizes `stream`.  The handle's configuration is
 * unchanged if an error is returned. */
idbf_status idbf_tune_apply(idbf_handle h, int64_t nrhs, int32_t dtype, const char* cache_path, void* stream,
                            idbf_apply_config* chosen);

/* Wave shapes of the batched pivoted QR (Section 2.1, eq. pivotedQR2, on
 * the sampled block) for IDs of up to 64 candidates with 65..80, 81..96 and
 * 97..112 sampled rows: bit b of the mask for the b-th range.  A clear bit
 * (the default) runs four wavefronts of 20, 24 or 28 rows; a set bit runs
 * five of 16, eight of 12 or eight of 14.  Both take the same steps; only
 * the sums across wavefronts round differently, so T agrees to rounding and
 * a pivot could differ only where two residual norms sit at the edge of the
 * tie band (the tests find identical skeletons).  The setting is
 * process-wide and read at every launch, so it should change only
 * while no construction runs.  idbf_set_qr_shapes: IDBF_EINVAL for bits
 * above the three; idbf_get_qr_shapes: IDBF_EINVAL for a NULL mask. */
idbf_status idbf_set_qr_shapes(uint32_t mask);
idbf_status idbf_get_qr_shapes(uint32_t* mask);

/* Autotuner of those shapes.  Builds the factorization of (phase, X, Omega,
 * N, tol, leaf, opts) as idbf_construct does, with IDBF_FLAG_PROFILE added,
 * and times its ID kernels (the id_qr records; the better of two
 * constructions after one warm-up) for the current mask and then for each
 * one-bit change of the best mask so far, keeping a change that is faster.
 * The chosen mask is then set process-wide (idbf_set_qr_shapes).  With
 * cache_path, a line "<key>\t<mask> <ms>" (key: GPU architecture, N, phase,
 * tol, leaf, oversampling, kmax) answers later calls without timing; the
 * last line for a key wins.  *mask, *ms (the ID kernels of one construction
 * with the chosen shapes; 0 from the cache if it held no time) and
 * *from_cache are written when non-NULL.  Errors of idbf_construct are
 * returned as they are, with the shape mask left as it was. */
idbf_status idbf_tune_construct(const idbf_phase* phase, const double* X, const double* Omega, int64_t N,
                                double tol, int32_t leaf, const idbf_opts* opts, const char* cache_path,
                                uint32_t* mask, float* ms, int32_t* from_cache);

/* Thread-local description of the last failure on this thread ("" if none). */
const char* idbf_last_error(void);

typedef struct idbf_info {
  int64_t N;
  int32_t leaf, L, H, oversample;
  double tol;
  int64_t n_ids;          /* interpolative decompositions performed */
  int64_t nnz_T;          /* complex entries of all T blocks (sum of k (c - k)) */
  int64_t nnz_S;          /* complex entries of the middle factor (in use) */
  int64_t n_skel;         /* skeleton indices stored over all levels */
  int32_t rank_min, rank_max;
  int32_t cand_max, samples_max;
  int64_t device_bytes;   /* device memory held by the handle */
  double construct_ms;    /* host wall time of idbf_construct */
  double id_flops;        /* FP64 flops of the IDs: sum 16 sum_{j<k} (s-j)(c-j) + 4 k^2 (c-k) */
  int64_t sampled_entries;/* kernel entries sampled by the IDs: sum s c */
  int64_t proposed;       /* IDs first computed from a proposal (0 without a proposer) */
  int64_t rejected;       /* proposals the residual test rejected (recomputed plainly) */
} idbf_info;

/* Summary of a handle (host *info). */
idbf_status idbf_get_info(idbf_handle h, idbf_info* info);

/*
 * Per-level statistics of a construction (Section 2.4's factors, level by
 * level): for level t = 1..H and side IDBF_SIDE_U / IDBF_SIDE_V the rank
 * histogram of its 2^(L+1) IDs and what the level stores and cost.
 * idbf_stats fills *out (host) for levels 1..min(H, IDBF_STATS_LEVELS);
 * entries of other levels are zero.  It reads the ranks back from the device
 * (a small temporary device buffer; synchronizes the handle's stream).
 */
#define IDBF_STATS_LEVELS 16
#define IDBF_STATS_RANKS 65   /* ranks 0..64 */
typedef struct idbf_level_stats_t {
  int64_t n_ids;            /* IDs of the level (2^(L+1)) */
  int64_t rank_hist[IDBF_STATS_RANKS];  /* rank_hist[r]: IDs of rank r */
  int32_t rank_min, rank_max, cand_max, samples_max;
  int64_t n_skel;           /* skeleton indices (sum of ranks) */
  int64_t nnz_T;            /* T entries in use: sum k (c - k) */
  int64_t sampled_entries;  /* kernel entries the IDs sampled: sum s c */
  int64_t tall;             /* IDs with more than 128 samples (row-reduced first) */
  int64_t proposed;         /* IDs first computed from a proposal */
  int64_t accepted;         /* proposals the residual test accepted */
  int64_t rejected;         /* proposals recomputed by the plain ID */
  double id_flops;          /* FP64 flops of the level's IDs (as idbf_info.id_flops) */
  double wall_ms;           /* host wall time of the level inside idbf_construct (shared by all
                               instances of a batched construction) */
} idbf_level_stats_t;
typedef struct idbf_stats_t {
  int32_t L, H;
  int32_t levels;           /* levels filled: min(H, IDBF_STATS_LEVELS) */
  int32_t reserved;
  idbf_level_stats_t level[IDBF_STATS_LEVELS][2];  /* [t - 1][side] */
  int64_t nnz_S;            /* middle-factor entries in use */
  int64_t n_blocks_S;       /* middle-factor blocks */
  int64_t apply_bytes_c64;  /* factor bytes one complex64 apply streams: 8 (nnz_T + nnz_S) + 40 per ID record */
  int64_t apply_bytes_c128; /* the same for complex128: 16 (nnz_T + nnz_S) + 40 per ID record */
  int64_t device_bytes;     /* device memory held by the handle */
  double construct_ms;      /* host wall time of idbf_construct */
} idbf_stats_t;
idbf_status idbf_stats(idbf_handle h, idbf_stats_t* out);

/* Per-kernel device time of a handle built with IDBF_FLAG_PROFILE: HIP events
 * recorded around every launch of idbf_construct, idbf_apply and
 * idbf_apply_adjoint on the stream
 * the kernel runs on.  bytes / flops are the algorithmic work of those
 * launches: factor entries streamed plus the vectors read or written once
 * (apply), FP64 flops of the pivoted QR and solve (IDs). */
typedef struct idbf_kernel_stat {
  char name[24];
  int32_t launches;
  int32_t reserved;
  double ms;      /* summed device time of the launches */
  double bytes;   /* summed algorithmic bytes */
  double flops;   /* summed algorithmic flops */
} idbf_kernel_stat;

/* Aggregate recorded launches by kernel name into out[0 .. *n) (host, at most
 * max entries); reset != 0 discards the records afterwards.  Synchronizes
 * with the recorded events.  IDBF_EINVAL if profiling is off. */
idbf_status idbf_profile_read(idbf_handle h, idbf_kernel_stat* out, int32_t max, int32_t* n,
                              int32_t reset);

/* Switch the recording of those events on (on != 0) or off for later calls on
 * h, whatever the construction flags were.  Each record costs the stream a
 * marker of a few microseconds (a 1-RHS apply records 2H + 2 of them), so a
 * caller that times the path itself can leave the markers out of the calls it
 * times.  Records already taken stay until idbf_profile_read(reset != 0)
 * discards them; idbf_profile_read answers IDBF_EINVAL only while profiling is
 * off and no records are held.  IDBF_EINVAL for a NULL handle. */
idbf_status idbf_profile_enable(idbf_handle h, int32_t on);

/*
 * Inspection of one level's IDs, for verification.  side IDBF_SIDE_U or
 * IDBF_SIDE_V, level t in [1, H].  IDs are numbered q = partner * 2^(L-t+1)
 * + node, where node is the tree node at depth L-t+1 whose candidates the ID
 * compresses and partner the node at depth t of the other tree.
 *   idbf_batch_sizes: *n_ids, *n_skel (sum of ranks), *n_T (T entries stored).
 *   idbf_batch_export (all host arrays, sized by idbf_batch_sizes):
 *     rank[n_ids], cand_len[n_ids], mask[2 * n_ids] (bit l of the 128-bit
 *     word pair (mask[2q], mask[2q+1]) set: candidate l is a skeleton), skel[n_skel] (global indices, ascending within each ID,
 *     IDs consecutive), T[2 * n_T] (complex128), T_off[n_ids] (entry offset
 *     of each ID's T).  T of an ID with rank k and r = cand_len - k redundant
 *     candidates is k x r, stored from the even offset T_off[q]; V IDs store it
 *     column-major (entry j*k + i), U IDs row-major (entry i*r + j); rows
 *     follow ascending skeletons, columns ascending redundant candidates.
 *     n_T counts the reserved entries (per-ID rank bounds, rounded even);
 *     the reserved entries past an ID's k r are unspecified.
 */
idbf_status idbf_batch_sizes(idbf_handle h, int32_t side, int32_t level, int64_t* n_ids,
                             int64_t* n_skel, int64_t* n_T);
/*
 * idbf_batch_proposal -- sample counts of one level's IDs (host arrays of
 * n_ids, each nullable): proposed[q] the count the proposal network set
 * before the residual test, used[q] the count the stored ID was computed
 * from (the proposal, or the plain t |cand| when rejected), rejected[q] 1
 * when the residual test rejected the proposal.  Without a proposer all
 * three describe the plain construction (proposed = used, rejected = 0).
 * Synchronizes the handle's stream.
 */
idbf_status idbf_batch_proposal(idbf_handle h, int32_t side, int32_t level, int32_t* proposed,
                                int32_t* used, int32_t* rejected);
idbf_status idbf_batch_export(idbf_handle h, int32_t side, int32_t level, int32_t* rank,
                              int32_t* cand_len, uint64_t* mask, int32_t* skel, double* T,
                              int64_t* T_off);

/*
 * Middle factor S (Section 2.4): for rows R and columns C' at depth
 * d = L-H+1, block b = (C'' * 2^d + R) * 2^(d-H) + j holds
 * K(skel of U_H ID (R, C''), skel of V_H ID (C', R >> (d-H))) with
 * C' = C'' * 2^(d-H) + j, stored column-major from the even offset S_off[b].
 * When H = 0 there is one N x N block, K itself.  n_entries counts the
 * stored entries including the alignment padding.  Host arrays:
 * S[2 * n_entries], S_off[n_blocks].
 */
idbf_status idbf_middle_sizes(idbf_handle h, int64_t* n_blocks, int64_t* n_entries);
idbf_status idbf_middle_export(idbf_handle h, double* S, int64_t* S_off);

/*
 * idbf_sample -- entry sampler: out[i * ncols + j] = K(X[rows[i]], Omega[cols[j]])
 * as complex128 (Introduction: each entry in O(1) operations).  The phase is
 * formed with an error-free product and reduced modulo 1 in FP64 before the
 * exponential; J_0 entries are real (imaginary part 0).  rows, cols, out:
 * device; X, Omega: device.
 */
idbf_status idbf_sample(const idbf_phase* phase, const double* X, const double* Omega,
                        const int32_t* rows, int64_t nrows, const int32_t* cols, int64_t ncols,
                        double* out, void* stream);

/*
 * idbf_id_batch -- n_ids independent (tol, kmax)-IDs on explicit index sets
 * (Section 2.1, Lemma 2.1, eqs. pivotedQR2, acc, R2), the kernel every level
 * of idbf_construct runs.  ID q compresses candidates
 * cand_idx[cand_beg[q] .. cand_beg[q] + cand_len[q]) (ascending global
 * indices, <= 128) against allowed points allow_idx[allow_beg[q] .. + allow_len[q])
 * (ascending).  side IDBF_SIDE_V: candidates are columns (Omega) and the ID
 * is a column ID of K(samples, cand); IDBF_SIDE_U: candidates are rows (X)
 * and it is a row ID of K(cand, samples).  s = min(oversample * cand_len,
 * allow_len) samples are picked by the Mock-Chebyshev rule (an ID with
 * s > 256: IDBF_EUNSUPPORTED, nothing computed).
 * Outputs (device): rank[q]; mask[2q], mask[2q+1] (128-bit skeleton mask);
 * skel[q * 128 + i] ascending skeleton global indices;
 * T[(q * 4096 + e) * 2 ..] complex128 in the layout of idbf_batch_export.
 * Ranks above 64 give IDBF_ERANK.  Asynchronous on stream.
 */
idbf_status idbf_id_batch(const idbf_phase* phase, const double* X, const double* Omega,
                          int32_t side, int64_t n_ids, const int32_t* cand_idx,
                          const int32_t* cand_beg, const int32_t* cand_len,
                          const int32_t* allow_idx, const int32_t* allow_beg,
                          const int32_t* allow_len, double tol, int32_t kmax,
                          int32_t oversample, int32_t* rank, uint64_t* mask, int32_t* skel,
                          double* T, void* stream);

/*
 * Rank-proposal network (not in the paper; the learned-proposal extension of
 * the construction).  A perceptron with IDBF_MLP_INPUTS inputs, two hidden
 * ReLU layers of `hidden` units (16, 32, 64 or 128) and one output, FP32 on
 * the GPU.  Parameters are one flat vector: W1 (inputs x hidden, row-major),
 * b1, W2 (hidden x hidden), b2, W3 (hidden), b3.  Inputs of an ID (level t,
 * side 0 = U / 1 = V; x_c, xi_c the centres of its row and column nodes
 * scaled to [0, 1)): t/8, side, x_c, xi_c, a, m/4, 1 for the FIO kernel,
 * a m |cos 2 pi m x_c| / 4 (a = m = 0 and 0 for the DFT); the target is
 * rank / 16.
 *   idbf_mlp_create: params (host, idbf_mlp_param_count floats) are copied.
 *   idbf_mlp_forward: y[i] = f(X[i * 8 ..]) (device arrays, asynchronous).
 *   idbf_mlp_loss_grad: grad (device, param-count floats) of
 *       mean((f(X) - y)^2) / 2 over the n rows; *loss (host) = that mean.
 *   idbf_mlp_train: `epochs` passes of Adam (lr, betas 0.9 / 0.999) over
 *       minibatches of `batch` rows in a SplitMix64 order; loss_per_epoch
 *       (host, nullable) receives each epoch's mean loss.  Synchronizes.
 *   idbf_mlp_params: copy the parameters to host.
 *   idbf_rank_samples: training data from a built handle: features[n_ids * 8]
 *       and targets[n_ids] (device floats) of one level's IDs.
 */
#define IDBF_MLP_INPUTS 8
int32_t idbf_mlp_param_count(int32_t hidden);
idbf_status idbf_mlp_create(int32_t hidden, const float* params, idbf_mlp* out);
idbf_status idbf_mlp_destroy(idbf_mlp m);
idbf_status idbf_mlp_params(idbf_mlp m, float* params);
idbf_status idbf_mlp_forward(idbf_mlp m, const float* X, int64_t n, float* y, void* stream);
idbf_status idbf_mlp_loss_grad(idbf_mlp m, const float* X, const float* y, int64_t n, float* grad, float* loss,
                               void* stream);
idbf_status idbf_mlp_train(idbf_mlp m, const float* X, const float* y, int64_t n, int32_t epochs, int32_t batch,
                           float lr, uint64_t seed, float* loss_per_epoch, void* stream);
idbf_status idbf_rank_samples(idbf_handle h, int32_t side, int32_t level, float* features, float* targets);
/* Training data of the skeleton network from a built handle: *cmax (host)
 * receives the level's largest candidate count; with features and targets
 * (device, n_ids * cmax * 8 and n_ids * cmax floats) given, row q * cmax + l
 * holds the features of candidate l of ID q and target 1 (a skeleton of the
 * plain construction) or 0, and -1 for l >= cand_len[q] (padding).
 * Synchronizes the handle's stream. */
idbf_status idbf_skeleton_samples(idbf_handle h, int32_t side, int32_t level, int32_t* cmax, float* features,
                                  float* targets);
/* The proposed skeleton sets of one level (host arrays, nullable): n_prop[q]
 * proposed columns of ID q, order[q * 64 + j] the j-th of them (candidate
 * position, best score first, j < n_prop[q]).  IDBF_EINVAL without a
 * skeleton proposer.  Synchronizes the handle's stream. */
idbf_status idbf_batch_skeleton_proposal(idbf_handle h, int32_t side, int32_t level, int32_t* n_prop,
                                        uint8_t* order);

#ifdef __cplusplus
}
#endif

#endif /* IDBF_H */
