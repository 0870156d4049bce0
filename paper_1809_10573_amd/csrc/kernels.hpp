// Launchers of the IDBF HIP kernels (one translation unit per kernel family).
#pragma once

#include "common.hpp"

namespace idbf {

// Error bits a kernel may raise in its status word.
enum : int32_t { kErrRank = 1, kErrSize = 2 };

// QR kernel variant of an ID with c candidates and s samples: buckets 0..7
// take up to 64 candidates by ceil(s / 16) (one to four wavefronts of 16
// rows up to 64 samples, four of 20, 24 or 28 rows up to 112, eight of 16
// up to 128), buckets 8..23 up to 128 with ceil(s / 8) wavefronts of 8
// rows; buckets 24..27 pack two IDs of up to 32 candidates
// and 64 samples per workgroup, 28..29 four IDs of up to 16 and 32.  A tall
// ID (s > kQrRows) enters the one-ID kernels with its reduced block of c
// rows.  Slot kQrBuckets of the bucket counters counts the tall IDs.
constexpr int kQrBuckets = 30;
constexpr int kBucketSlots = kQrBuckets + 1;
constexpr int kFirstPackedBucket = 24;
__host__ __device__ inline bool is_tall(int s) { return s > kQrRows; }
__host__ __device__ inline int qr_rows(int c, int s) { return is_tall(s) ? c : s; }
__host__ __device__ inline int qr_bucket(int c, int s) {
  const bool tall = is_tall(s);
  s = qr_rows(c, s);
  s = s < 1 ? 1 : s;
  if (!tall && c <= 16 && s <= 32) return 28 + (s + 15) / 16 - 1;  // four IDs per workgroup
  if (!tall && c <= 32 && s <= 64) return 24 + (s + 15) / 16 - 1;  // two IDs per workgroup
  if (c <= kWave) {
    const int w = (s + 15) / 16;
    return (w > 8 ? 8 : w) - 1;
  }
  const int w = (s + 7) / 8;
  return 8 + (w > 16 ? 16 : w) - 1;
}

// ------------------------------------------------------------- batched ID
struct IdArgs {
  PhaseDev ph;
  const double* X;
  const double* Om;
  int side;  // IDBF_SIDE_U: candidates are rows (row ID); IDBF_SIDE_V: columns (column ID)
  int64_t n_ids;
  const int32_t* cand_idx;
  const int32_t* cand_beg;
  const int32_t* cand_len;
  const double* cand_coord;   // coordinate of cand_idx[p] at [p], or null (then looked up)
  const int32_t* allow_idx;
  const int32_t* allow_beg;
  const int32_t* allow_len;
  const double* allow_coord;  // same for the allowed points
  double tol;
  int kmax;
  bool truncate;              // ranks above kMaxRank stop at kMaxRank instead of an error
  int oversample;
  int s_max;                  // largest sample count of the batch
  int c_max;                  // largest candidate count of the batch (sizes the launch)
  int rows_max;               // largest qr_rows(c, s) of the batch (sizes an unordered launch)
  const int32_t* samples;     // per-ID sample counts, or null: s = min(t c, |allowed|)
  int sampler;                // IDBF_SAMPLER_MOCKCHEB or IDBF_SAMPLER_RANDOM
  int level;                  // level t of the batch (random sampler counters)
  uint64_t seed;              // random sampler seed
  const int32_t* sel_list;    // selection: the IDs to process (sel_n of them), or null: all n_ids
  int64_t sel_n;
  int32_t* samp_pos;          // sample positions, samp_ld per ID (scratch)
  int64_t samp_ld;            // >= the largest sample count of the batch
  const int32_t* order;       // QR launch: IDs grouped by kernel variant (qr_bucket), or null
  int64_t bucket_off[kQrBuckets + 1];  // host: order[bucket_off[b] .. bucket_off[b + 1]) are bucket b
  // tall IDs (s > kQrRows): the row reduction writes each one's c x c
  // triangular factor to tall_R + tall_slot[q] * tall_ld2 (column-major,
  // leading dimension c), which the QR kernels read instead of sampling
  const int32_t* tall_list;   // the tall IDs; slot i is tall_list[i]
  int64_t n_tall;
  int32_t* tall_slot;         // per ID: its slot (tall IDs only)
  double2* tall_R;
  int64_t tall_ld2;           // entries per slot: >= c_max^2
  double2* tall_work;         // reduction scratch: tall_chunk blocks of tall_work_ld entries
  int64_t tall_work_ld;       // >= s_max c_max
  int64_t tall_chunk;         // tall IDs per reduction launch
  // skeleton proposal: the number of proposed columns of each ID and their
  // candidate positions (kMaxRank per ID, best first); the pivot search of
  // the QR runs over these columns only, with the eps-rank threshold still
  // taken against the block's largest column norm.  An ID none of whose
  // proposed columns is above it gets prop_fail[q] = 1 (the caller clears
  // the array).  Null: the pivoted QR of Section 2.1 over every column.
  const int32_t* prop_k;
  const uint8_t* prop_cols;
  int32_t* prop_fail;
  int32_t* rank;
  uint64_t* mask;        // two words per ID: bit l of (mask[2q], mask[2q+1]) = candidate l is a skeleton
  int32_t* skel_out;     // kMaxCand entries per ID
  double2* T128;
  float2* T64;           // may be null
  const int64_t* T_off;  // null: ID q writes at q * kSlot
  int32_t* status;
};
// Selection (one wavefront per ID), then sampling + QR + solve (one
// workgroup per ID, variant by qr_bucket); launch_qr first runs the row
// reduction of the tall IDs (chunks of tall_chunk); launch_id_batch runs
// selection and QR.
hipError_t launch_select(const IdArgs& a, hipStream_t st);
hipError_t launch_qr(const IdArgs& a, hipStream_t st);
hipError_t launch_id_batch(const IdArgs& a, hipStream_t st);
// Wave shapes of QR buckets 4..6 (65..80, 81..96, 97..112 sampled rows, up to
// 64 candidates): bit b set runs bucket 4 + b on short wavefronts (five of 16
// rows, eight of 12, eight of 14) instead of four tall ones (20, 24, 28 rows).
// Process-wide; read at each launch.
constexpr uint32_t kQrShapeBits = 7u;
uint32_t qr_shape_mask();
void set_qr_shape_mask(uint32_t mask);
// IDs grouped by qr_bucket: counts[0..kQrBuckets) += bucket sizes and
// counts[kQrBuckets] += tall IDs (pass 1), then order[] (and tall[] for the
// tall IDs) filled from per-slot cursors (pass 2, cursors pre-set to the
// bucket offsets; cursors[kQrBuckets] to 0).
// keep (nullable): only IDs with keep[q] != 0 are counted / placed.
hipError_t launch_bucket_count(const int32_t* samples, const int32_t* cand_len, const int32_t* keep, int64_t n,
                               unsigned long long* counts, hipStream_t st);
hipError_t launch_bucket_fill(const int32_t* samples, const int32_t* cand_len, const int32_t* keep, int64_t n,
                              unsigned long long* cursors, int32_t* order, int32_t* tall, hipStream_t st);

// ------------------------------------------------------------- learned proposal
constexpr int kProposalInputs = 8;       // features per ID
constexpr float kProposalScale = 16.f;   // network output x 16 = proposed rank
int mlp_param_count(int n_in, int hidden);
// y = network(X) for n rows of n_in features; z1, z2 (nullable, n x hidden):
// pre-activations kept for the backward pass
hipError_t launch_mlp_forward(const float* P, int n_in, int hidden, const float* X, int64_t n, float* y,
                              float* z1, float* z2, hipStream_t st);
// G = d/dP of mean((y - t)^2) / 2 over the n rows, *loss_dev = sum (y - t)^2;
// ws: (4 hidden + 2) n floats
hipError_t launch_mlp_loss_grad(const float* P, int n_in, int hidden, const float* X, const float* t, int64_t n,
                                float* G, float* loss_dev, float* ws, hipStream_t st);
hipError_t launch_adam(float* P, const float* G, float* M, float* V, int np, float lr, int step, hipStream_t st);
hipError_t launch_gather_rows(const float* X, const float* t, const int32_t* idx, int64_t n, int n_in, float* Xb,
                              float* tb, hipStream_t st);
// features of the n IDs of level t, side (0 U, 1 V): F[q * kProposalInputs + i]
hipError_t launch_features(int64_t n, int L, int t, int side, const PhaseDev& ph, float* F, hipStream_t st);
// s_prop[q] = clamp(t (ceil(16 y[q]) + margin), 1, samples[q])
hipError_t launch_propose(const float* y, const int32_t* samples, int64_t n, int oversample, int margin,
                          int32_t* s_prop, hipStream_t st);
struct ResidualArgs {
  IdArgs id;                    // the level batch, after its IDs are written
  int level;
  uint64_t seed;
  double factor;                // accept when ||E||_F <= factor tol ||A||_F
  bool force_reject;            // reject every proposal (the fallback then recomputes all IDs)
  bool skeletons;               // the IDs took proposed skeletons: every one is tested
  int32_t* reject;              // out: 1 = rejected
  int32_t* s_prop;              // rejected IDs get samples_plain[q] (the fallback's count)
  const int32_t* samples_plain;
};
hipError_t launch_residual(const ResidualArgs& a, hipStream_t st);
// Skeleton proposal.  Features of candidate l of ID q (row q * cmax + l;
// rows l >= c zero): t/8, side, x_c, xi_c, a, m/4, l/c, and the candidate's
// coordinate relative to the first and last candidates of its ID.
hipError_t launch_cand_features(int64_t n, int L, int t, int side, const PhaseDev& ph, const int32_t* cand_beg,
                                const int32_t* cand_len, const double* cand_coord, int cmax, float* F,
                                hipStream_t st);
// per ID: k_f = min(c, s_prop[q], kMaxRank, ceil(16 y_rank[q]) + margin) and the k_f candidates of highest
// score (score[q * cmax + l]), best first
hipError_t launch_pick_skeletons(const float* score, int cmax, const float* y_rank, const int32_t* s_prop,
                                 const int32_t* cand_len, int64_t n, int margin, int32_t* prop_k,
                                 uint8_t* prop_cols, hipStream_t st);
// training targets: out[q * cmax + l] = 1 (skeleton) / 0 (redundant), -1 for l >= c
hipError_t launch_skel_targets(const uint64_t* mask, const int32_t* cand_len, int64_t n, int cmax, float* out,
                               hipStream_t st);
// hist[r] += #{q : rank[q] == r} for r <= kMaxRank (hist zeroed by the caller)
hipError_t launch_rank_hist(const int32_t* rank, int64_t n, unsigned long long* hist, hipStream_t st);
// out[q] = rank[q] / kProposalScale (training targets)
hipError_t launch_rank_targets(const int32_t* rank, int64_t n, float* out, hipStream_t st);

// Work of a finished level (IDs with keep[q] != 0, keep nullable):
// out[0] += sum 16 sum_{j<k}(s-j)(c-j) + 4 k^2 (c-k) (FP64 flops),
// out[1] += sum k (c - k) (T entries), out[2] += sum s c (samples).
hipError_t launch_id_work(const int32_t* rank, const int32_t* cand_len, const int32_t* samples, const int32_t* keep,
                          int64_t n, unsigned long long* out, hipStream_t st);

// ------------------------------------------------------------- level plumbing
struct DescArgs {
  int side, t, L, leaf;
  int64_t N, n_ids;
  int oversample, kmax;
  const int32_t* prev_skel_off;   // same side, level t-1 (t > 1)
  const int32_t* allow_skel_off;  // U: V_{t-1} (t > 1); V: U_t
  int32_t* cand_beg;
  int32_t* cand_len;
  int32_t* allow_beg;
  int32_t* allow_len;
  int64_t* t_bound;               // upper bound of k (c - k) per ID
  int32_t* samples;               // s = min(t c, |allowed|) per ID (Section 2.1: t k rows, k = c)
};
hipError_t launch_desc(const DescArgs& a, hipStream_t st);

// Exclusive scan of n values into off[0..n] (off[n] = total) plus the sum,
// max and min of the values and the max of an optional second array, written
// to stats[0..3].  ws: kScanWs int64 of device workspace (tile partials).
constexpr int kScanMaxTiles = 1024;
constexpr int64_t kScanWs = 5 * kScanMaxTiles;
hipError_t launch_scan_i64(const int64_t* v, int64_t n, int64_t* off, const int32_t* aux,
                           int64_t* stats, int64_t* ws, hipStream_t st);
hipError_t launch_scan_i32(const int32_t* v, int64_t n, int32_t* off, const int32_t* aux,
                           int64_t* stats, int64_t* ws, hipStream_t st);

hipError_t launch_iota(int32_t* p, int64_t n, hipStream_t st);
// packed skeleton lists and their coordinates (base[index])
hipError_t launch_compact_skel(const int32_t* scratch, const int32_t* rank, const int32_t* off,
                               int64_t n_ids, const double* base, int32_t* out, double* out_coord,
                               hipStream_t st);

// Middle factor: per block b rows skel_r[rbeg .. +rlen), cols skel_c[cbeg .. +clen).
struct MiddleDescArgs {
  int L, H;
  int64_t n_blocks;
  const int32_t* u_off;  // U_H skeleton offsets
  const int32_t* v_off;  // V_H skeleton offsets
  int32_t* rbeg;
  int32_t* rlen;
  int32_t* cbeg;
  int32_t* clen;
  int64_t* size;               // entries reserved per block (rounded up to even)
  unsigned long long* nnz;     // += sum of rlen * clen (entries in use)
};
hipError_t launch_middle_desc(const MiddleDescArgs& a, hipStream_t st);
struct SampleBlocksArgs {
  PhaseDev ph;
  const double* X;
  const double* Om;
  int64_t n_blocks;
  const int32_t* row_idx;
  const int32_t* col_idx;
  const int32_t* rbeg;
  const int32_t* rlen;
  const int32_t* cbeg;
  const int32_t* clen;
  const int64_t* off;
  double2* out128;
  float2* out64;  // may be null
};
// block b stored column-major at off[b]: entry (i, j) at off[b] + j * rlen[b] + i
hipError_t launch_sample_blocks(const SampleBlocksArgs& a, hipStream_t st);

// dense sampler: out[i * nc + j] = K(X[rows[i]], Om[cols[j]])
hipError_t launch_sample_dense(const PhaseDev& ph, const double* X, const double* Om,
                               const int32_t* rows, int64_t nr, const int32_t* cols, int64_t nc,
                               double2* out, hipStream_t st);

// ------------------------------------------------------------- apply
// Everything one apply stage needs of an ID, in one 40-byte record.
struct ApplyMeta {
  int64_t t_off;     // first T entry (even)
  uint64_t mask;     // bit l: candidate l is a skeleton (l < 64)
  uint64_t mask_hi;  // bit l - 64: candidate l is a skeleton (64 <= l < 128)
  int32_t cand_beg;  // input (V) / output (U) segment start
  int32_t skel_off;  // output (V) / input (U) segment start
  int32_t c;         // candidates
  int32_t k;         // rank
};
hipError_t launch_pack_meta(const int64_t* t_off, const uint64_t* mask, const int32_t* cand_beg,
                            const int32_t* skel_off, const int32_t* cand_len, const int32_t* rank, int64_t n,
                            ApplyMeta* out, hipStream_t st);

struct StageArgs {
  const ApplyMeta* meta;   // per ID (V, U stages)
  int64_t n;               // IDs (V stage) or units (U stage) or U_H IDs (S stage)
  int nn;                  // U stage: nodes per partner row of the level (2^(L-t+1));
                           // adjoint S stage: 2^d
  int64_t nrhs;
  const int32_t* cand_beg;
  const int32_t* cand_len;
  const int32_t* rank;
  const int32_t* skel_off;
  const uint64_t* mask;
  const int64_t* T_off;
  const void* T;           // double2 or float2 entries
  const void* in;
  void* out;
  int pmax;                // largest factor block (entries) of the stage: LDS per ID
  int cmax;                // largest candidate set of the stage (1-RHS: IDs per wavefront)
  int gemm_rows;           // matrix-core stage: rows of A staged per unit (multiple of 16 for FP32, 32 for BF16)
  int rhs_iter;            // matrix-core stage: right-hand-side blocks a workgroup walks through per staged A
                           // (0: the kernel's default)
  // middle stage
  bool dense;              // H = 0: one N x N block
  int64_t rlen_host;       // its row count
  int nsub;                // blocks per output: 2^(d-H) (1 when H = 0)
  const int32_t* rbeg;
  const int32_t* rlen;
  const int32_t* cbeg;
  const int32_t* clen;
};
// Block jb of the middle-stage group q.  Forward: the U_H ID q owns the
// consecutive blocks q nsub + jb.  Adjoint: the V_H ID q = p 2^d + C' meets
// the blocks S(R, C') of the U_H IDs (R, C' >> sh), R = (p << sh) + jb
// (A.nn = 2^d, A.nsub = 2^sh).
template <bool ADJ>
__device__ __forceinline__ int64_t middle_block(const StageArgs& A, int64_t q, int jb) {
  if constexpr (!ADJ) {
    return q * A.nsub + jb;
  } else {
    const int sh = __builtin_ctz((unsigned)A.nsub);
    const int64_t p = q / A.nn, cn = q % A.nn;
    return ((cn >> sh) * A.nn + (p << sh) + jb) * A.nsub + (cn & (A.nsub - 1));
  }
}

// Stage launchers, named by the shape of the stage (V: IDs read a candidate
// segment and write their skeleton rows; U: ID pairs write a shared
// candidate segment; S: the middle factor).  adj: the adjoint of the other
// factor of that shape -- V-shaped over U factors (conj(T), T row-major),
// U-shaped over V factors (conj(T), T column-major), S^H grouped by V_H ID
// (nn = 2^d).
hipError_t launch_apply_v(const StageArgs& a, bool fp64, hipStream_t st, bool adj = false);
hipError_t launch_apply_u(const StageArgs& a, bool fp64, hipStream_t st, bool adj = false);
hipError_t launch_apply_s(const StageArgs& a, bool fp64, hipStream_t st, bool adj = false);
// matrix-core stage kernels: mode 0 V, 1 S, 2 U (the shape, as above, with
// adj selecting the adjoint of the other factor); kmax_unit and mmax_unit
// bound the K and M of every unit of the stage (size the LDS of A); prec:
// FP32 or BF16 split on complex64 data, FP64 on complex128 data.  A stage
// whose A would need more than kMaxGemmLds bytes of LDS is refused
// (hipErrorInvalidValue): gemm_lds_bytes tells beforehand.
enum { kGemmF32 = 0, kGemmBf16 = 1, kGemmF64 = 2 };
constexpr size_t kMaxGemmLds = size_t(156) << 10;  // 160 KB less the kernels' static arrays
size_t gemm_lds_bytes(int kmax_unit, int mmax_unit, int prec);
// Fused two-stage groups of the complex64 many-RHS apply (forward; prec
// kGemmF32 or kGemmBf16):
// V stages t, t + 1 (mode 0; a1 the level-t units, a2 the level-(t+1) ones)
// or U stages t, t - 1 (mode 2), every ID of both levels of rank <= 16 tk
// (tk = 1 or 2), stage-1 units' K <= kmax1, stage-2 units' M <= mmax2 <= 64.
// a1.in is read and a2.out written; the intermediate stays in registers.
constexpr size_t kMaxFusedLds = size_t(152) << 10;  // 160 KB less the kernel's static arrays
constexpr int kMaxRhsIter = 64;                      // largest StageArgs::rhs_iter
size_t fused2_lds_bytes(int tk, int kmax1, int mmax2);
hipError_t launch_apply_fused2(const StageArgs& a1, const StageArgs& a2, int mode, int tk, int kmax1, int mmax2,
                               int prec, hipStream_t st);
hipError_t launch_apply_gemm(const StageArgs& a, int mode, int kmax_unit, int mmax_unit, int prec,
                             hipStream_t st, bool adj = false);

}  // namespace idbf
