// Batched linear-scaling interpolative decomposition (Section 2.1, Lemma 2.1,
// eqs. pivotedQR2, acc, R2) on gfx950, in FP64.  Two kernels:
//
// select_kernel -- Mock-Chebyshev sample selection, one wavefront per ID.
//   Targets are searched in parallel (one lane per target) by an
//   interpolation-then-bisection search over the sorted allowed coordinates;
//   the sequential "nearest unused point" rule runs only for IDs where two
//   targets share a nearest point (otherwise it gives the same picks).
//
// id_kernel -- sampling + pivoted QR + interpolation solve, one ID per
//   workgroup of W wavefronts.  Lane l owns candidate l (a column of the
//   sampled matrix B = K(samples, cand) for a column ID, or of
//   B = K(cand, samples)^T for a row ID); wave w holds sampled rows
//   [R w, R w + R) of every column in registers, so the Householder sweep,
//   column norms and dot products are lane-local.  Per step: residual norms
//   are recomputed; M = max (DPP reduction); stop when M <= eps |R_00|; the
//   pivot is the smallest candidate index with norm >= (1 - 1e-8) M (ballot);
//   the pivot column's Householder vector goes through LDS, and only the
//   wavefront that holds row j applies row masks.  Then T = R11^{-1} R12 by
//   back-substitution over R rows staged in LDS, one redundant candidate per
//   thread, rows permuted to ascending skeletons.
// id_kernel_g -- the same, with two (up to 32 candidates) or four (up to 16)
//   IDs per workgroup, each on its own group of lanes.
#include <algorithm>
#include <atomic>
#include <climits>

#include "kernels.hpp"

namespace idbf {

namespace {

constexpr int kSelIds = 4;  // IDs (wavefronts) per selection workgroup
constexpr uint64_t kSamplerSalt = 0xA0761D6478BD642Full;  // keeps sampler counters apart from other draws

__device__ double cheb_fraction(int j, int s) {
  if (s == 1) return 0.5;
  const int n = s - 1;
  if (j == 0) return 0.0;
  if (j == n) return 1.0;
  if (3 * j == n) return 0.25;
  if (2 * j == n) return 0.5;
  if (3 * j == 2 * n) return 0.75;
  return 0.5 * (1.0 - cos(M_PI * (double)j / (double)n));
}

// Target lo + (hi - lo) f, with the product and the sum rounded separately as
// the definition is written: a fused multiply-add rounds once and can move a
// target that sits on the midpoint of two inexact coordinates (points n pi,
// f = 1/4) to the other side.
__device__ __forceinline__ double cheb_target(double lo, double hi, double f) {
#pragma clang fp contract(off)
  const double span = hi - lo;
  return lo + span * f;
}

// Coordinates of an index segment: direct[p] when a coordinate array is
// given, else base[idx[p]].
struct Seg {
  const double* direct;
  const double* base;
  const int32_t* idx;
  __device__ __forceinline__ double operator()(int64_t p) const { return direct ? direct[p] : base[idx[p]]; }
};

// Position of the point nearest to z in the ascending segment a[0..n), the
// smaller position on a tie.  Up to four interpolation probes, then bisection.
__device__ int nearest_pos(const Seg& a, int n, double z) {
  const double a0 = a(0);
  if (n == 1 || z <= a0) return 0;
  const double an = a(n - 1);
  if (z > an) return n - 1;
  int lo = 0, hi = n - 1;  // a[lo] < z <= a[hi]
  double alo = a0, ahi = an;
  for (int it = 0; hi - lo > 1; ++it) {
    int g;
    if (it < 4) {
      const double f = (z - alo) / (ahi - alo);
      g = lo + 1 + (int)(f * (double)(hi - lo - 1));
      g = min(max(g, lo + 1), hi - 1);
    } else {
      g = (lo + hi) >> 1;
    }
    const double ag = a(g);
    if (ag < z) {
      lo = g;
      alo = ag;
    } else {
      hi = g;
      ahi = ag;
    }
  }
  return (__builtin_fabs(alo - z) <= __builtin_fabs(ahi - z)) ? lo : hi;
}

// Sequential rule, given each target z[j] and its nearest point p0[j]: for
// targets in order, the nearest unused point (smaller position on a tie); then
// ascending order.  Used positions are a bitmap when the set is small enough,
// else a scan of the picks at or below the largest pick so far (later
// nearest points above it are free).
constexpr int kSelBitmapWords = 256;  // positions covered by the bitmap: 8192

__device__ void greedy_select(const Seg& a, int n, int s, const double* z, const int* p0, int* pos,
                              uint32_t* bits) {
  const bool use_bits = n <= kSelBitmapWords * 32;
  int maxpick = -1;
  auto used = [&](int p) -> bool {
    if (use_bits) return (bits[p >> 5] >> (p & 31)) & 1u;
    if (p > maxpick) return false;
    for (int t = 0; t < s; ++t)
      if (pos[t] == p) return true;
    return false;
  };
  // nearest unused position <= p (or -1) and >= p (or n); with the bitmap a
  // word of 32 positions per step (near-full selections collide at almost
  // every target)
  auto free_le = [&](int p) -> int {
    if (!use_bits) {
      while (p >= 0 && used(p)) --p;
      return p;
    }
    while (p >= 0) {
      const uint32_t f = ~bits[p >> 5] & (0xffffffffu >> (31 - (p & 31)));  // free bits <= p in its word
      if (f) return (p & ~31) + 31 - __clz(f);
      p = (p & ~31) - 1;
    }
    return -1;
  };
  auto free_ge = [&](int p) -> int {
    if (!use_bits) {
      while (p < n && used(p)) ++p;
      return p;
    }
    while (p < n) {
      const uint32_t f = ~bits[p >> 5] & (0xffffffffu << (p & 31));  // free bits >= p in its word
      if (f) return min((p & ~31) + __ffs(f) - 1, n);
      p = (p & ~31) + 32;
    }
    return n;
  };
  for (int j = 0; j < s; ++j) pos[j] = -1;
  for (int j = 0; j < s; ++j) {
    const int q0 = p0[j];
    int pick = q0;
    if (used(q0)) {
      const int l = free_le(q0 - 1);
      const int r = free_ge(q0 + 1);
      if (l < 0) {
        pick = r;
      } else if (r >= n) {
        pick = l;
      } else {
        pick = (__builtin_fabs(a(l) - z[j]) <= __builtin_fabs(a(r) - z[j])) ? l : r;
      }
    }
    pos[j] = pick;
    maxpick = max(maxpick, pick);
    if (use_bits) bits[pick >> 5] |= 1u << (pick & 31);
  }
  for (int i = 1; i < s; ++i) {
    const int v = pos[i];
    int k = i - 1;
    while (k >= 0 && pos[k] > v) {
      pos[k + 1] = pos[k];
      --k;
    }
    pos[k + 1] = v;
  }
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wavefront per ID; waves never synchronize with each other.  Six
// wavefronts per SIMD (80 VGPRs): the searches are latency-bound.
__global__ __launch_bounds__(64 * kSelIds) __attribute__((amdgpu_waves_per_eu(6, 8))) void select_kernel(IdArgs A) {
  __shared__ int s_pos[kSelIds][kMaxSamples];
  __shared__ int s_p0[kSelIds][kMaxSamples];
  __shared__ double s_z[kSelIds][kMaxSamples];
  __shared__ uint32_t s_bits[kSelIds][kSelBitmapWords];
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int64_t qi = blockIdx.x * (int64_t)kSelIds + w;
  if (qi >= (A.sel_list ? A.sel_n : A.n_ids)) return;
  const int64_t q = A.sel_list ? (int64_t)A.sel_list[qi] : qi;
  const int c = A.cand_len[q], na = A.allow_len[q];
  const int s = A.samples ? A.samples[q] : min(A.oversample * c, na);
  if (c < 1 || c > kMaxCand || na < 1 || s < 1 || s > kMaxSamples || s > A.samp_ld) return;  // the QR reports it
  int32_t* out = A.samp_pos + q * A.samp_ld;
  if (s >= na) {
    for (int j = lane; j < na; j += kWave) out[j] = j;
    return;
  }
  if (A.sampler == IDBF_SAMPLER_RANDOM) {
    // Floyd's algorithm: for j = na-s .. na-1 draw t uniform in [0, j] (SplitMix64
    // of a counter from seed, level, side, ID, draw); take t, or j if t is taken
    if (lane == 0) {
      const uint64_t base = ((A.seed & 0xffffffffull) << 32) ^ ((uint64_t)A.level << 24) ^
                            ((uint64_t)A.side << 23) ^ (uint64_t)q;
      for (int i = 0; i < s; ++i) {
        const int64_t j = (int64_t)na - s + i;
        uint64_t z = (((base << 8) | (uint64_t)i) ^ kSamplerSalt) + 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        int t = (int)(((z >> 32) * (uint64_t)(j + 1)) >> 32);
        for (int e = 0; e < i; ++e)
          if (s_pos[w][e] == t) {
            t = (int)j;
            break;
          }
        s_pos[w][i] = t;
      }
    }
    wave_lds_sync();
    // ascending: each chosen position goes to its rank (positions are distinct)
    for (int e = lane; e < s; e += kWave) {
      const int v = s_pos[w][e];
      int rank = 0;
      for (int f = 0; f < s; ++f) rank += s_pos[w][f] < v;
      out[rank] = v;
    }
    return;
  }
  const bool isV = (A.side == IDBF_SIDE_V);
  const int ab = A.allow_beg[q];
  const Seg a{A.allow_coord ? A.allow_coord + ab : nullptr, isV ? A.X : A.Om, A.allow_idx + ab};
  const double lo = a(0), hi = a(na - 1);
  int coll = 0;
  int prev_last = -1;
  for (int j0 = 0; j0 < s; j0 += kWave) {
    const int j = j0 + lane;
    int p = -1;
    if (j < s) {
      const double z = cheb_target(lo, hi, cheb_fraction(j, s));
      p = nearest_pos(a, na, z);
      s_z[w][j] = z;
      s_p0[w][j] = p;
    }
    const int left = __shfl_up(p, 1, kWave);
    const int before = (lane == 0) ? prev_last : left;
    if (j < s && j > 0 && p == before) coll = 1;
    prev_last = __shfl(p, kWave - 1, kWave);
  }
  if (__ballot(coll)) {
    if (na <= kSelBitmapWords * 32)
      for (int i = lane; i < (na + 31) / 32; i += kWave) s_bits[w][i] = 0u;
    wave_lds_sync();
    if (lane == 0) greedy_select(a, na, s, s_z[w], s_p0[w], s_pos[w], s_bits[w]);
    wave_lds_sync();
    for (int j = lane; j < s; j += kWave) out[j] = s_pos[w][j];
  } else {
    wave_lds_sync();
    for (int j = lane; j < s; j += kWave) out[j] = s_p0[w][j];
  }
}

// Maximum over the 64 lanes of a wavefront of values that are either >= 0 or
// negative placeholders.  Non-negative doubles order like their bit patterns,
// so the maximum is taken on the high words (signed, so that placeholders sort
// below every non-negative value), then on the low words of the lanes that
// share the largest high word.  Each pass is a DPP max: row_shr within rows of
// 16, then row broadcasts; lane 63 ends with the maximum.
template <typename T, int CTRL, int ROWMASK>
__device__ __forceinline__ T dpp_max(T v, T identity) {
  const T o = (T)__builtin_amdgcn_update_dpp((int)identity, (int)v, CTRL, ROWMASK, 0xf, false);
  return v > o ? v : o;
}
template <typename T>
__device__ __forceinline__ T wave_max32(T v, T identity) {
  v = dpp_max<T, 0x111, 0xf>(v, identity);  // row_shr:1
  v = dpp_max<T, 0x112, 0xf>(v, identity);  // row_shr:2
  v = dpp_max<T, 0x114, 0xf>(v, identity);  // row_shr:4
  v = dpp_max<T, 0x118, 0xf>(v, identity);  // row_shr:8
  v = dpp_max<T, 0x142, 0xa>(v, identity);  // row_bcast:15
  v = dpp_max<T, 0x143, 0xc>(v, identity);  // row_bcast:31
  return (T)__builtin_amdgcn_readlane((int)v, kWave - 1);
}
__device__ __forceinline__ double wave_max_nonneg(double v) {
  const int hi = __double2hiint(v);
  const int mh = wave_max32<int>(hi, INT_MIN);
  const unsigned lo = (hi == mh) ? (unsigned)__double2loint(v) : 0u;
  const unsigned ml = wave_max32<unsigned>(lo, 0u);
  return __hiloint2double(mh, (int)ml);
}

// Maximum over each group of 64 / G lanes (G = 2: lanes [32 g, 32 g + 32);
// G = 4: rows of 16), by the same two 32-bit passes, returned in every lane
// of the group: row_shr steps leave each row's maximum in its lane 15,
// row_bcast:15 joins rows 0-1 and 2-3, and the group's last lane is read.
template <typename T, int G>
__device__ __forceinline__ T group_max32(T v, T identity, int lane) {
  v = dpp_max<T, 0x111, 0xf>(v, identity);  // row_shr:1
  v = dpp_max<T, 0x112, 0xf>(v, identity);  // row_shr:2
  v = dpp_max<T, 0x114, 0xf>(v, identity);  // row_shr:4
  v = dpp_max<T, 0x118, 0xf>(v, identity);  // row_shr:8
  if constexpr (G == 2) v = dpp_max<T, 0x142, 0xa>(v, identity);  // row_bcast:15
  constexpr int last = kWave / G - 1;
  return (T)__shfl((int)v, lane | last, kWave);
}
template <int G>
__device__ __forceinline__ double group_max_nonneg(double v, int lane) {
  const int hi = __double2hiint(v);
  const int mh = group_max32<int, G>(hi, INT_MIN, lane);
  const unsigned lo = (hi == mh) ? (unsigned)__double2loint(v) : 0u;
  const unsigned ml = group_max32<unsigned, G>(lo, 0u, lane);
  return __hiloint2double(mh, (int)ml);
}

__device__ __forceinline__ bool skel_bit(uint64_t lo, uint64_t hi, int p) {
  return p < 64 ? ((lo >> p) & 1ull) : ((hi >> (p - 64)) & 1ull);
}

// Number of skeletons among candidate positions < p (128-bit mask lo | hi).
__device__ __forceinline__ int skel_below(uint64_t lo, uint64_t hi, int p) {
  return p < 64 ? __popcll(lo & lanes_below(p)) : __popcll(lo) + __popcll(hi & lanes_below(p - 64));
}

// One ID per workgroup of W wavefronts.  Lane l owns candidate columns
// l + 64 cs (cs < CPL); wavefront w holds sampled rows [R w, R w + R).
//   CPL = 1, R = 16: up to 64 candidates and 64 samples (W <= 4);
//   CPL = 1, W = 4:  65..80, 81..96 and 97..112 samples with R = 20, 24 and
//                    28 (three wavefronts per SIMD; 113..128 take W = 8,
//                    R = 16).  Each pivot step pays two workgroup barriers
//                    and cross-wave reductions, so at this register budget
//                    few tall wavefronts beat many short ones: three IDs per
//                    CU instead of two (W = 8), or the same three with
//                    four-wave instead of five-wave barriers (W = 5);
//   CPL = 2, R = 8:  up to 128 candidates (W <= 16), same registers per lane.
template <int W, int CPL, int R>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(R > 16 ? 3 : 4, 8))) void id_kernel(IdArgs A) {
  constexpr int SMAX = R * W;
  constexpr int NC = kWave * CPL;     // candidate columns covered
  // R rows staged in LDS per back-substitution chunk: 32 KiB where registers
  // already limit a CU to four workgroups, else 16 KiB
  constexpr int kChunk = (W >= 4 ? 32 : 16) / CPL;
  // partial sums of the QR loop and the R rows of the solve share LDS
  constexpr size_t kPart = (size_t)W * CPL * kWave * (sizeof(double) + sizeof(double2));
  constexpr size_t kRrows = (size_t)kChunk * NC * sizeof(double2);
  __shared__ __attribute__((aligned(16))) unsigned char s_raw[kPart > kRrows ? kPart : kRrows];
  __shared__ double s_coord[SMAX];
  __shared__ double s_cx[SMAX];
  __shared__ double2 s_v[SMAX];
  __shared__ int s_piv[kMaxRank];
  __shared__ int s_srank[kMaxRank];
  __shared__ double s_axj[2];
  __shared__ double2 s_diag[kMaxRank];  // R_jj of each step (1 / R_jj once the loop ends)
  double* s_part = reinterpret_cast<double*>(s_raw);                                         // [W][CPL][64]
  double2* s_partc = reinterpret_cast<double2*>(s_raw + W * CPL * kWave * sizeof(double));  // [W][CPL][64]
  double2* s_R = reinterpret_cast<double2*>(s_raw);                                          // [kChunk][NC]

  const int64_t q = A.order ? A.order[blockIdx.x] : (int64_t)blockIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform: row tests branch on SGPRs
  const int nthreads = kWave * W;
  const int cb = A.cand_beg[q], c = A.cand_len[q];
  const int ab = A.allow_beg[q], na = A.allow_len[q];
  const int s = A.samples ? A.samples[q] : min(A.oversample * c, na);
  const bool tall = is_tall(s);  // the block is the row reduction's c x c triangular factor
  const int srows = qr_rows(c, s);
  const int64_t tslot =
      (tall && A.tall_slot) ? (int64_t)__builtin_amdgcn_readfirstlane(A.tall_slot[q]) : -1;  // uniform
  if (c < 1 || c > NC || na < 1 || s < 1 || s > kMaxSamples || s > A.samp_ld || srows > SMAX || s > na ||
      (tall && (tslot < 0 || tslot >= A.n_tall || (int64_t)c * c > A.tall_ld2))) {
    if (threadIdx.x == 0) atomicOr(A.status, kErrSize);
    return;
  }
  const bool isV = (A.side == IDBF_SIDE_V);
  const bool fio = (A.ph.kind == IDBF_PHASE_FIO);
  const Seg cs_{A.cand_coord ? A.cand_coord + cb : nullptr, isV ? A.Om : A.X, A.cand_idx + cb};
  const Seg as{A.allow_coord ? A.allow_coord + ab : nullptr, isV ? A.X : A.Om, A.allow_idx + ab};

  int gidx[CPL];
  double ccoord[CPL], ccx[CPL];
#pragma unroll
  for (int cs = 0; cs < CPL; ++cs) {
    const int col = lane + kWave * cs;
    gidx[cs] = 0;
    ccoord[cs] = 0.0;
    ccx[cs] = 0.0;
    if (col < c) {
      gidx[cs] = A.cand_idx[cb + col];
      ccoord[cs] = cs_(col);
      if (!isV && fio) ccx[cs] = amplitude_shift(A.ph, ccoord[cs]);
    }
  }
  const int32_t* sp = A.samp_pos + q * A.samp_ld;
  for (int j = threadIdx.x; j < s && !tall; j += nthreads) {
    const double v = as(sp[j]);
    s_coord[j] = v;
    s_cx[j] = (isV && fio) ? amplitude_shift(A.ph, v) : 0.0;
  }
  __syncthreads();

  // sampled block: rows [R w, R w + R) of columns lane + 64 cs (rows >= srows stay zero)
  const int row0 = w * R;
  double2 a[CPL][R];
  if (tall) {  // upper triangle of the reduced block
    const double2* Rt = A.tall_R + tslot * A.tall_ld2;
#pragma unroll
    for (int cs = 0; cs < CPL; ++cs)
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int row = row0 + i, col = lane + kWave * cs;
        a[cs][i] = (col < c && row <= col) ? Rt[col * c + row] : make_double2(0.0, 0.0);
      }
  } else {
#pragma unroll
    for (int cs = 0; cs < CPL; ++cs)
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int row = row0 + i;
        double2 v = make_double2(0.0, 0.0);
        if (lane + kWave * cs < c && row < s) {  // one call site per row: K(sample, cand) or K(cand, sample)
          const double sc = s_coord[row];
          v = kernel_entry(A.ph, isV ? sc : ccoord[cs], isV ? s_cx[row] : ccx[cs], isV ? ccoord[cs] : sc);
        }
        a[cs][i] = v;
      }
  }

  const int kuser = min(min(min(s, c), A.kmax > 0 ? A.kmax : (1 << 30)), A.truncate ? kMaxRank : (1 << 30));
  // a skeleton proposal restricts the pivot search to the proposed columns
  // (a 128-bit mask, the same in every lane)
  const bool restricted = A.prop_k != nullptr;
  uint64_t pm0 = ~0ull, pm1 = ~0ull;
  if (restricted) {
    pm0 = pm1 = 0;
    const uint8_t* fpiv = A.prop_cols + q * (int64_t)kMaxRank;
    const int kf = __builtin_amdgcn_readfirstlane(min(A.prop_k[q], kMaxRank));
    for (int i = 0; i < kf; ++i) {
      const int p = __builtin_amdgcn_readfirstlane((int)fpiv[i]);
      if (p < kWave) pm0 |= 1ull << p;
      else if (p < 2 * kWave) pm1 |= 1ull << (p - kWave);
    }
  }
  bool proposed[CPL];
#pragma unroll
  for (int cs = 0; cs < CPL; ++cs) proposed[cs] = (((cs == 0 ? pm0 : pm1) >> lane) & 1ull) != 0;
  bool pivoted[CPL];
  int pstep[CPL];  // step at which the column became a pivot
#pragma unroll
  for (int cs = 0; cs < CPL; ++cs) {
    pivoted[cs] = false;
    pstep[cs] = 0;
  }
  double stop2 = 0.0;  // (tol |R_00|)^2
  int k = 0;
  bool zero_block = false, overflow = false;
  // residual column norms of this wave's rows, for step 0; later steps get
  // them from the update loop of the step before (rows >= j + 1)
  double part[CPL];
#pragma unroll
  for (int cs = 0; cs < CPL; ++cs) {
    double p0 = 0.0, p1 = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      if (i & 1) p1 = __builtin_fma(a[cs][i].y, a[cs][i].y, __builtin_fma(a[cs][i].x, a[cs][i].x, p1));
      else p0 = __builtin_fma(a[cs][i].y, a[cs][i].y, __builtin_fma(a[cs][i].x, a[cs][i].x, p0));
    }
    part[cs] = p0 + p1;
  }
  for (int j = 0;; ++j) {
    const bool live = row0 + R > j;   // wave-uniform: this wave holds rows >= j
    const bool edge = live && row0 <= j;  // ... and row j itself (rows < j must stay as they are)
    double nrm2[CPL];
#pragma unroll
    for (int cs = 0; cs < CPL; ++cs) nrm2[cs] = part[cs];
    if constexpr (W > 1) {
#pragma unroll
      for (int cs = 0; cs < CPL; ++cs) s_part[(w * CPL + cs) * kWave + lane] = part[cs];
      __syncthreads();
#pragma unroll
      for (int cs = 0; cs < CPL; ++cs) {
        nrm2[cs] = 0.0;
#pragma unroll(CPL == 1 ? W : 4)
        for (int ww = 0; ww < W; ++ww) nrm2[cs] += s_part[(ww * CPL + cs) * kWave + lane];
      }
    }
    // pivot search on squared norms (sqrt is monotone: the same maximum, and
    // the tie band below is far wider than a rounding of the square)
    bool active[CPL], eligible[CPL];  // not yet a pivot (updated) / and proposed (may become one)
    double nq[CPL];
    double nqmax = -1.0;
#pragma unroll
    for (int cs = 0; cs < CPL; ++cs) {
      active[cs] = (lane + kWave * cs < c) && !pivoted[cs];
      eligible[cs] = active[cs] && proposed[cs];
      nq[cs] = eligible[cs] ? nrm2[cs] : -1.0;
      nqmax = fmax(nqmax, nq[cs]);
    }
    // squared maximum residual norm; the stopping test M <= tol |R_00| is
    // taken on squares
    const double M2 = wave_max_nonneg(nqmax);
    if (j == 0) {
      // |R_00| of the unrestricted QR: the largest column norm of the block
      double all = M2;
      if (restricted) {
        double m = -1.0;
#pragma unroll
        for (int cs = 0; cs < CPL; ++cs)
          if (lane + kWave * cs < c) m = fmax(m, nrm2[cs]);
        all = wave_max_nonneg(m);
      }
      if (!(all > 0.0)) {
        zero_block = true;
        break;
      }
      const double b = A.tol * sqrt(all);
      stop2 = b * b;
    }
    if ((j > 0 || restricted) && M2 <= stop2) break;  // (a proposal may end at step 0)
    if (j == kuser) break;
    if (j == kMaxRank) {
      overflow = true;
      break;
    }
    int p;
    {
      constexpr double kTie2 = (1.0 - kPivotTie) * (1.0 - kPivotTie);
      const double thr2 = kTie2 * M2;
      const uint64_t near0 = __ballot(eligible[0] && nq[0] >= thr2);
      uint64_t near1 = 0;
      if constexpr (CPL > 1) near1 = __ballot(eligible[CPL - 1] && nq[CPL - 1] >= thr2);
      if (near0 == 0 && near1 == 0) break;  // no finite residual norm left (cannot happen for finite input)
      p = __builtin_amdgcn_readfirstlane(
          near0 ? __ffsll((unsigned long long)near0) - 1 : kWave + __ffsll((unsigned long long)near1) - 1);
    }
    const int pl = p & (kWave - 1), pc = p / kWave;  // pivot lane and column slot (uniform)
    // Householder vector of the pivot column (rows >= j): lane pl of every
    // live wave publishes its own rows to the wave's slice of LDS (no
    // workgroup barrier); the wave that holds row j zeroes the rows above it,
    // so that rows < j drop out of the dot and the update exactly, and forms
    // the head:
    //   v_i = a_i(p) for i > j, v_j = x_j - alpha,
    //   alpha = -(x_j/|x_j|) nu_p, tau = 2 / |v|^2 = 1 / (nu_p (nu_p + |x_j|)).
    // The pivot column's registers are left as they are: below the diagonal
    // they are never read again, and R_jj = alpha is kept in LDS.
    const double nup = sqrt(readlane(pc == 0 ? nq[0] : nq[CPL - 1], pl));
    if (lane == pl && live) {
      if (!edge) {
        if (pc == 0) {
#pragma unroll
          for (int i = 0; i < R; ++i) s_v[row0 + i] = a[0][i];
        } else {
#pragma unroll
          for (int i = 0; i < R; ++i) s_v[row0 + i] = a[CPL - 1][i];
        }
      } else {
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const double2 ai = (pc == 0) ? a[0][i] : a[CPL - 1][i];
          s_v[row0 + i] = (row0 + i >= j) ? ai : make_double2(0.0, 0.0);
        }
        const double2 xj = s_v[j];  // same-lane LDS accesses are ordered
        const double axj = sqrt(cabs2(xj));
        double2 vj;
        if (axj > 0.0) {
          const double g = nup / axj;  // alpha = -g x_j, v_j = (1 + g) x_j
          s_diag[j] = make_double2(-xj.x * g, -xj.y * g);
          vj = make_double2(xj.x + xj.x * g, xj.y + xj.y * g);
        } else {
          s_diag[j] = make_double2(-nup, 0.0);
          vj = make_double2(nup, 0.0);
        }
        s_v[j] = vj;
        s_axj[j & 1] = axj;
      }
    }
    wave_lds_sync();
    double2 dot[CPL];
#pragma unroll
    for (int cs = 0; cs < CPL; ++cs) {
      dot[cs] = make_double2(0.0, 0.0);
      if (live) {
        double2 d0 = make_double2(0.0, 0.0), d1 = make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < R; ++i) {
          if (i & 1) d1 = cfma_conj(s_v[row0 + i], a[cs][i], d1);
          else d0 = cfma_conj(s_v[row0 + i], a[cs][i], d0);
        }
        dot[cs] = cadd(d0, d1);
      }
    }
    if constexpr (W > 1) {
#pragma unroll
      for (int cs = 0; cs < CPL; ++cs) s_partc[(w * CPL + cs) * kWave + lane] = dot[cs];
      __syncthreads();
#pragma unroll
      for (int cs = 0; cs < CPL; ++cs) {
        dot[cs] = make_double2(0.0, 0.0);
#pragma unroll(CPL == 1 ? W : 4)
        for (int ww = 0; ww < W; ++ww) dot[cs] = cadd(dot[cs], s_partc[(ww * CPL + cs) * kWave + lane]);
      }
    }
    // tau = 1 / (nu_p (nu_p + |x_j|)): hardware reciprocal and two Newton steps
    const double den = nup * (nup + s_axj[j & 1]);
    double tau = __builtin_amdgcn_rcp(den);
    tau = __builtin_fma(tau, __builtin_fma(-den, tau, 1.0), tau);
    tau = __builtin_fma(tau, __builtin_fma(-den, tau, 1.0), tau);
#pragma unroll
    for (int cs = 0; cs < CPL; ++cs) {
      // update, and the residual norm of rows >= j + 1 for the next step (the
      // wave that holds row j recounts its rows below j)
      part[cs] = 0.0;
      if (live && active[cs] && !(lane == pl && cs == pc)) {
        const double2 sdot = make_double2(-tau * dot[cs].x, -tau * dot[cs].y);
        double p0 = 0.0, p1 = 0.0;
#pragma unroll
        for (int i = 0; i < R; ++i) {
          a[cs][i] = cfma(s_v[row0 + i], sdot, a[cs][i]);
          if (i & 1) p1 = __builtin_fma(a[cs][i].y, a[cs][i].y, __builtin_fma(a[cs][i].x, a[cs][i].x, p1));
          else p0 = __builtin_fma(a[cs][i].y, a[cs][i].y, __builtin_fma(a[cs][i].x, a[cs][i].x, p0));
        }
        if (edge) {  // rows <= j of this wave are final: recount without them
          p0 = 0.0;
          p1 = 0.0;
#pragma unroll
          for (int i = 0; i < R; ++i)
            if (row0 + i > j) {
              if (i & 1) p1 = __builtin_fma(a[cs][i].y, a[cs][i].y, __builtin_fma(a[cs][i].x, a[cs][i].x, p1));
              else p0 = __builtin_fma(a[cs][i].y, a[cs][i].y, __builtin_fma(a[cs][i].x, a[cs][i].x, p0));
            }
        }
        part[cs] = p0 + p1;
      }
    }
    if (lane == pl) {
#pragma unroll
      for (int cs = 0; cs < CPL; ++cs)
        if (cs == pc) {
          pivoted[cs] = true;
          pstep[cs] = j;
        }
    }
    if (threadIdx.x == 0) s_piv[j] = p;
    k = j + 1;
  }
  if (k == 0) {  // no pivot taken: keep the first candidate, T = 0
    if (restricted && !zero_block && threadIdx.x == 0) A.prop_fail[q] = 1;  // no proposed column above eps
    zero_block = true;
  }
  if (zero_block) {
    k = 1;
#pragma unroll
    for (int cs = 0; cs < CPL; ++cs) {
      pivoted[cs] = (cs == 0 && lane == 0);
      pstep[cs] = 0;
    }
    if (threadIdx.x == 0) s_piv[0] = 0;
  }
  if (overflow && threadIdx.x == 0) atomicOr(A.status, kErrRank);
  __syncthreads();  // s_piv complete; every read of the partial sums is done

  // skeleton masks (identical in every wave: pivot decisions are)
  const uint64_t msk0 = __ballot(pivoted[0] && lane < c);
  uint64_t msk1 = 0;
  if constexpr (CPL > 1) msk1 = __ballot(pivoted[CPL - 1] && lane + kWave < c);
  for (int i = threadIdx.x; i < k; i += nthreads) {
    s_srank[i] = skel_below(msk0, msk1, s_piv[i]);
    if (!zero_block) {  // 1 / R_ii, for the solve
      const double2 d = s_diag[i];
      const double inv = 1.0 / cabs2(d);
      s_diag[i] = make_double2(d.x * inv, -d.y * inv);
    }
  }
  if (w == 0) {
    if (lane == 0) {
      A.rank[q] = k;
      A.mask[2 * q] = msk0;
      A.mask[2 * q + 1] = msk1;
    }
#pragma unroll
    for (int cs = 0; cs < CPL; ++cs) {
      const int col = lane + kWave * cs;
      if (pivoted[cs] && col < c) A.skel_out[q * kMaxCand + skel_below(msk0, msk1, col)] = gidx[cs];
    }
  }
  // Back-substitution T = R11^{-1} R12 in chunks of kChunk R rows staged in
  // LDS, last chunk first, with the columns permuted: pivot l at slot l,
  // redundant candidate jr at slot k + jr, so both operands of
  //   t_ii = (r_ii - sum_{l > ii} R[ii][piv_l] t_l) / R[ii][piv_ii]
  // are direct loads.  Waves 0..CPL-1 own the redundant columns (one per
  // thread); t_l of earlier (higher) chunks are read back from this thread's
  // T entries.
  const int r = c - k;
  const int64_t off = A.T_off ? A.T_off[q] : q * (int64_t)kSlot;
  int slot[CPL];
#pragma unroll
  for (int cs = 0; cs < CPL; ++cs) {
    const int cc = lane + kWave * cs;
    slot[cs] = pivoted[cs] ? pstep[cs] : k + cc - skel_below(msk0, msk1, cc);
  }
  const int col = (w < CPL) ? w * kWave + lane : 0;
  const bool solver = (w < CPL) && col < c && !skel_bit(msk0, msk1, col);
  const int jr = solver ? col - skel_below(msk0, msk1, col) : 0;
  auto t_index = [&](int l) -> int64_t {  // T entry of (skeleton of pivot row l, this column)
    const int sr = s_srank[l];
    return off + (isV ? (int64_t)jr * k + sr : (int64_t)sr * r + jr);
  };
  for (int cb0 = ((k - 1) / kChunk) * kChunk; cb0 >= 0; cb0 -= kChunk) {
    const int ce = min(k, cb0 + kChunk);
    __syncthreads();  // the previous chunk's LDS reads are done
#pragma unroll
    for (int cs = 0; cs < CPL; ++cs)
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int row = row0 + i;
        if (row >= cb0 && row < ce && lane + kWave * cs < c)
          s_R[(row - cb0) * NC + slot[cs]] = zero_block ? make_double2(0.0, 0.0) : a[cs][i];
      }
    __syncthreads();
    if (!solver) continue;
    for (int ii = ce - 1; ii >= cb0; --ii) {
      const double2* Ri = s_R + (ii - cb0) * NC;
      double2 acc = Ri[k + jr];
      if (!zero_block) {
        double2 acc1 = make_double2(0.0, 0.0), acc2 = acc1, acc3 = acc1;
        const double2* tcol = s_R + k + jr - cb0 * NC;  // t_l at tcol[l * NC]
        int l = ii + 1;
        for (; l + 3 < ce; l += 4) {  // four independent chains
          const double2 r0 = Ri[l], r1 = Ri[l + 1], r2 = Ri[l + 2], r3 = Ri[l + 3];
          const double2 t0 = tcol[l * NC], t1 = tcol[(l + 1) * NC], t2 = tcol[(l + 2) * NC], t3 = tcol[(l + 3) * NC];
          acc = cfma(make_double2(-r0.x, -r0.y), t0, acc);
          acc1 = cfma(make_double2(-r1.x, -r1.y), t1, acc1);
          acc2 = cfma(make_double2(-r2.x, -r2.y), t2, acc2);
          acc3 = cfma(make_double2(-r3.x, -r3.y), t3, acc3);
        }
        for (; l < ce; ++l) {
          const double2 r0 = Ri[l];
          acc = cfma(make_double2(-r0.x, -r0.y), tcol[l * NC], acc);
        }
        for (l = ce; l < k; ++l) {
          const double2 rl = Ri[l];
          acc1 = cfma(make_double2(-rl.x, -rl.y), A.T128[t_index(l)], acc1);
        }
        acc = cadd(cadd(acc, acc1), cadd(acc2, acc3));
        acc = cmul(acc, s_diag[ii]);  // 1 / R_ii
      }
      s_R[(ii - cb0) * NC + k + jr] = acc;
      const int64_t e = t_index(ii);
      A.T128[e] = acc;
      if (A.T64) A.T64[e] = make_float2((float)acc.x, (float)acc.y);
    }
  }
}


// G IDs per workgroup of W wavefronts, for small IDs (G = 2: up to 32
// candidates and 64 samples; G = 4: up to 16 and 32).  ID g owns lanes
// [g GL, g GL + GL), GL = 64 / G, one candidate per lane, and wavefront w
// holds sampled rows [16 w, 16 w + 16) of every ID.  The IDs take their
// pivot steps together; an ID that has stopped sits out the remaining steps.
// The arithmetic of each ID is the one-ID kernel's.
template <int W, int G>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(4, 8))) void id_kernel_g(IdArgs A,
                                                                                                int64_t n) {
  constexpr int R = 16, SMAX = R * W, GL = kWave / G;
  constexpr int kChunk = W >= 3 ? 32 : 16;  // R rows staged per solve chunk
  constexpr size_t kPart = (size_t)W * kWave * (sizeof(double) + sizeof(double2));
  constexpr size_t kRrows = (size_t)kChunk * kWave * sizeof(double2);
  __shared__ __attribute__((aligned(16))) unsigned char s_raw[kPart > kRrows ? kPart : kRrows];
  __shared__ double s_coord[G][SMAX];
  __shared__ double s_cx[G][SMAX];
  __shared__ double2 s_v[G][SMAX];
  __shared__ int s_piv[G][GL];      // ranks are at most c <= GL
  __shared__ int s_srank[G][GL];
  __shared__ double s_axj[G][2];
  __shared__ double2 s_diag[G][GL];
  __shared__ int s_k[G];
  double* s_part = reinterpret_cast<double*>(s_raw);                                   // [W][64]
  double2* s_partc = reinterpret_cast<double2*>(s_raw + W * kWave * sizeof(double));  // [W][64]
  double2* s_R = reinterpret_cast<double2*>(s_raw);                                    // [kChunk][64]

  const int lane = threadIdx.x & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int nthreads = kWave * W;
  const int gi = lane / GL, gl = lane % GL;  // this lane's ID in the workgroup, and its column
  const bool isV = (A.side == IDBF_SIDE_V);
  const bool fio = (A.ph.kind == IDBF_PHASE_FIO);
  auto id_of = [&](int g) -> int64_t {  // -1 past the end of the bucket
    const int64_t qi = blockIdx.x * (int64_t)G + g;
    return qi < n ? (A.order ? (int64_t)A.order[qi] : qi) : -1;
  };
  auto samples_of = [&](int64_t q, int c, int na) {
    return A.samples ? A.samples[q] : min(A.oversample * c, na);
  };
  // this lane's ID; an ID outside the kernel's limits is reported and sits out
  const int64_t q = id_of(gi);
  int c = 0, cb = 0, s = 0;
  if (q >= 0) {
    c = A.cand_len[q];
    cb = A.cand_beg[q];
    const int na = A.allow_len[q];
    s = samples_of(q, c, na);
    // tall IDs (reduced blocks) always run on the one-ID kernels
    if (c < 1 || c > GL || na < 1 || s < 1 || s > SMAX || s > A.samp_ld || s > na) {
      if (w == 0 && gl == 0) atomicOr(A.status, kErrSize);
      c = 0;
      s = 0;
    }
  }
  const bool member = c > 0;  // this lane's ID takes part

  const int col = gl;
  int gidx = 0;
  double ccoord = 0.0, ccx = 0.0;
  if (col < c) {
    gidx = A.cand_idx[cb + col];
    ccoord = A.cand_coord ? A.cand_coord[cb + col] : (isV ? A.Om : A.X)[gidx];
    if (!isV && fio) ccx = amplitude_shift(A.ph, ccoord);
  }
  for (int e = threadIdx.x; e < G * SMAX; e += nthreads) {  // sampled coordinates of every ID
    const int g = e / SMAX, j = e % SMAX;
    const int64_t qg = id_of(g);
    if (qg < 0) continue;
    const int cg = A.cand_len[qg], nag = A.allow_len[qg];
    const int sg = samples_of(qg, cg, nag);
    if (j >= sg || j >= nag || sg > SMAX || sg > A.samp_ld) continue;
    const int ab = A.allow_beg[qg];
    const int pos = A.samp_pos[qg * A.samp_ld + j];
    const double v = A.allow_coord ? A.allow_coord[ab + pos] : (isV ? A.X : A.Om)[A.allow_idx[ab + pos]];
    s_coord[g][j] = v;
    s_cx[g][j] = (isV && fio) ? amplitude_shift(A.ph, v) : 0.0;
  }
  __syncthreads();

  const int row0 = w * R;
  double2 a[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int row = row0 + i;
    double2 v = make_double2(0.0, 0.0);
    if (col < c && row < s)
      v = isV ? kernel_entry(A.ph, s_coord[gi][row], s_cx[gi][row], ccoord)
              : kernel_entry(A.ph, ccoord, ccx, s_coord[gi][row]);
    a[i] = v;
  }

  const int kuser = min(min(min(s, c), A.kmax > 0 ? A.kmax : (1 << 30)), A.truncate ? kMaxRank : (1 << 30));
  // a skeleton proposal restricts the pivot search to the proposed columns
  const bool restricted = A.prop_k != nullptr;
  bool proposed = !restricted;
  if (restricted && member) {
    const int kf = min(A.prop_k[q], kMaxRank);
    for (int i = 0; i < kf; ++i) proposed = proposed || (int)A.prop_cols[q * (int64_t)kMaxRank + i] == col;
  }
  bool pivoted = false;
  int pstep = 0;
  double stop2 = 0.0;
  int k = 0;
  bool done = !member, zero_block = false, overflow = false;
  double part;
  {
    double p0 = 0.0, p1 = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      if (i & 1) p1 = __builtin_fma(a[i].y, a[i].y, __builtin_fma(a[i].x, a[i].x, p1));
      else p0 = __builtin_fma(a[i].y, a[i].y, __builtin_fma(a[i].x, a[i].x, p0));
    }
    part = p0 + p1;
  }
  const uint64_t gmask = (GL == 64) ? ~0ull : ((1ull << GL) - 1ull);
  for (int j = 0;; ++j) {
    const bool live = row0 + R > j;
    const bool edge = live && row0 <= j;
    double nrm2 = part;
    if constexpr (W > 1) {
      s_part[w * kWave + lane] = part;
      __syncthreads();
      nrm2 = 0.0;
#pragma unroll
      for (int ww = 0; ww < W; ++ww) nrm2 += s_part[ww * kWave + lane];
    }
    const bool active = !done && col < c && !pivoted;  // not yet a pivot: updated
    const bool eligible = active && proposed;          // ... and a pivot candidate
    const double nq = eligible ? nrm2 : -1.0;
    const double M2 = group_max_nonneg<G>(nq, lane);
    // |R_00| of the unrestricted QR: the largest column norm of the block
    const double all = (restricted && j == 0) ? group_max_nonneg<G>(!done && col < c ? nrm2 : -1.0, lane) : M2;
    if (!done) {  // this ID's stopping rules, in the one-ID kernel's order
      if (j == 0) {
        if (!(all > 0.0)) {
          zero_block = true;
          done = true;
        } else {
          const double b = A.tol * sqrt(all);
          stop2 = b * b;
        }
      }
      if (!done && (j > 0 || restricted) && M2 <= stop2) done = true;  // (a proposal may end at step 0)
      if (!done && j == kuser) done = true;
      if (!done && j == kMaxRank) {
        overflow = true;
        done = true;
      }
    }
    constexpr double kTie2 = (1.0 - kPivotTie) * (1.0 - kPivotTie);
    const uint64_t near = __ballot(!done && eligible && nq >= kTie2 * M2);
    const uint64_t gbits = (near >> (gi * GL)) & gmask;
    if (!done && gbits == 0) done = true;  // no finite residual norm left (cannot happen for finite input)
    if (__ballot(!done) == 0) break;       // every ID has stopped (the same in every wavefront)
    const int p = done ? 0 : __ffsll((unsigned long long)gbits) - 1;  // pivot column of this ID
    const int pl = gi * GL + p;                                         // its lane
    const double nup = sqrt(__shfl(nq, pl, kWave));
    if (!done && lane == pl && live) {
#pragma unroll
      for (int i = 0; i < R; ++i) s_v[gi][row0 + i] = (!edge || row0 + i >= j) ? a[i] : make_double2(0.0, 0.0);
      if (edge) {  // same-lane LDS accesses are ordered
        const double2 xj = s_v[gi][j];
        const double axj = sqrt(cabs2(xj));
        double2 vj;
        if (axj > 0.0) {
          const double g = nup / axj;  // alpha = -g x_j, v_j = (1 + g) x_j
          s_diag[gi][j] = make_double2(-xj.x * g, -xj.y * g);
          vj = make_double2(xj.x + xj.x * g, xj.y + xj.y * g);
        } else {
          s_diag[gi][j] = make_double2(-nup, 0.0);
          vj = make_double2(nup, 0.0);
        }
        s_v[gi][j] = vj;
        s_axj[gi][j & 1] = axj;
      }
    }
    wave_lds_sync();
    double2 dot = make_double2(0.0, 0.0);
    if (live && !done) {
      double2 d0 = make_double2(0.0, 0.0), d1 = make_double2(0.0, 0.0);
#pragma unroll
      for (int i = 0; i < R; ++i) {
        if (i & 1) d1 = cfma_conj(s_v[gi][row0 + i], a[i], d1);
        else d0 = cfma_conj(s_v[gi][row0 + i], a[i], d0);
      }
      dot = cadd(d0, d1);
    }
    if constexpr (W > 1) {
      s_partc[w * kWave + lane] = dot;
      __syncthreads();
      dot = make_double2(0.0, 0.0);
#pragma unroll
      for (int ww = 0; ww < W; ++ww) dot = cadd(dot, s_partc[ww * kWave + lane]);
    }
    part = 0.0;
    if (!done) {
      const double den = nup * (nup + s_axj[gi][j & 1]);
      double tau = __builtin_amdgcn_rcp(den);
      tau = __builtin_fma(tau, __builtin_fma(-den, tau, 1.0), tau);
      tau = __builtin_fma(tau, __builtin_fma(-den, tau, 1.0), tau);
      if (live && active && lane != pl) {
        const double2 sdot = make_double2(-tau * dot.x, -tau * dot.y);
        double p0 = 0.0, p1 = 0.0;
#pragma unroll
        for (int i = 0; i < R; ++i) {
          a[i] = cfma(s_v[gi][row0 + i], sdot, a[i]);
          if (i & 1) p1 = __builtin_fma(a[i].y, a[i].y, __builtin_fma(a[i].x, a[i].x, p1));
          else p0 = __builtin_fma(a[i].y, a[i].y, __builtin_fma(a[i].x, a[i].x, p0));
        }
        if (edge) {
          p0 = 0.0;
          p1 = 0.0;
#pragma unroll
          for (int i = 0; i < R; ++i)
            if (row0 + i > j) {
              if (i & 1) p1 = __builtin_fma(a[i].y, a[i].y, __builtin_fma(a[i].x, a[i].x, p1));
              else p0 = __builtin_fma(a[i].y, a[i].y, __builtin_fma(a[i].x, a[i].x, p0));
            }
        }
        part = p0 + p1;
      }
      if (lane == pl) {
        pivoted = true;
        pstep = j;
      }
      if (w == 0 && lane == pl) s_piv[gi][j] = p;
      k = j + 1;
    }
  }
  if (member && k == 0) {
    if (restricted && !zero_block && w == 0 && gl == 0) A.prop_fail[q] = 1;  // no proposed column above eps
    zero_block = true;
  }
  if (zero_block) {
    k = 1;
    pivoted = (gl == 0);
    pstep = 0;
    if (w == 0 && gl == 0) s_piv[gi][0] = 0;
  }
  if (overflow && w == 0 && gl == 0) atomicOr(A.status, kErrRank);
  if (w == 0 && gl == 0) s_k[gi] = member ? k : 0;
  __syncthreads();  // s_piv, s_k complete; every read of the partial sums is done

  const uint64_t msk = (__ballot(pivoted && col < c) >> (gi * GL)) & gmask;  // this ID's skeleton mask
  for (int e = threadIdx.x; e < G * GL; e += nthreads) {
    const int g = e / GL, i = e % GL;
    if (i >= s_k[g]) continue;
    const int pc = s_piv[g][i];
    // skeleton rank of pivot column pc: the pivots of ID g below pc
    int below = 0;
    for (int l = 0; l < s_k[g]; ++l) below += s_piv[g][l] < pc;
    s_srank[g][i] = below;
  }
  if (member && !zero_block) {
    for (int i = gl + GL * w; i < k; i += GL * W) {  // 1 / R_ii of this ID
      const double2 d = s_diag[gi][i];
      const double inv = 1.0 / cabs2(d);
      s_diag[gi][i] = make_double2(d.x * inv, -d.y * inv);
    }
  }
  if (w == 0 && member) {
    if (gl == 0) {
      A.rank[q] = k;
      A.mask[2 * q] = msk;
      A.mask[2 * q + 1] = 0;
    }
    if (pivoted && col < c) A.skel_out[q * kMaxCand + __popcll(msk & lanes_below(col))] = gidx;
  }
  // Back-substitution as in the one-ID kernel: R rows staged with ID g's
  // pivots at slots g GL + l and its redundant candidates at g GL + k_g + jr;
  // wavefront 0 solves, one redundant column per lane.
  int kall = 0;
#pragma unroll
  for (int g = 0; g < G; ++g) kall = max(kall, s_k[g]);
  const int r = c - k;
  const int64_t off = member ? (A.T_off ? A.T_off[q] : q * (int64_t)kSlot) : 0;
  const bool skel = (msk >> col) & 1ull;
  const int below = __popcll(msk & lanes_below(col));
  const int slot = gi * GL + (pivoted ? pstep : k + col - below);
  const bool solver = (w == 0) && member && col < c && !skel;
  const int jr = solver ? col - below : 0;
  const int gb = gi * GL;
  auto t_index = [&](int l) -> int64_t {
    const int sr = s_srank[gi][l];
    return off + (isV ? (int64_t)jr * k + sr : (int64_t)sr * r + jr);
  };
  for (int cb0 = kall > 0 ? ((kall - 1) / kChunk) * kChunk : -1; cb0 >= 0; cb0 -= kChunk) {
    const int ce = min(kall, cb0 + kChunk);
    __syncthreads();  // the previous chunk's LDS reads are done
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int row = row0 + i;
      if (row >= cb0 && row < ce && row < k && col < c)
        s_R[(row - cb0) * kWave + slot] = zero_block ? make_double2(0.0, 0.0) : a[i];
    }
    __syncthreads();
    if (!solver) continue;
    const int cek = min(ce, k);
    for (int ii = cek - 1; ii >= cb0; --ii) {
      const double2* Ri = s_R + (ii - cb0) * kWave + gb;
      double2 acc = Ri[k + jr];
      if (!zero_block) {
        double2 acc1 = make_double2(0.0, 0.0);
        const double2* tcol = s_R + gb + k + jr - cb0 * kWave;  // t_l at tcol[l * 64]
        int l = ii + 1;
        for (; l + 1 < cek; l += 2) {
          const double2 r0 = Ri[l], r1 = Ri[l + 1];
          acc = cfma(make_double2(-r0.x, -r0.y), tcol[l * kWave], acc);
          acc1 = cfma(make_double2(-r1.x, -r1.y), tcol[(l + 1) * kWave], acc1);
        }
        if (l < cek) {
          const double2 r0 = Ri[l];
          acc = cfma(make_double2(-r0.x, -r0.y), tcol[l * kWave], acc);
        }
        for (l = ce; l < k; ++l) {
          const double2 rl = Ri[l];
          acc1 = cfma(make_double2(-rl.x, -rl.y), A.T128[t_index(l)], acc1);
        }
        acc = cmul(cadd(acc, acc1), s_diag[gi][ii]);
      }
      s_R[(ii - cb0) * kWave + gb + k + jr] = acc;
      const int64_t e = t_index(ii);
      A.T128[e] = acc;
      if (A.T64) A.T64[e] = make_float2((float)acc.x, (float)acc.y);
    }
  }
}

// Row reduction of a tall sampled block (s > kQrRows rows, c <= 128
// columns): B = Q0 R0 by unpivoted Householder QR in FP64, keeping the c x c
// upper triangular R0.  Column pivoting picks each pivot by the norms of the
// columns' components orthogonal to the columns already taken; these depend
// on B only through B^H B = R0^H R0.  So the pivoted QR of R0 takes the
// pivots and |R_jj| that the pivoted QR of B takes, its R differs only by row
// phases, and T = R11^{-1} R12 is the same (in exact arithmetic).
// One workgroup per tall ID; the s x c block lives in a global scratch slot
// (column-major, leading dimension s), each wavefront updating whole columns.
constexpr int kTallThreads = 256;

__device__ __forceinline__ double2 wave_sum(double2 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, kWave);
    v.y += __shfl_xor(v.y, off, kWave);
  }
  return v;
}

__global__ __launch_bounds__(kTallThreads) void tall_reduce_kernel(IdArgs A, int64_t slot0) {
  constexpr int NW = kTallThreads / kWave;
  __shared__ double s_coord[kMaxSamples];
  __shared__ double s_cx[kMaxSamples];
  __shared__ double s_ccoord[kMaxCand];
  __shared__ double s_ccx[kMaxCand];
  __shared__ double2 s_v[kMaxSamples];
  __shared__ double s_red[NW];
  __shared__ double s_tau;
  const int64_t slot = slot0 + blockIdx.x;
  if (slot >= A.n_tall) return;
  const int64_t q = A.tall_list[slot];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const int c = A.cand_len[q], cb = A.cand_beg[q], na = A.allow_len[q], ab = A.allow_beg[q];
  const int s = A.samples ? A.samples[q] : min(A.oversample * c, na);
  if (c < 1 || c > kMaxCand || !is_tall(s) || s > kMaxSamples || s > na || s > A.samp_ld ||
      (int64_t)s * c > A.tall_work_ld || (int64_t)c * c > A.tall_ld2) {
    if (tid == 0) {
      A.tall_slot[q] = -1;  // the QR kernel reports it
      atomicOr(A.status, kErrSize);
    }
    return;
  }
  const bool isV = (A.side == IDBF_SIDE_V);
  const bool fio = (A.ph.kind == IDBF_PHASE_FIO);
  const Seg cs_{A.cand_coord ? A.cand_coord + cb : nullptr, isV ? A.Om : A.X, A.cand_idx + cb};
  const Seg as{A.allow_coord ? A.allow_coord + ab : nullptr, isV ? A.X : A.Om, A.allow_idx + ab};
  const int32_t* sp = A.samp_pos + q * A.samp_ld;
  for (int j = tid; j < s; j += kTallThreads) {
    const double v = as(sp[j]);
    s_coord[j] = v;
    s_cx[j] = (isV && fio) ? amplitude_shift(A.ph, v) : 0.0;
  }
  for (int l = tid; l < c; l += kTallThreads) {
    const double v = cs_(l);
    s_ccoord[l] = v;
    s_ccx[l] = (!isV && fio) ? amplitude_shift(A.ph, v) : 0.0;
  }
  __syncthreads();
  double2* W = A.tall_work + (int64_t)blockIdx.x * A.tall_work_ld;
  for (int e = tid; e < s * c; e += kTallThreads) {
    const int i = e % s, l = e / s;
    W[(int64_t)l * s + i] = isV ? kernel_entry(A.ph, s_coord[i], s_cx[i], s_ccoord[l])
                                : kernel_entry(A.ph, s_ccoord[l], s_ccx[l], s_coord[i]);
  }
  __syncthreads();
  for (int j = 0; j < c; ++j) {
    // column j below the diagonal, its norm and the Householder vector
    double p = 0.0;
    for (int i = j + tid; i < s; i += kTallThreads) {
      const double2 v = W[(int64_t)j * s + i];
      s_v[i] = v;
      p = __builtin_fma(v.y, v.y, __builtin_fma(v.x, v.x, p));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) p += __shfl_xor(p, off, kWave);
    if (lane == 0) s_red[w] = p;
    __syncthreads();
    if (tid == 0) {
      double nu2 = 0.0;
#pragma unroll
      for (int k = 0; k < NW; ++k) nu2 += s_red[k];
      const double nu = sqrt(nu2);
      double tau = 0.0;
      if (nu > 0.0) {
        const double2 xj = s_v[j];
        const double axj = sqrt(cabs2(xj));
        double2 alpha, vj;
        if (axj > 0.0) {
          const double g = nu / axj;  // alpha = -g x_j, v_j = (1 + g) x_j
          alpha = make_double2(-xj.x * g, -xj.y * g);
          vj = make_double2(xj.x + xj.x * g, xj.y + xj.y * g);
        } else {
          alpha = make_double2(-nu, 0.0);
          vj = make_double2(nu, 0.0);
        }
        s_v[j] = vj;
        W[(int64_t)j * s + j] = alpha;
        tau = 1.0 / (nu * (nu + axj));  // 2 / |v|^2
      }
      s_tau = tau;
    }
    __syncthreads();
    const double tau = s_tau;
    if (tau != 0.0) {
      for (int l = j + 1 + w; l < c; l += NW) {
        double2* col = W + (int64_t)l * s;
        double2 d = make_double2(0.0, 0.0);
        for (int i = j + lane; i < s; i += kWave) d = cfma_conj(s_v[i], col[i], d);
        d = wave_sum(d);
        const double2 f = make_double2(-tau * d.x, -tau * d.y);
        for (int i = j + lane; i < s; i += kWave) col[i] = cfma(s_v[i], f, col[i]);
      }
    }
    __syncthreads();  // the columns are updated before the next step reads them
  }
  double2* Rt = A.tall_R + slot * A.tall_ld2;
  for (int e = tid; e < c * c; e += kTallThreads) {
    const int i = e % c, l = e / c;
    Rt[e] = i <= l ? W[(int64_t)l * s + i] : make_double2(0.0, 0.0);
  }
  if (tid == 0) A.tall_slot[q] = (int32_t)slot;
}

}  // namespace

hipError_t launch_qr_bucket(const IdArgs& a, int64_t n, int bucket, hipStream_t st);

namespace {
std::atomic<uint32_t> g_qr_shapes{0};  // bit b: bucket 4 + b runs on its short wavefronts
}

uint32_t qr_shape_mask() { return g_qr_shapes.load(std::memory_order_relaxed); }
void set_qr_shape_mask(uint32_t mask) { g_qr_shapes.store(mask & kQrShapeBits, std::memory_order_relaxed); }

hipError_t launch_select(const IdArgs& a, hipStream_t st) {
  const int64_t n = a.sel_list ? a.sel_n : a.n_ids;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(select_kernel, dim3((unsigned)((n + kSelIds - 1) / kSelIds)), dim3(64 * kSelIds), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_id_batch(const IdArgs& a, hipStream_t st) {
  hipError_t e = launch_select(a, st);
  if (e != hipSuccess) return e;
  return launch_qr(a, st);
}

hipError_t launch_qr(const IdArgs& a, hipStream_t st) {
  if (a.n_ids <= 0) return hipSuccess;
  if (a.n_tall > 0) {  // reduced blocks of the tall IDs first, tall_chunk per launch (scratch slots)
    if (!a.tall_list || !a.tall_slot || !a.tall_R || !a.tall_work || a.tall_chunk < 1) return hipErrorInvalidValue;
    for (int64_t b0 = 0; b0 < a.n_tall; b0 += a.tall_chunk) {
      const int64_t n = std::min<int64_t>(a.tall_chunk, a.n_tall - b0);
      hipLaunchKernelGGL(tall_reduce_kernel, dim3((unsigned)n), dim3(kTallThreads), 0, st, a, b0);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  if (!a.order) {
    int bk = qr_bucket(a.c_max, a.rows_max);
    if (a.n_tall > 0 && bk >= kFirstPackedBucket) bk = (a.rows_max + 15) / 16 - 1;  // tall IDs: one-ID kernels
    return launch_qr_bucket(a, a.n_ids, bk, st);
  }
  // one launch per bucket of IDs that need the same kernel variant
  IdArgs b = a;
  for (int bk = 0; bk < kQrBuckets; ++bk) {
    const int64_t cnt = a.bucket_off[bk + 1] - a.bucket_off[bk];
    if (cnt <= 0) continue;
    b.order = a.order + a.bucket_off[bk];
    hipError_t e = launch_qr_bucket(b, cnt, bk, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int W, int CPL, int R>
hipError_t launch_one(const IdArgs& a, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((id_kernel<W, CPL, R>), dim3((unsigned)n), dim3(64 * W), 0, st, a);
  return hipGetLastError();
}

template <int W, int G>
hipError_t launch_packed(const IdArgs& a, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((id_kernel_g<W, G>), dim3((unsigned)((n + G - 1) / G)), dim3(64 * W), 0, st, a, n);
  return hipGetLastError();
}

hipError_t launch_qr_bucket(const IdArgs& a, int64_t n, int bucket, hipStream_t st) {
  const uint32_t shapes = qr_shape_mask();
  switch (bucket) {
    // up to 64 candidates: 16 rows per wavefront up to 64 samples, then four
    // wavefronts of 20, 24 or 28 rows up to 112 (or, with the bucket's bit of
    // the shape mask set, five or eight short ones)
    case 0: return launch_one<1, 1, 16>(a, n, st);
    case 1: return launch_one<2, 1, 16>(a, n, st);
    case 2: return launch_one<3, 1, 16>(a, n, st);
    case 3: return launch_one<4, 1, 16>(a, n, st);
    case 4: return (shapes & 1u) ? launch_one<5, 1, 16>(a, n, st) : launch_one<4, 1, 20>(a, n, st);
    case 5: return (shapes & 2u) ? launch_one<8, 1, 12>(a, n, st) : launch_one<4, 1, 24>(a, n, st);
    case 6: return (shapes & 4u) ? launch_one<8, 1, 14>(a, n, st) : launch_one<4, 1, 28>(a, n, st);
    case 7: return launch_one<8, 1, 16>(a, n, st);
    // 65..128 candidates: two per lane, 8 rows per wavefront
    case 8: return launch_one<1, 2, 8>(a, n, st);
    case 9: return launch_one<2, 2, 8>(a, n, st);
    case 10: return launch_one<3, 2, 8>(a, n, st);
    case 11: return launch_one<4, 2, 8>(a, n, st);
    case 12: return launch_one<5, 2, 8>(a, n, st);
    case 13: return launch_one<6, 2, 8>(a, n, st);
    case 14: return launch_one<7, 2, 8>(a, n, st);
    case 15: return launch_one<8, 2, 8>(a, n, st);
    case 16: return launch_one<9, 2, 8>(a, n, st);
    case 17: return launch_one<10, 2, 8>(a, n, st);
    case 18: return launch_one<11, 2, 8>(a, n, st);
    case 19: return launch_one<12, 2, 8>(a, n, st);
    case 20: return launch_one<13, 2, 8>(a, n, st);
    case 21: return launch_one<14, 2, 8>(a, n, st);
    case 22: return launch_one<15, 2, 8>(a, n, st);
    case 23: return launch_one<16, 2, 8>(a, n, st);
    // two IDs per workgroup: up to 32 candidates and 64 samples
    case 24: return launch_packed<1, 2>(a, n, st);
    case 25: return launch_packed<2, 2>(a, n, st);
    case 26: return launch_packed<3, 2>(a, n, st);
    case 27: return launch_packed<4, 2>(a, n, st);
    // four IDs per workgroup: up to 16 candidates and 32 samples
    case 28: return launch_packed<1, 4>(a, n, st);
    default: return launch_packed<2, 4>(a, n, st);
  }
}

}  // namespace idbf
