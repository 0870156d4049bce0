// Learned proposal for the construction (not in the paper).  Per level
// batch: features of every ID -> the rank network's estimate k^ ->
// proposed sample counts s' = min(s, t (ceil k^ + margin)); optionally a
// second network scores every candidate of every ID and the k_f best become
// the ID's proposed skeleton, which the QR takes as its pivots in that order
// (no pivot search, no eps-rank stop).  The IDs are computed from s' samples,
// then a randomized residual test on r = 8 fresh allowed points accepts or
// rejects each one,
//   || A(r, red) - A(r, skel) T ||_F <= 10 eps || A(r, cand) ||_F,
// and rejected IDs are recomputed by the plain pivoted ID from the plain s
// samples (a rank-only proposal that kept s' = s is the plain ID and is
// accepted as it is).
#include <algorithm>

#include "kernels.hpp"

namespace idbf {

namespace {

// Features of ID q = partner * nn + node of level t (side 0: U, 1: V), with
// the row node's centre x_c and the column node's centre xi_c (both scaled to
// [0, 1)), whichever of the two the ID compresses:
//   t / 8, side, x_c, xi_c, a, m / 4, FIO?, a m |cos 2 pi m x_c| / 4
// (the last: the local rate of change of c(x), which drives the rank).
__global__ void features_kernel(int64_t n, int L, int t, int side, PhaseDev ph, float* F) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int64_t nn = 1ll << (L - t + 1);
  const int64_t node = q % nn, partner = q / nn;
  const double cn = ((double)node + 0.5) / (double)nn;
  const double cp = ((double)partner + 0.5) / (double)(1ll << t);
  const double xc = side == 0 ? cn : cp, xic = side == 0 ? cp : cn;
  const bool fio = ph.kind == IDBF_PHASE_FIO;
  float* f = F + q * kProposalInputs;
  f[0] = (float)t / 8.f;
  f[1] = (float)side;
  f[2] = (float)xc;
  f[3] = (float)xic;
  f[4] = fio ? (float)ph.a : 0.f;
  f[5] = fio ? (float)(ph.freq / 4.0) : 0.f;
  f[6] = fio ? 1.f : 0.f;
  f[7] = fio ? (float)(ph.a * ph.freq * fabs(cospi(2.0 * ph.freq * xc)) / 4.0) : 0.f;
}

__global__ void propose_kernel(const float* y, const int32_t* samples, int64_t n, int oversample, int margin,
                               int32_t* s_prop) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float kh = fminf(fmaxf(ceilf(y[q] * kProposalScale), 1.f), (float)kMaxRank);
  const int64_t s = (int64_t)oversample * ((int64_t)kh + margin);
  s_prop[q] = (int32_t)max((int64_t)1, min((int64_t)samples[q], s));
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double coord_of(const double* direct, const double* base, const int32_t* idx, int64_t p) {
  return direct ? direct[p] : base[idx[p]];
}

constexpr int kCheckRows = 8;
constexpr int kWavesRC = 4;

// One wavefront per ID; lanes own candidates lane and lane + 64.
__global__ __launch_bounds__(64 * kWavesRC) void residual_kernel(ResidualArgs R) {
  __shared__ double2 s_S[kWavesRC][kCheckRows][kMaxRank];
  const IdArgs& A = R.id;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x & (kWave - 1);
  const int64_t q = blockIdx.x * (int64_t)kWavesRC + w;
  if (q >= A.n_ids) return;
  const bool isV = (A.side == IDBF_SIDE_V);
  const bool fio = (A.ph.kind == IDBF_PHASE_FIO);
  const int c = A.cand_len[q], cb = A.cand_beg[q], na = A.allow_len[q], ab = A.allow_beg[q];
  const int k = A.rank[q], r = c - k;
  const uint64_t m0 = A.mask[2 * q], m1 = A.mask[2 * q + 1];
  const int64_t off = A.T_off[q];
  // check points: the high 32 bits of SplitMix64 of (seed, level, side, q, i), scaled to [0, na)
  const uint64_t base = ((R.seed & 0xffffffffull) << 32) ^ ((uint64_t)R.level << 24) ^ ((uint64_t)A.side << 23) ^
                        (uint64_t)q;
  double pc[kCheckRows], pcx[kCheckRows];
#pragma unroll
  for (int i = 0; i < kCheckRows; ++i) {
    const uint64_t z = splitmix64(base * 16ull + (uint64_t)i);
    const int64_t pos = (int64_t)(((z >> 32) * (uint64_t)na) >> 32);
    pc[i] = coord_of(A.allow_coord ? A.allow_coord + ab : nullptr, isV ? A.X : A.Om, A.allow_idx + ab, pos);
    pcx[i] = (isV && fio) ? amplitude_shift(A.ph, pc[i]) : 0.0;
  }
  double2 a[2][kCheckRows];
  bool red[2];
  int idx[2];
  double na2 = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int l = lane + kWave * h;
    red[h] = false;
    idx[h] = 0;
    if (l < c) {
      const double cc = coord_of(A.cand_coord ? A.cand_coord + cb : nullptr, isV ? A.Om : A.X, A.cand_idx + cb, l);
      const double ccx = (!isV && fio) ? amplitude_shift(A.ph, cc) : 0.0;
      const bool sk = l < 64 ? ((m0 >> l) & 1ull) : ((m1 >> (l - 64)) & 1ull);
      const int below = l < 64 ? __popcll(m0 & lanes_below(l)) : __popcll(m0) + __popcll(m1 & lanes_below(l - 64));
      red[h] = !sk;
      idx[h] = sk ? below : l - below;
#pragma unroll
      for (int i = 0; i < kCheckRows; ++i) {
        a[h][i] = isV ? kernel_entry(A.ph, pc[i], pcx[i], cc) : kernel_entry(A.ph, cc, ccx, pc[i]);
        na2 += cabs2(a[h][i]);
        if (sk) s_S[w][i][below] = a[h][i];
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  double e2 = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (!red[h]) continue;
    const int j = idx[h];
#pragma unroll
    for (int i = 0; i < kCheckRows; ++i) {
      double2 e = a[h][i];
      for (int b = 0; b < k; ++b) {
        const double2 t = A.T128[off + (isV ? (int64_t)j * k + b : (int64_t)b * r + j)];
        const double2 s = s_S[w][i][b];
        e = cfma(make_double2(-s.x, -s.y), t, e);
      }
      e2 += cabs2(e);
    }
  }
  for (int d = 32; d > 0; d >>= 1) {
    e2 += __shfl_xor(e2, d, kWave);
    na2 += __shfl_xor(na2, d, kWave);
  }
  if (lane == 0) {
    const double bound = R.factor * A.tol;
    // a rank proposal that kept the plain sample count is the plain ID itself
    // (a skeleton proposal is not: it is always tested)
    const bool same = !R.skeletons && R.s_prop[q] == R.samples_plain[q];
    // a skeleton proposal none of whose columns the QR could keep is unusable
    const bool kept = !R.skeletons || R.reject[q] == 0;
    const bool ok = !R.force_reject && kept && (same || e2 <= bound * bound * na2);
    R.reject[q] = ok ? 0 : 1;
    if (!ok) R.s_prop[q] = R.samples_plain[q];  // the fallback samples the plain count
  }
}

// Candidate features, one thread per (ID, candidate position).
__global__ void cand_features_kernel(int64_t n, int L, int t, int side, PhaseDev ph, const int32_t* cand_beg,
                                     const int32_t* cand_len, const double* cand_coord, int cmax, float* F) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * cmax) return;
  const int64_t q = e / cmax;
  const int l = (int)(e % cmax);
  float* f = F + e * kProposalInputs;
  const int c = cand_len[q];
  if (l >= c) {
#pragma unroll
    for (int i = 0; i < kProposalInputs; ++i) f[i] = 0.f;
    return;
  }
  const int64_t nn = 1ll << (L - t + 1);
  const int64_t node = q % nn, partner = q / nn;
  const double cn = ((double)node + 0.5) / (double)nn;
  const double cp = ((double)partner + 0.5) / (double)(1ll << t);
  const bool fio = ph.kind == IDBF_PHASE_FIO;
  const double* cc = cand_coord + cand_beg[q];
  const double lo = cc[0], hi = cc[c - 1];
  f[0] = (float)t / 8.f;
  f[1] = (float)side;
  f[2] = (float)(side == 0 ? cn : cp);
  f[3] = (float)(side == 0 ? cp : cn);
  f[4] = fio ? (float)ph.a : 0.f;
  f[5] = fio ? (float)(ph.freq / 4.0) : 0.f;
  f[6] = (float)l / (float)c;
  f[7] = c > 1 && hi > lo ? (float)((cc[l] - lo) / (hi - lo)) : 0.5f;
}

// One wavefront per ID: each candidate's place in the descending score order
// (ties to the lower position) by counting; the first k_f are the pivots.
__global__ __launch_bounds__(256) void pick_skeletons_kernel(const float* score, int cmax, const float* y_rank,
                                                             const int32_t* s_prop, const int32_t* cand_len,
                                                             int64_t n, int margin, int32_t* prop_k,
                                                             uint8_t* prop_cols) {
  const int64_t q = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (q >= n) return;
  const int c = cand_len[q];
  const float kh = fminf(fmaxf(ceilf(y_rank[q] * kProposalScale), 1.f), (float)kMaxRank);
  // the proposed set: room for the proposed rank and twice the margin (the
  // restricted pivot search chooses within it)
  const int kf = max(1, min(c, min(kMaxRank, (int)kh + 2 * margin)));
  if (lane == 0) prop_k[q] = kf;
  const float* sc = score + q * cmax;
  for (int l = lane; l < c; l += kWave) {
    const float v = sc[l];
    int place = 0;
    for (int m = 0; m < c; ++m) {
      const float w = sc[m];
      place += (w > v) || (w == v && m < l);
    }
    if (place < kf) prop_cols[q * kMaxRank + place] = (uint8_t)l;
  }
}

__global__ void skel_targets_kernel(const uint64_t* mask, const int32_t* cand_len, int64_t n, int cmax, float* out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * cmax) return;
  const int64_t q = e / cmax;
  const int l = (int)(e % cmax);
  if (l >= cand_len[q]) {
    out[e] = -1.f;
    return;
  }
  const uint64_t w = l < 64 ? mask[2 * q] : mask[2 * q + 1];
  out[e] = (float)((w >> (l & 63)) & 1ull);
}

__global__ __launch_bounds__(256) void rank_hist_kernel(const int32_t* rank, int64_t n, unsigned long long* hist) {
  __shared__ unsigned int s_h[kMaxRank + 1];
  for (int i = threadIdx.x; i <= kMaxRank; i += blockDim.x) s_h[i] = 0;
  __syncthreads();
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
    const int r = rank[q];
    if (r >= 0 && r <= kMaxRank) atomicAdd(&s_h[r], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= kMaxRank; i += blockDim.x)
    if (s_h[i]) atomicAdd(hist + i, (unsigned long long)s_h[i]);
}

__global__ void targets_kernel(const int32_t* rank, int64_t n, float* out) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q < n) out[q] = (float)rank[q] / kProposalScale;
}

inline unsigned blocks(int64_t n, int per = 256) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_rank_targets(const int32_t* rank, int64_t n, float* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(targets_kernel, dim3(blocks(n)), dim3(256), 0, st, rank, n, out);
  return hipGetLastError();
}

hipError_t launch_cand_features(int64_t n, int L, int t, int side, const PhaseDev& ph, const int32_t* cand_beg,
                                const int32_t* cand_len, const double* cand_coord, int cmax, float* F,
                                hipStream_t st) {
  if (n <= 0 || cmax <= 0) return hipSuccess;
  hipLaunchKernelGGL(cand_features_kernel, dim3(blocks(n * cmax)), dim3(256), 0, st, n, L, t, side, ph, cand_beg,
                     cand_len, cand_coord, cmax, F);
  return hipGetLastError();
}

hipError_t launch_pick_skeletons(const float* score, int cmax, const float* y_rank, const int32_t* s_prop,
                                 const int32_t* cand_len, int64_t n, int margin, int32_t* prop_k,
                                 uint8_t* prop_cols, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(pick_skeletons_kernel, dim3(blocks(n, 4)), dim3(256), 0, st, score, cmax, y_rank, s_prop,
                     cand_len, n, margin, prop_k, prop_cols);
  return hipGetLastError();
}

hipError_t launch_skel_targets(const uint64_t* mask, const int32_t* cand_len, int64_t n, int cmax, float* out,
                               hipStream_t st) {
  if (n <= 0 || cmax <= 0) return hipSuccess;
  hipLaunchKernelGGL(skel_targets_kernel, dim3(blocks(n * cmax)), dim3(256), 0, st, mask, cand_len, n, cmax, out);
  return hipGetLastError();
}

hipError_t launch_rank_hist(const int32_t* rank, int64_t n, unsigned long long* hist, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(rank_hist_kernel, dim3(std::min<unsigned>(blocks(n), 256u)), dim3(256), 0, st, rank, n, hist);
  return hipGetLastError();
}

hipError_t launch_features(int64_t n, int L, int t, int side, const PhaseDev& ph, float* F, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(features_kernel, dim3(blocks(n)), dim3(256), 0, st, n, L, t, side, ph, F);
  return hipGetLastError();
}

hipError_t launch_propose(const float* y, const int32_t* samples, int64_t n, int oversample, int margin,
                          int32_t* s_prop, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(propose_kernel, dim3(blocks(n)), dim3(256), 0, st, y, samples, n, oversample, margin, s_prop);
  return hipGetLastError();
}

hipError_t launch_residual(const ResidualArgs& a, hipStream_t st) {
  if (a.id.n_ids <= 0) return hipSuccess;
  hipLaunchKernelGGL(residual_kernel, dim3(blocks(a.id.n_ids, kWavesRC)), dim3(64 * kWavesRC), 0, st, a);
  return hipGetLastError();
}

}  // namespace idbf
