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
//   [16 w, 16 w + 16) of every column in registers, so the Householder sweep,
//   column norms and dot products are lane-local.  Per step: residual norms
//   are recomputed; M = max (DPP reduction); stop when M <= eps |R_00|; the
//   pivot is the smallest candidate index with norm >= (1 - 1e-8) M (ballot);
//   the pivot column's Householder vector goes through LDS.  Then
//   T = R11^{-1} R12 by back-substitution in registers, one redundant
//   candidate per lane, rows permuted to ascending skeletons.
#include <algorithm>

#include "kernels.hpp"

namespace idbf {

namespace {

constexpr int kRPW = 16;    // sampled rows per wavefront in the QR kernel
constexpr int kSelIds = 4;  // IDs (wavefronts) per selection workgroup

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

// Sequential rule: for targets in order, the nearest unused point; then sort.
__device__ void greedy_select(const Seg& a, int n, int s, double lo, double hi, int* pos) {
  for (int j = 0; j < s; ++j) {
    const double z = lo + (hi - lo) * cheb_fraction(j, s);
    const int p0 = nearest_pos(a, n, z);
    auto used = [&](int p) {
      for (int t = 0; t < j; ++t)
        if (pos[t] == p) return true;
      return false;
    };
    int pick = p0;
    if (used(p0)) {
      int l = p0 - 1;
      while (l >= 0 && used(l)) --l;
      int r = p0 + 1;
      while (r < n && used(r)) ++r;
      if (l < 0) {
        pick = r;
      } else if (r >= n) {
        pick = l;
      } else {
        pick = (__builtin_fabs(a(l) - z) <= __builtin_fabs(a(r) - z)) ? l : r;
      }
    }
    pos[j] = pick;
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

// One wavefront per ID; waves never synchronize with each other.
__global__ __launch_bounds__(64 * kSelIds) void select_kernel(IdArgs A) {
  __shared__ int s_pos[kSelIds][kMaxSamples];
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int64_t q = blockIdx.x * (int64_t)kSelIds + w;
  if (q >= A.n_ids) return;
  const int c = A.cand_len[q], na = A.allow_len[q];
  const int s = min(A.oversample * c, na);
  if (c < 1 || c > kMaxCand || na < 1 || s > kMaxSamples) return;  // id_kernel reports it
  int32_t* out = A.samp_pos + q * (int64_t)kMaxSamples;
  if (s >= na) {
    for (int j = lane; j < na; j += kWave) out[j] = j;
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
    if (j < s) p = nearest_pos(a, na, lo + (hi - lo) * cheb_fraction(j, s));
    const int left = __shfl_up(p, 1, kWave);
    const int before = (lane == 0) ? prev_last : left;
    if (j < s && j > 0 && p == before) coll = 1;
    prev_last = __shfl(p, kWave - 1, kWave);
    if (j < s) s_pos[w][j] = p;
  }
  if (__ballot(coll)) {
    wave_lds_sync();
    if (lane == 0) greedy_select(a, na, s, lo, hi, s_pos[w]);
  }
  wave_lds_sync();
  for (int j = lane; j < s; j += kWave) out[j] = s_pos[w][j];
}

// DPP max over the 64 lanes of a wavefront: row_shr within rows of 16, then
// row broadcasts; lane 63 ends with the maximum.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int l2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWMASK, 0xf, false);
  const int h2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWMASK, 0xf, false);
  return __hiloint2double(h2, l2);
}
__device__ __forceinline__ double wave_max_dpp(double v) {
  v = fmax(v, dpp_d<0x111, 0xf>(v));  // row_shr:1
  v = fmax(v, dpp_d<0x112, 0xf>(v));  // row_shr:2
  v = fmax(v, dpp_d<0x114, 0xf>(v));  // row_shr:4
  v = fmax(v, dpp_d<0x118, 0xf>(v));  // row_shr:8
  v = fmax(v, dpp_d<0x142, 0xa>(v));  // row_bcast:15
  v = fmax(v, dpp_d<0x143, 0xc>(v));  // row_bcast:31
  return readlane(v, kWave - 1);
}

template <int W>
__global__ __launch_bounds__(64 * W) void id_kernel(IdArgs A) {
  constexpr int R = kRPW;
  constexpr int SMAX = R * W;
  __shared__ double s_part[W > 1 ? W : 1][kWave];
  __shared__ double2 s_partc[W > 1 ? W : 1][kWave];
  __shared__ double s_coord[SMAX];
  __shared__ double s_cx[SMAX];
  __shared__ double2 s_v[SMAX];
  __shared__ double2 s_col[2][kMaxRank];  // back-substitution: a column of R11
  __shared__ double2 s_t[2][kWave];       // back-substitution: one row of T
  __shared__ int s_piv[kMaxRank];
  __shared__ int s_srank[kMaxRank];
  __shared__ double2 s_alpha;
  __shared__ double s_tau;

  const int64_t q = blockIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int nthreads = kWave * W;
  const int cb = A.cand_beg[q], c = A.cand_len[q];
  const int ab = A.allow_beg[q], na = A.allow_len[q];
  const int s = min(A.oversample * c, na);
  if (c < 1 || c > kMaxCand || na < 1 || s > SMAX) {
    if (threadIdx.x == 0) atomicOr(A.status, kErrSize);
    return;
  }
  const bool isV = (A.side == IDBF_SIDE_V);
  const bool fio = (A.ph.kind == IDBF_PHASE_FIO);
  const Seg cs{A.cand_coord ? A.cand_coord + cb : nullptr, isV ? A.Om : A.X, A.cand_idx + cb};
  const Seg as{A.allow_coord ? A.allow_coord + ab : nullptr, isV ? A.X : A.Om, A.allow_idx + ab};

  int gidx = 0;
  double ccoord = 0.0, ccx = 0.0;
  if (lane < c) {
    gidx = A.cand_idx[cb + lane];
    ccoord = cs(lane);
    if (!isV && fio) ccx = amplitude_shift(A.ph, ccoord);
  }
  const int32_t* sp = A.samp_pos + q * (int64_t)kMaxSamples;
  for (int j = threadIdx.x; j < s; j += nthreads) {
    const double v = as(sp[j]);
    s_coord[j] = v;
    s_cx[j] = (isV && fio) ? amplitude_shift(A.ph, v) : 0.0;
  }
  __syncthreads();

  // sampled block: rows [R w, R w + R) of column `lane`
  const int row0 = w * R;
  const bool wave_has_rows = row0 < s;
  double2 a[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int row = row0 + i;
    double2 v = make_double2(0.0, 0.0);
    if (lane < c && row < s)
      v = isV ? kernel_entry(A.ph, s_coord[row], s_cx[row], ccoord)
              : kernel_entry(A.ph, ccoord, ccx, s_coord[row]);
    a[i] = v;
  }

  const int kuser = min(min(s, c), A.kmax > 0 ? A.kmax : (1 << 30));
  bool pivoted = false;
  double r00 = 0.0;
  int k = 0;
  bool zero_block = false, overflow = false;
  for (int j = 0;; ++j) {
    double part = 0.0;
    if (wave_has_rows) {
#pragma unroll
      for (int i = 0; i < R; ++i)
        if (row0 + i >= j) part += cabs2(a[i]);
    }
    double nrm2 = part;
    if constexpr (W > 1) {
      s_part[w][lane] = part;
      __syncthreads();
      nrm2 = 0.0;
#pragma unroll
      for (int ww = 0; ww < W; ++ww) nrm2 += s_part[ww][lane];
    }
    const bool eligible = (lane < c) && !pivoted;
    const double nu = eligible ? sqrt(nrm2) : -1.0;
    const double M = wave_max_dpp(nu);
    if (j == 0) {
      r00 = M;
      if (M == 0.0) {
        zero_block = true;
        break;
      }
    } else if (M <= A.tol * r00) {
      break;
    }
    if (j == kuser) break;
    if (j == kMaxRank) {
      overflow = true;
      break;
    }
    const uint64_t near = __ballot(eligible && nu >= (1.0 - kPivotTie) * M);
    if (near == 0) break;  // no finite residual norm left (cannot happen for finite input)
    const int p = __builtin_amdgcn_readfirstlane(__ffsll((unsigned long long)near) - 1);
    if (lane == p) {
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int row = row0 + i;
        if (row > j && row < s) s_v[row] = a[i];
        if (row == j) {
          const double2 xj = a[i];
          const double axj = sqrt(cabs2(xj));
          double2 alpha, vj;
          if (axj > 0.0) {
            alpha = make_double2(-xj.x / axj * nu, -xj.y / axj * nu);
            const double sc = (axj + nu) / axj;
            vj = make_double2(xj.x * sc, xj.y * sc);
          } else {
            alpha = make_double2(-nu, 0.0);
            vj = make_double2(nu, 0.0);
          }
          s_v[row] = vj;
          s_alpha = alpha;
          s_tau = 1.0 / (nu * (nu + axj));
        }
      }
      if (w == 0) s_piv[j] = p;
    }
    __syncthreads();
    const double tau = s_tau;
    double2 dot = make_double2(0.0, 0.0);
    if (wave_has_rows) {
#pragma unroll
      for (int i = 0; i < R; ++i)
        if (row0 + i >= j && row0 + i < s) dot = cfma_conj(s_v[row0 + i], a[i], dot);
    }
    if constexpr (W > 1) {
      s_partc[w][lane] = dot;
      __syncthreads();
      dot = make_double2(0.0, 0.0);
#pragma unroll
      for (int ww = 0; ww < W; ++ww) dot = cadd(dot, s_partc[ww][lane]);
    }
    if (lane == p) {
      const double2 alpha = s_alpha;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int row = row0 + i;
        if (row == j) a[i] = alpha;
        if (row > j) a[i] = make_double2(0.0, 0.0);
      }
      pivoted = true;
    } else if (eligible && wave_has_rows) {
      const double2 sdot = make_double2(-tau * dot.x, -tau * dot.y);
#pragma unroll
      for (int i = 0; i < R; ++i)
        if (row0 + i >= j && row0 + i < s) a[i] = cfma(s_v[row0 + i], sdot, a[i]);
    }
    k = j + 1;
    if constexpr (W == 1) __syncthreads();
  }
  if (k == 0) zero_block = true;  // no pivot taken: keep the first candidate, T = 0
  if (zero_block) {
    k = 1;
    pivoted = (lane == 0);
    if (threadIdx.x == 0) s_piv[0] = 0;
  }
  if (overflow && threadIdx.x == 0) atomicOr(A.status, kErrRank);
  __syncthreads();
  const uint64_t msk = __ballot(pivoted && lane < c);
  if (threadIdx.x < k) s_srank[threadIdx.x] = __popcll(msk & lanes_below(s_piv[threadIdx.x]));
  __syncthreads();

  const int below = __popcll(msk & lanes_below(lane));
  const int r = c - k;
  const bool redundant = (lane < c) && !pivoted;
  if (w == 0) {
    if (lane == 0) {
      A.rank[q] = k;
      A.mask[q] = msk;
    }
    if (pivoted && lane < c) A.skel_out[q * kMaxCand + below] = gidx;
  }
  // Back-substitution T = R11^{-1} R12, one redundant candidate per lane, rows
  // from the last up: t_ii = r_ii / R[ii][piv_ii], then r_i -= R[i][piv_ii] t_ii
  // for i < ii.  Column piv_ii of R11 and the row t_ii go through double-buffered
  // LDS slots, so each step needs two barriers.
  const int jr = lane - below;
  const int64_t off = A.T_off ? A.T_off[q] : q * (int64_t)kSlot;
  for (int ii = k - 1; ii >= 0; --ii) {
    const int buf = ii & 1;
    const int pp = s_piv[ii];
    if (lane == pp) {
#pragma unroll
      for (int i = 0; i < R; ++i)
        if (row0 + i <= ii) s_col[buf][row0 + i] = a[i];
    }
    __syncthreads();
    if (redundant && row0 <= ii && ii < row0 + R) {
      double2 t = make_double2(0.0, 0.0);
      if (!zero_block) {
        const double2 d = s_col[buf][ii];
        const double inv = 1.0 / cabs2(d);
#pragma unroll
        for (int i = 0; i < R; ++i)
          if (row0 + i == ii) t = cmul(a[i], make_double2(d.x * inv, -d.y * inv));
      }
      s_t[buf][lane] = t;
      const int sr = s_srank[ii];
      const int64_t e = off + (isV ? (int64_t)jr * k + sr : (int64_t)sr * r + jr);
      A.T128[e] = t;
      if (A.T64) A.T64[e] = make_float2((float)t.x, (float)t.y);
    }
    __syncthreads();
    if (redundant && row0 < ii) {
      const double2 t = s_t[buf][lane];
      const double2 mt = make_double2(-t.x, -t.y);
#pragma unroll
      for (int i = 0; i < R; ++i)
        if (row0 + i < ii) a[i] = cfma(s_col[buf][row0 + i], mt, a[i]);
    }
  }
}

}  // namespace

int id_batch_waves(int s_max) { return std::max(1, std::min(kMaxSamples / kRPW, (s_max + kRPW - 1) / kRPW)); }

hipError_t launch_select(const IdArgs& a, hipStream_t st) {
  if (a.n_ids <= 0) return hipSuccess;
  hipLaunchKernelGGL(select_kernel, dim3((unsigned)((a.n_ids + kSelIds - 1) / kSelIds)), dim3(64 * kSelIds), 0,
                     st, a);
  return hipGetLastError();
}

hipError_t launch_id_batch(const IdArgs& a, hipStream_t st) {
  hipError_t e = launch_select(a, st);
  if (e != hipSuccess) return e;
  return launch_qr(a, st);
}

hipError_t launch_qr(const IdArgs& a, hipStream_t st) {
  if (a.n_ids <= 0) return hipSuccess;
  const dim3 grid((unsigned)a.n_ids);
  switch (id_batch_waves(a.s_max)) {
    case 1: hipLaunchKernelGGL(id_kernel<1>, grid, dim3(64), 0, st, a); break;
    case 2: hipLaunchKernelGGL(id_kernel<2>, grid, dim3(128), 0, st, a); break;
    case 3: hipLaunchKernelGGL(id_kernel<3>, grid, dim3(192), 0, st, a); break;
    case 4: hipLaunchKernelGGL(id_kernel<4>, grid, dim3(256), 0, st, a); break;
    case 5: hipLaunchKernelGGL(id_kernel<5>, grid, dim3(320), 0, st, a); break;
    case 6: hipLaunchKernelGGL(id_kernel<6>, grid, dim3(384), 0, st, a); break;
    case 7: hipLaunchKernelGGL(id_kernel<7>, grid, dim3(448), 0, st, a); break;
    default: hipLaunchKernelGGL(id_kernel<8>, grid, dim3(512), 0, st, a); break;
  }
  return hipGetLastError();
}

}  // namespace idbf
