// Batched linear-scaling interpolative decomposition (Section 2.1, Lemma 2.1,
// eqs. pivotedQR2, acc, R2) on gfx950, in FP64.
//
// One ID per workgroup of W wavefronts.  Lane l owns candidate l (a column of
// the sampled matrix B = K(samples, cand) for a column ID, or of
// B = K(cand, samples)^T for a row ID); wave w holds sampled rows
// [32 w, 32 w + 32) of every column in registers, so the Householder sweep,
// column norms and dot products are lane-local and only the per-step pivot
// vector goes through LDS.  Steps of the sweep:
//   1. Mock-Chebyshev selection of s = min(t c, |allowed|) allowed points
//      (targets in parallel; a sequential "nearest unused" pass only when two
//      targets share a nearest point).
//   2. Entry sampling in FP64 with exact phase reduction.
//   3. Column-pivoted Householder QR stopped at the eps-rank: before step j,
//      residual norms are recomputed, M = max; stop when M <= eps |R_00|; the
//      pivot is the smallest candidate index with norm >= (1 - 1e-8) M.
//   4. T = R11^{-1} R12 by back-substitution (wave 0; R11 entries read from
//      the pivot lanes' registers), rows permuted to ascending skeletons.
#include "kernels.hpp"

namespace idbf {

namespace {

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

// Position of the allowed point nearest to z (smaller position on a tie).
__device__ int nearest_pos(const double* coord, const int32_t* idx, int n, double z) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (coord[idx[mid]] < z) lo = mid + 1; else hi = mid;
  }
  if (lo == 0) return 0;
  if (lo == n) return n - 1;
  const double dl = __builtin_fabs(coord[idx[lo - 1]] - z);
  const double dr = __builtin_fabs(coord[idx[lo]] - z);
  return (dl <= dr) ? lo - 1 : lo;
}

// Sequential rule: for targets in order, the nearest unused point.
__device__ void greedy_select(const double* coord, const int32_t* idx, int n, int s, double lo,
                              double hi, int* pos) {
  for (int j = 0; j < s; ++j) {
    const double z = lo + (hi - lo) * cheb_fraction(j, s);
    const int p0 = nearest_pos(coord, idx, n, z);
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
        const double dl = __builtin_fabs(coord[idx[l]] - z);
        const double dr = __builtin_fabs(coord[idx[r]] - z);
        pick = (dl <= dr) ? l : r;
      }
    }
    pos[j] = pick;
  }
  for (int i = 1; i < s; ++i) {  // ascending order
    const int v = pos[i];
    int k = i - 1;
    while (k >= 0 && pos[k] > v) {
      pos[k + 1] = pos[k];
      --k;
    }
    pos[k + 1] = v;
  }
}

template <int W>
__global__ __launch_bounds__(64 * W) void id_kernel(IdArgs A) {
  constexpr int R = kRowsPerWave;
  constexpr int SMAX = R * W;
  __shared__ double s_coord[SMAX];
  __shared__ double s_cx[SMAX];
  __shared__ int s_pos[SMAX];
  __shared__ double2 s_v[SMAX];
  __shared__ double s_part[W][kWave];
  __shared__ double2 s_partc[W][kWave];
  __shared__ int s_piv[kMaxRank];
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
  const double* candX = isV ? A.Om : A.X;
  const double* allowX = isV ? A.X : A.Om;
  const int32_t* aidx = A.allow_idx + ab;

  int gidx = 0;
  double ccoord = 0.0, ccx = 0.0;
  if (lane < c) {
    gidx = A.cand_idx[cb + lane];
    ccoord = candX[gidx];
    if (!isV && fio) ccx = amplitude_shift(A.ph, ccoord);
  }

  // ---- 1. Mock-Chebyshev sample selection
  if (s >= na) {
    for (int j = threadIdx.x; j < na; j += nthreads) s_pos[j] = j;
  } else {
    const double lo = allowX[aidx[0]], hi = allowX[aidx[na - 1]];
    for (int j = threadIdx.x; j < s; j += nthreads)
      s_pos[j] = nearest_pos(allowX, aidx, na, lo + (hi - lo) * cheb_fraction(j, s));
    __syncthreads();
    int coll = 0;
    for (int j = threadIdx.x + 1; j < s; j += nthreads) coll |= (s_pos[j] == s_pos[j - 1]);
    if (__syncthreads_or(coll)) {
      if (threadIdx.x == 0) greedy_select(allowX, aidx, na, s, lo, hi, s_pos);
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < s; j += nthreads) {
    const double v = allowX[aidx[s_pos[j]]];
    s_coord[j] = v;
    s_cx[j] = (isV && fio) ? amplitude_shift(A.ph, v) : 0.0;
  }
  __syncthreads();

  // ---- 2. sampled block, rows [R w, R w + R) of column `lane`
  const int row0 = w * R;
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

  // ---- 3. column-pivoted Householder QR with eps-rank stop
  const int kuser = min(min(s, c), A.kmax > 0 ? A.kmax : (1 << 30));
  bool pivoted = false;
  double r00 = 0.0;
  int k = 0;
  bool zero_block = false, overflow = false;
  for (int j = 0;; ++j) {
    double part = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i)
      if (row0 + i >= j) part += cabs2(a[i]);
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
    const double M = wave_max(nu);
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
    const int p = __builtin_amdgcn_readfirstlane(
        wave_min((eligible && nu >= (1.0 - kPivotTie) * M) ? lane : kWave));
    if (p >= kWave) break;  // no finite residual norm left (cannot happen for finite input)
    // pivot lane publishes the Householder vector v (rows >= j) and alpha, tau
    if (lane == p) {
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int row = row0 + i;
        if (row > j) s_v[row] = a[i];
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
    }
    __syncthreads();
    const double tau = s_tau;
    double2 dot = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < R; ++i)
      if (row0 + i >= j) dot = cfma_conj(s_v[row0 + i], a[i], dot);
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
      if (w == 0) s_piv[j] = p;
    } else if (eligible) {
      const double2 sdot = make_double2(tau * dot.x, tau * dot.y);
#pragma unroll
      for (int i = 0; i < R; ++i)
        if (row0 + i >= j) a[i] = cfma(make_double2(-s_v[row0 + i].x, -s_v[row0 + i].y), sdot, a[i]);
    }
    k = j + 1;
    __syncthreads();
  }
  if (k == 0) zero_block = true;  // no pivot was taken: keep the first candidate, T = 0
  if (zero_block) {
    k = 1;
    pivoted = (lane == 0);
    if (threadIdx.x == 0) s_piv[0] = 0;
  }
  if (overflow && threadIdx.x == 0) atomicOr(A.status, kErrRank);
  __syncthreads();
  if (w != 0) return;

  const uint64_t msk = __ballot(pivoted && lane < c);
  const int below = __popcll(msk & lanes_below(lane));
  const int r = c - k;

  // ---- 4. T = R11^{-1} R12 on the redundant lanes, in place in a[0..k)
  const bool redundant = (lane < c) && !pivoted;
  if (zero_block) {
#pragma unroll
    for (int i = 0; i < R; ++i) a[i] = make_double2(0.0, 0.0);
  } else {
#pragma unroll
    for (int ii = R - 1; ii >= 0; --ii) {
      if (ii < k) {
        const int pp = __builtin_amdgcn_readfirstlane(s_piv[ii]);
        const double2 d = readlane(a[ii], pp);
        const double inv = 1.0 / cabs2(d);
        const double2 t = cmul(a[ii], make_double2(d.x * inv, -d.y * inv));
        if (redundant) a[ii] = t;
#pragma unroll
        for (int i = 0; i < ii; ++i) {
          const double2 rr = readlane(a[i], pp);
          if (redundant) a[i] = cfma(make_double2(-rr.x, -rr.y), t, a[i]);
        }
      }
    }
  }

  // ---- outputs
  if (lane == 0) {
    A.rank[q] = k;
    A.mask[q] = msk;
  }
  if (pivoted && lane < c) A.skel_out[q * kMaxCand + below] = gidx;
  if (redundant) {
    const int jr = lane - below;
    const int64_t off = A.T_off ? A.T_off[q] : q * (int64_t)kSlot;
#pragma unroll
    for (int ii = 0; ii < R; ++ii) {
      if (ii < k) {
        const int pp = s_piv[ii];
        const int sr = min(__popcll(msk & lanes_below(pp)), k - 1);
        const int64_t e = off + (isV ? (int64_t)jr * k + sr : (int64_t)sr * r + jr);
        A.T128[e] = a[ii];
        if (A.T64) A.T64[e] = make_float2((float)a[ii].x, (float)a[ii].y);
      }
    }
  }
}

}  // namespace

hipError_t launch_id_batch(const IdArgs& a, int waves, hipStream_t st) {
  if (a.n_ids <= 0) return hipSuccess;
  dim3 grid((unsigned)a.n_ids);
  switch (waves) {
    case 1: hipLaunchKernelGGL(id_kernel<1>, grid, dim3(64), 0, st, a); break;
    case 2: hipLaunchKernelGGL(id_kernel<2>, grid, dim3(128), 0, st, a); break;
    case 3: hipLaunchKernelGGL(id_kernel<3>, grid, dim3(192), 0, st, a); break;
    default: hipLaunchKernelGGL(id_kernel<4>, grid, dim3(256), 0, st, a); break;
  }
  return hipGetLastError();
}

}  // namespace idbf
