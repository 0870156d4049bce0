// Apply of the IDBF factors (eq. finishIDBF read right to left): H V stages,
// the middle factor, H U stages.
//
//  V stage: z_t(ID) = u[skel] + T u[red], u = the ID's candidate segment of
//           z_{t-1} (x at t = 1).  T is column-major (entry j*k + i).
//  S stage: w_H(U_H ID) = sum of its 2^(d-H) blocks times V_H segments.
//  U stage: each unit (one node, one parent partner) owns the two IDs of the
//           partner's children; they share one candidate segment, which the
//           unit writes whole: v[skel] = w, v[red] = T^T w, summed over both
//           IDs (T row-major, entry i*r + j).  No atomics, no zero fill.
//
// nrhs == 1: one wavefront per ID (unit), lane = candidate position.
// nrhs > 1:  one workgroup per (ID, 64 right-hand sides); lanes over
//            right-hand sides, so every load of z / w / x / y is coalesced.
#include "kernels.hpp"

namespace idbf {

namespace {

constexpr int kIdsPerBlock = 4;  // wavefronts (IDs) per 256-thread workgroup

// ---------------------------------------------------------------- 1 RHS
template <typename C>
__global__ __launch_bounds__(256) void apply_v1(StageArgs A) {
  __shared__ C s_u[kIdsPerBlock][kWave];
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int64_t q = blockIdx.x * (int64_t)kIdsPerBlock + w;
  const bool ok = q < A.n;
  const C* in = static_cast<const C*>(A.in);
  C* out = static_cast<C*>(A.out);
  const C* T = static_cast<const C*>(A.T);
  int c = 0, k = 0, cb = 0;
  uint64_t msk = 0;
  if (ok) {
    c = A.cand_len[q];
    k = A.rank[q];
    cb = A.cand_beg[q];
    msk = A.mask[q];
  }
  C u = czero(C{});
  if (lane < c) u = in[cb + lane];
  const int below = __popcll(msk & lanes_below(lane));
  const bool sk = (msk >> lane) & 1ull;
  if (lane < c && !sk) s_u[w][lane - below] = u;
  __syncthreads();
  if (lane < c && sk) {
    const int r = c - k;
    const C* Tq = T + A.T_off[q] + below;
    C acc = u;
    for (int j = 0; j < r; ++j) acc = cfma(Tq[(int64_t)j * k], s_u[w][j], acc);
    out[A.skel_off[q] + below] = acc;
  }
}

template <typename C>
__global__ __launch_bounds__(256) void apply_u1(StageArgs A) {
  __shared__ C s_w[kIdsPerBlock][2][kMaxRank];
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int64_t unit = blockIdx.x * (int64_t)kIdsPerBlock + w;
  const bool ok = unit < A.n;
  const C* in = static_cast<const C*>(A.in);
  C* out = static_cast<C*>(A.out);
  const C* T = static_cast<const C*>(A.T);
  int64_t qid[2] = {0, 0};
  int kk[2] = {0, 0}, c = 0, cb = 0;
  uint64_t mk[2] = {0, 0};
  if (ok) {
    const int64_t P = unit / A.nn, node = unit % A.nn;
    qid[0] = 2 * P * A.nn + node;
    qid[1] = qid[0] + A.nn;
    c = A.cand_len[qid[0]];
    cb = A.cand_beg[qid[0]];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      kk[h] = A.rank[qid[h]];
      mk[h] = A.mask[qid[h]];
      if (lane < kk[h]) s_w[w][h][lane] = in[A.skel_off[qid[h]] + lane];
    }
  }
  __syncthreads();
  if (lane < c) {
    C acc = czero(C{});
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int below = __popcll(mk[h] & lanes_below(lane));
      if ((mk[h] >> lane) & 1ull) {
        acc = cadd(acc, s_w[w][h][below]);
      } else {
        const int k = kk[h], r = c - k, jr = lane - below;
        const C* Tq = T + A.T_off[qid[h]] + jr;
        for (int i = 0; i < k; ++i) acc = cfma(Tq[(int64_t)i * r], s_w[w][h][i], acc);
      }
    }
    out[cb + lane] = acc;
  }
}

template <typename C>
__global__ __launch_bounds__(256) void apply_s1(StageArgs A) {
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int64_t q = blockIdx.x * (int64_t)kIdsPerBlock + w;
  if (q >= A.n) return;
  const C* in = static_cast<const C*>(A.in);
  C* out = static_cast<C*>(A.out);
  const C* S = static_cast<const C*>(A.T);
  const int64_t b0 = q * A.nsub;
  const int rl = A.rlen[b0], rb = A.rbeg[b0];
  for (int i0 = 0; i0 < rl; i0 += kWave) {
    const int i = i0 + lane;
    if (i >= rl) break;
    C acc = czero(C{});
    for (int jb = 0; jb < A.nsub; ++jb) {
      const int64_t b = b0 + jb;
      const int cl = A.clen[b], cbg = A.cbeg[b];
      const C* Sb = S + A.T_off[b] + i;
      for (int col = 0; col < cl; ++col) acc = cfma(Sb[(int64_t)col * rl], in[cbg + col], acc);
    }
    out[rb + i] = acc;
  }
}

// ---------------------------------------------------------------- many RHS
constexpr int kRhsChunk = 64;

template <typename C>
__global__ __launch_bounds__(256) void apply_vn(StageArgs A) {
  __shared__ int s_skel[kMaxCand];
  __shared__ int s_red[kMaxCand];
  const int64_t q = blockIdx.x;
  const int64_t rhs = blockIdx.y * (int64_t)kRhsChunk + (threadIdx.x & (kRhsChunk - 1));
  const int g = threadIdx.x / kRhsChunk;
  const int c = A.cand_len[q], k = A.rank[q], cb = A.cand_beg[q];
  const uint64_t msk = A.mask[q];
  if (threadIdx.x < c) {
    const int l = threadIdx.x;
    const int below = __popcll(msk & lanes_below(l));
    if ((msk >> l) & 1ull) s_skel[below] = l; else s_red[l - below] = l;
  }
  __syncthreads();
  if (rhs >= A.nrhs) return;
  const C* in = static_cast<const C*>(A.in);
  C* out = static_cast<C*>(A.out);
  const C* Tq = static_cast<const C*>(A.T) + A.T_off[q];
  const int64_t nr = A.nrhs;
  const int r = c - k;
  for (int i = g; i < k; i += 256 / kRhsChunk) {
    C acc = in[(int64_t)(cb + s_skel[i]) * nr + rhs];
    for (int j = 0; j < r; ++j) acc = cfma(Tq[(int64_t)j * k + i], in[(int64_t)(cb + s_red[j]) * nr + rhs], acc);
    out[(int64_t)(A.skel_off[q] + i) * nr + rhs] = acc;
  }
}

template <typename C>
__global__ __launch_bounds__(256) void apply_un(StageArgs A) {
  const int64_t unit = blockIdx.x;
  const int64_t rhs = blockIdx.y * (int64_t)kRhsChunk + (threadIdx.x & (kRhsChunk - 1));
  const int g = threadIdx.x / kRhsChunk;
  if (rhs >= A.nrhs) return;
  const int64_t P = unit / A.nn, node = unit % A.nn;
  const int64_t qid[2] = {2 * P * A.nn + node, 2 * P * A.nn + node + A.nn};
  const int c = A.cand_len[qid[0]], cb = A.cand_beg[qid[0]];
  const C* in = static_cast<const C*>(A.in);
  C* out = static_cast<C*>(A.out);
  const C* T = static_cast<const C*>(A.T);
  const int64_t nr = A.nrhs;
  for (int l = g; l < c; l += 256 / kRhsChunk) {
    C acc = czero(C{});
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint64_t msk = A.mask[qid[h]];
      const int k = A.rank[qid[h]], so = A.skel_off[qid[h]];
      const int below = __popcll(msk & lanes_below(l));
      if ((msk >> l) & 1ull) {
        acc = cadd(acc, in[(int64_t)(so + below) * nr + rhs]);
      } else {
        const int r = c - k, jr = l - below;
        const C* Tq = T + A.T_off[qid[h]] + jr;
        for (int i = 0; i < k; ++i) acc = cfma(Tq[(int64_t)i * r], in[(int64_t)(so + i) * nr + rhs], acc);
      }
    }
    out[(int64_t)(cb + l) * nr + rhs] = acc;
  }
}

template <typename C>
__global__ __launch_bounds__(256) void apply_sn(StageArgs A) {
  const int64_t q = blockIdx.x;
  const int64_t rhs = blockIdx.y * (int64_t)kRhsChunk + (threadIdx.x & (kRhsChunk - 1));
  const int g = threadIdx.x / kRhsChunk;
  if (rhs >= A.nrhs) return;
  const C* in = static_cast<const C*>(A.in);
  C* out = static_cast<C*>(A.out);
  const C* S = static_cast<const C*>(A.T);
  const int64_t nr = A.nrhs;
  const int64_t b0 = q * A.nsub;
  const int rl = A.rlen[b0], rb = A.rbeg[b0];
  for (int i = g; i < rl; i += 256 / kRhsChunk) {
    C acc = czero(C{});
    for (int jb = 0; jb < A.nsub; ++jb) {
      const int64_t b = b0 + jb;
      const int cl = A.clen[b], cbg = A.cbeg[b];
      const C* Sb = S + A.T_off[b] + i;
      for (int col = 0; col < cl; ++col) acc = cfma(Sb[(int64_t)col * rl], in[(int64_t)(cbg + col) * nr + rhs], acc);
    }
    out[(int64_t)(rb + i) * nr + rhs] = acc;
  }
}

inline unsigned grid1(int64_t n) { return (unsigned)((n + kIdsPerBlock - 1) / kIdsPerBlock); }
inline dim3 gridn(int64_t n, int64_t nrhs) {
  return dim3((unsigned)n, (unsigned)((nrhs + kRhsChunk - 1) / kRhsChunk));
}

}  // namespace

hipError_t launch_apply_v(const StageArgs& a, bool fp64, hipStream_t st) {
  if (a.n <= 0 || a.nrhs <= 0) return hipSuccess;
  if (a.nrhs == 1) {
    if (fp64) hipLaunchKernelGGL(apply_v1<double2>, dim3(grid1(a.n)), dim3(256), 0, st, a);
    else hipLaunchKernelGGL(apply_v1<float2>, dim3(grid1(a.n)), dim3(256), 0, st, a);
  } else {
    if (fp64) hipLaunchKernelGGL(apply_vn<double2>, gridn(a.n, a.nrhs), dim3(256), 0, st, a);
    else hipLaunchKernelGGL(apply_vn<float2>, gridn(a.n, a.nrhs), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_apply_u(const StageArgs& a, bool fp64, hipStream_t st) {
  if (a.n <= 0 || a.nrhs <= 0) return hipSuccess;
  if (a.nrhs == 1) {
    if (fp64) hipLaunchKernelGGL(apply_u1<double2>, dim3(grid1(a.n)), dim3(256), 0, st, a);
    else hipLaunchKernelGGL(apply_u1<float2>, dim3(grid1(a.n)), dim3(256), 0, st, a);
  } else {
    if (fp64) hipLaunchKernelGGL(apply_un<double2>, gridn(a.n, a.nrhs), dim3(256), 0, st, a);
    else hipLaunchKernelGGL(apply_un<float2>, gridn(a.n, a.nrhs), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_apply_s(const StageArgs& a, bool fp64, hipStream_t st) {
  if (a.n <= 0 || a.nrhs <= 0) return hipSuccess;
  if (a.nrhs == 1) {
    if (fp64) hipLaunchKernelGGL(apply_s1<double2>, dim3(grid1(a.n)), dim3(256), 0, st, a);
    else hipLaunchKernelGGL(apply_s1<float2>, dim3(grid1(a.n)), dim3(256), 0, st, a);
  } else {
    if (fp64) hipLaunchKernelGGL(apply_sn<double2>, gridn(a.n, a.nrhs), dim3(256), 0, st, a);
    else hipLaunchKernelGGL(apply_sn<float2>, gridn(a.n, a.nrhs), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace idbf
