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
// Adjoint (K~^H, the stages in reverse order, conjugate transposed): U_t^H has
// a V stage's shape over the U factors (T row-major), V_t^H a U stage's
// over the V factors (T column-major), and S^H groups the middle blocks by
// V_H ID; the same kernels take an ADJ template flag.
//
// nrhs == 1: one wavefront per ID (unit), lane = candidate position; IDs
//            with at most 16 (32) candidates four (two) per wavefront.
// nrhs > 1:  one workgroup per (ID or unit, 256 right-hand sides), one
//            thread per right-hand side, so every load of z / w / x / y is
//            coalesced (complex128; complex64 runs on the matrix cores).
#include <algorithm>

#include "kernels.hpp"

namespace idbf {

namespace {

constexpr int kIdsPerBlock = 4;  // wavefronts (IDs) per 256-thread workgroup

// ---------------------------------------------------------------- 1 RHS
// Each wavefront streams the factor block(s) of its ID (unit) with 16-byte
// loads per lane, all issued before the first use, multiplies each entry by
// the input it meets (from LDS) and writes the product to LDS; lanes then sum
// the products of their output.  Block offsets are even, so every block
// starts 16-byte aligned.

template <typename C> struct Vec;
template <> struct Vec<float2> { using type = float4; static constexpr int epl = 2; };
template <> struct Vec<double2> { using type = double2; static constexpr int epl = 1; };

template <typename C>
__device__ __forceinline__ C vec_entry(const typename Vec<C>::type& v, int t);
template <>
__device__ __forceinline__ float2 vec_entry<float2>(const float4& v, int t) {
  return t == 0 ? make_float2(v.x, v.y) : make_float2(v.z, v.w);
}
template <>
__device__ __forceinline__ double2 vec_entry<double2>(const double2& v, int) { return v; }

__device__ __forceinline__ float2 conj_if(float2 v, bool c) { return c ? make_float2(v.x, -v.y) : v; }
__device__ __forceinline__ double2 conj_if(double2 v, bool c) { return c ? make_double2(v.x, -v.y) : v; }

// Products P[e] = blk[e] * in[e / div] (ADJ: conj(blk[e]) * in[e % div]) for
// e < n, streamed NV vector loads per lane at a time (all issued before the
// first use).
template <typename C, int NV, bool ADJ = false>
__device__ __forceinline__ void stream_products(const C* blk, int n, int div, const C* in_lds, C* out_lds,
                                                int lane) {
  using V = typename Vec<C>::type;
  constexpr int EPL = Vec<C>::epl;
  const V* src = reinterpret_cast<const V*>(blk);
  const int nv = (n + EPL - 1) / EPL;
  const float rdiv = 1.0f / (float)div;
  for (int v0 = 0; v0 < nv; v0 += NV * kWave) {
    V buf[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      const int v = v0 + lane + m * kWave;
      if (v0 + m * kWave < nv && v < nv) buf[m] = src[v];
    }
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      const int v = v0 + lane + m * kWave;
      if (v0 + m * kWave < nv && v < nv) {
#pragma unroll
        for (int t = 0; t < EPL; ++t) {
          const int e = v * EPL + t;
          if (e < n) {
            const int j = (int)(((float)e + 0.5f) * rdiv);  // e / div, exact for e < 2^16
            const int jin = ADJ ? e - j * div : j;
            out_lds[e] = cfma(conj_if(vec_entry<C>(buf[m], t), ADJ), in_lds[jin], czero(C{}));
          }
        }
      }
    }
  }
}

// vector loads in flight per lane: one product slot (kProdSlot entries) per round
template <typename C> constexpr int nv_for();

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bool mbit(const ApplyMeta& m, int p) {
  return p < 64 ? ((m.mask >> p) & 1ull) : ((m.mask_hi >> (p - 64)) & 1ull);
}
// skeletons among candidate positions < p
__device__ __forceinline__ int mbelow(const ApplyMeta& m, int p) {
  return p < 64 ? __popcll(m.mask & lanes_below(p)) : __popcll(m.mask) + __popcll(m.mask_hi & lanes_below(p - 64));
}

// Every 1-RHS wavefront stages its products in a fixed slot of kProdSlot
// entries (LDS), whatever the block size: a block is processed in chunks of
// whole columns (V, S) or rows (U), partial sums kept in registers.
constexpr int kProdSlot = 512;
template <typename C> constexpr int nv_for() { return kProdSlot * (int)sizeof(C) / (kWave * 16); }

// V stage: z(ID) = u[skel] + T u[red]; T column-major (entry j*k + i).
// One wavefront per ID, candidate positions lane and lane + 64; the ID's
// packed record is read with a wave-uniform index (scalar loads).
// ADJ: the adjoint of a U stage, which has the same shape: per U ID,
// w(ID) = u[skel] + conj(T) u[red] with T row-major (entry i*r + j), taken in
// chunks of whole rows.
template <typename C, bool ADJ = false>
__global__ __launch_bounds__(256) void apply_v1(StageArgs A) {
  __shared__ C s_prod[kIdsPerBlock][kProdSlot];
  __shared__ C s_u[kIdsPerBlock][kMaxCand];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x & (kWave - 1);
  const int64_t q = blockIdx.x * (int64_t)(blockDim.x / kWave) + w;
  if (q >= A.n) return;
  C* s_p = s_prod[w];
  const C* in = static_cast<const C*>(A.in);
  C* out = static_cast<C*>(A.out);
  const ApplyMeta m = A.meta[q];
  const int c = m.c, k = m.k, r = c - k;
  const int halves = c > kWave ? 2 : 1;  // wave-uniform
  C acc[2];
  int below[2];
  bool sk[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int pos = lane + kWave * h;
    acc[h] = czero(C{});
    below[h] = 0;
    sk[h] = false;
    if (h < halves && pos < c) {
      const C u = in[m.cand_beg + pos];
      below[h] = mbelow(m, pos);
      sk[h] = mbit(m, pos);
      if (sk[h]) acc[h] = u; else s_u[w][pos - below[h]] = u;
    }
  }
  wave_sync_lds();
  const C* T = static_cast<const C*>(A.T) + m.t_off;
  if constexpr (!ADJ) {
    const int cols = max(1, kProdSlot / max(k, 1));  // whole columns per chunk
    for (int j0 = 0; j0 < r; j0 += cols) {
      const int nj = min(cols, r - j0);
      stream_products<C, nv_for<C>()>(T + (int64_t)j0 * k, nj * k, k, s_u[w] + j0, s_p, lane);
      wave_sync_lds();
#pragma unroll
      for (int h = 0; h < 2; ++h)
        if (h < halves && lane + kWave * h < c && sk[h])
          for (int j = 0; j < nj; ++j) acc[h] = cadd(acc[h], s_p[j * k + below[h]]);
      wave_sync_lds();
    }
  } else if (r > 0) {
    const int rows = max(1, kProdSlot / r);  // whole rows per chunk
    for (int i0 = 0; i0 < k; i0 += rows) {
      const int ni = min(rows, k - i0);
      stream_products<C, nv_for<C>(), true>(T + (int64_t)i0 * r, ni * r, r, s_u[w], s_p, lane);
      wave_sync_lds();
#pragma unroll
      for (int h = 0; h < 2; ++h)
        if (h < halves && lane + kWave * h < c && sk[h] && below[h] >= i0 && below[h] < i0 + ni) {
          const C* p = s_p + (below[h] - i0) * r;
          for (int j = 0; j < r; ++j) acc[h] = cadd(acc[h], p[j]);
        }
      wave_sync_lds();
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h)
    if (h < halves && lane + kWave * h < c && sk[h]) out[m.skel_off + below[h]] = acc[h];
}

// U stage: one unit = the two IDs of one node with the two children of one
// partner; they share the candidate segment, which the unit writes whole.
// T row-major (entry i*r + j), processed in chunks of whole rows.
// ADJ: the adjoint of a V stage, which has the same shape: the V IDs (C, 2P)
// and (C, 2P + 1) share their candidate segment; v[skel] = w,
// v[red_j] = sum_i conj(T(i, j)) w_i with T column-major (entry j*k + i),
// taken in chunks of whole columns.
template <typename C, bool ADJ = false>
__global__ __launch_bounds__(256) void apply_u1(StageArgs A) {
  __shared__ C s_prod[kIdsPerBlock][kProdSlot];
  __shared__ C s_w[kIdsPerBlock][2][kMaxRank];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x & (kWave - 1);
  const int64_t unit = blockIdx.x * (int64_t)(blockDim.x / kWave) + w;
  if (unit >= A.n) return;
  C* s_p = s_prod[w];
  const C* in = static_cast<const C*>(A.in);
  C* out = static_cast<C*>(A.out);
  const int64_t P = unit / A.nn, node = unit % A.nn;
  ApplyMeta m[2];
  m[0] = A.meta[2 * P * A.nn + node];
  m[1] = A.meta[2 * P * A.nn + node + A.nn];
  const int c = m[0].c;
  const int halves = c > kWave ? 2 : 1;  // wave-uniform
#pragma unroll
  for (int h = 0; h < 2; ++h)
    if (lane < m[h].k) s_w[w][h][lane] = in[m[h].skel_off + lane];
  wave_sync_lds();
  C acc[2];
  int below[2][2];
  bool sk[2][2];
#pragma unroll
  for (int hp = 0; hp < 2; ++hp) {
    const int pos = lane + kWave * hp;
    acc[hp] = czero(C{});
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      below[hp][h] = mbelow(m[h], pos);
      sk[hp][h] = mbit(m[h], pos);
      if (hp < halves && pos < c && sk[hp][h]) acc[hp] = cadd(acc[hp], s_w[w][h][below[hp][h]]);
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int k = m[h].k, r = c - k;
    if (r == 0) continue;
    const C* T = static_cast<const C*>(A.T) + m[h].t_off;
    if constexpr (!ADJ) {
      const int rows = max(1, kProdSlot / r);  // whole rows per chunk
      for (int i0 = 0; i0 < k; i0 += rows) {
        const int ni = min(rows, k - i0);
        stream_products<C, nv_for<C>()>(T + (int64_t)i0 * r, ni * r, r, s_w[w][h] + i0, s_p, lane);
        wave_sync_lds();
#pragma unroll
        for (int hp = 0; hp < 2; ++hp) {
          const int pos = lane + kWave * hp;
          if (hp < halves && pos < c && !sk[hp][h]) {
            const C* p = s_p + (pos - below[hp][h]);
            for (int i = 0; i < ni; ++i) acc[hp] = cadd(acc[hp], p[i * r]);
          }
        }
        wave_sync_lds();
      }
    } else {
      const int cols = max(1, kProdSlot / k);  // whole columns per chunk
      for (int j0 = 0; j0 < r; j0 += cols) {
        const int nj = min(cols, r - j0);
        stream_products<C, nv_for<C>(), true>(T + (int64_t)j0 * k, nj * k, k, s_w[w][h], s_p, lane);
        wave_sync_lds();
#pragma unroll
        for (int hp = 0; hp < 2; ++hp) {
          const int pos = lane + kWave * hp;
          const int j = pos - below[hp][h];
          if (hp < halves && pos < c && !sk[hp][h] && j >= j0 && j < j0 + nj) {
            const C* p = s_p + (j - j0) * k;
            for (int i = 0; i < k; ++i) acc[hp] = cadd(acc[hp], p[i]);
          }
        }
        wave_sync_lds();
      }
    }
  }
#pragma unroll
  for (int hp = 0; hp < 2; ++hp) {
    const int pos = lane + kWave * hp;
    if (hp < halves && pos < c) out[m[0].cand_beg + pos] = acc[hp];
  }
}

// Middle factor, one U_H ID per wavefront: the 2^(d-H) blocks S(R, C') are
// consecutive, column-major, rows of the output; each block is processed in
// chunks of whole columns.
// ADJ: one V_H ID per wavefront, z(C') = sum over its blocks of S(R, C')^H
// w(R); columns of each block are the outputs, again in chunks of whole
// columns.
template <typename C, bool ADJ = false>
__global__ __launch_bounds__(256) void apply_s1(StageArgs A) {
  __shared__ C s_prod[kIdsPerBlock][kProdSlot];
  __shared__ C s_z[kIdsPerBlock][kMaxRank];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x & (kWave - 1);
  const int64_t q = blockIdx.x * (int64_t)(blockDim.x / kWave) + w;
  if (q >= A.n) return;
  C* s_p = s_prod[w];
  const C* in = static_cast<const C*>(A.in);
  C* out = static_cast<C*>(A.out);
  const C* S = static_cast<const C*>(A.T);
  const int64_t b0 = middle_block<ADJ>(A, q, 0);
  C acc = czero(C{});
  if constexpr (!ADJ) {
    const int rl = A.rlen[b0], rb = A.rbeg[b0];
    for (int jb = 0; jb < A.nsub; ++jb) {
      const int cl = A.clen[b0 + jb];
      if (lane < cl) s_z[w][lane] = in[A.cbeg[b0 + jb] + lane];
      wave_sync_lds();
      const C* Sb = S + A.T_off[b0 + jb];
      const int cols = max(1, kProdSlot / max(rl, 1));
      for (int c0 = 0; c0 < cl; c0 += cols) {
        const int nc = min(cols, cl - c0);
        stream_products<C, nv_for<C>()>(Sb + (int64_t)c0 * rl, nc * rl, rl, s_z[w] + c0, s_p, lane);
        wave_sync_lds();
        if (lane < rl)
          for (int col = 0; col < nc; ++col) acc = cadd(acc, s_p[col * rl + lane]);
        wave_sync_lds();
      }
    }
    if (lane < rl) out[rb + lane] = acc;
  } else {
    const int cl = A.clen[b0], cb = A.cbeg[b0];
    for (int jb = 0; jb < A.nsub; ++jb) {
      const int64_t b = middle_block<ADJ>(A, q, jb);
      const int rl = A.rlen[b];
      if (lane < rl) s_z[w][lane] = in[A.rbeg[b] + lane];
      wave_sync_lds();
      if (rl > 0) {
        const C* Sb = S + A.T_off[b];
        const int cols = max(1, kProdSlot / rl);
        for (int c0 = 0; c0 < cl; c0 += cols) {
          const int nc = min(cols, cl - c0);
          stream_products<C, nv_for<C>(), true>(Sb + (int64_t)c0 * rl, nc * rl, rl, s_z[w], s_p, lane);
          wave_sync_lds();
          if (lane >= c0 && lane < c0 + nc) {
            const C* pp = s_p + (lane - c0) * rl;
            for (int i = 0; i < rl; ++i) acc = cadd(acc, pp[i]);
          }
          wave_sync_lds();
        }
      }
    }
    if (lane < cl) out[cb + lane] = acc;
  }
}

// 1-RHS V- and U-shaped stages whose candidate sets have at most 64 / G
// points (the lowest levels: 16 at t = 1): G IDs (units) per wavefront, each
// on its own group of 64 / G lanes (lane = candidate position), all of an
// ID's products in one slot of kProdSlot / G entries.  Same products and
// summation order as apply_v1 / apply_u1 (ADJ included), so the same results.
template <typename C, int G, bool ADJ>
__global__ __launch_bounds__(256) void apply_v1g(StageArgs A) {
  constexpr int GL = kWave / G, SLOT = kProdSlot / G;
  using V = typename Vec<C>::type;
  constexpr int EPL = Vec<C>::epl;
  constexpr int NV = SLOT / EPL / GL;  // vector loads per lane
  __shared__ C s_prod[kIdsPerBlock][kProdSlot];
  __shared__ C s_u[kIdsPerBlock][kWave];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x & (kWave - 1);
  const int g = lane / GL, l = lane % GL;
  const int64_t q0 = (blockIdx.x * (int64_t)kIdsPerBlock + w) * G;
  if (q0 >= A.n) return;
  const int64_t q = q0 + g;
  const bool valid = q < A.n;
  const ApplyMeta m = A.meta[valid ? q : A.n - 1];
  const int c = m.c, k = m.k, r = c - k;
  C* s_p = s_prod[w] + g * SLOT;
  C* s_ug = s_u[w] + g * GL;
  const C* in = static_cast<const C*>(A.in);
  C* out = static_cast<C*>(A.out);
  const bool on = valid && l < c;
  C acc = czero(C{});
  int below = 0;
  bool sk = false;
  if (on) {
    const C u = in[m.cand_beg + l];
    below = mbelow(m, l);
    sk = mbit(m, l);
    if (sk) acc = u; else s_ug[l - below] = u;
  }
  wave_sync_lds();
  // P[e] = T[e] u[red_{e / k}], T column-major (entry j*k + i); ADJ (U_t^H):
  // P[e] = conj(T[e]) u[red_{e % r}], T row-major (entry i*r + j)
  const int n = k * r, nv = (n + EPL - 1) / EPL;
  const V* src = reinterpret_cast<const V*>(static_cast<const C*>(A.T) + m.t_off);
  const int div = ADJ ? r : k;
  const float rk = 1.0f / (float)max(div, 1);
  V buf[NV];
#pragma unroll
  for (int mm = 0; mm < NV; ++mm) {
    const int v = l + GL * mm;
    if (valid && v < nv) buf[mm] = src[v];
  }
#pragma unroll
  for (int mm = 0; mm < NV; ++mm) {
    const int v = l + GL * mm;
    if (valid && v < nv) {
#pragma unroll
      for (int t = 0; t < EPL; ++t) {
        const int e = v * EPL + t;
        if (e < n) {
          const int q = (int)(((float)e + 0.5f) * rk);  // e / div
          s_p[e] = cfma(conj_if(vec_entry<C>(buf[mm], t), ADJ), s_ug[ADJ ? e - q * div : q], czero(C{}));
        }
      }
    }
  }
  wave_sync_lds();
  if (on && sk) {
    if constexpr (!ADJ) {
      for (int j = 0; j < r; ++j) acc = cadd(acc, s_p[j * k + below]);
    } else {
      for (int j = 0; j < r; ++j) acc = cadd(acc, s_p[below * r + j]);
    }
    out[m.skel_off + below] = acc;
  }
}

template <typename C, int G, bool ADJ>
__global__ __launch_bounds__(256) void apply_u1g(StageArgs A) {
  constexpr int GL = kWave / G, SLOT = kProdSlot / G;
  using V = typename Vec<C>::type;
  constexpr int EPL = Vec<C>::epl;
  constexpr int NV = SLOT / EPL / GL;
  __shared__ C s_prod[kIdsPerBlock][kProdSlot];
  __shared__ C s_w[kIdsPerBlock][2][kWave];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x & (kWave - 1);
  const int g = lane / GL, l = lane % GL;
  const int64_t u0 = (blockIdx.x * (int64_t)kIdsPerBlock + w) * G;
  if (u0 >= A.n) return;
  const int64_t unit = u0 + g;
  const bool valid = unit < A.n;
  const int64_t un = valid ? unit : A.n - 1;
  const int64_t P = un / A.nn, node = un % A.nn;
  ApplyMeta m[2];
  m[0] = A.meta[2 * P * A.nn + node];
  m[1] = A.meta[2 * P * A.nn + node + A.nn];
  const int c = m[0].c;
  C* s_p = s_prod[w] + g * SLOT;
  const C* in = static_cast<const C*>(A.in);
  C* out = static_cast<C*>(A.out);
#pragma unroll
  for (int h = 0; h < 2; ++h)
    if (valid && l < m[h].k) s_w[w][h][g * GL + l] = in[m[h].skel_off + l];
  wave_sync_lds();
  const bool on = valid && l < c;
  C acc = czero(C{});
  int below[2];
  bool sk[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    below[h] = mbelow(m[h], l);
    sk[h] = mbit(m[h], l);
    if (on && sk[h]) acc = cadd(acc, s_w[w][h][g * GL + below[h]]);
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    // P[e] = T_h[e] w_h[e / r], T row-major (entry i*r + j); ADJ (V_t^H):
    // P[e] = conj(T_h[e]) w_h[e % k], T column-major (entry j*k + i)
    const int k = m[h].k, r = c - k, n = k * r, nv = (n + EPL - 1) / EPL;
    const V* src = reinterpret_cast<const V*>(static_cast<const C*>(A.T) + m[h].t_off);
    const int div = ADJ ? k : r;
    const float rr = 1.0f / (float)max(div, 1);
    V buf[NV];
#pragma unroll
    for (int mm = 0; mm < NV; ++mm) {
      const int v = l + GL * mm;
      if (valid && v < nv) buf[mm] = src[v];
    }
#pragma unroll
    for (int mm = 0; mm < NV; ++mm) {
      const int v = l + GL * mm;
      if (valid && v < nv) {
#pragma unroll
        for (int t = 0; t < EPL; ++t) {
          const int e = v * EPL + t;
          if (e < n) {
            const int q = (int)(((float)e + 0.5f) * rr);  // e / div
            s_p[e] = cfma(conj_if(vec_entry<C>(buf[mm], t), ADJ), s_w[w][h][g * GL + (ADJ ? e - q * div : q)],
                          czero(C{}));
          }
        }
      }
    }
    wave_sync_lds();
    if (on && !sk[h]) {
      if constexpr (!ADJ) {
        const C* p = s_p + (l - below[h]);
        for (int i = 0; i < k; ++i) acc = cadd(acc, p[i * r]);
      } else {
        const C* p = s_p + (l - below[h]) * k;
        for (int i = 0; i < k; ++i) acc = cadd(acc, p[i]);
      }
    }
    wave_sync_lds();
  }
  if (on) out[m[0].cand_beg + l] = acc;
}

// The whole matrix when the tree has no levels (N <= 2 leaf): lanes over rows
// (ADJ: over columns, with conjugated entries).
template <typename C, bool ADJ = false>
__global__ __launch_bounds__(256) void apply_dense(StageArgs A) {
  const C* in = static_cast<const C*>(A.in);
  C* out = static_cast<C*>(A.out);
  const C* S = static_cast<const C*>(A.T);
  const int rl = A.rlen[0], cl = A.clen[0];
  const int no = ADJ ? cl : rl, ni = ADJ ? rl : cl;
  const int64_t nr = A.nrhs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)no * nr;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int o = (int)(e / nr);
    const int64_t rhs = e % nr;
    C acc = czero(C{});
    for (int l = 0; l < ni; ++l) {
      const C sv = ADJ ? conj_if(S[(int64_t)o * rl + l], true) : S[(int64_t)l * rl + o];
      acc = cfma(sv, in[(int64_t)l * nr + rhs], acc);
    }
    out[(int64_t)o * nr + rhs] = acc;
  }
}

// ---------------------------------------------------------------- many RHS
// One thread per right-hand side, a workgroup per (ID or unit, 256 RHS).  The
// ID's factor block is staged in LDS once; each thread keeps its outputs (or,
// for U stages, its inputs) in registers, indexed statically up to the rank
// bound, and every global load and store is coalesced across right-hand sides.
constexpr int kRhsTile = 256;

template <typename C>
__device__ __forceinline__ void stage_block(const C* src, int n, C* dst) {
  for (int e = threadIdx.x; e < n; e += blockDim.x) dst[e] = src[e];
}

constexpr int kRankChunk = 16;  // outputs (V, S) or inputs (U) held in registers per pass

// V stage: the ID's T (dynamic LDS, k r entries) is applied to one RHS per
// thread, kRankChunk outputs per pass.  ADJ: the adjoint of a U stage (per U
// ID, conj(T) with T row-major).
template <typename C, bool ADJ = false>
__global__ __launch_bounds__(256) void apply_vn(StageArgs A) {
  extern __shared__ __attribute__((aligned(16))) unsigned char s_dyn[];
  C* s_T = reinterpret_cast<C*>(s_dyn);
  __shared__ int s_skel[kMaxCand];
  __shared__ int s_red[kMaxCand];
  const int64_t q = blockIdx.x;
  const int64_t n = blockIdx.y * (int64_t)kRhsTile + threadIdx.x;
  const ApplyMeta m = A.meta[q];
  const int c = m.c, k = m.k, cb = m.cand_beg, so = m.skel_off;
  const int r = c - k;
  for (int l = threadIdx.x; l < c; l += blockDim.x) {
    const int below = mbelow(m, l);
    if (mbit(m, l)) s_skel[below] = l; else s_red[l - below] = l;
  }
  stage_block(static_cast<const C*>(A.T) + m.t_off, k * r, s_T);
  __syncthreads();
  if (n >= A.nrhs) return;
  const C* in = static_cast<const C*>(A.in) + n;
  C* out = static_cast<C*>(A.out) + n;
  const int64_t nr = A.nrhs;
  for (int i0 = 0; i0 < k; i0 += kRankChunk) {
    C acc[kRankChunk];
#pragma unroll
    for (int i = 0; i < kRankChunk; ++i) acc[i] = czero(C{});
    for (int j = 0; j < r; ++j) {
      const C uj = in[(int64_t)(cb + s_red[j]) * nr];
      if constexpr (!ADJ) {
        const C* t = s_T + j * k + i0;
#pragma unroll
        for (int i = 0; i < kRankChunk; ++i)
          if (i0 + i < k) acc[i] = cfma(t[i], uj, acc[i]);
      } else {
        const C* t = s_T + i0 * r + j;
#pragma unroll
        for (int i = 0; i < kRankChunk; ++i)
          if (i0 + i < k) acc[i] = cfma(conj_if(t[i * r], true), uj, acc[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < kRankChunk; ++i)
      if (i0 + i < k) out[(int64_t)(so + i0 + i) * nr] = cadd(acc[i], in[(int64_t)(cb + s_skel[i0 + i]) * nr]);
  }
}

// U stage: the unit's two T blocks (dynamic LDS, 2 pmax entries); one RHS per
// thread; each pass takes kRankChunk inputs of one ID and adds their
// contribution to every candidate position (the first pass writes).  ADJ:
// the adjoint of a V stage (the V ID pair of one segment, conj(T) with T
// column-major).
template <typename C, bool ADJ = false>
__global__ __launch_bounds__(256) void apply_un(StageArgs A) {
  extern __shared__ __attribute__((aligned(16))) unsigned char s_dyn[];
  C* s_T = reinterpret_cast<C*>(s_dyn);
  const int64_t unit = blockIdx.x;
  const int64_t n = blockIdx.y * (int64_t)kRhsTile + threadIdx.x;
  const int64_t P = unit / A.nn, node = unit % A.nn;
  ApplyMeta m[2];
  m[0] = A.meta[2 * P * A.nn + node];
  m[1] = A.meta[2 * P * A.nn + node + A.nn];
  const int c = m[0].c, cb = m[0].cand_beg;
  const C* T = static_cast<const C*>(A.T);
  stage_block(T + m[0].t_off, m[0].k * (c - m[0].k), s_T);
  stage_block(T + m[1].t_off, m[1].k * (c - m[1].k), s_T + A.pmax);
  __syncthreads();
  if (n >= A.nrhs) return;
  const C* in = static_cast<const C*>(A.in) + n;
  C* out = static_cast<C*>(A.out) + n;
  const int64_t nr = A.nrhs;
  bool first = true;
  for (int h = 0; h < 2; ++h) {
    const int k = m[h].k, r = c - k, so = m[h].skel_off;
    const C* Th = s_T + h * A.pmax;
    for (int i0 = 0; i0 < k; i0 += kRankChunk) {
      C wv[kRankChunk];
#pragma unroll
      for (int i = 0; i < kRankChunk; ++i) wv[i] = (i0 + i < k) ? in[(int64_t)(so + i0 + i) * nr] : czero(C{});
      for (int l = 0; l < c; ++l) {
        C acc = first ? czero(C{}) : out[(int64_t)(cb + l) * nr];
        const int below = mbelow(m[h], l);
        if (mbit(m[h], l)) {
          if (below >= i0 && below < i0 + kRankChunk) acc = cadd(acc, in[(int64_t)(so + below) * nr]);
        } else {
          if constexpr (!ADJ) {
            const C* t = Th + (int64_t)i0 * r + (l - below);
#pragma unroll
            for (int i = 0; i < kRankChunk; ++i)
              if (i0 + i < k) acc = cfma(t[i * r], wv[i], acc);
          } else {
            const C* t = Th + (int64_t)(l - below) * k + i0;
#pragma unroll
            for (int i = 0; i < kRankChunk; ++i)
              if (i0 + i < k) acc = cfma(conj_if(t[i], true), wv[i], acc);
          }
        }
        out[(int64_t)(cb + l) * nr] = acc;
      }
      first = false;
    }
  }
}

// Middle stage: one U_H ID per workgroup, its blocks staged in dynamic LDS
// one at a time (pmax entries); kRankChunk outputs per pass.  ADJ: one V_H ID
// per workgroup, conj(S)^T of each of its blocks.
template <typename C, bool ADJ = false>
__global__ __launch_bounds__(256) void apply_sn(StageArgs A) {
  extern __shared__ __attribute__((aligned(16))) unsigned char s_dyn[];
  C* s_S = reinterpret_cast<C*>(s_dyn);
  const int64_t q = blockIdx.x;
  const int64_t n = blockIdx.y * (int64_t)kRhsTile + threadIdx.x;
  const int64_t b0 = middle_block<ADJ>(A, q, 0);
  const int ol = ADJ ? A.clen[b0] : A.rlen[b0];   // outputs
  const int ob = ADJ ? A.cbeg[b0] : A.rbeg[b0];
  const bool live = n < A.nrhs;
  const C* in = static_cast<const C*>(A.in) + (live ? n : 0);
  C* out = static_cast<C*>(A.out) + (live ? n : 0);
  const int64_t nr = A.nrhs;
  for (int i0 = 0; i0 < ol; i0 += kRankChunk) {
    C acc[kRankChunk];
#pragma unroll
    for (int i = 0; i < kRankChunk; ++i) acc[i] = czero(C{});
    for (int jb = 0; jb < A.nsub; ++jb) {
      const int64_t b = middle_block<ADJ>(A, q, jb);
      const int rl = A.rlen[b], cl = A.clen[b];
      const int il = ADJ ? rl : cl, ib = ADJ ? A.rbeg[b] : A.cbeg[b];  // inputs of this block
      __syncthreads();
      stage_block(static_cast<const C*>(A.T) + A.T_off[b], rl * cl, s_S);
      __syncthreads();
      if (!live) continue;
      for (int l = 0; l < il; ++l) {
        const C zc = in[(int64_t)(ib + l) * nr];
        if constexpr (!ADJ) {
          const C* sc = s_S + l * rl + i0;
#pragma unroll
          for (int i = 0; i < kRankChunk; ++i)
            if (i0 + i < ol) acc[i] = cfma(sc[i], zc, acc[i]);
        } else {
          const C* sc = s_S + i0 * rl + l;
#pragma unroll
          for (int i = 0; i < kRankChunk; ++i)
            if (i0 + i < ol) acc[i] = cfma(conj_if(sc[i * rl], true), zc, acc[i]);
        }
      }
    }
    if (!live) continue;
#pragma unroll
    for (int i = 0; i < kRankChunk; ++i)
      if (i0 + i < ol) out[(int64_t)(ob + i0 + i) * nr] = acc[i];
  }
}

// Raise a kernel's dynamic LDS limit once when a launch needs more than the
// default (gfx950 workgroups may use up to 160 KB).
template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= (size_t(64) << 10)) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

inline unsigned grid1(int64_t n, int ipb = kIdsPerBlock) { return (unsigned)((n + ipb - 1) / ipb); }
inline dim3 gridn(int64_t n, int64_t nrhs) {
  return dim3((unsigned)n, (unsigned)((nrhs + kRhsTile - 1) / kRhsTile));
}

template <bool ADJ>
hipError_t launch_v_shaped(const StageArgs& a, bool fp64, hipStream_t st) {
  if (a.nrhs == 1 && a.cmax > 0 && a.cmax <= kWave / 2) {  // small candidate sets: IDs share wavefronts
    if (a.cmax <= kWave / 4) {
      if (fp64) hipLaunchKernelGGL((apply_v1g<double2, 4, ADJ>), dim3(grid1(a.n, 4 * kIdsPerBlock)), dim3(256), 0, st, a);
      else hipLaunchKernelGGL((apply_v1g<float2, 4, ADJ>), dim3(grid1(a.n, 4 * kIdsPerBlock)), dim3(256), 0, st, a);
    } else {
      if (fp64) hipLaunchKernelGGL((apply_v1g<double2, 2, ADJ>), dim3(grid1(a.n, 2 * kIdsPerBlock)), dim3(256), 0, st, a);
      else hipLaunchKernelGGL((apply_v1g<float2, 2, ADJ>), dim3(grid1(a.n, 2 * kIdsPerBlock)), dim3(256), 0, st, a);
    }
  } else if (a.nrhs == 1) {
    if (fp64) hipLaunchKernelGGL((apply_v1<double2, ADJ>), dim3(grid1(a.n)), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((apply_v1<float2, ADJ>), dim3(grid1(a.n)), dim3(256), 0, st, a);
  } else {
    if (!fp64) return hipErrorInvalidValue;  // complex64 runs on the matrix cores (complex128 there too when A fits LDS)
    const size_t lds = (size_t)a.pmax * sizeof(double2);
    if (hipError_t e = allow_lds(apply_vn<double2, ADJ>, lds); e != hipSuccess) return e;
    hipLaunchKernelGGL((apply_vn<double2, ADJ>), gridn(a.n, a.nrhs), dim3(256), lds, st, a);
  }
  return hipGetLastError();
}

template <bool ADJ>
hipError_t launch_u_shaped(const StageArgs& a, bool fp64, hipStream_t st) {
  if (a.nrhs == 1 && a.cmax > 0 && a.cmax <= kWave / 2) {  // small candidate sets: units share wavefronts
    if (a.cmax <= kWave / 4) {
      if (fp64) hipLaunchKernelGGL((apply_u1g<double2, 4, ADJ>), dim3(grid1(a.n, 4 * kIdsPerBlock)), dim3(256), 0, st, a);
      else hipLaunchKernelGGL((apply_u1g<float2, 4, ADJ>), dim3(grid1(a.n, 4 * kIdsPerBlock)), dim3(256), 0, st, a);
    } else {
      if (fp64) hipLaunchKernelGGL((apply_u1g<double2, 2, ADJ>), dim3(grid1(a.n, 2 * kIdsPerBlock)), dim3(256), 0, st, a);
      else hipLaunchKernelGGL((apply_u1g<float2, 2, ADJ>), dim3(grid1(a.n, 2 * kIdsPerBlock)), dim3(256), 0, st, a);
    }
  } else if (a.nrhs == 1) {
    if (fp64) hipLaunchKernelGGL((apply_u1<double2, ADJ>), dim3(grid1(a.n)), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((apply_u1<float2, ADJ>), dim3(grid1(a.n)), dim3(256), 0, st, a);
  } else {
    if (!fp64) return hipErrorInvalidValue;  // complex64 runs on the matrix cores (complex128 there too when A fits LDS)
    const size_t lds = 2 * (size_t)a.pmax * sizeof(double2);
    if (hipError_t e = allow_lds(apply_un<double2, ADJ>, lds); e != hipSuccess) return e;
    hipLaunchKernelGGL((apply_un<double2, ADJ>), gridn(a.n, a.nrhs), dim3(256), lds, st, a);
  }
  return hipGetLastError();
}

template <bool ADJ>
hipError_t launch_s_stage(const StageArgs& a, bool fp64, hipStream_t st) {
  if (a.dense) {
    const unsigned blocks = (unsigned)std::min<int64_t>((a.rlen_host * a.nrhs + 255) / 256, 65535);
    if (fp64) hipLaunchKernelGGL((apply_dense<double2, ADJ>), dim3(blocks), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((apply_dense<float2, ADJ>), dim3(blocks), dim3(256), 0, st, a);
  } else if (a.nrhs == 1) {
    if (fp64) hipLaunchKernelGGL((apply_s1<double2, ADJ>), dim3(grid1(a.n)), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((apply_s1<float2, ADJ>), dim3(grid1(a.n)), dim3(256), 0, st, a);
  } else {
    if (!fp64) return hipErrorInvalidValue;  // complex64 runs on the matrix cores (complex128 there too when A fits LDS)
    const size_t lds = (size_t)a.pmax * sizeof(double2);
    if (hipError_t e = allow_lds(apply_sn<double2, ADJ>, lds); e != hipSuccess) return e;
    hipLaunchKernelGGL((apply_sn<double2, ADJ>), gridn(a.n, a.nrhs), dim3(256), lds, st, a);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_apply_v(const StageArgs& a, bool fp64, hipStream_t st, bool adj) {
  if (a.n <= 0 || a.nrhs <= 0) return hipSuccess;
  return adj ? launch_v_shaped<true>(a, fp64, st) : launch_v_shaped<false>(a, fp64, st);
}

hipError_t launch_apply_u(const StageArgs& a, bool fp64, hipStream_t st, bool adj) {
  if (a.n <= 0 || a.nrhs <= 0) return hipSuccess;
  return adj ? launch_u_shaped<true>(a, fp64, st) : launch_u_shaped<false>(a, fp64, st);
}

hipError_t launch_apply_s(const StageArgs& a, bool fp64, hipStream_t st, bool adj) {
  if (a.n <= 0 || a.nrhs <= 0) return hipSuccess;
  return adj ? launch_s_stage<true>(a, fp64, st) : launch_s_stage<false>(a, fp64, st);
}

}  // namespace idbf
