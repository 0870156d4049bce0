// Many-RHS apply of the IDBF factors on the matrix cores, complex64 in/out
// (eq. finishIDBF read right to left, the same stages as the VALU apply).
//
// Every stage unit is a small dense product on a block of right-hand sides:
//   V stage (the two IDs (C, 2P), (C, 2P + 1) sharing one candidate segment):
//                       z_h[skel_off_h + i] = u[skel_h,i] + sum_j T_h(i, j) u[red_h,j] (M = k_0 + k_1, K = c)
//   S stage (U_H ID):   w[rbeg + i]       = sum_b sum_col S_b(i, col) z[cbeg_b + col] (M = k_R, K = sum k_C')
//   U stage (a unit):   v[cand_beg + l]   = sum_h ( l in skel_h ? w_h[b] : sum_i T_h(i, red(l)) w_h[i] )
//                                                                          (M = c, K = k_0 + k_1)
// The adjoint stages stage A^H of the other factor of the same shape (U_t^H
// as a V unit, V_t^H as a U unit, S^H per V_H ID); the product is unchanged.
// A (M x K complex: the factor entries and the identity parts) is staged in
// LDS once per workgroup; every input row is read once per unit.  Rows of the
// stage vectors are (row, rhs) complex64, right-hand sides fastest.
//
// Complex arithmetic on real MFMA: with B' the interleaved (re, im) rows and
// B~ the same rows with each pair mapped (re, im) -> (-im, re),
//   C' = A_re B' + A_im B~
// gives the interleaved complex product.  A lane holds two complex right-hand
// sides (4 real columns): real column 4 j + t of the wave's block belongs to
// N-tile t, so B~ is a register shuffle, never a cross-lane move.
//
// Precision: FP64 MFMA for complex128 data (v_mfma_f64_16x16x4_f64, the
// FP32 layout with one complex right-hand side per lane), FP32 MFMA
// (v_mfma_f32_16x16x4_f32, 16-row M tiles, one wavefront over all M tiles of
// a unit), or the BF16 hi/lo split
// a ~= a_hi + a_lo with a b ~= a_hi b_hi + a_hi b_lo + a_lo b_hi on
// v_mfma_f32_32x32x16_bf16 (32-row M tiles), FP32 accumulation.  A unit's A
// is staged once per workgroup and serves up to 1024 right-hand sides.
#include <algorithm>

#include "kernels.hpp"

namespace idbf {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kMaxKg = 256;  // largest K of a unit (S stage: 4 blocks of <= 64 columns)
constexpr int kMaxMg = 128;  // largest M of a unit (V: k_0 + k_1, U: c)
constexpr int kRhsPerWave = 64;
constexpr int kWavesG = 4;

enum { kModeV = 0, kModeS = 1, kModeU = 2 };

struct Unit {
  int M, K;
};

__host__ __device__ __forceinline__ int lda_for(int K) { return ((K + 15) & ~15) + 2; }

// Stage the unit's A (M x K complex, zero padded to Mpad x roundup(K, 16))
// into LDS with the input row of every K index (s_src) and the output row of
// every M index (s_out).
//   V unit (C, P): the IDs (C, 2P) and (C, 2P + 1) share the candidate
//     segment: rows [0, k0) of A are [I T_0] of the first (skeleton columns
//     carry the identity), rows [k0, k0 + k1) those of the second.
//   U unit: A = [P_0 P_1], P_h(l, i) = 1 if l is the i-th skeleton of ID h,
//     T_h(i, j) if l is its j-th redundant candidate.
//   S (U_H ID): A = [S_1 ... S_nsub].
// ADJ (the adjoint, stages in reverse): a V-shaped unit over the U ID pair
// of one segment, A = [P_0 P_1]^H; a U-shaped unit over the V ID pair of one
// segment, A = ([I T_0]; [I T_1])^H; S^H per V_H ID, A = [S(R_1, C')^H ...].
__device__ __forceinline__ float2 cplx(float2, float re, float im) { return make_float2(re, im); }
__device__ __forceinline__ double2 cplx(double2, double re, double im) { return make_double2(re, im); }

// Where the entries of a V or U unit go in A: the row of output i of ID h
// and the column of candidate l (V), or the row of candidate l and the
// column of input b of ID h (U).  The plain stage packs them densely; the
// fused two-stage groups place them on their register tiles.
struct DenseMap {
  __device__ int vrow(int h, int i, int k0) const { return (h ? k0 : 0) + i; }
  __device__ int vcol(int l) const { return l; }
  __device__ int urow(int l) const { return l; }
  __device__ int ucol(int h, int b, int k0) const { return (h ? k0 : 0) + b; }
  __device__ Unit vdims(int k0, int k1, int c) const { return Unit{k0 + k1, c}; }
  __device__ Unit udims(int k0, int k1, int c) const { return Unit{c, k0 + k1}; }
};

template <int MODE, bool ADJ, typename C = float2, typename Map = DenseMap>
__device__ Unit stage_unit(const StageArgs& A, C* s_A, int* s_src, int* s_out, int* s_red, int64_t q = -1,
                           int rows = 0, const Map& mp = Map{}) {
  if (q < 0) q = blockIdx.x;
  if (rows == 0) rows = A.gemm_rows;
  const C* T = static_cast<const C*>(A.T);
  const C zero = cplx(C{}, 0.f, 0.f), one = cplx(C{}, 1.f, 0.f);
  Unit u{};
  if constexpr (MODE == kModeS) {
    const int64_t b0 = middle_block<ADJ>(A, q, 0);
    const int ol = ADJ ? A.clen[b0] : A.rlen[b0], obg = ADJ ? A.cbeg[b0] : A.rbeg[b0];  // outputs
    int K = 0;
    for (int jb = 0; jb < A.nsub; ++jb) {
      const int64_t b = middle_block<ADJ>(A, q, jb);
      K += ADJ ? A.rlen[b] : A.clen[b];
    }
    u = Unit{ol, K};
    const int lda = lda_for(K);
    for (int e = threadIdx.x; e < rows * lda; e += blockDim.x) s_A[e] = zero;
    for (int i = threadIdx.x; i < ol; i += blockDim.x) s_out[i] = obg + i;
    __syncthreads();
    int off = 0;
    for (int jb = 0; jb < A.nsub; ++jb) {
      const int64_t b = middle_block<ADJ>(A, q, jb);
      const int rl = A.rlen[b], cl = A.clen[b];
      const int il = ADJ ? rl : cl, ibg = ADJ ? A.rbeg[b] : A.cbeg[b];  // inputs of this block
      const int64_t so = A.T_off[b];
      for (int l = threadIdx.x; l < il; l += blockDim.x) s_src[off + l] = ibg + l;
      for (int e = threadIdx.x; e < rl * cl; e += blockDim.x) {
        const C v = T[so + e];  // S(e % rl, e / rl)
        if (ADJ) s_A[(e / rl) * lda + off + e % rl] = cplx(C{}, v.x, -v.y);
        else s_A[(e % rl) * lda + off + e / rl] = v;
      }
      off += il;
    }
  } else {
    const int64_t P = q / A.nn, node = q % A.nn;
    const ApplyMeta m0 = A.meta[2 * P * A.nn + node];
    const ApplyMeta m1 = A.meta[2 * P * A.nn + node + A.nn];
    const int c = m0.c, k0 = m0.k;
    const bool isV = (MODE == kModeV);
    u = isV ? mp.vdims(k0, m1.k, c) : mp.udims(k0, m1.k, c);
    const int lda = lda_for(u.K);
    for (int e = threadIdx.x; e < rows * lda; e += blockDim.x) s_A[e] = zero;
    __syncthreads();  // zero fill before the identity entries
    for (int e = threadIdx.x; e < 2 * kMaxMg; e += blockDim.x) {  // (ID h, candidate position l)
      const int h = e / kMaxMg, l = e % kMaxMg;
      const ApplyMeta& m = h ? m1 : m0;
      if (l < m.k) {
        if (isV) s_out[mp.vrow(h, l, k0)] = m.skel_off + l;
        else s_src[mp.ucol(h, l, k0)] = m.skel_off + l;
      }
      if (l < c) {
        if (h == 0) {
          if (isV) s_src[mp.vcol(l)] = m.cand_beg + l;
          else s_out[mp.urow(l)] = m.cand_beg + l;
        }
        const int below = l < 64 ? __popcll(m.mask & lanes_below(l))
                                 : __popcll(m.mask) + __popcll(m.mask_hi & lanes_below(l - 64));
        if (l < 64 ? ((m.mask >> l) & 1ull) : ((m.mask_hi >> (l - 64)) & 1ull)) {
          if (isV) s_A[mp.vrow(h, below, k0) * lda + mp.vcol(l)] = one;
          else s_A[mp.urow(l) * lda + mp.ucol(h, below, k0)] = one;
        } else {
          s_red[h * kMaxMg + l - below] = l;
        }
      }
    }
    __syncthreads();
    // T_h(i, j) at j k + i for V factors, at i r + j for U factors
    constexpr bool colmajor = (MODE == kModeV) != ADJ;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const ApplyMeta& m = h ? m1 : m0;
      const int k = m.k, r = c - k;
      for (int e = threadIdx.x; e < k * r; e += blockDim.x) {
        const int i = colmajor ? e % k : e / r, j = colmajor ? e / k : e % r;
        C v = T[m.t_off + e];
        if (ADJ) v.y = -v.y;
        if (isV) s_A[mp.vrow(h, i, k0) * lda + mp.vcol(s_red[h * kMaxMg + j])] = v;
        else s_A[mp.urow(s_red[h * kMaxMg + j]) * lda + mp.ucol(h, i, k0)] = v;
      }
    }
  }
  __syncthreads();
  return u;
}

__device__ __forceinline__ float2 ld2(const float2* p, bool ok) { return ok ? *p : make_float2(0.f, 0.f); }

__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

// BF16 split on v_mfma_f32_32x32x16_bf16: one wavefront per (32-row M tile,
// block of 64 right-hand sides); the workgroup's wavefronts cover
// kRhsIterB such blocks in turn, so the staged A serves them all.
constexpr int kRhsIterB = 8;

template <int MODE, bool ADJ>
__global__ __launch_bounds__(64 * kWavesG) void apply_gemm_bf16(StageArgs A) {
  extern __shared__ __attribute__((aligned(16))) float2 s_A[];
  __shared__ int s_src[kMaxKg];
  __shared__ int s_out[kMaxMg];
  __shared__ int s_red[2 * kMaxMg];
  const Unit u = stage_unit<MODE, ADJ>(A, s_A, s_src, s_out, s_red);
  const int lane = threadIdx.x & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int tiles = A.gemm_rows / 32;
  const int mt = w % tiles;
  if (mt * 32 >= u.M) return;
  const int blocks = blockDim.x / kWave / tiles;  // right-hand-side blocks per pass
  const int half = lane >> 5, jj = lane & 31;
  const int64_t nr = A.nrhs;
  const float2* in = static_cast<const float2*>(A.in);
  float2* out = static_cast<float2*>(A.out);
  const int lda = lda_for(u.K);
  for (int it = 0; it < A.rhs_iter; ++it) {
    const int64_t rhs0 = ((blockIdx.y * (int64_t)A.rhs_iter + it) * blocks + w / tiles) * kRhsPerWave;
    if (rhs0 >= nr) return;
    const int64_t n0 = rhs0 + 2 * jj;
    const bool ok0 = n0 < nr, ok1 = n0 + 1 < nr;
    f32x16 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f32x16{};
    for (int kc = 0; kc < u.K; kc += 16) {
      float4 b[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int kk = kc + 8 * half + e;
        const int row = kk < u.K ? s_src[kk] : -1;
        const float2* p = in + (int64_t)(row < 0 ? 0 : row) * nr + n0;
        const float2 v0 = ld2(p, row >= 0 && ok0), v1 = ld2(p + 1, row >= 0 && ok1);
        b[e] = make_float4(v0.x, v0.y, v1.x, v1.y);
      }
      const float2* ap = s_A + (mt * 32 + jj) * lda + kc + 8 * half;
      bf16x8 arh, arl, aih, ail;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float2 av = ap[e];
        __bf16 h, l;
        split_bf16(av.x, h, l);
        arh[e] = h;
        arl[e] = l;
        split_bf16(av.y, h, l);
        aih[e] = h;
        ail[e] = l;
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        bf16x8 bh, bl, sh, sl;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float bt[4] = {b[e].x, b[e].y, b[e].z, b[e].w};
          const float bs[4] = {-b[e].y, b[e].x, -b[e].w, b[e].z};
          __bf16 h, l;
          split_bf16(bt[t], h, l);
          bh[e] = h;
          bl[e] = l;
          split_bf16(bs[t], h, l);
          sh[e] = h;
          sl[e] = l;
        }
        f32x16 c = acc[t];
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, bh, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, bl, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arl, bh, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, sh, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, sl, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ail, sh, c, 0, 0, 0);
        acc[t] = c;
      }
    }
    // epilogue: C row i = 32 mt + 8 (v / 4) + 4 half + v % 4, real column 4 jj + t
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = mt * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
      if (i >= u.M) continue;
      float2* p = out + (int64_t)s_out[i] * nr + n0;
      if (ok0) p[0] = make_float2(acc[0][v], acc[1][v]);
      if (ok1) p[1] = make_float2(acc[2][v], acc[3][v]);
    }
  }
}

// FP32 on v_mfma_f32_16x16x4_f32: 16-row M tiles (a unit of M rows pads to
// a multiple of 16, not 32).  One wavefront per block of 32 right-hand sides
// covers every M tile of the unit (up to TM), so each input row is loaded
// once per wavefront.  Lane (kq = lane / 16, c = lane % 16) feeds K index
// kc + kq: A row 16 mt + c, and the two complex right-hand sides rhs0 + 2c,
// rhs0 + 2c + 1 as real columns 4c + t of N-tiles t = 0..3; D row 4 kq + v,
// column c of tile t is the output of row 16 mt + 4 kq + v, real column
// 4c + t.
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kRhsPerWave16 = 32;
constexpr int kWavesG16 = 4;   // wavefronts per workgroup
constexpr int kRhsIter16 = 8;  // right-hand-side blocks per wavefront: the staged A serves kRhsIter16 kWavesG16 blocks

template <int MODE, bool ADJ, int TM>
__global__ __launch_bounds__(64 * kWavesG16) void apply_gemm16(StageArgs A) {
  extern __shared__ __attribute__((aligned(16))) float2 s_A[];
  __shared__ int s_src[kMaxKg];
  __shared__ int s_out[kMaxMg];
  __shared__ int s_red[2 * kMaxMg];
  const Unit u = stage_unit<MODE, ADJ>(A, s_A, s_src, s_out, s_red);
  const int lane = threadIdx.x & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int kq = lane >> 4, c16 = lane & 15;
  const int tiles = (u.M + 15) / 16;  // <= TM
  const int lda = lda_for(u.K);
  const int64_t nr = A.nrhs;
  const float2* in = static_cast<const float2*>(A.in);
  float2* out = static_cast<float2*>(A.out);
  for (int it = 0; it < A.rhs_iter; ++it) {
    const int64_t rhs0 = ((blockIdx.y * (int64_t)A.rhs_iter + it) * kWavesG16 + w) * kRhsPerWave16;
    if (rhs0 >= nr) return;
    const int64_t n0 = rhs0 + 2 * c16;
    const bool ok0 = n0 < nr, ok1 = n0 + 1 < nr;
    f32x4 acc[TM][4];
#pragma unroll
    for (int mt = 0; mt < TM; ++mt)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[mt][t] = f32x4{};
    for (int kc = 0; kc < u.K; kc += 16) {
      float4 b[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int kk = kc + 4 * e + kq;
        const int row = kk < u.K ? s_src[kk] : -1;
        const float2* p = in + (int64_t)(row < 0 ? 0 : row) * nr + n0;
        const float2 v0 = ld2(p, row >= 0 && ok0), v1 = ld2(p + 1, row >= 0 && ok1);
        b[e] = make_float4(v0.x, v0.y, v1.x, v1.y);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (kc + 4 * e >= u.K) break;  // K steps of 4 wholly past K add nothing
        const float bt[4] = {b[e].x, b[e].y, b[e].z, b[e].w};
        const float bs[4] = {-b[e].y, b[e].x, -b[e].w, b[e].z};
#pragma unroll
        for (int mt = 0; mt < TM; ++mt) {
          if (mt >= tiles) break;
          const float2 av = s_A[(mt * 16 + c16) * lda + kc + 4 * e + kq];  // zero past K (padded to 16)
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bt[t], acc[mt][t], 0, 0, 0);
            acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bs[t], acc[mt][t], 0, 0, 0);
          }
        }
      }
    }
#pragma unroll
    for (int mt = 0; mt < TM; ++mt) {
      if (mt >= tiles) break;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = mt * 16 + 4 * kq + v;
        if (i >= u.M) continue;
        float2* p = out + (int64_t)s_out[i] * nr + n0;
        if (ok0) p[0] = make_float2(acc[mt][0][v], acc[mt][1][v]);
        if (ok1) p[1] = make_float2(acc[mt][2][v], acc[mt][3][v]);
      }
    }
  }
}

// Fused two-stage groups (forward, FP32 MFMA).  Two consecutive V stages
// t, t + 1 (or U stages t, t - 1) form closed groups: the level-t units
// (2 C', P), (2 C' + 1, P) produce exactly the candidate segments of the
// level-(t+1) units (C', 2 P), (C', 2 P + 1) -- part h of stage-1 unit u is
// the outputs of its ID h, which stage-2 unit h reads as its u-th child.
// The U groups are the transpose: level-t units (C, 2 Q + u) write the
// candidates of the level-(t-1) IDs (2 C + h, 2 Q + u), the inputs of the
// level-(t-1) units (2 C + h, Q).  A group's intermediate never leaves the
// registers: stage 1 places part h of unit u on its own TK row tiles, so the
// FP32 16x16x4 accumulator of tile h TK + i (lane (kq, c), register v: row
// 16 i + 4 kq + v of the part, real column 4 c + t) is directly the B
// operand of stage 2 for K index u 16 TK + 16 i + 4 kq + v, once stage 2's A
// carries its columns at those indices.  All four units' A sit in LDS;
// every ID of both levels has rank <= 16 TK.
template <int TK>
struct Fuse1Map {  // stage 1: each ID's (V) or child's (U) rows on TK tiles of their own
  int c0;          // U: candidates of the first child
  __device__ int vrow(int h, int i, int) const { return h * 16 * TK + i; }
  __device__ int vcol(int l) const { return l; }
  __device__ int urow(int l) const { return l < c0 ? l : 16 * TK + l - c0; }
  __device__ int ucol(int h, int b, int k0) const { return (h ? k0 : 0) + b; }
  __device__ Unit vdims(int, int, int c) const { return Unit{32 * TK, c}; }
  __device__ Unit udims(int k0, int k1, int) const { return Unit{32 * TK, k0 + k1}; }
};
template <int TK>
struct Fuse2Map {  // stage 2: inputs at the register tiles of stage 1
  int kf;          // V: candidates of the first child (its rank)
  __device__ int vrow(int h, int i, int k0) const { return (h ? k0 : 0) + i; }
  __device__ int vcol(int l) const { return l < kf ? l : 16 * TK + l - kf; }
  __device__ int urow(int l) const { return l; }
  __device__ int ucol(int h, int b, int) const { return h * 16 * TK + b; }
  __device__ Unit vdims(int k0, int k1, int) const { return Unit{k0 + k1, 32 * TK}; }
  __device__ Unit udims(int, int, int c) const { return Unit{c, 32 * TK}; }
};

constexpr int kWavesF = 8;    // wavefronts per workgroup, 32 right-hand sides each
constexpr int kRhsIterF = 8;  // right-hand-side blocks per wavefront

// The group of workgroup blockIdx.x: its four units' A staged in LDS (stage
// 1 at sA1[u], stage 2 at sA2[h]) with their index lists; returns the
// units' shapes.
template <int MODE, int TK>
__device__ void stage_group(const StageArgs& A1, const StageArgs& A2, int lda1max, int rows2, float2* s_A,
                            int (*s_src)[kMaxKg], int (*s_out)[kMaxMg], int* s_red, Unit* u1, Unit* u2,
                            float2** sA1, float2** sA2) {
  constexpr int R1 = 32 * TK;
  const int64_t g = blockIdx.x;
  int64_t q1[2], q2[2];
  int cut[2];  // V: rank of stage-2 unit h's first child; U: candidates of stage-1 unit u's first child
  if constexpr (MODE == kModeV) {
    const int64_t node = g % A2.nn, P = g / A2.nn;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      q1[u] = P * A1.nn + 2 * node + u;
      q2[u] = (2 * P + u) * A2.nn + node;
      cut[u] = A1.meta[(2 * P + u) * A1.nn + 2 * node].k;
    }
  } else {
    const int64_t node = g % A1.nn, Q = g / A1.nn;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      q1[u] = (2 * Q + u) * A1.nn + node;
      q2[u] = Q * A2.nn + 2 * node + u;
      cut[u] = A2.meta[(2 * Q + u) * A2.nn + 2 * node].k;
    }
  }
  const int lda2 = lda_for(32 * TK);
  sA1[0] = s_A;
  sA1[1] = s_A + R1 * lda1max;
  sA2[0] = s_A + 2 * R1 * lda1max;
  sA2[1] = s_A + 2 * R1 * lda1max + rows2 * lda2;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    u1[u] = stage_unit<MODE, false, float2, Fuse1Map<TK>>(A1, sA1[u], s_src[u], s_out[u], s_red, q1[u], R1,
                                                          Fuse1Map<TK>{MODE == kModeU ? cut[u] : 0});
    u2[u] = stage_unit<MODE, false, float2, Fuse2Map<TK>>(A2, sA2[u], s_src[2 + u], s_out[2 + u], s_red, q2[u],
                                                          rows2, Fuse2Map<TK>{MODE == kModeV ? cut[u] : 0});
  }
}

template <int MODE, int TK>
__global__ __launch_bounds__(64 * kWavesF) void apply_fused2(StageArgs A1, StageArgs A2, int lda1max, int rows2) {
  extern __shared__ __attribute__((aligned(16))) float2 s_A[];
  __shared__ int s_src[4][kMaxKg];
  __shared__ int s_out[4][kMaxMg];
  __shared__ int s_red[2 * kMaxMg];
  constexpr int TM1 = 2 * TK;  // stage-1 tiles per unit
  const int lda2 = lda_for(32 * TK);
  Unit u1[2], u2[2];
  float2 *sA1[2], *sA2[2];
  stage_group<MODE, TK>(A1, A2, lda1max, rows2, s_A, s_src, s_out, s_red, u1, u2, sA1, sA2);
  const int lane = threadIdx.x & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int kq = lane >> 4, c16 = lane & 15;
  const int64_t nr = A1.nrhs;
  const float2* in = static_cast<const float2*>(A1.in);
  float2* out = static_cast<float2*>(A2.out);
  for (int it = 0; it < A1.rhs_iter; ++it) {
    const int64_t rhs0 = ((blockIdx.y * (int64_t)A1.rhs_iter + it) * kWavesF + w) * kRhsPerWave16;
    if (rhs0 >= nr) return;
    const int64_t n0 = rhs0 + 2 * c16;
    const bool ok0 = n0 < nr, ok1 = n0 + 1 < nr;
    f32x4 acc1[2][TM1][4];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int mt = 0; mt < TM1; ++mt)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc1[u][mt][t] = f32x4{};
      const int K = u1[u].K, lda = lda_for(K);
      const float2* sA = sA1[u];
      // the rows of K block kc, four per lane (zero past K)
      auto load = [&](float4* b, int kc) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int kk = kc + 4 * e + kq;
          const int row = kk < K ? s_src[u][kk] : -1;
          const float2* p = in + (int64_t)(row < 0 ? 0 : row) * nr + n0;
          const float2 v0 = ld2(p, row >= 0 && ok0), v1 = ld2(p + 1, row >= 0 && ok1);
          b[e] = make_float4(v0.x, v0.y, v1.x, v1.y);
        }
      };
      float4 b[4], bn[4];
      load(b, 0);
      for (int kc = 0; kc < K; kc += 16) {
        if (kc + 16 < K) load(bn, kc + 16);  // next block in flight during this one's products
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (kc + 4 * e >= K) break;
          const float bt[4] = {b[e].x, b[e].y, b[e].z, b[e].w};
          const float bs[4] = {-b[e].y, b[e].x, -b[e].w, b[e].z};
#pragma unroll
          for (int mt = 0; mt < TM1; ++mt) {
            const float2 av = sA[(mt * 16 + c16) * lda + kc + 4 * e + kq];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              acc1[u][mt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bt[t], acc1[u][mt][t], 0, 0, 0);
              acc1[u][mt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bs[t], acc1[u][mt][t], 0, 0, 0);
            }
          }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) b[e] = bn[e];
      }
    }
    // stage 2: unit h reads part h of both stage-1 units from the registers
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int tiles = (u2[h].M + 15) / 16;  // <= 4
      const float2* sA = sA2[h];
      f32x4 acc[4][4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[mt][t] = f32x4{};
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int i = 0; i < TK; ++i)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const f32x4* d = acc1[u][h * TK + i];
            const float bt[4] = {d[0][v], d[1][v], d[2][v], d[3][v]};
            const float bs[4] = {-d[1][v], d[0][v], -d[3][v], d[2][v]};
            const int col = u * 16 * TK + 16 * i + 4 * kq + v;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
              if (mt >= tiles) break;
              const float2 av = sA[(mt * 16 + c16) * lda2 + col];
#pragma unroll
              for (int t = 0; t < 4; ++t) {
                acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bt[t], acc[mt][t], 0, 0, 0);
                acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bs[t], acc[mt][t], 0, 0, 0);
              }
            }
          }
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        if (mt >= tiles) break;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = mt * 16 + 4 * kq + v;
          if (i >= u2[h].M) continue;
          float2* p = out + (int64_t)s_out[2 + h][i] * nr + n0;
          if (ok0) p[0] = make_float2(acc[mt][0][v], acc[mt][1][v]);
          if (ok1) p[1] = make_float2(acc[mt][2][v], acc[mt][3][v]);
        }
      }
    }
  }
}

// The fused groups with BF16 hi/lo split products on
// v_mfma_f32_16x16x16_bf16 (FP32 accumulation).  Lane (kq, c) feeds K
// indices kc + 4 kq .. kc + 4 kq + 3 of A row 16 mt + c and of its two
// complex right-hand sides; the 16x16 accumulator layout (register v: row
// 4 kq + v, column c) is then exactly stage 2's B operand for one 16-row
// tile.  Each complex product is A_re B' + A_im B~ with both factors split,
// a b ~= a_hi b_hi + a_hi b_lo + a_lo b_hi.
typedef short s16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split4(const float* x, s16x4& hi, s16x4& lo) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const __bf16 h = (__bf16)x[e];
    const __bf16 l = (__bf16)(x[e] - (float)h);
    hi[e] = __builtin_bit_cast(short, h);
    lo[e] = __builtin_bit_cast(short, l);
  }
}

// A staged block rewritten in place, four K entries at a time, as the split
// operands (re hi, re lo, im hi, im lo; four BF16 each): 32 bytes, the size
// of the four complex FP32 entries they replace.  kcols is a multiple of 16.
__device__ void presplit(float2* sA, int rows, int lda, int kcols) {
  const int groups = kcols / 4;
  for (int e = threadIdx.x; e < rows * groups; e += blockDim.x) {
    float2* g = sA + (e / groups) * lda + 4 * (e % groups);
    float re[4], im[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      re[i] = g[i].x;
      im[i] = g[i].y;
    }
    s16x4 part[4];
    split4(re, part[0], part[1]);
    split4(im, part[2], part[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i) reinterpret_cast<s16x4*>(g)[i] = part[i];
  }
}

struct BOp {  // the split B operand of one K step: N-tile t, and its (re, im) -> (-im, re) rotation
  s16x4 h[4], l[4], sh[4], sl[4];
};

__device__ __forceinline__ BOp make_bop(const float (*b)[4]) {
  BOp o;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    float bs[4];
    const int tp = t ^ 1;  // the other part of the same right-hand side
#pragma unroll
    for (int e = 0; e < 4; ++e) bs[e] = (t & 1) ? b[tp][e] : -b[tp][e];
    split4(b[t], o.h[t], o.l[t]);
    split4(bs, o.sh[t], o.sl[t]);
  }
  return o;
}

// acc[t] += A (4 K of one row, pre-split at ap) times B
__device__ __forceinline__ void mma_bf16(const float2* ap, const BOp& B, f32x4* acc) {
  const s16x4* g = reinterpret_cast<const s16x4*>(ap);
  const s16x4 arh = g[0], arl = g[1], aih = g[2], ail = g[3];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 c = acc[t];
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(arh, B.h[t], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(arh, B.l[t], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(arl, B.h[t], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aih, B.sh[t], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aih, B.sl[t], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ail, B.sh[t], c, 0, 0, 0);
    acc[t] = c;
  }
}

template <int MODE, int TK>
__global__ __launch_bounds__(64 * kWavesF) void apply_fused2b(StageArgs A1, StageArgs A2, int lda1max, int rows2) {
  extern __shared__ __attribute__((aligned(16))) float2 s_A[];
  __shared__ int s_src[4][kMaxKg];
  __shared__ int s_out[4][kMaxMg];
  __shared__ int s_red[2 * kMaxMg];
  constexpr int TM1 = 2 * TK;
  const int lda2 = lda_for(32 * TK);
  Unit u1[2], u2[2];
  float2 *sA1[2], *sA2[2];
  stage_group<MODE, TK>(A1, A2, lda1max, rows2, s_A, s_src, s_out, s_red, u1, u2, sA1, sA2);
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    presplit(sA1[u], 32 * TK, lda_for(u1[u].K), lda_for(u1[u].K) - 2);
    presplit(sA2[u], rows2, lda2, 32 * TK);
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int kq = lane >> 4, c16 = lane & 15;
  const int64_t nr = A1.nrhs;
  const float2* in = static_cast<const float2*>(A1.in);
  float2* out = static_cast<float2*>(A2.out);
  for (int it = 0; it < A1.rhs_iter; ++it) {
    const int64_t rhs0 = ((blockIdx.y * (int64_t)A1.rhs_iter + it) * kWavesF + w) * kRhsPerWave16;
    if (rhs0 >= nr) return;
    const int64_t n0 = rhs0 + 2 * c16;
    const bool ok0 = n0 < nr, ok1 = n0 + 1 < nr;
    f32x4 acc1[2][TM1][4];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int mt = 0; mt < TM1; ++mt)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc1[u][mt][t] = f32x4{};
      const int K = u1[u].K, lda = lda_for(K);
      const float2* sA = sA1[u];
      for (int kc = 0; kc < K; kc += 16) {
        float b[4][4];  // N-tile t (re, im of the two right-hand sides), K index kc + 4 kq + e
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int kk = kc + 4 * kq + e;
          const int row = kk < K ? s_src[u][kk] : -1;
          const float2* p = in + (int64_t)(row < 0 ? 0 : row) * nr + n0;
          const float2 v0 = ld2(p, row >= 0 && ok0), v1 = ld2(p + 1, row >= 0 && ok1);
          b[0][e] = v0.x;
          b[1][e] = v0.y;
          b[2][e] = v1.x;
          b[3][e] = v1.y;
        }
        const BOp B = make_bop(b);
#pragma unroll
        for (int mt = 0; mt < TM1; ++mt) mma_bf16(sA + (mt * 16 + c16) * lda + kc + 4 * kq, B, acc1[u][mt]);
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int tiles = (u2[h].M + 15) / 16;  // <= 4
      const float2* sA = sA2[h];
      f32x4 acc[4][4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[mt][t] = f32x4{};
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int i = 0; i < TK; ++i) {
          const f32x4* d = acc1[u][h * TK + i];
          float b[4][4];
#pragma unroll
          for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int e = 0; e < 4; ++e) b[t][e] = d[t][e];
          const BOp B = make_bop(b);
          const int col = u * 16 * TK + 16 * i + 4 * kq;
#pragma unroll
          for (int mt = 0; mt < 4; ++mt) {
            if (mt >= tiles) break;
            mma_bf16(sA + (mt * 16 + c16) * lda2 + col, B, acc[mt]);
          }
        }
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        if (mt >= tiles) break;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = mt * 16 + 4 * kq + v;
          if (i >= u2[h].M) continue;
          float2* p = out + (int64_t)s_out[2 + h][i] * nr + n0;
          if (ok0) p[0] = make_float2(acc[mt][0][v], acc[mt][1][v]);
          if (ok1) p[1] = make_float2(acc[mt][2][v], acc[mt][3][v]);
        }
      }
    }
  }
}

// FP64 on v_mfma_f64_16x16x4_f64 (complex128 data): the FP32 kernel's
// operand layout with one complex right-hand side per lane, so a wavefront
// covers 16 right-hand sides in two N-tiles (real and imaginary parts); lane
// (kq, c) feeds K index kc + kq and right-hand side rhs0 + c.  The f64
// instruction orders D differently from the f32 one: register v of lane
// (kq, c) holds row 4 v + kq, column c, i.e. output row 16 mt + 4 v + kq,
// part t of tile t.
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int kRhsPerWaveD = 16;
constexpr int kWavesD = 8;     // wavefronts per workgroup
constexpr int kRhsIterD = 8;   // right-hand-side blocks per wavefront: A serves kRhsIterD kWavesD blocks

template <int MODE, bool ADJ, int TM>
__global__ __launch_bounds__(64 * kWavesD) void apply_gemm16d(StageArgs A) {
  extern __shared__ __attribute__((aligned(16))) double2 s_Ad[];
  __shared__ int s_src[kMaxKg];
  __shared__ int s_out[kMaxMg];
  __shared__ int s_red[2 * kMaxMg];
  const Unit u = stage_unit<MODE, ADJ, double2>(A, s_Ad, s_src, s_out, s_red);
  const int lane = threadIdx.x & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int kq = lane >> 4, c16 = lane & 15;
  const int tiles = (u.M + 15) / 16;  // <= TM
  const int lda = lda_for(u.K);
  const int64_t nr = A.nrhs;
  const double2* in = static_cast<const double2*>(A.in);
  double2* out = static_cast<double2*>(A.out);
  for (int it = 0; it < A.rhs_iter; ++it) {
    const int64_t rhs0 = ((blockIdx.y * (int64_t)A.rhs_iter + it) * kWavesD + w) * kRhsPerWaveD;
    if (rhs0 >= nr) return;
    const int64_t n0 = rhs0 + c16;
    const bool ok = n0 < nr;
    f64x4 acc[TM][2];
#pragma unroll
    for (int mt = 0; mt < TM; ++mt)
#pragma unroll
      for (int t = 0; t < 2; ++t) acc[mt][t] = f64x4{};
    auto load = [&](double2* b, int kc) {  // the rows of K block kc, four per lane (zero past K)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int kk = kc + 4 * e + kq;
        const int row = kk < u.K ? s_src[kk] : -1;
        b[e] = (row >= 0 && ok) ? in[(int64_t)row * nr + n0] : make_double2(0.0, 0.0);
      }
    };
    double2 b[4], bn[4];
    load(b, 0);
    for (int kc = 0; kc < u.K; kc += 16) {
      if (kc + 16 < u.K) load(bn, kc + 16);  // next block in flight during this one's products
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (kc + 4 * e >= u.K) break;  // K steps of 4 wholly past K add nothing
        const double bt[2] = {b[e].x, b[e].y};
        const double bs[2] = {-b[e].y, b[e].x};
#pragma unroll
        for (int mt = 0; mt < TM; ++mt) {
          if (mt >= tiles) break;
          const double2 av = s_Ad[(mt * 16 + c16) * lda + kc + 4 * e + kq];  // zero past K (padded to 16)
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            acc[mt][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bt[t], acc[mt][t], 0, 0, 0);
            acc[mt][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bs[t], acc[mt][t], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) b[e] = bn[e];
    }
#pragma unroll
    for (int mt = 0; mt < TM; ++mt) {
      if (mt >= tiles) break;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = mt * 16 + 4 * v + kq;  // the f64 instruction's D: register v holds row 4 v + lane / 16
        if (i >= u.M || !ok) continue;
        out[(int64_t)s_out[i] * nr + n0] = make_double2(acc[mt][0][v], acc[mt][1][v]);
      }
    }
  }
}

}  // namespace

size_t gemm_lds_bytes(int kmax_unit, int mmax_unit, int prec) {
  const int rows = prec == kGemmBf16 ? ((mmax_unit + 31) & ~31) : ((mmax_unit + 15) & ~15);
  const size_t elem = prec == kGemmF64 ? sizeof(double2) : sizeof(float2);
  return (size_t)rows * (size_t)(((kmax_unit + 15) & ~15) + 2) * elem;
}

size_t fused2_lds_bytes(int tk, int kmax1, int mmax2) {
  const int r1 = 32 * tk, r2 = (mmax2 + 15) & ~15;
  return sizeof(float2) * (2 * (size_t)r1 * lda_for(kmax1) + 2 * (size_t)r2 * lda_for(32 * tk));
}

hipError_t launch_apply_fused2(const StageArgs& a1, const StageArgs& a2, int mode, int tk, int kmax1, int mmax2,
                               int prec, hipStream_t st) {
  if (a1.n <= 0 || a1.nrhs <= 0) return hipSuccess;
  if ((tk != 1 && tk != 2) || kmax1 < 1 || kmax1 > kMaxKg || mmax2 < 1 || mmax2 > 64 || (a1.n & 1) ||
      (prec != kGemmF32 && prec != kGemmBf16) ||
      a1.rhs_iter < 0 || a1.rhs_iter > kMaxRhsIter)
    return hipErrorInvalidValue;
  const size_t lds = fused2_lds_bytes(tk, kmax1, mmax2);
  if (lds > kMaxFusedLds) return hipErrorInvalidValue;
  const int rows2 = (mmax2 + 15) & ~15, lda1 = lda_for(kmax1);
  StageArgs b1 = a1;
  if (b1.rhs_iter == 0) b1.rhs_iter = kRhsIterF;
  const int64_t per_block = (int64_t)b1.rhs_iter * kWavesF * kRhsPerWave16;
  const dim3 grid((unsigned)(a1.n / 2), (unsigned)((a1.nrhs + per_block - 1) / per_block));
#define IDBF_FUSED2(KERNEL, M, TK)                                                                   \
  do {                                                                                               \
    if (lds > (size_t(64) << 10)) {                                                                  \
      hipError_t e_ = hipFuncSetAttribute(reinterpret_cast<const void*>(&KERNEL<M, TK>),             \
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);     \
      if (e_ != hipSuccess) return e_;                                                               \
    }                                                                                                \
    hipLaunchKernelGGL((KERNEL<M, TK>), grid, dim3(64 * kWavesF), lds, st, b1, a2, lda1, rows2);     \
  } while (0)
#define IDBF_FUSED2_ALL(KERNEL)                                                                      \
  do {                                                                                               \
    if (mode == kModeV) {                                                                            \
      if (tk == 1) IDBF_FUSED2(KERNEL, kModeV, 1); else IDBF_FUSED2(KERNEL, kModeV, 2);              \
    } else {                                                                                         \
      if (tk == 1) IDBF_FUSED2(KERNEL, kModeU, 1); else IDBF_FUSED2(KERNEL, kModeU, 2);              \
    }                                                                                                \
  } while (0)
  if (prec == kGemmBf16) IDBF_FUSED2_ALL(apply_fused2b);
  else IDBF_FUSED2_ALL(apply_fused2);
#undef IDBF_FUSED2_ALL
#undef IDBF_FUSED2
  return hipGetLastError();
}

hipError_t launch_apply_gemm(const StageArgs& a0, int mode, int kmax_unit, int mmax_unit, int prec,
                             hipStream_t st, bool adj) {
  if (a0.n <= 0 || a0.nrhs <= 0) return hipSuccess;
  if (kmax_unit < 1 || kmax_unit > kMaxKg || mmax_unit < 1 || mmax_unit > kMaxMg) return hipErrorInvalidValue;
  if (gemm_lds_bytes(kmax_unit, mmax_unit, prec) > kMaxGemmLds) return hipErrorInvalidValue;
  if (a0.rhs_iter < 0 || a0.rhs_iter > kMaxRhsIter) return hipErrorInvalidValue;
  StageArgs a = a0;
  const bool bf16 = prec == kGemmBf16;
  if (prec == kGemmF64) {  // FP64: the FP32 kernel's layout, 16 right-hand sides per wavefront
    a.gemm_rows = (mmax_unit + 15) & ~15;
    if (a.rhs_iter == 0) a.rhs_iter = kRhsIterD;
    const int64_t per_block = (int64_t)a.rhs_iter * kWavesD * kRhsPerWaveD;
    const dim3 grid((unsigned)a.n, (unsigned)((a.nrhs + per_block - 1) / per_block));
    const size_t lds = gemm_lds_bytes(kmax_unit, mmax_unit, prec);
#define IDBF_GEMM16D(M, J, TM)                                                                       \
  do {                                                                                               \
    if (lds > (size_t(64) << 10)) {                                                                  \
      hipError_t e_ = hipFuncSetAttribute(reinterpret_cast<const void*>(&apply_gemm16d<M, J, TM>),   \
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);     \
      if (e_ != hipSuccess) return e_;                                                               \
    }                                                                                                \
    hipLaunchKernelGGL((apply_gemm16d<M, J, TM>), grid, dim3(64 * kWavesD), lds, st, a);             \
  } while (0)
#define IDBF_GEMM16D_TM(M, J)                                                                        \
  do {                                                                                               \
    if (a.gemm_rows <= 64) IDBF_GEMM16D(M, J, 4); else IDBF_GEMM16D(M, J, 8);                        \
  } while (0)
    switch (mode) {
      case kModeV: if (adj) IDBF_GEMM16D_TM(kModeV, true); else IDBF_GEMM16D_TM(kModeV, false); break;
      case kModeS: if (adj) IDBF_GEMM16D_TM(kModeS, true); else IDBF_GEMM16D_TM(kModeS, false); break;
      default: if (adj) IDBF_GEMM16D_TM(kModeU, true); else IDBF_GEMM16D_TM(kModeU, false); break;
    }
#undef IDBF_GEMM16D_TM
#undef IDBF_GEMM16D
    return hipGetLastError();
  }
  if (!bf16) {  // FP32: 16-row tiles, one wavefront per 32 right-hand sides over all of them
    a.gemm_rows = (mmax_unit + 15) & ~15;
    if (a.rhs_iter == 0) a.rhs_iter = kRhsIter16;
    const int64_t per_block = (int64_t)a.rhs_iter * kWavesG16 * kRhsPerWave16;
    const dim3 grid((unsigned)a.n, (unsigned)((a.nrhs + per_block - 1) / per_block));
    const size_t lds = (size_t)a.gemm_rows * (size_t)(((kmax_unit + 15) & ~15) + 2) * sizeof(float2);
#define IDBF_GEMM16(M, J, TM)                                                                        \
  do {                                                                                               \
    if (lds > (size_t(64) << 10)) {                                                                  \
      hipError_t e_ = hipFuncSetAttribute(reinterpret_cast<const void*>(&apply_gemm16<M, J, TM>),    \
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);     \
      if (e_ != hipSuccess) return e_;                                                               \
    }                                                                                                \
    hipLaunchKernelGGL((apply_gemm16<M, J, TM>), grid, dim3(64 * kWavesG16), lds, st, a);            \
  } while (0)
#define IDBF_GEMM16_TM(M, J)                                                                         \
  do {                                                                                               \
    if (a.gemm_rows <= 64) IDBF_GEMM16(M, J, 4); else IDBF_GEMM16(M, J, 8);                          \
  } while (0)
    switch (mode) {
      case kModeV: if (adj) IDBF_GEMM16_TM(kModeV, true); else IDBF_GEMM16_TM(kModeV, false); break;
      case kModeS: if (adj) IDBF_GEMM16_TM(kModeS, true); else IDBF_GEMM16_TM(kModeS, false); break;
      default: if (adj) IDBF_GEMM16_TM(kModeU, true); else IDBF_GEMM16_TM(kModeU, false); break;
    }
#undef IDBF_GEMM16_TM
#undef IDBF_GEMM16
    return hipGetLastError();
  }
  a.gemm_rows = (mmax_unit + 31) & ~31;  // BF16 split: 32-row tiles
  const int tiles_m = a.gemm_rows / 32;
  const int blocks_rhs = std::max(1, kWavesG / tiles_m);
  if (a.rhs_iter == 0) a.rhs_iter = kRhsIterB;
  const int64_t per_block = (int64_t)blocks_rhs * kRhsPerWave * a.rhs_iter;
  const dim3 grid((unsigned)a.n, (unsigned)((a.nrhs + per_block - 1) / per_block));
  const dim3 block(64 * blocks_rhs * tiles_m);
  const size_t lds = (size_t)a.gemm_rows * (size_t)(((kmax_unit + 15) & ~15) + 2) * sizeof(float2);
#define IDBF_GEMM(M, J)                                                                              \
  do {                                                                                               \
    if (lds > (size_t(64) << 10)) {                                                                  \
      hipError_t e_ = hipFuncSetAttribute(reinterpret_cast<const void*>(&apply_gemm_bf16<M, J>),     \
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);     \
      if (e_ != hipSuccess) return e_;                                                               \
    }                                                                                                \
    hipLaunchKernelGGL((apply_gemm_bf16<M, J>), grid, block, lds, st, a);                            \
  } while (0)
  switch (mode) {
    case kModeV: if (adj) IDBF_GEMM(kModeV, true); else IDBF_GEMM(kModeV, false); break;
    case kModeS: if (adj) IDBF_GEMM(kModeS, true); else IDBF_GEMM(kModeS, false); break;
    default: if (adj) IDBF_GEMM(kModeU, true); else IDBF_GEMM(kModeU, false); break;
  }
#undef IDBF_GEMM
  return hipGetLastError();
}

}  // namespace idbf
