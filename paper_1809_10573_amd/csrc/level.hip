// Level plumbing of the construction (Sections 2.2-2.4): per-ID candidate and
// allowed index segments, prefix scans that size the packed factor arrays,
// skeleton compaction, and the middle factor's block list.
//
// IDs of level t are numbered q = partner * 2^(L-t+1) + node.  In that order
//  - the candidates of a level-t ID (the merged skeletons of its node's two
//    children for the same parent partner) are one contiguous segment of the
//    level t-1 skeleton list of the same side, and
//  - its allowed points (skeletons of the other side for every descendant at
//    the right depth, with the partner the tree algebra fixes) are one
//    contiguous segment of the other side's list,
// so every ID reads two contiguous index segments.
#include <algorithm>

#include "kernels.hpp"

namespace idbf {

namespace {

__global__ void desc_kernel(DescArgs A) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= A.n_ids) return;
  const int t = A.t, L = A.L;
  const int64_t nn = 1ll << (L - t + 1);
  const int64_t node = q % nn, partner = q / nn;
  int32_t cb, cl, ab, al;
  if (t == 1) {
    cb = (int32_t)(node * A.leaf);
    cl = A.leaf;
  } else {
    // children 2 node, 2 node + 1 of the parent partner at level t-1
    const int64_t qp = (partner >> 1) * (2 * nn) + 2 * node;
    cb = A.prev_skel_off[qp];
    cl = A.prev_skel_off[qp + 2] - cb;
  }
  if (A.side == IDBF_SIDE_U) {
    if (t == 1) {
      ab = (int32_t)(partner * (A.N / 2));
      al = (int32_t)(A.N / 2);
    } else {
      // V_{t-1} IDs (C'' below partner at depth L-t+2, ancestor of node at depth t-1)
      const int sh = L - 2 * t + 2;
      const int64_t lo = (node >> sh) * (2 * nn) + (partner << sh);
      ab = A.allow_skel_off[lo];
      al = A.allow_skel_off[lo + (1ll << sh)] - ab;
    }
  } else {
    // U_t IDs (R'' below partner at depth L-t+1, ancestor of node at depth t)
    const int sh = L - 2 * t + 1;
    const int64_t lo = (node >> sh) * nn + (partner << sh);
    ab = A.allow_skel_off[lo];
    al = A.allow_skel_off[lo + (1ll << sh)] - ab;
  }
  A.cand_beg[q] = cb;
  A.cand_len[q] = cl;
  A.allow_beg[q] = ab;
  A.allow_len[q] = al;
  // Section 2.1: t k rows with k = |cand|, at most the allowed set (above
  // kMaxSamples the construction stops with IDBF_EUNSUPPORTED)
  const int64_t s = min((int64_t)A.oversample * cl, (int64_t)al);
  int64_t kcap = min((int64_t)cl, s);
  if (A.kmax > 0) kcap = min(kcap, (int64_t)A.kmax);
  kcap = min(kcap, (int64_t)kMaxRank);
  const int64_t half = cl / 2;
  const int64_t bound = (kcap >= half) ? half * (cl - half) : kcap * (cl - kcap);
  A.t_bound[q] = (bound + 1) & ~int64_t(1);  // even: every T block starts 16-byte aligned
  A.samples[q] = (int32_t)s;
}

// Exclusive prefix sums over a level's values (off[0 .. n], off[n] = total)
// with their sum, max and min and the max of an optional second array, in
// three launches: coalesced tile reductions, one workgroup scanning the tile
// partials (stats and tile offsets), and a rescan of every tile.
constexpr int kScanThreads = 256;

__device__ __forceinline__ int64_t wave_incl_sum(int64_t x, int lane) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int64_t y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  return x;
}

template <typename V>
__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const V* v, int64_t n, const int32_t* aux,
                                                                  int64_t tile, int64_t* ws) {
  __shared__ int64_t s_p[4][kScanThreads / kWave];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const int64_t beg = blockIdx.x * tile, end = min(n, beg + tile);
  int64_t sum = 0, mx = INT64_MIN, mn = INT64_MAX, ax = INT64_MIN;
  for (int64_t i = beg + tid; i < end; i += kScanThreads) {
    const int64_t x = (int64_t)v[i];
    sum += x;
    mx = max(mx, x);
    mn = min(mn, x);
    if (aux) ax = max(ax, (int64_t)aux[i]);
  }
  for (int d = kWave / 2; d > 0; d >>= 1) {
    sum += __shfl_xor(sum, d, kWave);
    mx = max(mx, __shfl_xor(mx, d, kWave));
    mn = min(mn, __shfl_xor(mn, d, kWave));
    ax = max(ax, __shfl_xor(ax, d, kWave));
  }
  if (lane == 0) {
    s_p[0][w] = sum;
    s_p[1][w] = mx;
    s_p[2][w] = mn;
    s_p[3][w] = ax;
  }
  __syncthreads();
  if (tid == 0) {
    for (int k = 1; k < kScanThreads / kWave; ++k) {
      sum += s_p[0][k];
      mx = max(mx, s_p[1][k]);
      mn = min(mn, s_p[2][k]);
      ax = max(ax, s_p[3][k]);
    }
    int64_t* o = ws + 4 * blockIdx.x;
    o[0] = sum;
    o[1] = mx;
    o[2] = mn;
    o[3] = ax;
  }
}

// One workgroup: exclusive offsets of the nb <= kScanMaxTiles tile sums (to
// ws[4 kScanMaxTiles + b]), the totals to stats, and off[n].
template <typename O>
__global__ __launch_bounds__(kScanMaxTiles) void scan_partials_kernel(int nb, int64_t n, int64_t* ws,
                                                                     int64_t* stats, O* off) {
  __shared__ int64_t s_w[4][kScanMaxTiles / kWave];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const bool on = tid < nb;
  const int64_t x = on ? ws[4 * tid] : 0;
  const int64_t incl = wave_incl_sum(x, lane);
  int64_t mx = on ? ws[4 * tid + 1] : INT64_MIN, mn = on ? ws[4 * tid + 2] : INT64_MAX;
  int64_t ax = on ? ws[4 * tid + 3] : INT64_MIN;
  for (int d = kWave / 2; d > 0; d >>= 1) {
    mx = max(mx, __shfl_xor(mx, d, kWave));
    mn = min(mn, __shfl_xor(mn, d, kWave));
    ax = max(ax, __shfl_xor(ax, d, kWave));
  }
  if (lane == kWave - 1) s_w[0][w] = incl;
  if (lane == 0) {
    s_w[1][w] = mx;
    s_w[2][w] = mn;
    s_w[3][w] = ax;
  }
  __syncthreads();
  int64_t before = 0;
  for (int k = 0; k < w; ++k) before += s_w[0][k];
  if (on) ws[4 * kScanMaxTiles + tid] = before + incl - x;
  if (tid == 0) {
    int64_t tot = 0;
    for (int k = 0; k < kScanMaxTiles / kWave; ++k) {
      tot += s_w[0][k];
      mx = max(mx, s_w[1][k]);
      mn = min(mn, s_w[2][k]);
      ax = max(ax, s_w[3][k]);
    }
    stats[0] = tot;
    stats[1] = mx;
    stats[2] = mn;
    stats[3] = ax;
    off[n] = (O)tot;
  }
}

template <typename V, typename O>
__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(const V* v, int64_t n, int64_t tile,
                                                                 const int64_t* ws, O* off) {
  __shared__ int64_t s_w[kScanThreads / kWave];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const int64_t beg = blockIdx.x * tile, end = min(n, beg + tile);
  int64_t carry = ws[4 * kScanMaxTiles + blockIdx.x];
  for (int64_t c0 = beg; c0 < end; c0 += kScanThreads) {
    const int64_t i = c0 + tid;
    const int64_t x = i < end ? (int64_t)v[i] : 0;
    const int64_t incl = wave_incl_sum(x, lane);
    if (lane == kWave - 1) s_w[w] = incl;
    __syncthreads();
    int64_t before = 0, total = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / kWave; ++k) {
      if (k < w) before += s_w[k];
      total += s_w[k];
    }
    if (i < end) off[i] = (O)(carry + before + incl - x);
    carry += total;
    __syncthreads();  // s_w is rewritten by the next chunk
  }
}

__global__ void iota_kernel(int32_t* p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

__global__ void compact_kernel(const int32_t* scratch, const int32_t* rank, const int32_t* off,
                               int64_t n_ids, const double* base, int32_t* out, double* out_coord) {
  const int64_t q = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (q >= n_ids) return;
  if (lane < rank[q]) {
    const int32_t g = scratch[q * kMaxCand + lane];
    out[off[q] + lane] = g;
    out_coord[off[q] + lane] = base[g];
  }
}

__device__ unsigned long long middle_desc_one(const MiddleDescArgs& A, int64_t b) {
  const int H = A.H, d = A.L - A.H + 1, sh = d - H;
  const int64_t nsub = 1ll << sh;
  const int64_t qu = b / nsub, j = b % nsub;
  const int64_t r = qu & ((1ll << d) - 1), cpart = qu >> d;   // U_H ID (node r, partner cpart)
  const int64_t cnode = (cpart << sh) + j;                      // column node at depth d
  const int64_t qv = (r >> sh) * (1ll << d) + cnode;            // V_H ID (node cnode, partner r >> sh)
  const int32_t rb = A.u_off[qu], rl = A.u_off[qu + 1] - rb;
  const int32_t cb = A.v_off[qv], cl = A.v_off[qv + 1] - cb;
  A.rbeg[b] = rb;
  A.rlen[b] = rl;
  A.cbeg[b] = cb;
  A.clen[b] = cl;
  A.size[b] = ((int64_t)rl * cl + 1) & ~int64_t(1);  // even: blocks start 16-byte aligned
  return (unsigned long long)rl * cl;
}

__global__ __launch_bounds__(256) void middle_desc_kernel(MiddleDescArgs A) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  unsigned long long used = 0;
  if (b < A.n_blocks) used = middle_desc_one(A, b);
  for (int off = 32; off > 0; off >>= 1) used += __shfl_xor(used, off, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0 && used) atomicAdd(A.nnz, used);
}

// One workgroup per block; lanes over rows, loop over columns.
__global__ __launch_bounds__(256) void sample_blocks_kernel(SampleBlocksArgs A) {
  const int64_t b = blockIdx.x;
  const int rl = A.rlen[b], cl = A.clen[b];
  const int32_t* ri = A.row_idx + A.rbeg[b];
  const int32_t* ci = A.col_idx + A.cbeg[b];
  const int64_t off = A.off[b];
  const bool fio = (A.ph.kind == IDBF_PHASE_FIO);
  for (int64_t e = threadIdx.x; e < (int64_t)rl * cl; e += blockDim.x) {
    const int i = (int)(e % rl), jc = (int)(e / rl);
    const double x = A.X[ri[i]];
    const double cx = fio ? amplitude_shift(A.ph, x) : 0.0;
    const double2 v = kernel_entry(A.ph, x, cx, A.Om[ci[jc]]);
    A.out128[off + e] = v;
    if (A.out64) A.out64[off + e] = make_float2((float)v.x, (float)v.y);
  }
}

__global__ void sample_dense_kernel(PhaseDev ph, const double* X, const double* Om, const int32_t* rows,
                                    int64_t nr, const int32_t* cols, int64_t nc, double2* out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nr * nc) return;
  const int64_t i = e / nc, j = e % nc;
  const double x = X[rows[i]];
  const double cx = (ph.kind == IDBF_PHASE_FIO) ? amplitude_shift(ph, x) : 0.0;
  out[e] = kernel_entry(ph, x, cx, Om[cols[j]]);
}

__global__ __launch_bounds__(256) void id_work_kernel(const int32_t* rank, const int32_t* cand_len,
                                                      const int32_t* samples, const int32_t* keep, int64_t n,
                                                      unsigned long long* out) {
  __shared__ unsigned long long s_w[3][256];
  unsigned long long fl = 0, te = 0, se = 0;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
    if (keep && !keep[q]) continue;
    const int64_t k = rank[q], c = cand_len[q], sq = samples[q];
    unsigned long long h = 0;
    for (int64_t j = 0; j < k; ++j) h += (unsigned long long)((sq - j) * (c - j));
    fl += 16 * h + 4 * (unsigned long long)(k * k * (c - k));
    te += (unsigned long long)(k * (c - k));
    se += (unsigned long long)(sq * c);
  }
  s_w[0][threadIdx.x] = fl;
  s_w[1][threadIdx.x] = te;
  s_w[2][threadIdx.x] = se;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d)
      for (int m = 0; m < 3; ++m) s_w[m][threadIdx.x] += s_w[m][threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x < 3) atomicAdd(out + threadIdx.x, s_w[threadIdx.x][0]);
}

__global__ __launch_bounds__(256) void bucket_count_kernel(const int32_t* samples, const int32_t* cand_len,
                                                           const int32_t* keep, int64_t n,
                                                           unsigned long long* counts) {
  __shared__ unsigned int s_c[kBucketSlots];
  if (threadIdx.x < kBucketSlots) s_c[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    if (!keep || keep[q]) {
      atomicAdd(&s_c[qr_bucket(cand_len[q], samples[q])], 1u);
      if (is_tall(samples[q])) atomicAdd(&s_c[kQrBuckets], 1u);
    }
  __syncthreads();
  if (threadIdx.x < kBucketSlots && s_c[threadIdx.x])
    atomicAdd(counts + threadIdx.x, (unsigned long long)s_c[threadIdx.x]);
}

// Slots are reserved per workgroup (one global atomic per bucket and
// workgroup), then handed out inside the workgroup with LDS atomics.
__global__ __launch_bounds__(256) void bucket_fill_kernel(const int32_t* samples, const int32_t* cand_len,
                                                          const int32_t* keep, int64_t n,
                                                          unsigned long long* cursors, int32_t* order, int32_t* tall) {
  __shared__ unsigned int s_cnt[kBucketSlots];
  __shared__ unsigned long long s_base[kBucketSlots];
  if (threadIdx.x < kBucketSlots) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool in = q < n && (!keep || keep[q]);
  const bool tl = in && is_tall(samples[q]);
  int b = 0;
  unsigned int local = 0, local_t = 0;
  if (in) {
    b = qr_bucket(cand_len[q], samples[q]);
    local = atomicAdd(&s_cnt[b], 1u);
    if (tl) local_t = atomicAdd(&s_cnt[kQrBuckets], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kBucketSlots && s_cnt[threadIdx.x])
    s_base[threadIdx.x] = atomicAdd(cursors + threadIdx.x, (unsigned long long)s_cnt[threadIdx.x]);
  __syncthreads();
  if (in) order[s_base[b] + local] = (int32_t)q;
  if (tl) tall[s_base[kQrBuckets] + local_t] = (int32_t)q;
}

__global__ void pack_meta_kernel(const int64_t* t_off, const uint64_t* mask, const int32_t* cand_beg,
                                 const int32_t* skel_off, const int32_t* cand_len, const int32_t* rank, int64_t n,
                                 ApplyMeta* out) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= n) return;
  out[q] = ApplyMeta{t_off[q], mask[2 * q], mask[2 * q + 1], cand_beg[q], skel_off[q], cand_len[q], rank[q]};
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_desc(const DescArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(desc_kernel, dim3(blocks_for(a.n_ids, 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename V, typename O>
hipError_t launch_scan(const V* v, int64_t n, O* off, const int32_t* aux, int64_t* stats, int64_t* ws,
                       hipStream_t st) {
  // tiles: at most kScanMaxTiles, each a whole number of kScanThreads chunks
  const int64_t chunks = std::max<int64_t>(1, (n + kScanThreads - 1) / kScanThreads);
  const int64_t per = (chunks + kScanMaxTiles - 1) / kScanMaxTiles;
  const int64_t tile = per * kScanThreads;
  const int nb = (int)std::max<int64_t>(1, (n + tile - 1) / tile);
  hipLaunchKernelGGL((scan_reduce_kernel<V>), dim3(nb), dim3(kScanThreads), 0, st, v, n, aux, tile, ws);
  hipLaunchKernelGGL((scan_partials_kernel<O>), dim3(1), dim3(kScanMaxTiles), 0, st, nb, n, ws, stats, off);
  hipLaunchKernelGGL((scan_apply_kernel<V, O>), dim3(nb), dim3(kScanThreads), 0, st, v, n, tile, ws, off);
  return hipGetLastError();
}

hipError_t launch_scan_i64(const int64_t* v, int64_t n, int64_t* off, const int32_t* aux, int64_t* stats,
                           int64_t* ws, hipStream_t st) {
  return launch_scan(v, n, off, aux, stats, ws, st);
}

hipError_t launch_scan_i32(const int32_t* v, int64_t n, int32_t* off, const int32_t* aux, int64_t* stats,
                           int64_t* ws, hipStream_t st) {
  return launch_scan(v, n, off, aux, stats, ws, st);
}

hipError_t launch_iota(int32_t* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(iota_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_compact_skel(const int32_t* scratch, const int32_t* rank, const int32_t* off, int64_t n_ids,
                               const double* base, int32_t* out, double* out_coord, hipStream_t st) {
  if (n_ids <= 0) return hipSuccess;
  hipLaunchKernelGGL(compact_kernel, dim3(blocks_for(n_ids, 4)), dim3(256), 0, st, scratch, rank, off, n_ids,
                     base, out, out_coord);
  return hipGetLastError();
}

hipError_t launch_id_work(const int32_t* rank, const int32_t* cand_len, const int32_t* samples, const int32_t* keep, int64_t n,
                          unsigned long long* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(id_work_kernel, dim3(std::min<unsigned>(blocks_for(n, 256), 1024u)), dim3(256), 0, st, rank,
                     cand_len, samples, keep, n, out);
  return hipGetLastError();
}

hipError_t launch_bucket_count(const int32_t* samples, const int32_t* cand_len, const int32_t* keep, int64_t n,
                               unsigned long long* counts, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(bucket_count_kernel, dim3(std::min<unsigned>(blocks_for(n, 256), 1024u)), dim3(256), 0, st,
                     samples, cand_len, keep, n, counts);
  return hipGetLastError();
}

hipError_t launch_bucket_fill(const int32_t* samples, const int32_t* cand_len, const int32_t* keep, int64_t n,
                              unsigned long long* cursors, int32_t* order, int32_t* tall, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(bucket_fill_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, samples, cand_len, keep, n,
                     cursors, order, tall);
  return hipGetLastError();
}

hipError_t launch_pack_meta(const int64_t* t_off, const uint64_t* mask, const int32_t* cand_beg,
                            const int32_t* skel_off, const int32_t* cand_len, const int32_t* rank, int64_t n,
                            ApplyMeta* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(pack_meta_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, t_off, mask, cand_beg, skel_off,
                     cand_len, rank, n, out);
  return hipGetLastError();
}

hipError_t launch_middle_desc(const MiddleDescArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(middle_desc_kernel, dim3(blocks_for(a.n_blocks, 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_sample_blocks(const SampleBlocksArgs& a, hipStream_t st) {
  if (a.n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(sample_blocks_kernel, dim3((unsigned)a.n_blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_sample_dense(const PhaseDev& ph, const double* X, const double* Om, const int32_t* rows,
                               int64_t nr, const int32_t* cols, int64_t nc, double2* out, hipStream_t st) {
  if (nr * nc <= 0) return hipSuccess;
  hipLaunchKernelGGL(sample_dense_kernel, dim3(blocks_for(nr * nc, 256)), dim3(256), 0, st, ph, X, Om, rows, nr,
                     cols, nc, out);
  return hipGetLastError();
}

}  // namespace idbf
