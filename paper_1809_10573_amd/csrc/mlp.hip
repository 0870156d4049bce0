// Rank-proposal network (not in the paper: the learned-proposal extension of
// the construction).  y = W3^T relu(W2^T relu(W1^T x + b1) + b2) + b3 with
// n_in = 8 inputs and H hidden units per layer, FP32.  Parameters are one
// flat vector: W1 (n_in x H, row-major), b1, W2 (H x H), b2, W3 (H), b3.
//
// Forward: a workgroup takes kTile samples; layer-1 and layer-2 activations
// live in LDS, each thread owns one hidden unit for kTile / (256 / H) samples
// and reads its W2 column once per tile.
// Backward (mean squared error / 2): one kernel per gradient block, each
// output element summed over the batch by one thread in a fixed order, so the
// gradient is deterministic (no atomics).
#include "kernels.hpp"

namespace idbf {

namespace {

constexpr int kTile = 64;      // samples per forward workgroup
constexpr int kMaxHidden = 128;

struct Layout {
  int n_in, H;
  __host__ __device__ int w1() const { return 0; }
  __host__ __device__ int b1() const { return n_in * H; }
  __host__ __device__ int w2() const { return n_in * H + H; }
  __host__ __device__ int b2() const { return n_in * H + H + H * H; }
  __host__ __device__ int w3() const { return n_in * H + 2 * H + H * H; }
  __host__ __device__ int b3() const { return n_in * H + 3 * H + H * H; }
};

// z1, z2 (optional, n x H each) keep the pre-activations for the backward pass.
__global__ __launch_bounds__(256) void mlp_fwd_kernel(const float* P, Layout lo, const float* X, int64_t n,
                                                      float* y, float* z1, float* z2) {
  __shared__ float s_h1[kTile][kMaxHidden + 1];
  __shared__ float s_h2[kTile][kMaxHidden + 1];
  __shared__ float s_x[kTile][8];
  const int H = lo.H, n_in = lo.n_in;
  const int64_t s0 = blockIdx.x * (int64_t)kTile;
  const int ns = (int)min((int64_t)kTile, n - s0);
  for (int e = threadIdx.x; e < kTile * n_in; e += blockDim.x) {
    const int s = e / n_in, i = e % n_in;
    s_x[s][i] = (s < ns) ? X[(s0 + s) * n_in + i] : 0.f;
  }
  __syncthreads();
  const int h = threadIdx.x % H, g = threadIdx.x / H, G = blockDim.x / H;  // G sample groups
  // layer 1
  {
    float w[8];
    for (int i = 0; i < n_in; ++i) w[i] = P[lo.w1() + i * H + h];
    const float b = P[lo.b1() + h];
    for (int s = g; s < kTile; s += G) {
      float acc = b;
      for (int i = 0; i < n_in; ++i) acc = fmaf(s_x[s][i], w[i], acc);
      if (z1 && s < ns) z1[(s0 + s) * H + h] = acc;
      s_h1[s][h] = fmaxf(acc, 0.f);
    }
  }
  __syncthreads();
  // layer 2: thread (h, g) accumulates samples g, g + G, ...
  {
    constexpr int kPer = kTile;  // upper bound of samples per thread (G >= 1)
    float acc[kPer];
    const int cnt = (kTile + G - 1 - g) / G;
    const float b = P[lo.b2() + h];
#pragma unroll
    for (int j = 0; j < kPer; ++j) acc[j] = b;
    for (int k = 0; k < H; ++k) {
      const float wk = P[lo.w2() + k * H + h];
#pragma unroll
      for (int j = 0; j < kPer; ++j)
        if (j < cnt) acc[j] = fmaf(s_h1[g + j * G][k], wk, acc[j]);
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j)
      if (j < cnt) {
        const int s = g + j * G;
        if (z2 && s < ns) z2[(s0 + s) * H + h] = acc[j];
        s_h2[s][h] = fmaxf(acc[j], 0.f);
      }
  }
  __syncthreads();
  // layer 3: one thread per sample
  if ((int)threadIdx.x < ns) {
    const int s = threadIdx.x;
    float acc = P[lo.b3()];
    for (int k = 0; k < H; ++k) acc = fmaf(s_h2[s][k], P[lo.w3() + k], acc);
    y[s0 + s] = acc;
  }
}

// d_out[s] = (y[s] - t[s]) / n; loss parts: (y - t)^2 per sample
__global__ void mlp_dout_kernel(const float* y, const float* t, int64_t n, float* d_out, float* sq) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  const float r = y[s] - t[s];
  d_out[s] = r / (float)n;
  sq[s] = r * r;
}

// d_z2[s][h] = d_out[s] W3[h] [z2 > 0]
__global__ void mlp_dz2_kernel(const float* P, Layout lo, const float* d_out, const float* z2, int64_t n,
                               float* dz2) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * lo.H) return;
  const int64_t s = e / lo.H;
  const int h = (int)(e % lo.H);
  dz2[e] = (z2[e] > 0.f) ? d_out[s] * P[lo.w3() + h] : 0.f;
}

// d_z1[s][k] = sum_h d_z2[s][h] W2[k][h]  [z1 > 0]
__global__ void mlp_dz1_kernel(const float* P, Layout lo, const float* dz2, const float* z1, int64_t n,
                               float* dz1) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * lo.H) return;
  const int64_t s = e / lo.H;
  const int k = (int)(e % lo.H);
  float acc = 0.f;
  if (z1[e] > 0.f)
    for (int h = 0; h < lo.H; ++h) acc = fmaf(dz2[s * lo.H + h], P[lo.w2() + k * lo.H + h], acc);
  dz1[e] = acc;
}

// Parameter gradients, one thread per parameter, batch sums in sample order:
//   W1[i][h] = sum_s x[s][i] dz1[s][h]     b1[h] = sum_s dz1[s][h]
//   W2[k][h] = sum_s relu(z1[s][k]) dz2[s][h]   b2[h] = sum_s dz2[s][h]
//   W3[h]    = sum_s relu(z2[s][h]) d_out[s]    b3 = sum_s d_out[s]
__global__ void mlp_grad_kernel(Layout lo, const float* X, const float* z1, const float* z2, const float* dz1,
                                const float* dz2, const float* d_out, int64_t n, float* G) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int H = lo.H;
  if (p >= lo.b3() + 1) return;
  float acc = 0.f;
  if (p < lo.b1()) {
    const int i = p / H, h = p % H;
    for (int64_t s = 0; s < n; ++s) acc = fmaf(X[s * lo.n_in + i], dz1[s * H + h], acc);
  } else if (p < lo.w2()) {
    const int h = p - lo.b1();
    for (int64_t s = 0; s < n; ++s) acc += dz1[s * H + h];
  } else if (p < lo.b2()) {
    const int k = (p - lo.w2()) / H, h = (p - lo.w2()) % H;
    for (int64_t s = 0; s < n; ++s) acc = fmaf(fmaxf(z1[s * H + k], 0.f), dz2[s * H + h], acc);
  } else if (p < lo.w3()) {
    const int h = p - lo.b2();
    for (int64_t s = 0; s < n; ++s) acc += dz2[s * H + h];
  } else if (p < lo.b3()) {
    const int h = p - lo.w3();
    for (int64_t s = 0; s < n; ++s) acc = fmaf(fmaxf(z2[s * H + h], 0.f), d_out[s], acc);
  } else {
    for (int64_t s = 0; s < n; ++s) acc += d_out[s];
  }
  G[p] = acc;
}

__global__ void adam_kernel(float* P, const float* G, float* M, float* V, int np, float lr, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const float g = G[p];
  const float m = 0.9f * M[p] + 0.1f * g;
  const float v = 0.999f * V[p] + 0.001f * g * g;
  M[p] = m;
  V[p] = v;
  P[p] -= lr * (m / c1) / (sqrtf(v / c2) + 1e-8f);
}

__global__ void gather_rows_kernel(const float* X, const float* t, const int32_t* idx, int64_t n, int n_in,
                                   float* Xb, float* tb) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int64_t src = idx[e];
  for (int i = 0; i < n_in; ++i) Xb[e * n_in + i] = X[src * n_in + i];
  tb[e] = t[src];
}

// sum of v[0..n) by one workgroup, fixed order per thread then a tree
__global__ __launch_bounds__(256) void sum_kernel(const float* v, int64_t n, float* out) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += v[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) s[threadIdx.x] += s[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = (float)s[0];
}

inline unsigned blocks(int64_t n, int per = 256) { return (unsigned)((n + per - 1) / per); }

}  // namespace

int mlp_param_count(int n_in, int hidden) { return Layout{n_in, hidden}.b3() + 1; }

hipError_t launch_mlp_forward(const float* P, int n_in, int hidden, const float* X, int64_t n, float* y,
                              float* z1, float* z2, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n_in > 8 || hidden > kMaxHidden || 256 % hidden != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mlp_fwd_kernel, dim3(blocks(n, kTile)), dim3(256), 0, st, P, Layout{n_in, hidden}, X, n, y,
                     z1, z2);
  return hipGetLastError();
}

// ws: 4 n H + 2 n floats of scratch
hipError_t launch_mlp_loss_grad(const float* P, int n_in, int hidden, const float* X, const float* t, int64_t n,
                                float* G, float* loss_dev, float* ws, hipStream_t st) {
  if (n <= 0) return hipErrorInvalidValue;
  const Layout lo{n_in, hidden};
  float* z1 = ws;
  float* z2 = z1 + n * hidden;
  float* dz1 = z2 + n * hidden;
  float* dz2 = dz1 + n * hidden;
  float* y = dz2 + n * hidden;
  float* d_out = y + n;
  hipError_t e = launch_mlp_forward(P, n_in, hidden, X, n, y, z1, z2, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_dout_kernel, dim3(blocks(n)), dim3(256), 0, st, y, t, n, d_out, y);  // y <- (y - t)^2
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, y, n, loss_dev);
  hipLaunchKernelGGL(mlp_dz2_kernel, dim3(blocks(n * hidden)), dim3(256), 0, st, P, lo, d_out, z2, n, dz2);
  hipLaunchKernelGGL(mlp_dz1_kernel, dim3(blocks(n * hidden)), dim3(256), 0, st, P, lo, dz2, z1, n, dz1);
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(blocks(lo.b3() + 1)), dim3(256), 0, st, lo, X, z1, z2, dz1, dz2, d_out, n,
                     G);
  return hipGetLastError();
}

hipError_t launch_adam(float* P, const float* G, float* M, float* V, int np, float lr, int step, hipStream_t st) {
  const float c1 = 1.f - powf(0.9f, (float)step), c2 = 1.f - powf(0.999f, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks(np)), dim3(256), 0, st, P, G, M, V, np, lr, c1, c2);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const float* X, const float* t, const int32_t* idx, int64_t n, int n_in, float* Xb,
                              float* tb, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks(n)), dim3(256), 0, st, X, t, idx, n, n_in, Xb, tb);
  return hipGetLastError();
}

}  // namespace idbf
