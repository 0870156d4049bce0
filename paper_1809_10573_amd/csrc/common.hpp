// Shared device helpers of the IDBF library: complex arithmetic, the kernel
// entry K(x, xi) = exp(2 pi i Phi(x, xi)), wavefront reductions and host
// error plumbing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/idbf.h"

namespace idbf {

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kMaxCand = 128;    // candidates per ID (two lanes' worth above 64)
constexpr int kMaxSamples = 128; // sampled rows per ID: s = min(t c, |allowed|, 128)
constexpr int kMaxRank = 64;     // rank of an ID
constexpr int kSlot = 4096;      // T entries per ID in slot layout (max k (c - k))
constexpr double kPivotTie = 1e-8;

struct PhaseDev {
  int kind;
  double c0, a, freq, cdiv;
};

// ---------------------------------------------------------------- complex
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// acc + a * b
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 acc) {
  acc.x = __builtin_fma(a.x, b.x, acc.x);
  acc.x = __builtin_fma(-a.y, b.y, acc.x);
  acc.y = __builtin_fma(a.x, b.y, acc.y);
  acc.y = __builtin_fma(a.y, b.x, acc.y);
  return acc;
}
// acc + conj(a) * b
__device__ __forceinline__ double2 cfma_conj(double2 a, double2 b, double2 acc) {
  acc.x = __builtin_fma(a.x, b.x, acc.x);
  acc.x = __builtin_fma(a.y, b.y, acc.x);
  acc.y = __builtin_fma(a.x, b.y, acc.y);
  acc.y = __builtin_fma(-a.y, b.x, acc.y);
  return acc;
}
__device__ __forceinline__ double cabs2(double2 a) { return __builtin_fma(a.x, a.x, a.y * a.y); }

__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 acc) {
  acc.x = __builtin_fmaf(a.x, b.x, acc.x);
  acc.x = __builtin_fmaf(-a.y, b.y, acc.x);
  acc.y = __builtin_fmaf(a.x, b.y, acc.y);
  acc.y = __builtin_fmaf(a.y, b.x, acc.y);
  return acc;
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }

template <typename C> struct Real;
template <> struct Real<double2> { using type = double; };
template <> struct Real<float2> { using type = float; };

__device__ __forceinline__ double2 czero(double2) { return make_double2(0.0, 0.0); }
__device__ __forceinline__ float2 czero(float2) { return make_float2(0.f, 0.f); }

// ---------------------------------------------------------------- phase
// a*b - round(a*b), to within one rounding of the exact product: p = fl(a b),
// e = a b - p exactly (fused multiply-add), p - rint(p) is exact for |p| < 2^52.
__device__ __forceinline__ double frac_of_product(double a, double b) {
  double p = a * b;
  double e = __builtin_fma(a, b, -p);
  return (p - __builtin_rint(p)) + e;
}

// c(x) = (c0 + a sin(2 pi freq x)) / cdiv  (Example 1's amplitude of |xi|)
__device__ __forceinline__ double amplitude_shift(const PhaseDev& ph, double x) {
  return (ph.c0 + ph.a * sinpi(2.0 * ph.freq * x)) / ph.cdiv;
}

// K(x, xi) = exp(2 pi i Phi(x, xi)); cx = c(x) (unused for the DFT kernel).
// The phase is reduced to [-1/2, 1/2] turns before the exponential.
__device__ __forceinline__ double2 kernel_entry(const PhaseDev& ph, double x, double cx, double xi) {
  double th;
  if (ph.kind == IDBF_PHASE_DFT) {
    th = -frac_of_product(x, xi);
  } else {
    th = frac_of_product(x, xi) + frac_of_product(cx, __builtin_fabs(xi));
  }
  th -= __builtin_rint(th);
  double s, c;
  sincospi(2.0 * th, &s, &c);
  return make_double2(c, s);
}

// ---------------------------------------------------------------- wave ops
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, kWave));
  return v;
}
__device__ __forceinline__ double readlane(double v, int lane) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double2 readlane(double2 v, int lane) {
  return make_double2(readlane(v.x, lane), readlane(v.y, lane));
}
__device__ __forceinline__ uint64_t lanes_below(int lane) {
  return lane >= 64 ? ~0ull : ((1ull << lane) - 1ull);
}

}  // namespace idbf

// ------------------------------------------------------------------ host side
namespace idbf {
void set_error(const char* fmt, ...);
}

#define IDBF_HIP_CHECK(call)                                                          \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      idbf::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                      __LINE__);                                                      \
      return IDBF_EHIP;                                                               \
    }                                                                                 \
  } while (0)
