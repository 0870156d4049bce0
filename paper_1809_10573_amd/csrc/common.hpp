// Shared device helpers of the IDBF library: complex arithmetic, the kernel
// entry K(x, xi) = exp(2 pi i Phi(x, xi)) or J_0(x xi), wavefront reductions
// and host error plumbing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/idbf.h"

namespace idbf {

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kMaxCand = 128;    // candidates per ID (two lanes' worth above 64)
constexpr int kMaxSamples = 256; // sampled rows per ID: s = min(t c, |allowed|) <= 256
constexpr int kQrRows = 128;     // rows the register-resident QR kernels hold; taller sample
                                 // blocks are first reduced to their c x c triangular factor
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

// ---------------------------------------------------------------- J_0
// J_0 for Example 2's Schloemilch kernel K(g, w) = J_0(g w), by two
// published methods, in the operation order of the oracle's and without
// fused multiply-adds, so the two agree to the rounding of sin, cos, sqrt:
//  z < 25:  Miller's normalized backward recurrence, f_{n-1} = (2n/z) f_n -
//           f_{n+1} from f_{n0} = 1e-30 at n0 = 2 floor((z + 40)/2), and
//           J_0 = f_0 / (f_0 + 2 sum_{k>=1} f_{2k}) (A&S 9.12, 9.1.46);
//  z >= 25: Hankel's asymptotic expansion (A&S 9.2.5, 9.2.9, 9.2.10) with 11
//           terms of P and Q: J_0 = ((P + Q) cos z + (P - Q) sin z) / sqrt(pi z),
//           z reduced modulo pi/2 by a three-part split C1 + C2 + C3 of pi/2
//           (27 and 29 significant bits, then 53: n C1, n C2 exact for
//           n < 2^24; Cody and Waite).
constexpr int kHankelTerms = 11;
struct HankelB {
  double b[2 * kHankelTerms];
};
// b_k = (1 3 ... (2k-1))^2 / (k! 8^k) by b_k = b_{k-1} (2k-1)^2 / (8k)
constexpr HankelB hankel_b() {
  HankelB h{};
  h.b[0] = 1.0;
  for (int k = 1; k < 2 * kHankelTerms; ++k) h.b[k] = h.b[k - 1] * (double)((2 * k - 1) * (2 * k - 1)) / (double)(8 * k);
  return h;
}

__device__ inline double j0_miller(double z) {
#pragma clang fp contract(off)
  const int n0 = 2 * (int)floor((z + 40.0) / 2.0);
  const double r = 2.0 / z;
  double f = 1e-30, fn = 0.0, s = 1e-30;  // n0 is even: J_{n0} opens the sum
  for (int n = n0; n >= 1; --n) {
    const double fp = ((double)n * r) * f - fn;  // f_{n-1}
    fn = f;
    f = fp;
    if (((n - 1) & 1) == 0 && n - 1 >= 2) s = s + f;
    if (fabs(f) > 1e200) {
      f = f * 1e-200;
      fn = fn * 1e-200;
      s = s * 1e-200;
    }
  }
  return f / (f + 2.0 * s);
}

__device__ inline double j0_hankel(double z) {
#pragma clang fp contract(off)
  constexpr HankelB H = hankel_b();
  constexpr double kC1 = 0x1.921fb54000000p+0, kC2 = 0x1.10b4611000000p-30, kC3 = 0x1.4c4c6628b80dcp-59;
  constexpr double kTwoOverPi = 2.0 / M_PI;
  const double u = 1.0 / (z * z);
  constexpr double sgn_last = ((kHankelTerms - 1) & 1) ? -1.0 : 1.0;
  double p = sgn_last * H.b[2 * kHankelTerms - 2], q = sgn_last * H.b[2 * kHankelTerms - 1];
#pragma unroll
  for (int m = kHankelTerms - 2; m >= 0; --m) {
    const double sg = (m & 1) ? -1.0 : 1.0;
    p = p * u + sg * H.b[2 * m];
    q = q * u + sg * H.b[2 * m + 1];
  }
  q = -q / z;
  const double n = rint(z * kTwoOverPi);
  const double r = ((z - n * kC1) - n * kC2) - n * kC3;
  double sr, cr;
  sincos(r, &sr, &cr);
  const int quad = (int)((long long)n & 3);
  const double cz = quad == 0 ? cr : quad == 1 ? -sr : quad == 2 ? -cr : sr;
  const double sz = quad == 0 ? sr : quad == 1 ? cr : quad == 2 ? -sr : -cr;
  return ((p + q) * cz + (p - q) * sz) / sqrt(M_PI * z);
}

__device__ inline double bessel_j0(double z) {
  z = fabs(z);
  if (z == 0.0) return 1.0;
  return z < 25.0 ? j0_miller(z) : j0_hankel(z);
}

// K(x, xi) = exp(2 pi i Phi(x, xi)); cx = c(x) (unused for the DFT kernel);
// the Schloemilch kernel J_0(x xi) is real.
// The phase is reduced to [-1/2, 1/2] turns before the exponential.
__device__ __forceinline__ double2 kernel_entry(const PhaseDev& ph, double x, double cx, double xi) {
  if (ph.kind == IDBF_PHASE_J0) return make_double2(bessel_j0(x * xi), 0.0);
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
