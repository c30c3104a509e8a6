// Device-side helpers shared by the Debye kernels (gfx950).
//
// FP64 trigonometry for the per-pair set-up of the q recurrence.  The set-up
// runs once per atom pair and q chunk, the recurrence itself runs in FP32, so
// these helpers favour clear, branch-free FP64 code over speed:
//   * sin/cos on |x| <= pi/4 by their Taylor series in Horner form;
//   * additive range reduction by Cody & Waite (1980) with pi/2 and pi split
//     into three parts of 33 significant bits each, so k * part is exact for
//     |k| < 2^20 (|argument| < 1.6e6 rad).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sas {

// pi/2 = kPio2A + kPio2B + kPio2C (each part rounded to 33 bits); pi = 2 x that.
constexpr double kPio2A = 0x1.921fb54400000p+0;
constexpr double kPio2B = 0x1.0b4611a600000p-34;
constexpr double kPio2C = 0x1.3198a2e037073p-69;
constexpr double kPiA = 0x1.921fb54400000p+1;
constexpr double kPiB = 0x1.0b4611a600000p-33;
constexpr double kPiC = 0x1.3198a2e037073p-68;
constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;
constexpr double kOneOverPi = 0x1.45f306dc9c883p-2;
constexpr double kTwoPi = 0x1.921fb54442d18p+2;

// 1/n! for the Taylor coefficients (n! is exact in FP64 up to 22!).
constexpr double fact(int n) { return n <= 1 ? 1.0 : n * fact(n - 1); }

struct SinCos {
  double s, c;
};

// Taylor coefficients, evaluated at compile time.  Terms through x^11 (sin)
// and x^12 (cos) leave a truncation below 1e-11 relative for |x| <= pi/4;
// every value derived from them is rounded to FP32 (6e-8) afterwards, so the
// truncation adds no measurable bias.
constexpr double kS3 = -1.0 / fact(3), kS5 = 1.0 / fact(5), kS7 = -1.0 / fact(7), kS9 = 1.0 / fact(9);
constexpr double kS11 = -1.0 / fact(11);
constexpr double kC2 = -1.0 / fact(2), kC4 = 1.0 / fact(4), kC6 = -1.0 / fact(6), kC8 = 1.0 / fact(8);
constexpr double kC10 = -1.0 / fact(10), kC12 = 1.0 / fact(12);

// a * b + c with the constant c taken from an SGPR pair.  Written as inline
// assembly because the compiler otherwise keeps every FP64 polynomial
// coefficient in a VGPR pair, which costs the forward kernel its second wave
// per SIMD.
__device__ __forceinline__ double fma_vvs(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}
__device__ __forceinline__ double mul_vs(double a, double b) {
  double r;
  asm("v_mul_f64 %0, %1, %2" : "=v"(r) : "v"(a), "s"(b));
  return r;
}
__device__ __forceinline__ double add_vs(double a, double b) {
  double r;
  asm("v_add_f64 %0, %1, %2" : "=v"(r) : "v"(a), "s"(b));
  return r;
}

// sin and cos of |x| <= pi/4.
__device__ __forceinline__ SinCos sincos_small(double x) {
  const double x2 = x * x;
  double ps = add_vs(mul_vs(x2, kS11), kS9);
  ps = fma_vvs(ps, x2, kS7);
  ps = fma_vvs(ps, x2, kS5);
  ps = fma_vvs(ps, x2, kS3);
  double pc = add_vs(mul_vs(x2, kC12), kC10);
  pc = fma_vvs(pc, x2, kC8);
  pc = fma_vvs(pc, x2, kC6);
  pc = fma_vvs(pc, x2, kC4);
  pc = fma_vvs(pc, x2, kC2);
  SinCos r;
  r.s = fma(x * x2, ps, x);
  r.c = fma(x2, pc, 1.0);
  return r;
}

// sin and cos of any |x| < 1.6e6 (quadrant reduction by pi/2).
__device__ __forceinline__ SinCos sincos_any(double x) {
  const double k = rint(x * kTwoOverPi);
  double y = fma(-k, kPio2A, x);
  y = fma(-k, kPio2B, y);
  y = fma(-k, kPio2C, y);
  const SinCos b = sincos_small(y);
  const int quad = static_cast<int>(static_cast<int64_t>(k) & 3);
  SinCos r;
  // x = y + quad * pi/2
  r.s = (quad & 1) ? b.c : b.s;
  r.c = (quad & 1) ? b.s : b.c;
  if (quad == 1 || quad == 2) r.c = -r.c;
  if (quad & 2) r.s = -r.s;
  return r;
}

// 1/sqrt(a) for a > 0 in FP64: hardware estimate refined by one Newton step.
// The step squares the estimate's relative error, leaving it below 1e-13:
// enough for q r to 1e-9 rad at r = 10^4 A, far below the FP32 rounding of
// every value derived from it.
__device__ __forceinline__ double rsqrt_f64(double a) {
  const double y = __builtin_amdgcn_rsq(a);
  return y * fma(-0.5 * a, y * y, 1.5);
}

// +1.0f or -1.0f for an even or odd integer k held in a double.
__device__ __forceinline__ float parity_sign(double k) {
  const unsigned bits = static_cast<unsigned>(static_cast<int>(k)) << 31;
  return __uint_as_float(bits ^ 0x3f800000u);
}

// Direct form: acc + sin(q r) * w, for any q >= 0, from rp = r / pi.
// t = q * rp is rounded to the nearest integer k by adding 1.5 * 2^52 in the
// same FMA (the sum's low word then holds k), x = t - k lies in [-1/2, 1/2]
// and is exact to FP64 rounding, and sin(q r) = (-1)^k sin(pi x) =
// sin(pi (-1)^k x): the parity of k flips the sign bit of x.  sin(pi x) is
// x * P(x^2) with P the degree-4 minimax fit of relative error 5e-9
// (coefficients rounded to FP32, 4e-8; fit_sinpi.py beside this file
// reproduces them and the cosine's below).  Four FP64 and eight FP32
// instructions per call.
constexpr double kRoundMagic = 0x1.8p+52;
constexpr float kSinPi0 = 0x1.921fb6p+1f, kSinPi1 = -0x1.4abbc2p+2f, kSinPi2 = 0x1.4668b0p+1f,
                kSinPi3 = -0x1.324ccap-1f, kSinPi4 = 0x1.3daff6p-4f;

constexpr float kCosPi0 = 0x1.000000p+0f, kCosPi1 = -0x1.3bd3ccp+2f, kCosPi2 = 0x1.03c1e4p+2f,
                kCosPi3 = -0x1.55d076p+0f, kCosPi4 = 0x1.e126f2p-3f, kCosPi5 = -0x1.8fb73ep-6f;

// sin(q r) and cos(q r) in FP32 for the direct adjoint, by the same reduction:
// sin(q r) = sin(pi (-1)^k x), cos(q r) = (-1)^k cos(pi x), cos(pi x) = Q(x^2)
// with Q the degree-5 minimax fit of absolute error 2e-10 (2e-8 with FP32
// coefficients).
struct SinCosF {
  float s, c;
};

__device__ __forceinline__ SinCosF sincos_qr(double q, double rp) {
  const double s = fma(q, rp, kRoundMagic);
  const double k = s - kRoundMagic;
  const float x = static_cast<float>(fma(q, rp, -k));
  const unsigned flip = static_cast<unsigned>(__double2loint(s)) << 31;
  const float xs = __uint_as_float(__float_as_uint(x) + flip);
  const float y = x * x;
  float p = fmaf(y, kSinPi4, kSinPi3);
  p = fmaf(p, y, kSinPi2);
  p = fmaf(p, y, kSinPi1);
  p = fmaf(p, y, kSinPi0);
  float c = fmaf(y, kCosPi5, kCosPi4);
  c = fmaf(c, y, kCosPi3);
  c = fmaf(c, y, kCosPi2);
  c = fmaf(c, y, kCosPi1);
  c = fmaf(c, y, kCosPi0);
  SinCosF r;
  r.s = xs * p;
  r.c = __uint_as_float(__float_as_uint(c) + flip);
  return r;
}

__device__ __forceinline__ float sin_qr_acc(double q, double rp, float w, float acc) {
  const double s = fma(q, rp, kRoundMagic);
  const double k = s - kRoundMagic;
  const float x = static_cast<float>(fma(q, rp, -k));
  const unsigned lo = static_cast<unsigned>(__double2loint(s));
  const float xs = __uint_as_float(__float_as_uint(x) + (lo << 31));
  const float y = xs * xs;
  float p = fmaf(y, kSinPi4, kSinPi3);
  p = fmaf(p, y, kSinPi2);
  p = fmaf(p, y, kSinPi1);
  p = fmaf(p, y, kSinPi0);
  return fmaf(xs * w, p, acc);
}

}  // namespace sas
