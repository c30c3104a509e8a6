// Device-side helpers shared by the Debye kernels (gfx950).
//
// FP64 trigonometry for the per-pair set-up of the q recurrence.  The set-up
// runs once per atom pair and q chunk, the recurrence itself runs in FP32, and
// every value the set-up produces is rounded to FP32 once, so these helpers
// need relative accuracy well below FP32's 6e-8, not full FP64:
//   * sin/cos on |x| <= pi/4 by minimax polynomials of relative error 5e-12
//     and 7e-11 (fit_halfangle.py beside this file derives them);
//   * additive range reduction by Cody & Waite (1980) with pi/2 split into
//     parts of 33 significant bits, so k * part is exact for |k| < 2^20; the
//     quotient k comes from one FMA that adds 1.5 * 2^52, which leaves k in
//     the low word of the sum (its parity without a conversion).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sas {

// pi/2 = kPio2A + kPio2B + kPio2C (each part rounded to 33 bits).
constexpr double kPio2A = 0x1.921fb54400000p+0;
constexpr double kPio2B = 0x1.0b4611a600000p-34;
constexpr double kPio2C = 0x1.3198a2e037073p-69;
constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;
constexpr double kOneOverPi = 0x1.45f306dc9c883p-2;
constexpr double kTwoPi = 0x1.921fb54442d18p+2;
// Adding 1.5 * 2^52 rounds a double of magnitude below 2^51 to an integer k
// and leaves k (two's complement) in the low word of the sum.
constexpr double kRoundMagic = 0x1.8p+52;

struct SinCos {
  double s, c;
};

// sin(x) = x + x y P(y), cos(x) = 1 + y Q(y), y = x^2, on |x| <= pi/4 (1 + 1e-4):
// minimax coefficients of P and Q (fit_halfangle.py).
constexpr double kHs1 = -0x1.5555554c6ffb7p-3, kHs2 = 0x1.111108690b3d5p-7, kHs3 = -0x1.a00f7e144cf98p-13,
                 kHs4 = 0x1.6cd1b07f8e9f5p-19;
constexpr double kHc1 = -0x1.ffffffcb77e03p-2, kHc2 = 0x1.55553c74b32fap-5, kHc3 = -0x1.6c07efdea28fcp-10,
                 kHc4 = 0x1.991642d7d2148p-16;

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

// sin and cos of |x| <= pi/4 (1 + 1e-4).
__device__ __forceinline__ SinCos sincos_small(double x) {
  const double y = x * x;
  double ps = add_vs(mul_vs(y, kHs4), kHs3);
  ps = fma_vvs(ps, y, kHs2);
  ps = fma_vvs(ps, y, kHs1);
  double pc = add_vs(mul_vs(y, kHc4), kHc3);
  pc = fma_vvs(pc, y, kHc2);
  pc = fma_vvs(pc, y, kHc1);
  SinCos r;
  r.s = fma(x * y, ps, x);
  r.c = fma(y, pc, 1.0);
  return r;
}

// x = k pi/2 + h with |h| <= pi/4 (1 + 1e-4) for |x| < 1.6e6: returns h and
// writes the quotient's low word (k mod 2^32) to *klo.  Two parts of pi/2
// for the set-up's step angles (|k| < 2^20; the third part changes h by
// |k| 2e-21), three for seed angles.
template <int PARTS>
__device__ __forceinline__ double reduce_pio2(double x, int* klo) {
  const double s = fma(x, kTwoOverPi, kRoundMagic);
  const double k = s - kRoundMagic;
  double h = fma(-k, kPio2A, x);
  h = fma(-k, kPio2B, h);
  if constexpr (PARTS > 2) h = fma(-k, kPio2C, h);
  *klo = __double2loint(s);
  return h;
}

// sin and cos of any |x| < 1.6e6 (quadrant reduction by pi/2).
__device__ __forceinline__ SinCos sincos_any(double x) {
  int quad = 0;
  const SinCos b = sincos_small(reduce_pio2<3>(x, &quad));
  SinCos r;
  // x = h + quad * pi/2
  r.s = (quad & 1) ? b.c : b.s;
  r.c = (quad & 1) ? b.s : b.c;
  if ((quad & 3) == 1 || (quad & 3) == 2) r.c = -r.c;
  if (quad & 2) r.s = -r.s;
  return r;
}

// The step angle of a pair's recurrence: for hd = dq r / 2, dq r = k pi + dp
// with |dp| <= pi/2 (1 + 1e-4).  Returns sin and cos of dp/2 and writes
// (-1)^k to *sg.
__device__ __forceinline__ SinCos half_step(double hd, float* sg) {
  int klo = 0;
  const SinCos hh = sincos_small(reduce_pio2<2>(hd, &klo));
  *sg = __uint_as_float((static_cast<unsigned>(klo) << 31) ^ 0x3f800000u);
  return hh;
}

// 1/sqrt(a) for a > 0 in FP64: hardware estimate refined by one Newton step.
// The step squares the estimate's relative error, leaving it below 1e-13:
// enough for q r to 1e-9 rad at r = 10^4 A, far below the FP32 rounding of
// every value derived from it.
__device__ __forceinline__ double rsqrt_f64(double a) {
  const double y = __builtin_amdgcn_rsq(a);
  return y * fma(-0.5 * a, y * y, 1.5);
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
  const double s = fma_vvs(q, rp, kRoundMagic);
  const double k = add_vs(s, -kRoundMagic);
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

// sin(pi b) and cos(pi b) for |b| <= 1/2 by the two polynomials above.
__device__ __forceinline__ SinCosF sincos_pi(float b) {
  const float y = b * b;
  float p = fmaf(y, kSinPi4, kSinPi3);
  p = fmaf(p, y, kSinPi2);
  p = fmaf(p, y, kSinPi1);
  p = fmaf(p, y, kSinPi0);
  float c = fmaf(y, kCosPi5, kCosPi4);
  c = fmaf(c, y, kCosPi3);
  c = fmaf(c, y, kCosPi2);
  c = fmaf(c, y, kCosPi1);
  c = fmaf(c, y, kCosPi0);
  return {b * p, c};
}
// The direct adjoint's three evaluations of sin(q r) and cos(q r) from
// rp = r / pi, with q uniform (an SGPR):
//  - sincos_qr_small for t = q rp <= 1/2: b = t, the FP64 product rounded
//    once to FP32, no reduction;
//  - sincos_qr_frac for 1/4 <= t < 2^19: the one-FMA reduction (b = |v| - 1/2
//    with v = t + 1/2 mod 2, v in [-1, 1)); sin(pi t) = sin(pi b) and
//    cos(pi t) = sin(pi v) = sign(v) cos(pi b), the sign being that of the
//    sum's low word; `magic` (1.5 2^21 + 1/2) and `scale` (2^-31) in VGPRs;
//  - sincos_qr_exact for any t: the reduction of sincos_qr, its first FMA's
//    constant in the VGPR pair `rmagic`.
__device__ __forceinline__ SinCosF sincos_qr_small(double q, double rp) {
  double t;
  asm("v_mul_f64 %0, %1, %2" : "=v"(t) : "s"(q), "v"(rp));
  return sincos_pi(static_cast<float>(t));
}
__device__ __forceinline__ SinCosF sincos_qr_frac(double q, double rp, double magic, float scale) {
  double s;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(s) : "s"(q), "v"(rp), "v"(magic));
  const unsigned lo = static_cast<unsigned>(__double2loint(s));
  float b = static_cast<float>(static_cast<int>(lo));
  asm("v_fma_f32 %0, |%1|, %2, -0.5" : "=v"(b) : "v"(b), "v"(scale));
  SinCosF r = sincos_pi(b);
  r.c = __uint_as_float(__float_as_uint(r.c) ^ (lo & 0x80000000u));
  return r;
}
__device__ __forceinline__ SinCosF sincos_qr_exact(double q, double rp, double rmagic) {
  double s, x;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(s) : "s"(q), "v"(rp), "v"(rmagic));
  const double k = add_vs(s, -kRoundMagic);
  asm("v_fma_f64 %0, %1, %2, -%3" : "=v"(x) : "s"(q), "v"(rp), "v"(k));
  const unsigned flip = static_cast<unsigned>(__double2loint(s)) << 31;
  SinCosF r = sincos_pi(static_cast<float>(x));
  r.s = __uint_as_float(__float_as_uint(r.s) + flip);
  r.c = __uint_as_float(__float_as_uint(r.c) + flip);
  return r;
}

// acc + a * b written in place (v_fmac_f32), so that the accumulators of the
// direct forms' two sine evaluations keep their registers.
__device__ __forceinline__ float fmac_inplace(float a, float b, float acc) {
  asm("v_fmac_f32 %0, %1, %2" : "+v"(acc) : "v"(a), "v"(b));
  return acc;
}

// The direct form's one-FMA reduction of t = q rp (rp = r / pi), for
// 1/4 <= t < 2^19.  One FMA adds 1.5 * 2^21 + 1/2, which puts the sum in
// [2^21, 2^22), where its last bit is worth 2^-31: it holds t + 1/2 rounded to
// a multiple of 2^-31 (to nearest), and its low word read as a signed integer
// is v 2^31 with v = t + 1/2 (mod 2), v in [-1, 1).  Then sin(pi t) =
// -cos(pi v) = -cos(pi |v|) = sin(pi b) with b = |v| - 1/2 in [-1/2, 1/2]:
// one conversion and one FMA give b, with no sign to apply, and
// sin(pi b) = b P(b^2).  The conversion rounds |v| to FP32, an absolute error
// of at most 2^-25 in b, so the relative accuracy of the smallest sines holds
// for t >= 1/4 (smaller t take the product or the exact form).  On gfx950
// FP32 additions, products and FMAs whose operands are VGPRs, literals or
// inline constants issue at twice the rate of conversions, FP64 operations
// and FP32 operations that read an SGPR; so the scale 2^-31 comes in a VGPR
// (`scale`), and the four values' steps are issued stage by stage (one FP64
// FMA and one conversion, then the full-rate operations), which lets their
// latencies overlap.
constexpr double kHalfMagic = 0x1.8p+21 + 0.5;
constexpr double kFracMinT = 0x1p-2, kFracMaxT = 0x1p+19;
// The type form's weight folded into the polynomial: with wc[k] = w c_k (c_k
// the coefficients of sin(pi b) = b P(b^2)), w sin(pi b) = b (w P)(b^2) needs
// no product by w per q.  The five products are formed once per pair; each
// rounds once, as a product b w would, so the accuracy is that of the
// unweighted form to within about one FP32 rounding of the term.
struct SinPiW {
  float c[5];
};
__device__ __forceinline__ SinPiW sinpi_weighted(float w) {
  return {{w * kSinPi0, w * kSinPi1, w * kSinPi2, w * kSinPi3, w * kSinPi4}};
}
// acc[g] + b[g] (w P)(b[g]^2) for four values, stage by stage.  (The squares
// and the first step are issued in the rotated orders 1, 2, 3, 0 and 2, 3, 0,
// 1, which places b[g], y[g] and p[g] in three register banks: the steps read
// three VGPRs, and three from one bank halve the issue rate.)
// With a per-q factor fq (the per-atom form's f_b(q)), b[g] fq[g] takes the
// place of b[g] in the last step.
template <bool PER_Q>
__device__ __forceinline__ void acc4_weighted_sine(float (&b)[4], const SinPiW& wc, const float* fq, float* acc) {
  float y[4], p[4];
#pragma unroll
  for (int h = 1; h <= 4; ++h) y[h & 3] = b[h & 3] * b[h & 3];
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (PER_Q) {
#pragma unroll
    for (int g = 0; g < 4; ++g) b[g] *= fq[g];
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int h = 2; h <= 5; ++h) p[h & 3] = fmaf(y[h & 3], wc.c[4], wc.c[3]);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int k = 2; k >= 0; --k) {
#pragma unroll
    for (int g = 0; g < 4; ++g) p[g] = fmaf(p[g], y[g], wc.c[k]);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int g = 0; g < 4; ++g) acc[g] = fmac_inplace(b[g], p[g], acc[g]);
  __builtin_amdgcn_sched_barrier(0);
}

// The three direct-form evaluations of acc[g] + w sin(q[g] r) for four q
// values from rp = r / pi, the q values uniform (SGPRs, read through the
// scalar cache, which spares the LDS traffic of per-lane copies):
//  - sin_qr_acc4_frac_w, the one-FMA reduction above, for 1/4 <= t < 2^19;
//    its FMA's constant comes in the VGPR pair `magic` (one SGPR operand per
//    instruction);
//  - sin_qr_acc4_small_w, for t <= 1/2: b = t itself, the FP64 product
//    rounded once to FP32 (relative error 2^-24), inside the polynomial's
//    range, so no reduction at all;
//  - sin_qr_acc4_exact_w, for any t: k = round(t) by one FMA that adds
//    kRoundMagic (from the VGPR pair `rmagic`), t - k exact by a second,
//    and the parity of k as the sign (the reduction of sincos_qr).
template <bool PER_Q = false>
__device__ __forceinline__ void sin_qr_acc4_frac_w(const double (&q)[4], double rp, const SinPiW& wc, float scale,
                                                   double magic, float* acc, const float* fq = nullptr) {
  double s[4];
  float b[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) asm("v_fma_f64 %0, %1, %2, %3" : "=v"(s[g]) : "s"(q[g]), "v"(rp), "v"(magic));
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int g = 0; g < 4; ++g) b[g] = static_cast<float>(__double2loint(s[g]));
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int g = 0; g < 4; ++g) asm("v_fma_f32 %0, |%1|, %2, -0.5" : "=v"(b[g]) : "v"(b[g]), "v"(scale));
  __builtin_amdgcn_sched_barrier(0);
  acc4_weighted_sine<PER_Q>(b, wc, fq, acc);
}
template <bool PER_Q = false>
__device__ __forceinline__ void sin_qr_acc4_small_w(const double (&q)[4], double rp, const SinPiW& wc, float* acc,
                                                    const float* fq = nullptr) {
  double t[4];
  float b[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) asm("v_mul_f64 %0, %1, %2" : "=v"(t[g]) : "s"(q[g]), "v"(rp));
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int g = 0; g < 4; ++g) b[g] = static_cast<float>(t[g]);
  __builtin_amdgcn_sched_barrier(0);
  acc4_weighted_sine<PER_Q>(b, wc, fq, acc);
}
template <bool PER_Q = false>
__device__ __forceinline__ void sin_qr_acc4_exact_w(const double (&q)[4], double rp, const SinPiW& wc, double rmagic,
                                                    float* acc, const float* fq = nullptr) {
  double s[4], x[4];
  float b[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) asm("v_fma_f64 %0, %1, %2, %3" : "=v"(s[g]) : "s"(q[g]), "v"(rp), "v"(rmagic));
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int g = 0; g < 4; ++g) x[g] = add_vs(s[g], -kRoundMagic);  // k = round(t)
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int g = 0; g < 4; ++g) asm("v_fma_f64 %0, %1, %2, -%3" : "=v"(x[g]) : "s"(q[g]), "v"(rp), "v"(x[g]));  // t - k
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int g = 0; g < 4; ++g) b[g] = static_cast<float>(x[g]);
  __builtin_amdgcn_sched_barrier(0);
  // sin(pi t) = (-1)^k sin(pi (t - k)): k's parity, the low bit of s, moved
  // to the sign bit
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    unsigned u;
    asm("v_lshl_add_u32 %0, %1, 31, %2"
        : "=v"(u)
        : "v"(static_cast<unsigned>(__double2loint(s[g]))), "v"(__float_as_uint(b[g])));
    b[g] = __uint_as_float(u);
  }
  __builtin_amdgcn_sched_barrier(0);
  acc4_weighted_sine<PER_Q>(b, wc, fq, acc);
}

// The squared distances r^2 in [r2_lo, r2_hi) for which sin_qr_acc4_frac_w
// holds its accuracy at every q in [q_lo, q_hi] (t = q r / pi from 1/4 at
// q_lo to 2^19 at q_hi; q_lo = 0 gives an empty range), and those below
// r2_small, for which sin_qr_acc4_small_w does (t <= 1/2 at q_hi).  Testing
// r^2 costs a pair FP64 comparisons instead of products and comparisons.
struct FracRange {
  double r2_lo, r2_hi, r2_small;
};
// (q = 0 adds sin(0) = 0 under every reduction, so the callers take q_lo as
// the chunk's smallest positive q)
__device__ __forceinline__ FracRange frac_range(double q_lo, double q_hi) {
  constexpr double kPi = 0x1.921fb54442d18p+1;
  const double a = kFracMinT * kPi / q_lo, b = kFracMaxT * kPi / q_hi, c = 0.5 * kPi / q_hi;
  return {a * a, b * b, c * c};
}
// Whether a pair admits sin_qr_acc4_small_w (t <= 1/2 at every q of the chunk).
__device__ __forceinline__ bool small_t_ok(const FracRange& fr, double r2, float w) {
  return w == 0.f || r2 < fr.r2_small;
}
// The smallest positive q of a chunk of an ascending grid (q[0] when it is
// the only value).
__device__ __forceinline__ double chunk_q_lo(const double* q, int nqc) { return q[0] > 0.0 || nqc == 1 ? q[0] : q[1]; }
// Whether a pair (w = 0: it adds nothing either way) admits sin_qr_acc4_frac_w.
__device__ __forceinline__ bool frac_reduction_ok(const FracRange& fr, double r2, float w) {
  return w == 0.f || (r2 >= fr.r2_lo && r2 < fr.r2_hi);
}

}  // namespace sas
