// Device pieces shared by the forward kernels (type-segment form in
// sas_kernels.hip, per-atom form in sas_peratom.hip): the FP64 set-up of one
// pair's q recurrence and the reductions over the 64 lanes of a wave.
#pragma once
#include <hip/hip_runtime.h>

#include "sas_device.hpp"
#include "sas_kernels.hpp"

namespace sas {

// ---------------------------------------------------------------------------
// The q recurrence of one pair.
//
// For an atom pair at distance r and the chunk's grid theta_m = (q_s + m dq) r,
// m = 0..nqc-1, the lane needs y_m = sin(theta_m)/r.  Write dq r = k pi + dp
// with |dp| <= pi/2 and sigma = (-1)^k; then y_m = sigma^m z_m with
// z_m = sin(q_s r + m dp)/r, and z obeys the second-order recurrence
//     z_{m+1} = z_m + d_m,   d_{m+1} = d_m - lambda z_{m+1},
// lambda = 4 sin^2(dp/2), in the difference form (Reinsch) that stays accurate
// for small dp.  The seeds z_0 = sin(q_s r)/r and d_0 = z_1 - z_0 and lambda
// come from FP64 trigonometry and are rounded to FP32 once.  Each q step then
// costs three FP32 operations: the accumulate (sign folded in on odd steps),
// z += d and d += -lambda z.  Coincident atoms (r = 0) use r^2 = 1e-60, for
// which the same formulas give the sinc limit y_m = q_m.
// ---------------------------------------------------------------------------
// FP32 start of one pair's recurrence: z_0, d_0, -lambda and sigma (see
// above), from the FP64 set-up.  `use` = 0 gives an all-zero sequence.
struct PairSeed {
  float z, d, nlam, sg;
};

// (hdq = dq / 2, the grid step halved)
__device__ __forceinline__ PairSeed pair_seed(const double4& pi, const double4& pj, bool use, double hdq, double qs) {
  const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
  double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
  r2 = fmax(r2, 1e-60);
  const double ir = rsqrt_f64(r2);
  const double r = r2 * ir;
  PairSeed p;
  const SinCos hh = half_step(hdq * r, &p.sg);
  const double s2 = hh.s + hh.s;  // 2 sin(dp/2)
  const double lam = s2 * s2;     // 4 sin^2(dp/2) = 2 (1 - cos(dp))
  const double sdp = s2 * hh.c;   // sin(dp)
  p.nlam = static_cast<float>(-lam);
  if (qs == 0.0) {
    // chunk starting at q = 0: z_0 = 0, d_0 = sin(dp)/r
    p.z = 0.f;
    p.d = use ? static_cast<float>(sdp * ir) : 0.f;
  } else {
    const SinCos t0 = sincos_any(qs * r);
    const double w = use ? ir : 0.0;
    const double S0 = t0.s * w, C0 = t0.c * w;
    p.z = static_cast<float>(S0);
    p.d = static_cast<float>(fma(C0, sdp, -0.5 * lam * S0));
  }
  return p;
}

// One q step of two pairs' recurrences (A and B) into one accumulator:
//     acc += z_a + z_b          (even step; odd: acc += sigma_a z_a + sigma_b z_b)
//     z_a += d_a,  z_b += d_b,  d_a += -lambda_a z_a,  d_b += -lambda_b z_b
// with the FP32 operations written out and the eight chain values held in
// fixed VGPRs.  On gfx950 a VALU instruction whose three VGPR operands sit in
// one register bank (register number mod 4) issues at about half rate; two in
// one bank cost nothing.  The accumulators cycle through all four banks, so a
// chain value and its multiplier must sit in different banks, which the
// register allocator does not know to arrange: the chain values go to
// z_a, z_b, sigma_a, sigma_b, d_a, d_b, -lambda_a, -lambda_b at BASE .. BASE+7
// (BASE a multiple of 8, so banks 0 1 2 3 0 1 2 3), and no instruction of the
// step reads three operands from one bank.  BASE is picked at the top of the
// kernel's register budget so that the pinned registers take no occupancy.
// The arithmetic and its order are those of the plain C++ form (v_fmac_f32 is
// the FMA; adds round once), so the results are bitwise the same.
#define SAS_PIN(r) "{v" #r "}"
#define SAS_STEP2_ASM(R0, R1, R2, R3, R4, R5, R6, R7)                                                   \
  do {                                                                                                 \
    if constexpr (ODD)                                                                                 \
      asm("v_fmac_f32 %0, %5, %1\n v_fmac_f32 %0, %6, %2\n v_add_f32 %1, %1, %3\n"                    \
          "v_add_f32 %2, %2, %4\n v_fmac_f32 %3, %7, %1\n v_fmac_f32 %4, %8, %2"                       \
          : "+v"(acc), "+" SAS_PIN(R0)(za), "+" SAS_PIN(R1)(zb), "+" SAS_PIN(R4)(da), "+" SAS_PIN(R5)(db) \
          : SAS_PIN(R2)(sga), SAS_PIN(R3)(sgb), SAS_PIN(R6)(nla), SAS_PIN(R7)(nlb));                     \
    else                                                                                               \
      asm("v_add_f32 %0, %0, %1\n v_add_f32 %0, %0, %2\n v_add_f32 %1, %1, %3\n"                      \
          "v_add_f32 %2, %2, %4\n v_fmac_f32 %3, %5, %1\n v_fmac_f32 %4, %6, %2"                       \
          : "+v"(acc), "+" SAS_PIN(R0)(za), "+" SAS_PIN(R1)(zb), "+" SAS_PIN(R4)(da), "+" SAS_PIN(R5)(db) \
          : SAS_PIN(R6)(nla), SAS_PIN(R7)(nlb));                                                        \
  } while (0)

template <int BASE, bool ODD>
__device__ __forceinline__ void rec_step2(float& acc, float& za, float& zb, float& da, float& db, float sga,
                                          float sgb, float nla, float nlb) {
  static_assert(BASE == 248 || BASE == 160 || BASE == 88, "pinned register base");
  if constexpr (BASE == 248)
    SAS_STEP2_ASM(248, 249, 250, 251, 252, 253, 254, 255);
  else if constexpr (BASE == 160)
    SAS_STEP2_ASM(160, 161, 162, 163, 164, 165, 166, 167);
  else
    SAS_STEP2_ASM(88, 89, 90, 91, 92, 93, 94, 95);
}
#undef SAS_STEP2_ASM

// Four consecutive q steps (m even: even, odd, even, odd) of the same two
// pairs in one asm block.  The compiler follows each inline asm statement
// with an s_nop; in the two-wave kernels (chunks above 128 q) one block per
// four steps instead of one per step made the rod's pair kernel 3.4% faster
// (the three-wave kernels, where the other waves hide the nops, were 1-2%
// slower with it and keep one step per block).
#define SAS_STEP8_ASM(R0, R1, R2, R3, R4, R5, R6, R7)                                                   \
  asm("v_add_f32 %0, %0, %4\n v_add_f32 %0, %0, %5\n v_add_f32 %4, %4, %6\n"                          \
      "v_add_f32 %5, %5, %7\n v_fmac_f32 %6, %10, %4\n v_fmac_f32 %7, %11, %5\n"                      \
      "v_fmac_f32 %1, %8, %4\n v_fmac_f32 %1, %9, %5\n v_add_f32 %4, %4, %6\n"                        \
      "v_add_f32 %5, %5, %7\n v_fmac_f32 %6, %10, %4\n v_fmac_f32 %7, %11, %5\n"                      \
      "v_add_f32 %2, %2, %4\n v_add_f32 %2, %2, %5\n v_add_f32 %4, %4, %6\n"                          \
      "v_add_f32 %5, %5, %7\n v_fmac_f32 %6, %10, %4\n v_fmac_f32 %7, %11, %5\n"                      \
      "v_fmac_f32 %3, %8, %4\n v_fmac_f32 %3, %9, %5\n v_add_f32 %4, %4, %6\n"                        \
      "v_add_f32 %5, %5, %7\n v_fmac_f32 %6, %10, %4\n v_fmac_f32 %7, %11, %5"                        \
      : "+v"(acc0), "+v"(acc1), "+v"(acc2), "+v"(acc3), "+" SAS_PIN(R0)(za), "+" SAS_PIN(R1)(zb),      \
        "+" SAS_PIN(R4)(da), "+" SAS_PIN(R5)(db)                                                      \
      : SAS_PIN(R2)(sga), SAS_PIN(R3)(sgb), SAS_PIN(R6)(nla), SAS_PIN(R7)(nlb))

template <int BASE>
__device__ __forceinline__ void rec_step8(float& acc0, float& acc1, float& acc2, float& acc3, float& za, float& zb,
                                          float& da, float& db, float sga, float sgb, float nla, float nlb) {
  static_assert(BASE == 248 || BASE == 160 || BASE == 88, "pinned register base");
  if constexpr (BASE == 248)
    SAS_STEP8_ASM(248, 249, 250, 251, 252, 253, 254, 255);
  else if constexpr (BASE == 160)
    SAS_STEP8_ASM(160, 161, 162, 163, 164, 165, 166, 167);
  else
    SAS_STEP8_ASM(88, 89, 90, 91, 92, 93, 94, 95);
}
#undef SAS_STEP8_ASM
#undef SAS_PIN

// Register base for rec_step2 in a kernel of `waves` waves per SIMD (512
// VGPRs per SIMD lane shared by the waves, allocated in blocks of 8): the top
// eight of the budget (256 or 168), or v88 for the short chunks (at most 32
// q values), whose kernels need about a hundred.
constexpr int pin_base(int waves, bool small) { return small ? 88 : (waves <= 2 ? 248 : 160); }

// Sum acc[0..64) over the 64 lanes; lane l receives the total of element l.
// Recursive halving: at the step for lane bit b the lane keeps the half of its
// live range selected by b and adds the partner's copy of that half.
__device__ __forceinline__ float lane_transpose_reduce64(float* acc, int lane) {
#pragma unroll
  for (int step = 0; step < 6; ++step) {
    const int half = 32 >> step;
    const int bit = (lane >> (5 - step)) & 1;
#pragma unroll
    for (int k = 0; k < half; ++k) {
      const float lo = acc[k], hi = acc[k + half];
      const float send = bit ? lo : hi;
      const float keep = bit ? hi : lo;
      acc[k] = keep + __shfl_xor(send, half, kWave);
    }
  }
  return acc[0];
}

// Sum acc[0..R) (R < 64) over the lanes; lane l < R receives element l.
template <int R>
__device__ __forceinline__ float lane_allreduce_tail(float* acc, int lane) {
  float mine = 0.f;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    float v = acc[k];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    mine = (lane == k) ? v : mine;
  }
  return mine;
}

}  // namespace sas
