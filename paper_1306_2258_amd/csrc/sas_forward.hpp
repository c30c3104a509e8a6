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

__device__ __forceinline__ PairSeed pair_seed(const double4& pi, const double4& pj, bool use, double dq, double qs) {
  const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
  double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
  r2 = fmax(r2, 1e-60);
  const double ir = rsqrt_f64(r2);
  const double r = r2 * ir;
  const double delta = dq * r;
  const double k = rint(delta * kOneOverPi);
  double dp = fma(-k, kPiA, delta);
  dp = fma(-k, kPiB, dp);
  dp = fma(-k, kPiC, dp);
  const SinCos hh = sincos_small(0.5 * dp);
  const double s2 = hh.s + hh.s;  // 2 sin(dp/2)
  const double lam = s2 * s2;     // 4 sin^2(dp/2) = 2 (1 - cos(dp))
  const double sdp = s2 * hh.c;   // sin(dp)
  PairSeed p;
  p.nlam = static_cast<float>(-lam);
  p.sg = parity_sign(k);
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
