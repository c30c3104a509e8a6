// Adjoint of the Debye profile with respect to the coordinates (gfx950).
//
// For weights w_m (dL/dI(q_m)) the derivative of Eq. 2 gives, per atom pair
// (i, j) at distance r with form factors f_a, f_b:
//     C = sum_m U_m cos(q_m r),  S = sum_m V_m sin(q_m r),
//     U_m = w_m f_a(q_m) f_b(q_m),  V_m = U_m / q_m   (both 0 where q_m = 0),
//     G = 2 (C / r^2 - S / r^3),  g_i += G (x_i - x_j),  g_j -= G (x_i - x_j).
// The pair loop follows the forward kernel: one 64-lane wave per (I block of
// 128 atoms, two per lane, strip of J blocks, q chunk), J blocks staged in
// LDS, the same FP64 set-up and the
// same FP32 recurrence z_{m+1} = z_m + d_m, d_{m+1} = d_m - lambda z_{m+1}
// with z_m = sin(phi_m), phi_m = q_s r + m dp.  The cosine comes from the
// recurrence state itself, cos(phi_m) = (d_m + (lambda/2) z_m) / sin(dp), so a
// q step costs five FP32 operations: two for the recurrence and three
// accumulations (U d, U z, V z), kept separately for even and odd m to fold
// in the sign (-1)^(k m) of the reduction dq r = k pi + dp.  Lanes of one
// wave may hold atoms of several types; the wave visits each type present
// (almost always one) with the other lanes masked, so that U and V are
// wave-uniform and read from LDS.  The i-side sums stay in the lane (FP64);
// the j-side sums (both atoms of a lane added first) are reduced over the 64
// lanes per j with DPP row operations and kept in FP64 in LDS.
// Partial sums go to per-strip rows that a second kernel adds in fixed order.
//
// A non-uniform q grid has no recurrence: the direct variant evaluates sin and
// cos of q_m r for every q (FP64 reduction of q r / pi, FP32 polynomials, as
// in the forward's direct form) and accumulates C and S with their signs,
// two FMAs per atom and q.
//
// Per-atom form factors (k_adjoint_pa: many table rows, no type sort): U_m
// is a product of the pair's own rows, U_m = (w_m f_i(q_m)) f_j(q_m).  Each
// lane holds w_m f_i for a chunk of up to 100 q values in registers, 1/q_m is
// read from LDS (the same address in every lane), and the J atoms' rows are
// staged in LDS in runs of kPaSub beside their positions, as in the
// per-atom forward; so a q step costs two FP32 products (U and V = U/q) more
// than the type form.  One atom per lane, and the same strip rows and final
// reduce as the type form.
#include <hip/hip_runtime.h>

#include "sas_device.hpp"
#include "sas_kernels.hpp"
#include "sas_schedule.hpp"

namespace sas {

// Sum over the 64 lanes with DPP row operations (pairs, quads, half rows,
// rows, then the row broadcasts); the total ends in lanes 48..63 and is
// returned from lane 63 as a wave-uniform value.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v) {
  const int moved = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false);
  return v + __int_as_float(moved);
}

__device__ __forceinline__ float wave_total(float v) {
  v = dpp_add<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v = dpp_add<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xF>(v);  // row_half_mirror
  v = dpp_add<0x140, 0xF>(v);  // row_mirror
  v = dpp_add<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Per-pair FP64 set-up shared by the two atoms of a lane.  The values the
// pair's force is formed from at the end (1/r, 1 - cos(dp), 1/sin(dp),
// cos(q_s r)) are kept in FP32: that force combines FP32 q sums, and each
// pair's force enters the gradient once, so one more FP32 rounding there is
// an unbiased 6e-8 per pair against the 1e-5 the gradient is held to.
struct AdjSeed {
  float z, d, nlam, sg;
  float ir, omc, isdp, c0;  // 1/r, 1 - cos(dp), 1/sin(dp), cos(q_s r)
  double dx, dy, dz;
  bool valid;
};

__device__ __forceinline__ AdjSeed adj_seed(const double4& pi, const double4& pj, bool use, double dq, double qs) {
  AdjSeed p;
  p.dx = pi.x - pj.x;
  p.dy = pi.y - pj.y;
  p.dz = pi.z - pj.z;
  const double r2raw = fma(p.dz, p.dz, fma(p.dy, p.dy, p.dx * p.dx));
  p.valid = use && r2raw > 0.0;
  const double r2 = fmax(r2raw, 1e-60);
  const double ir = rsqrt_f64(r2);
  const double r = r2 * ir;
  p.ir = static_cast<float>(ir);
  const SinCos hh = half_step(0.5 * dq * r, &p.sg);
  const double s2 = hh.s + hh.s;  // 2 sin(dp/2)
  const double lam = s2 * s2;     // 4 sin^2(dp/2)
  const double sdp = s2 * hh.c;   // sin(dp)
  const double omc = 0.5 * lam;   // 1 - cos(dp) = lambda / 2
  p.omc = static_cast<float>(omc);
  // 1/sin(dp) by the FP32 hardware reciprocal (0 when sin(dp) = 0)
  p.isdp = sdp != 0.0 ? __builtin_amdgcn_rcpf(static_cast<float>(sdp)) : 0.f;
  double S0 = 0.0, C0 = 1.0;
  if (qs != 0.0) {
    const SinCos t0 = sincos_any(qs * r);
    S0 = t0.s;
    C0 = t0.c;
  }
  p.c0 = static_cast<float>(C0);
  p.z = static_cast<float>(S0);
  p.d = static_cast<float>(fma(C0, sdp, -S0 * omc));
  p.nlam = static_cast<float>(-lam);
  return p;
}

// G of one pair (its force is G (x_i - x_j)) from its six accumulators, in FP32.
__device__ __forceinline__ double adj_force(const AdjSeed& p, float a1e, float a1o, float a2e, float a2o, float a3e,
                                            float a3o, double dq, float u0) {
  const float A1 = fmaf(p.sg, a1o, a1e);
  const float A2 = fmaf(p.sg, a2o, a2e);
  const float A3 = fmaf(p.sg, a3o, a3e);
  // sum_m U_m cos(q_m r); with a single q (dq = 0), or dq r an exact multiple
  // of pi, the recurrence is constant and the seed's cosine is used
  const float Cc = (dq != 0.0 && p.isdp != 0.f) ? fmaf(p.omc, A2, A1) * p.isdp : u0 * p.c0;
  return p.valid ? static_cast<double>((2.f * p.ir * p.ir) * fmaf(-A3, p.ir, Cc)) : 0.0;
}

// G of one atom of the direct variant from its sums C and S.
__device__ __forceinline__ double adj_force_direct(bool valid, double ir, float c, float s) {
  return valid ? 2.0 * ir * ir * (static_cast<double>(c) - static_cast<double>(s) * ir) : 0.0;
}

// The minimum and maximum over the 64 lanes, by the same DPP steps (lanes
// outside a step's rows take the identity), returned from lane 63.
template <int CTRL, int ROW_MASK, bool MAX>
__device__ __forceinline__ float dpp_ext(float v) {
  const float id = MAX ? 0.f : __builtin_huge_valf();
  const float moved =
      __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(id), __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
  return MAX ? fmaxf(v, moved) : fminf(v, moved);
}
template <bool MAX>
__device__ __forceinline__ float wave_extreme(float v) {
  v = dpp_ext<0xB1, 0xF, MAX>(v);
  v = dpp_ext<0x4E, 0xF, MAX>(v);
  v = dpp_ext<0x141, 0xF, MAX>(v);
  v = dpp_ext<0x140, 0xF, MAX>(v);
  v = dpp_ext<0x142, 0xA, MAX>(v);
  v = dpp_ext<0x143, 0xC, MAX>(v);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

template <int BJ, bool DIRECT>
__global__ __launch_bounds__(kWave) void k_adjoint(AdjArgs a) {
  __shared__ double4 sj[BJ];
  __shared__ float4 ul4[kAdjQ / 4];
  __shared__ float4 vl4[kAdjQ / 4];
  __shared__ double gjl[BJ * 3];
  float* ul = reinterpret_cast<float*>(ul4);
  float* vl = reinterpret_cast<float*>(vl4);

  const int lane = threadIdx.x;
  const int64_t t = blockIdx.x;
  const StructDesc d = a.sd.get(0);
  const StripPos sp = decode_strip(t, d.n, a.geo);
  const int n = d.n;
  // two atoms per lane: rows I*128 + lane and I*128 + 64 + lane
  const int i1 = sp.I * 2 * kWave + lane, i2 = i1 + kWave;
  const bool v1 = i1 < n, v2 = i2 < n;
  const double4 p1 = a.xyz[d.atom_off + (v1 ? i1 : n - 1)];
  const double4 p2 = a.xyz[d.atom_off + (v2 ? i2 : n - 1)];
  const int t1 = clamp_type(a.tsort[d.atom_off + (v1 ? i1 : n - 1)], a.T);
  const int t2 = clamp_type(a.tsort[d.atom_off + (v2 ? i2 : n - 1)], a.T);

  const int m0 = blockIdx.y * a.qa;
  const int nqa = min(a.qa, a.Nq - m0);
  const int nq8 = (nqa + 7) & ~7;
  const int nq4 = (nqa + 3) & ~3;
  const double qs = a.q0 + m0 * a.dq;
  const double dq = a.dq;
  const int64_t pidx = static_cast<int64_t>(blockIdx.y) * a.n_strips + t;
  const int32_t* toff = a.toff;

  double g1x = 0.0, g1y = 0.0, g1z = 0.0, g2x = 0.0, g2y = 0.0, g2z = 0.0;

#pragma unroll 1
  for (int J = sp.Ja; J < sp.Jb; ++J) {
    const int j0 = J * BJ;
    const int j1 = min(n, j0 + BJ);
    __syncthreads();
    for (int k = lane; k < j1 - j0; k += kWave) sj[k] = a.xyz[d.atom_off + j0 + k];
    for (int k = lane; k < 3 * BJ; k += kWave) gjl[k] = 0.0;
    __syncthreads();
    const int64_t aj0 = d.atom_off + j0, aj1 = d.atom_off + j1;
    int lo = 0, hi = a.T - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (toff[mid + 1] > aj0)
        hi = mid;
      else
        lo = mid + 1;
    }
#pragma unroll 1
    for (int tb = lo; tb < a.T && toff[tb] < aj1; ++tb) {
      const int sa = static_cast<int>(max(static_cast<int64_t>(toff[tb]), aj0) - d.atom_off);
      const int sb = static_cast<int>(min(static_cast<int64_t>(toff[tb + 1]), aj1) - d.atom_off);
      if (sa >= sb) continue;
      uint64_t rem1 = __ballot(v1), rem2 = __ballot(v2);
#pragma unroll 1
      while (rem1 | rem2) {
        // the next type present among the lanes' atoms (wave-uniform)
        const int at = rem1 ? __shfl(t1, __ffsll(static_cast<unsigned long long>(rem1)) - 1, kWave)
                            : __shfl(t2, __ffsll(static_cast<unsigned long long>(rem2)) - 1, kWave);
        const bool mine1 = v1 && t1 == at, mine2 = v2 && t2 == at;
        rem1 &= ~static_cast<uint64_t>(__ballot(mine1));
        rem2 &= ~static_cast<uint64_t>(__ballot(mine2));
        // wave-uniform weights of the (at, tb) type pair for this chunk
        __syncthreads();
        const float* fa = a.tabp + static_cast<int64_t>(at) * a.ldt + m0;
        const float* fb = a.tabp + static_cast<int64_t>(tb) * a.ldt + m0;
        for (int m = lane; m < nq8; m += kWave) {
          float u = 0.f, v = 0.f;
          const double qm = DIRECT ? (m < nqa ? a.qdev[m0 + m] : 0.0) : a.q0 + (m0 + m) * dq;
          if (m < nqa && qm > 0.0) {
            const double uu = a.w[m0 + m] * static_cast<double>(fa[m]) * static_cast<double>(fb[m]);
            u = static_cast<float>(uu);
            v = static_cast<float>(uu / qm);
          }
          ul[m] = u;
          vl[m] = v;
        }
        __syncthreads();
        const float u0 = ul[0];
        if constexpr (DIRECT) {
          // q through the scalar cache (uniform), weights from LDS; per group of four
          // q the cheapest evaluation that holds for every lane's pairs: the
          // product form when t = q r / pi <= 1/2 at the group's largest q,
          // the one-FMA reduction when 1/4 <= t < 2^19 over the group, the
          // exact reduction otherwise.  The bounds are on q: the wave's
          // extremes of 1/r (FP32; a bound off by a rounding moves t by
          // 2^-24 relative, well inside each form's margin).
          using ConstDouble = const __attribute__((address_space(4))) double;
          ConstDouble* qk = (ConstDouble*)(a.qdev + m0);
          double kMagicV = kHalfMagic, kRoundV = kRoundMagic;
          float kScale31 = 0x1p-31f;
          asm volatile("" : "+v"(kMagicV), "+v"(kRoundV), "+v"(kScale31));
#pragma unroll 1
          for (int jl = sa; jl < sb; ++jl) {
            const double4 pj = sj[jl - j0];
            const double ax = p1.x - pj.x, ay = p1.y - pj.y, az = p1.z - pj.z;
            const double bx = p2.x - pj.x, by = p2.y - pj.y, bz = p2.z - pj.z;
            const double ra2 = fma(az, az, fma(ay, ay, ax * ax));
            const double rb2 = fma(bz, bz, fma(by, by, bx * bx));
            const bool va = mine1 && jl > i1 && ra2 > 0.0, vb = mine2 && jl > i2 && rb2 > 0.0;
            const double ira = rsqrt_f64(fmax(ra2, 1e-60)), irb = rsqrt_f64(fmax(rb2, 1e-60));
            const double rpa = fmax(ra2, 1e-60) * ira * kOneOverPi, rpb = fmax(rb2, 1e-60) * irb * kOneOverPi;
            const float ifa = static_cast<float>(ira), ifb = static_cast<float>(irb);
            const float ir_min =
                wave_extreme<false>(fminf(va ? ifa : __builtin_huge_valf(), vb ? ifb : __builtin_huge_valf()));
            const float ir_max = wave_extreme<true>(fmaxf(va ? ifa : 0.f, vb ? ifb : 0.f));
            constexpr double kPi = 0x1.921fb54442d18p+1;
            const double q_small = 0.5 * kPi * ir_min;     // t <= 1/2 below
            const double q_frac = 0.25 * kPi * ir_max;     // t >= 1/4 above
            const double q_huge = 0x1p+19 * kPi * ir_min;  // t < 2^19 below
            float ca = 0.f, sa2 = 0.f, cb = 0.f, sb2 = 0.f;
#pragma unroll 1
            for (int m = 0; m < nqa; m += 4) {
              const float4 u4 = ul4[m >> 2], v4 = vl4[m >> 2];
              const float u[4] = {u4.x, u4.y, u4.z, u4.w}, v[4] = {v4.x, v4.y, v4.z, v4.w};
              // (past the chunk's end the last q is repeated: its weights
              // are zero, and a larger q from the next chunk could push the
              // chosen form past its range, to an infinite term times zero)
              double q[4];
#pragma unroll
              for (int k = 0; k < 4; ++k) q[k] = qk[min(m + k, nqa - 1)];
              const double q_last = q[3];
              auto acc4 = [&](auto&& eval) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                  const SinCosF ea = eval(q[k], rpa), eb = eval(q[k], rpb);
                  ca = fmaf(u[k], ea.c, ca);
                  sa2 = fmaf(v[k], ea.s, sa2);
                  cb = fmaf(u[k], eb.c, cb);
                  sb2 = fmaf(v[k], eb.s, sb2);
                }
              };
              if (q_last <= q_small)
                acc4([&](double qq, double rp) { return sincos_qr_small(qq, rp); });
              else if (q[0] >= q_frac && q_last < q_huge)
                acc4([&](double qq, double rp) { return sincos_qr_frac(qq, rp, kMagicV, kScale31); });
              else
                acc4([&](double qq, double rp) { return sincos_qr_exact(qq, rp, kRoundV); });
            }
            const double GA = adj_force_direct(va, ira, ca, sa2);
            const double GB = adj_force_direct(vb, irb, cb, sb2);
            const double cax = GA * ax, cay = GA * ay, caz = GA * az;
            const double cbx = GB * bx, cby = GB * by, cbz = GB * bz;
            g1x += cax;
            g1y += cay;
            g1z += caz;
            g2x += cbx;
            g2y += cby;
            g2z += cbz;
            const float sx = wave_total(static_cast<float>(cax + cbx));
            const float sy = wave_total(static_cast<float>(cay + cby));
            const float sz = wave_total(static_cast<float>(caz + cbz));
            if (lane == 0) {
              double* gj = gjl + 3 * (jl - j0);
              gj[0] -= sx;
              gj[1] -= sy;
              gj[2] -= sz;
            }
          }
          continue;
        }
#pragma unroll 1
        for (int jl = sa; jl < sb; ++jl) {
          const double4 pj = sj[jl - j0];
          const AdjSeed A = adj_seed(p1, pj, mine1 && jl > i1, dq, qs);
          const AdjSeed B = adj_seed(p2, pj, mine2 && jl > i2, dq, qs);
          float za = A.z, da = A.d, zb = B.z, db = B.d;
          // (laundered: a known negation would become a source modifier,
          // forcing the slower 64-bit encoding of every FMA that uses it)
          float nla = A.nlam, nlb = B.nlam;
          asm volatile("" : "+v"(nla), "+v"(nlb));
          float a1e = 0.f, a1o = 0.f, a2e = 0.f, a2o = 0.f, a3e = 0.f, a3o = 0.f;
          float b1e = 0.f, b1o = 0.f, b2e = 0.f, b2o = 0.f, b3e = 0.f, b3o = 0.f;
          // one even and one odd q step of both atoms
          auto two_steps = [&](float ue, float ve, float uo, float vo) {
            a1e = fmaf(ue, da, a1e);
            b1e = fmaf(ue, db, b1e);
            a2e = fmaf(ue, za, a2e);
            b2e = fmaf(ue, zb, b2e);
            a3e = fmaf(ve, za, a3e);
            b3e = fmaf(ve, zb, b3e);
            za += da;
            zb += db;
            da = fmaf(nla, za, da);
            db = fmaf(nlb, zb, db);
            a1o = fmaf(uo, da, a1o);
            b1o = fmaf(uo, db, b1o);
            a2o = fmaf(uo, za, a2o);
            b2o = fmaf(uo, zb, b2o);
            a3o = fmaf(vo, za, a3o);
            b3o = fmaf(vo, zb, b3o);
            za += da;
            zb += db;
            da = fmaf(nla, za, da);
            db = fmaf(nlb, zb, db);
          };
          // blocks of 8 q (the loop unrolled twice: one branch per 16 q),
          // then a block of 4 if the chunk's count (rounded up to 4) leaves
          // one: no steps past the chunk's last 4
#pragma unroll 2
          for (int m = 0; m + 8 <= nq4; m += 8) {
            const float4 ua = ul4[m >> 2], ub = ul4[(m >> 2) + 1];
            const float4 va = vl4[m >> 2], vb = vl4[(m >> 2) + 1];
            two_steps(ua.x, va.x, ua.y, va.y);
            two_steps(ua.z, va.z, ua.w, va.w);
            two_steps(ub.x, vb.x, ub.y, vb.y);
            two_steps(ub.z, vb.z, ub.w, vb.w);
          }
          if (nq4 & 4) {
            const float4 ua = ul4[(nq4 - 4) >> 2], va = vl4[(nq4 - 4) >> 2];
            two_steps(ua.x, va.x, ua.y, va.y);
            two_steps(ua.z, va.z, ua.w, va.w);
          }
          const double GA = adj_force(A, a1e, a1o, a2e, a2o, a3e, a3o, dq, u0);
          const double GB = adj_force(B, b1e, b1o, b2e, b2o, b3e, b3o, dq, u0);
          const double cax = GA * A.dx, cay = GA * A.dy, caz = GA * A.dz;
          const double cbx = GB * B.dx, cby = GB * B.dy, cbz = GB * B.dz;
          g1x += cax;
          g1y += cay;
          g1z += caz;
          g2x += cbx;
          g2y += cby;
          g2z += cbz;
          const float sx = wave_total(static_cast<float>(cax + cbx));
          const float sy = wave_total(static_cast<float>(cay + cby));
          const float sz = wave_total(static_cast<float>(caz + cbz));
          if (lane == 0) {
            double* gj = gjl + 3 * (jl - j0);
            gj[0] -= sx;
            gj[1] -= sy;
            gj[2] -= sz;
          }
        }
      }
    }
    __syncthreads();
    double* outj = a.gJ + (pidx * a.geo.g * BJ + static_cast<int64_t>(J - sp.Ja) * BJ) * 3;
    for (int k = lane; k < 3 * (j1 - j0); k += kWave) outj[k] = gjl[k];
  }
  double* outi = a.gI + pidx * (2 * kWave) * 3;
  outi[3 * lane + 0] = g1x;
  outi[3 * lane + 1] = g1y;
  outi[3 * lane + 2] = g1z;
  outi[3 * (lane + kWave) + 0] = g2x;
  outi[3 * (lane + kWave) + 1] = g2y;
  outi[3 * (lane + kWave) + 2] = g2z;
}

template <int QA, bool DIRECT>
__global__ __launch_bounds__(kWave, 2) void k_adjoint_pa(AdjArgs a) {
  static_assert(QA % 4 == 0, "table rows are staged as float4");
  constexpr int BJ = kAdjPaBJ;
  constexpr int Q4 = QA / 4;
  constexpr int E4 = kPaSub * Q4;  // float4 elements of one run's rows
  __shared__ double4 sj[kPaSub];
  __shared__ __align__(16) float fj[kPaSub][QA];
  __shared__ double gjl[BJ * 3];
  __shared__ __align__(16) float iql[QA];

  const int lane = threadIdx.x;
  const int64_t t = blockIdx.x;
  const StructDesc d = a.sd.get(0);
  const StripPos sp = decode_strip(t, d.n, a.geo);
  const int n = d.n;
  const int i = sp.I * kWave + lane;
  const bool vi = i < n;
  const int ic = vi ? i : n - 1;
  const double4 pi = a.xyz[d.atom_off + ic];
  const int ti = clamp_type(a.tsort[d.atom_off + ic], a.T);

  const int m0 = blockIdx.y * a.qa;
  const int nqa = min(a.qa, a.Nq - m0);  // <= QA
  const double qs = a.q0 + m0 * a.dq;
  const double dq = a.dq;
  const int64_t pidx = static_cast<int64_t>(blockIdx.y) * a.n_strips + t;
  // this lane's weights w_m f_i(q_m) (zero at q = 0, where I does not depend
  // on the positions, and past the chunk) and the chunk's 1/q_m
  float wi[QA];
  const float* fi = a.tabp + static_cast<int64_t>(ti) * a.ldt + m0;
#pragma unroll
  for (int m = 0; m < QA; ++m) {
    const double qm = m < nqa ? (DIRECT ? a.qdev[m0 + m] : a.q0 + (m0 + m) * dq) : 0.0;
    wi[m] = qm > 0.0 ? static_cast<float>(a.w[m0 + m] * static_cast<double>(fi[m])) : 0.f;
  }
  for (int m = lane; m < QA; m += kWave) {
    const double qm = m < nqa ? (DIRECT ? a.qdev[m0 + m] : a.q0 + (m0 + m) * dq) : 0.0;
    iql[m] = qm > 0.0 ? static_cast<float>(1.0 / qm) : 0.f;
  }

  double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll 1
  for (int J = sp.Ja; J < sp.Jb; ++J) {
    const int j0 = J * BJ;
    const int j1 = min(n, j0 + BJ);
    __syncthreads();
    for (int k = lane; k < 3 * BJ; k += kWave) gjl[k] = 0.0;
#pragma unroll 1
    for (int u0 = j0; u0 < j1; u0 += kPaSub) {
      const int ns = min(kPaSub, j1 - u0);
      __syncthreads();
      const int ty = lane < ns ? clamp_type(a.tsort[d.atom_off + u0 + lane], a.T) : 0;  // row 0 past the run
      if (lane < ns) sj[lane] = a.xyz[d.atom_off + u0 + lane];
      for (int e = lane; e < E4; e += kWave) {
        const int r = e / Q4;
        const int c = e - r * Q4;
        const int tr = __shfl(ty, r, kWave);
        reinterpret_cast<float4*>(&fj[0][0])[e] =
            *reinterpret_cast<const float4*>(a.tabp + static_cast<int64_t>(tr) * a.ldt + m0 + 4 * c);
      }
      __syncthreads();
      if constexpr (DIRECT) {
        // per group of four q the product form, the one-FMA reduction or the
        // exact one, chosen from the wave's extremes of 1/r as in k_adjoint;
        // q through the scalar cache, groups past the chunk skipped, and the
        // last q repeated inside the chunk's last group
        using ConstDouble = const __attribute__((address_space(4))) double;
        ConstDouble* qk = (ConstDouble*)(a.qdev + m0);
        double kMagicV = kHalfMagic, kRoundV = kRoundMagic;
        float kScale31 = 0x1p-31f;
        asm volatile("" : "+v"(kMagicV), "+v"(kRoundV), "+v"(kScale31));
#pragma unroll 1
        for (int jl = u0; jl < u0 + ns; ++jl) {
          asm volatile("" ::: "memory");
          const double4 pj = sj[jl - u0];
          const float* f = fj[jl - u0];
          const bool use = vi && jl > i;
          const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
          const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
          const double ir = rsqrt_f64(fmax(r2, 1e-60));
          const double rp = fmax(r2, 1e-60) * ir * kOneOverPi;
          const bool ok = use && r2 > 0.0;
          const float irf = static_cast<float>(ir);
          const float ir_min = wave_extreme<false>(ok ? irf : __builtin_huge_valf());
          const float ir_max = wave_extreme<true>(ok ? irf : 0.f);
          constexpr double kPi = 0x1.921fb54442d18p+1;
          const double q_small = 0.5 * kPi * ir_min, q_frac = 0.25 * kPi * ir_max, q_huge = 0x1p+19 * kPi * ir_min;
          float cc = 0.f, ss = 0.f;
          // (fully unrolled: a runtime index would put wi and wiq in scratch)
#pragma unroll
          for (int m = 0; m < QA; m += 4) {
            if (m < nqa) {
              double q[4];
#pragma unroll
              for (int k = 0; k < 4; ++k) q[k] = qk[min(m + k, nqa - 1)];
              auto acc4 = [&](auto&& eval) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                  const SinCosF e = eval(q[k], rp);
                  const float u = wi[m + k] * f[m + k];
                  cc = fmaf(u, e.c, cc);
                  ss = fmaf(u * iql[m + k], e.s, ss);
                }
              };
              if (q[3] <= q_small)
                acc4([&](double qq, double r) { return sincos_qr_small(qq, r); });
              else if (q[0] >= q_frac && q[3] < q_huge)
                acc4([&](double qq, double r) { return sincos_qr_frac(qq, r, kMagicV, kScale31); });
              else
                acc4([&](double qq, double r) { return sincos_qr_exact(qq, r, kRoundV); });
            }
          }
          const double G = adj_force_direct(use && r2 > 0.0, ir, cc, ss);
          const double cx = G * dx, cy = G * dy, cz = G * dz;
          gx += cx;
          gy += cy;
          gz += cz;
          const float sx = wave_total(static_cast<float>(cx));
          const float sy = wave_total(static_cast<float>(cy));
          const float sz = wave_total(static_cast<float>(cz));
          if (lane == 0) {
            double* gj = gjl + 3 * (jl - j0);
            gj[0] -= sx;
            gj[1] -= sy;
            gj[2] -= sz;
          }
        }
      } else {
        // two pairs (j, j+1) per iteration sharing the lane's weights and 1/q:
        // two independent recurrence chains for the scheduler to interleave; an
        // odd run ends with a masked partner (zero seeds, zero force)
#pragma unroll 1
        for (int jl = u0; jl < u0 + ns; jl += 2) {
          const bool two = jl + 1 < u0 + ns;
          const int jb = two ? jl + 1 : jl;
          const AdjSeed A = adj_seed(pi, sj[jl - u0], vi && jl > i, dq, qs);
          asm volatile("" ::: "memory");
          const AdjSeed B = adj_seed(pi, sj[jb - u0], vi && jb > i && two, dq, qs);
          asm volatile("" ::: "memory");
          const float* fa = fj[jl - u0];
          const float* fb = fj[jb - u0];
          float za = A.z, da = A.d, zb = B.z, db = B.d;
          float nla = A.nlam, nlb = B.nlam;  // laundered, as in k_adjoint
          asm volatile("" : "+v"(nla), "+v"(nlb));
          float a1e = 0.f, a1o = 0.f, a2e = 0.f, a2o = 0.f, a3e = 0.f, a3o = 0.f;
          float b1e = 0.f, b1o = 0.f, b2e = 0.f, b2o = 0.f, b3e = 0.f, b3o = 0.f;
          // the rows' values and 1/q for each 4 q steps are loaded one group
          // ahead, so the LDS latency overlaps the previous group's steps
          const float4* fa4 = reinterpret_cast<const float4*>(fa);
          const float4* fb4 = reinterpret_cast<const float4*>(fb);
          const float4* iq4 = reinterpret_cast<const float4*>(iql);
          float4 ca = fa4[0], cb = fb4[0], ci = iq4[0];
#pragma unroll
          for (int g4 = 0; g4 < QA / 4; ++g4) {
            float4 na = ca, nb = cb, ni = ci;
            if (g4 + 1 < QA / 4) {
              na = fa4[g4 + 1];
              nb = fb4[g4 + 1];
              ni = iq4[g4 + 1];
            }
            __builtin_amdgcn_sched_barrier(0);  // keep the loads issued here
            const float fav[4] = {ca.x, ca.y, ca.z, ca.w}, fbv[4] = {cb.x, cb.y, cb.z, cb.w};
            const float iqv[4] = {ci.x, ci.y, ci.z, ci.w};
#pragma unroll
            for (int k = 0; k < 4; k += 2) {
              const int m = 4 * g4 + k;
              const float iqe = iqv[k], iqo = iqv[k + 1];
              const float uae = wi[m] * fav[k], ube = wi[m] * fbv[k];
              const float vae = uae * iqe, vbe = ube * iqe;
              a1e = fmaf(uae, da, a1e);
              b1e = fmaf(ube, db, b1e);
              a2e = fmaf(uae, za, a2e);
              b2e = fmaf(ube, zb, b2e);
              a3e = fmaf(vae, za, a3e);
              b3e = fmaf(vbe, zb, b3e);
              za += da;
              zb += db;
              da = fmaf(nla, za, da);
              db = fmaf(nlb, zb, db);
              const float uao = wi[m + 1] * fav[k + 1], ubo = wi[m + 1] * fbv[k + 1];
              const float vao = uao * iqo, vbo = ubo * iqo;
              a1o = fmaf(uao, da, a1o);
              b1o = fmaf(ubo, db, b1o);
              a2o = fmaf(uao, za, a2o);
              b2o = fmaf(ubo, zb, b2o);
              a3o = fmaf(vao, za, a3o);
              b3o = fmaf(vbo, zb, b3o);
              za += da;
              zb += db;
              da = fmaf(nla, za, da);
              db = fmaf(nlb, zb, db);
            }
            ca = na;
            cb = nb;
            ci = ni;
          }
          const double GA = adj_force(A, a1e, a1o, a2e, a2o, a3e, a3o, dq, wi[0] * fa[0]);
          const double GB = adj_force(B, b1e, b1o, b2e, b2o, b3e, b3o, dq, wi[0] * fb[0]);
          const double cax = GA * A.dx, cay = GA * A.dy, caz = GA * A.dz;
          const double cbx = GB * B.dx, cby = GB * B.dy, cbz = GB * B.dz;
          gx += cax;
          gy += cay;
          gz += caz;
          gx += cbx;
          gy += cby;
          gz += cbz;
          const float sax = wave_total(static_cast<float>(cax));
          const float say = wave_total(static_cast<float>(cay));
          const float saz = wave_total(static_cast<float>(caz));
          const float sbx = wave_total(static_cast<float>(cbx));
          const float sby = wave_total(static_cast<float>(cby));
          const float sbz = wave_total(static_cast<float>(cbz));
          if (lane == 0) {
            double* ga = gjl + 3 * (jl - j0);
            ga[0] -= sax;
            ga[1] -= say;
            ga[2] -= saz;
            if (two) {
              double* gb = gjl + 3 * (jb - j0);
              gb[0] -= sbx;
              gb[1] -= sby;
              gb[2] -= sbz;
            }
          }
        }
      }
    }
    __syncthreads();
    double* outj = a.gJ + (pidx * a.geo.g * BJ + static_cast<int64_t>(J - sp.Ja) * BJ) * 3;
    for (int k = lane; k < 3 * (j1 - j0); k += kWave) outj[k] = gjl[k];
  }
  double* outi = a.gI + pidx * kWave * 3;
  outi[3 * lane + 0] = gx;
  outi[3 * lane + 1] = gy;
  outi[3 * lane + 2] = gz;
}

// The i-side rows of each (sorted) atom's own row of strips and the j-side
// rows of every strip that holds its J block, summed in FP64; the sum is
// written to the caller's row perm[a].  A work-group takes 32 atoms and splits
// each atom's strips among 8 parts (part k takes every 8th strip from the
// k-th), the 32 threads of a part reading 32 consecutive atoms' rows; the 8
// partial sums are then added in part order.  (One thread per atom walking
// all its strips kept most CUs idle: 115 us for 20,000 atoms.)
constexpr int kGradParts = 8, kGradAtoms = 32;
__global__ __launch_bounds__(kGradParts * kGradAtoms) void k_grad_reduce(AdjArgs a, int32_t nchunks,
                                                                        const int32_t* __restrict__ perm,
                                                                        double* __restrict__ grad_out) {
  __shared__ double red[kGradParts][kGradAtoms][3];
  const StructDesc d = a.sd.get(0);
  const int part = threadIdx.x / kGradAtoms, al = threadIdx.x % kGradAtoms;
  const int64_t at = static_cast<int64_t>(blockIdx.x) * kGradAtoms + al;
  const int64_t n = d.n, c = a.geo.c, g = a.geo.g, bj = a.geo.bj, ib = a.geo.ib;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  if (at < n && n >= 2) {
    const int64_t nI = ceil_div(n, ib), nJ = ceil_div(n, bj);
    const int64_t I = at / ib, lane = at % ib, J = at / bj;
    for (int32_t ch = 0; ch < nchunks; ++ch) {
      const int64_t base = static_cast<int64_t>(ch) * a.n_strips;
      const int64_t first = row_first_strip(I, nJ, c, g);
      const int64_t spr = strips_in_row(I, nJ, c, g);
      for (int64_t s = first + part; s < first + spr; s += kGradParts) {
        const double* p = a.gI + ((base + s) * ib + lane) * 3;
        sx += p[0];
        sy += p[1];
        sz += p[2];
      }
      const int64_t rows = min(nI, (J + 1) * c);
      for (int64_t Ip = part; Ip < rows; Ip += kGradParts) {
        int64_t ja = 0;
        const int64_t s = strip_holding(Ip, J, nJ, c, g, &ja);
        const double* p = a.gJ + ((base + s) * g * bj + (at - ja * bj)) * 3;
        sx += p[0];
        sy += p[1];
        sz += p[2];
      }
    }
  }
  red[part][al][0] = sx;
  red[part][al][1] = sy;
  red[part][al][2] = sz;
  __syncthreads();
  if (part == 0 && at < n) {
    for (int k = 1; k < kGradParts; ++k) {
      sx += red[k][al][0];
      sy += red[k][al][1];
      sz += red[k][al][2];
    }
    const int64_t dst = perm[d.atom_off + at];
    grad_out[dst * 3 + 0] = sx;
    grad_out[dst * 3 + 1] = sy;
    grad_out[dst * 3 + 2] = sz;
  }
}

bool adjoint_bj_supported(int32_t bj) { return bj == 128 || bj == 256; }

hipError_t launch_adjoint(const AdjArgs& a, int32_t nchunks, hipStream_t st) {
  if (a.n_strips <= 0) return hipSuccess;
  if (!geometry_ok(a.geo) || a.geo.ib != 2 * kWave || a.geo.g != 1) return hipErrorInvalidValue;
  const dim3 grid(static_cast<uint32_t>(a.n_strips), nchunks);
  switch (a.geo.bj) {
    case 128:
      if (a.qdev)
        hipLaunchKernelGGL((k_adjoint<128, true>), grid, dim3(kWave), 0, st, a);
      else
        hipLaunchKernelGGL((k_adjoint<128, false>), grid, dim3(kWave), 0, st, a);
      break;
    case 256:
      if (a.qdev)
        hipLaunchKernelGGL((k_adjoint<256, true>), grid, dim3(kWave), 0, st, a);
      else
        hipLaunchKernelGGL((k_adjoint<256, false>), grid, dim3(kWave), 0, st, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_adjoint_pa(const AdjArgs& a, int32_t nchunks, int32_t qa_template, hipStream_t st) {
  if (a.n_strips <= 0) return hipSuccess;
  if (!geometry_ok(a.geo) || a.geo.bj != kAdjPaBJ || a.geo.ib != kWave || a.geo.g != 1 || a.qa > qa_template)
    return hipErrorInvalidValue;
  const dim3 grid(static_cast<uint32_t>(a.n_strips), nchunks);
  if (a.qdev) {
    if (qa_template != 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_adjoint_pa<64, true>), grid, dim3(kWave), 0, st, a);
    return hipGetLastError();
  }
  switch (qa_template) {
    case 32: hipLaunchKernelGGL((k_adjoint_pa<32, false>), grid, dim3(kWave), 0, st, a); break;
    case 64: hipLaunchKernelGGL((k_adjoint_pa<64, false>), grid, dim3(kWave), 0, st, a); break;
    case 100: hipLaunchKernelGGL((k_adjoint_pa<100, false>), grid, dim3(kWave), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_grad_reduce(const AdjArgs& a, int64_t n, int32_t nchunks, const int32_t* perm, double* grad_out,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (!geometry_ok(a.geo)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_grad_reduce, dim3(static_cast<uint32_t>(ceil_div(n, kGradAtoms))), dim3(kGradParts * kGradAtoms),
                     0, st, a, nchunks, perm, grad_out);
  return hipGetLastError();
}

}  // namespace sas
