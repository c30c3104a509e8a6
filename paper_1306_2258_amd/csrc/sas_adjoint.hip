// Adjoint of the Debye profile with respect to the coordinates (gfx950).
//
// For weights w_m (dL/dI(q_m)) the derivative of Eq. 2 gives, per atom pair
// (i, j) at distance r with form factors f_a, f_b:
//     C = sum_m U_m cos(q_m r),  S = sum_m V_m sin(q_m r),
//     U_m = w_m f_a(q_m) f_b(q_m),  V_m = U_m / q_m   (both 0 where q_m = 0),
//     G = 2 (C / r^2 - S / r^3),  g_i += G (x_i - x_j),  g_j -= G (x_i - x_j).
// The pair loop is the forward kernel's: one 64-lane wave per (I block, strip
// of J blocks, q chunk), J blocks staged in LDS, the same FP64 set-up and the
// same FP32 recurrence z_{m+1} = z_m + d_m, d_{m+1} = d_m - lambda z_{m+1}
// with z_m = sin(phi_m), phi_m = q_s r + m dp.  The cosine comes from the
// recurrence state itself, cos(phi_m) = (d_m + (lambda/2) z_m) / sin(dp), so a
// q step costs five FP32 operations: two for the recurrence and three
// accumulations (U d, U z, V z), kept separately for even and odd m to fold
// in the sign (-1)^(k m) of the reduction dq r = k pi + dp.  Lanes of one
// wave may hold atoms of several types; the wave visits each type present
// (almost always one) with the other lanes masked, so that U and V are
// wave-uniform and read from LDS.  The i-side sums stay in the lane (FP64);
// the j-side sums are reduced over the 64 lanes per j and kept in FP64 in LDS.
// Partial sums go to per-strip rows that a second kernel adds in fixed order.
#include <hip/hip_runtime.h>

#include "sas_device.hpp"
#include "sas_kernels.hpp"
#include "sas_schedule.hpp"

namespace sas {

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

template <int BJ>
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
  const int i = sp.I * kWave + lane;
  const bool vi = i < n;
  const int ic = vi ? i : n - 1;
  const double4 pi = a.xyz[d.atom_off + ic];
  const int ta = clamp_type(a.tsort[d.atom_off + ic], a.T);

  const int m0 = blockIdx.y * a.qa;
  const int nqa = min(a.qa, a.Nq - m0);
  const int nq8 = (nqa + 7) & ~7;
  const double qs = a.q0 + m0 * a.dq;
  const double dq = a.dq;
  const int64_t pidx = static_cast<int64_t>(blockIdx.y) * a.n_strips + t;
  const int32_t* toff = a.toff;

  double gx = 0.0, gy = 0.0, gz = 0.0;

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
      uint64_t remaining = __ballot(vi);
#pragma unroll 1
      while (remaining) {
        const int src = __ffsll(static_cast<unsigned long long>(remaining)) - 1;
        const int at = __shfl(ta, src, kWave);
        const bool mine = vi && ta == at;
        remaining &= ~static_cast<uint64_t>(__ballot(mine));
        // wave-uniform weights of the (at, tb) type pair for this chunk
        __syncthreads();
        const float* fa = a.tabp + static_cast<int64_t>(at) * a.ldt + m0;
        const float* fb = a.tabp + static_cast<int64_t>(tb) * a.ldt + m0;
        for (int m = lane; m < nq8; m += kWave) {
          float u = 0.f, v = 0.f;
          const double qm = a.q0 + (m0 + m) * dq;
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
#pragma unroll 1
        for (int jl = sa; jl < sb; ++jl) {
          const double4 pj = sj[jl - j0];
          const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
          const double r2raw = fma(dz, dz, fma(dy, dy, dx * dx));
          const bool valid = mine && jl > i && r2raw > 0.0;
          const double r2 = fmax(r2raw, 1e-60);
          const double ir = rsqrt_f64(r2);
          const double r = r2 * ir;
          const double delta = dq * r;
          const double k = rint(delta * kOneOverPi);
          double dp = fma(-k, kPiA, delta);
          dp = fma(-k, kPiB, dp);
          dp = fma(-k, kPiC, dp);
          const SinCos hh = sincos_small(0.5 * dp);
          const double sdp = 2.0 * hh.s * hh.c;  // sin(dp)
          const double omc = 2.0 * hh.s * hh.s;  // 1 - cos(dp) = lambda / 2
          const float nlam = static_cast<float>(-2.0 * omc);
          const float sg = (static_cast<int>(k) & 1) ? -1.f : 1.f;
          double S0 = 0.0, C0 = 1.0;
          if (qs != 0.0) {
            const SinCos t0 = sincos_any(qs * r);
            S0 = t0.s;
            C0 = t0.c;
          }
          float z = static_cast<float>(S0);
          float dd = static_cast<float>(fma(C0, sdp, -S0 * omc));
          float a1e = 0.f, a1o = 0.f, a2e = 0.f, a2o = 0.f, a3e = 0.f, a3o = 0.f;
#pragma unroll 1
          for (int m = 0; m < nq8; m += 8) {
            const float4 ua = ul4[m >> 2], ub = ul4[(m >> 2) + 1];
            const float4 va = vl4[m >> 2], vb = vl4[(m >> 2) + 1];
            const float uu[8] = {ua.x, ua.y, ua.z, ua.w, ub.x, ub.y, ub.z, ub.w};
            const float vv[8] = {va.x, va.y, va.z, va.w, vb.x, vb.y, vb.z, vb.w};
#pragma unroll
            for (int s = 0; s < 8; s += 2) {
              a1e = fmaf(uu[s], dd, a1e);
              a2e = fmaf(uu[s], z, a2e);
              a3e = fmaf(vv[s], z, a3e);
              z += dd;
              dd = fmaf(nlam, z, dd);
              a1o = fmaf(uu[s + 1], dd, a1o);
              a2o = fmaf(uu[s + 1], z, a2o);
              a3o = fmaf(vv[s + 1], z, a3o);
              z += dd;
              dd = fmaf(nlam, z, dd);
            }
          }
          const double A1 = static_cast<double>(a1e) + sg * static_cast<double>(a1o);
          const double A2 = static_cast<double>(a2e) + sg * static_cast<double>(a2o);
          const double A3 = static_cast<double>(a3e) + sg * static_cast<double>(a3o);
          // sum_m U_m cos(q_m r); with dq = 0 (a single q) the recurrence is
          // constant and the cosine is the seed's
          // (sdp = 0 with dq != 0 needs dq r to be an exact multiple of pi in
          // FP64; the seed's cosine is used there too)
          const double Cc = (dq != 0.0 && sdp != 0.0) ? (A1 + omc * A2) / sdp : static_cast<double>(u0) * C0;
          const double G = valid ? 2.0 * ir * ir * (Cc - A3 * ir) : 0.0;
          const double cx = G * dx, cy = G * dy, cz = G * dz;
          gx += cx;
          gy += cy;
          gz += cz;
          const float sx = wave_sum(static_cast<float>(cx));
          const float sy = wave_sum(static_cast<float>(cy));
          const float sz = wave_sum(static_cast<float>(cz));
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
  double* outi = a.gI + (pidx * kWave + lane) * 3;
  outi[0] = gx;
  outi[1] = gy;
  outi[2] = gz;
}

// One thread per (sorted) atom: the i-side rows of its own row of strips and
// the j-side rows of every strip that holds its J block, in a fixed order;
// the sum is written to the caller's row perm[a].
__global__ __launch_bounds__(256) void k_grad_reduce(AdjArgs a, int32_t nchunks, const int32_t* __restrict__ perm,
                                                     double* __restrict__ grad_out) {
  const StructDesc d = a.sd.get(0);
  const int64_t at = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (at >= d.n) return;
  const int64_t n = d.n, c = a.geo.c, g = a.geo.g, bj = a.geo.bj;
  const int64_t nI = ceil_div(n, kWave), nJ = ceil_div(n, bj);
  const int64_t I = at / kWave, lane = at % kWave, J = at / bj;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  if (n >= 2) {
    for (int32_t ch = 0; ch < nchunks; ++ch) {
      const int64_t base = static_cast<int64_t>(ch) * a.n_strips;
      const int64_t first = row_first_strip(I, nJ, c, g);
      const int64_t spr = ceil_div(nJ - I / c, g);
      for (int64_t s = first; s < first + spr; ++s) {
        const double* p = a.gI + ((base + s) * kWave + lane) * 3;
        sx += p[0];
        sy += p[1];
        sz += p[2];
      }
      const int64_t rows = min(nI, (J + 1) * c);
      for (int64_t Ip = 0; Ip < rows; ++Ip) {
        const int64_t u = Ip / c;
        const int64_t gi = (J - u) / g;
        const int64_t s = row_first_strip(Ip, nJ, c, g) + gi;
        const int64_t ja = u + gi * g;
        const double* p = a.gJ + ((base + s) * g * bj + (at - ja * bj)) * 3;
        sx += p[0];
        sy += p[1];
        sz += p[2];
      }
    }
  }
  const int64_t dst = perm[d.atom_off + at];
  grad_out[dst * 3 + 0] = sx;
  grad_out[dst * 3 + 1] = sy;
  grad_out[dst * 3 + 2] = sz;
}

bool adjoint_bj_supported(int32_t bj) { return bj == 64 || bj == 128 || bj == 256; }

hipError_t launch_adjoint(const AdjArgs& a, int32_t nchunks, hipStream_t st) {
  if (a.n_strips <= 0) return hipSuccess;
  const dim3 grid(static_cast<uint32_t>(a.n_strips), nchunks);
  switch (a.geo.bj) {
    case 64: hipLaunchKernelGGL((k_adjoint<64>), grid, dim3(kWave), 0, st, a); break;
    case 128: hipLaunchKernelGGL((k_adjoint<128>), grid, dim3(kWave), 0, st, a); break;
    case 256: hipLaunchKernelGGL((k_adjoint<256>), grid, dim3(kWave), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_grad_reduce(const AdjArgs& a, int64_t n, int32_t nchunks, const int32_t* perm, double* grad_out,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad_reduce, dim3(static_cast<uint32_t>((n + 255) / 256)), dim3(256), 0, st, a, nchunks, perm,
                     grad_out);
  return hipGetLastError();
}

}  // namespace sas
