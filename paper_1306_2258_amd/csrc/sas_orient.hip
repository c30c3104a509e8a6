// Orientation-averaged profile: Eq. 1 evaluated by quadrature over the
// sphere, the approximate family the Background section weighs against the
// direct sum (orientation sampling needs O(q^2 D^2) directions, so it pays
// only at low q).  For direction u,
//     A(q, u) = sum_j f_j(q) exp(i q u . (r_j - c)),   I(q) = <|A(q, u)|^2>_u,
// with c the molecule's centre.  |A|^2 is band-limited in u: its spherical
// harmonic content beyond degree 2L decays faster than exponentially once L
// exceeds q R (R the largest |r_j - c|), so a product rule with L + 1
// Gauss-Legendre nodes in cos(theta) and 2L + 1 uniform nodes in phi averages
// it to any wanted accuracy; the host picks L per chunk of q values.
//
// Kernels:
//   k_geometry      centre (mean position) and radius R, in FP64, fixed order;
//   k_orient_amp    one 64-lane wave per (64 directions, chunk of kOrientQ q,
//                   part of the atoms): the atoms (FP64 positions and their
//                   table rows, runs of kPaSub) are staged in LDS; per atom and
//                   direction the projection p = u . (r - c) in FP64, per q the
//                   sine and cosine of q p by the direct form's FP64 reduction
//                   and FP32 polynomials; FP32 sums over each run, FP64 across
//                   runs; one partial amplitude per (part, direction, q).
//                   On a uniform grid whose step turns the phase of the
//                   farthest atom by at most kRotMaxStep, the ROT variant
//                   evaluates exp(i q p) only at the chunk's first q and
//                   walks the rest by z <- z + z d, d = exp(i dq p) - 1:
//                   four FP32 FMAs per q instead of a reduction and two
//                   polynomials.  The start and d are FP64 (series
//                   truncation below 1e-11) rounded once to FP32, so their
//                   errors are plain roundings that differ from atom to
//                   atom; an error common to all atoms would not average
//                   out (see the kernel);
//   k_orient_reduce_slices, k_orient_reduce_final
//                   sum_k w_k |sum_parts A|^2 per q: per (slice of the
//                   directions, chunk) with coalesced reads, then the slices
//                   in order.
#include <hip/hip_runtime.h>

#include "sas_device.hpp"
#include "sas_kernels.hpp"
#include "sas_schedule.hpp"

namespace sas {

// cos(x) - 1 and sin(x) for |x| <= kRotMaxStep by their Taylor series, without
// forming cos(x) itself (1 + small would lose the small part's low bits).  The
// walk applies this increment at every step, so it keeps the series' exact
// leading coefficients (-1/2, -1/6): relative accuracy as x -> 0.  Terms
// through x^11 (sin) and x^12 (cos) leave a truncation below 1e-11 relative
// for |x| <= pi/4.
constexpr double fact(int n) { return n <= 1 ? 1.0 : n * fact(n - 1); }
constexpr double kS3 = -1.0 / fact(3), kS5 = 1.0 / fact(5), kS7 = -1.0 / fact(7), kS9 = 1.0 / fact(9);
constexpr double kS11 = -1.0 / fact(11);
constexpr double kC2 = -1.0 / fact(2), kC4 = 1.0 / fact(4), kC6 = -1.0 / fact(6), kC8 = 1.0 / fact(8);
constexpr double kC10 = -1.0 / fact(10), kC12 = 1.0 / fact(12);

struct StepInc {
  double cm1, s;
};
__device__ __forceinline__ StepInc step_increment(double x) {
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
  return StepInc{x2 * pc, fma(x * x2, ps, x)};
}

__global__ __launch_bounds__(1024) void k_geometry(const double4* __restrict__ xyz, int64_t n,
                                                   double* __restrict__ out) {
  __shared__ double red[1024][3];
  __shared__ double cen[3];
  const int t = threadIdx.x;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (int64_t k = t; k < n; k += blockDim.x) {
    const double4 p = xyz[k];
    sx += p.x;
    sy += p.y;
    sz += p.z;
  }
  red[t][0] = sx;
  red[t][1] = sy;
  red[t][2] = sz;
  __syncthreads();
  for (int h = 512; h >= 1; h >>= 1) {
    if (t < h)
      for (int d = 0; d < 3; ++d) red[t][d] += red[t + h][d];
    __syncthreads();
  }
  if (t == 0)
    for (int d = 0; d < 3; ++d) cen[d] = n > 0 ? red[0][d] / static_cast<double>(n) : 0.0;
  __syncthreads();
  double r2 = 0.0;
  for (int64_t k = t; k < n; k += blockDim.x) {
    const double4 p = xyz[k];
    const double dx = p.x - cen[0], dy = p.y - cen[1], dz = p.z - cen[2];
    r2 = fmax(r2, fma(dz, dz, fma(dy, dy, dx * dx)));
  }
  red[t][0] = r2;
  __syncthreads();
  for (int h = 512; h >= 1; h >>= 1) {
    if (t < h) red[t][0] = fmax(red[t][0], red[t + h][0]);
    __syncthreads();
  }
  if (t == 0) {
    out[0] = cen[0];
    out[1] = cen[1];
    out[2] = cen[2];
    out[3] = sqrt(red[0][0]);
  }
}

__device__ __forceinline__ int find_chunk(const OrientChunk* ch, int nchunks, int64_t blk) {
  int lo = 0, hi = nchunks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ch[mid].blk_off <= blk)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <bool ROT>
__global__ __launch_bounds__(kWave, 3) void k_orient_amp(OrientArgs a) {
  constexpr int QO = kOrientQ;
  __shared__ double4 sj[kPaSub];
  __shared__ __align__(16) float fj[kPaSub][QO];
  __shared__ double qs[QO];
  const int lane = threadIdx.x;
  const int64_t blk = blockIdx.x;
  const int part = blockIdx.y;
  const int c = find_chunk(a.chunks, a.nchunks, blk);
  const OrientChunk ch = a.chunks[c];
  const int64_t kdir = (blk - ch.blk_off) * kWave + lane;
  const int64_t ndir = static_cast<int64_t>(ch.nth) * ch.nph;
  const bool valid = kdir < ndir;
  const int64_t kk = valid ? kdir : 0;
  // this lane's direction: cos(theta) at a Gauss-Legendre node, phi uniform
  const int ith = static_cast<int>(kk / ch.nph);
  const int iph = static_cast<int>(kk - static_cast<int64_t>(ith) * ch.nph);
  const double ct = a.gl[2 * (ch.gl_off + ith)];
  const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
  const SinCos ph = sincos_any(kTwoPi * static_cast<double>(iph) / static_cast<double>(ch.nph));
  const double ux = st * ph.c, uy = st * ph.s, uz = ct;
  const double cx = a.center[0], cy = a.center[1], cz = a.center[2];
  for (int m = lane; m < QO; m += kWave) qs[m] = m < ch.nq ? a.qv[ch.m0 + m] : 0.0;

  double re[QO], im[QO];
#pragma unroll
  for (int m = 0; m < QO; ++m) re[m] = im[m] = 0.0;
  const int64_t a0 = static_cast<int64_t>(part) * a.atoms_per_part;
  const int64_t a1 = min(static_cast<int64_t>(a.n), a0 + a.atoms_per_part);
  constexpr int Q4 = QO / 4;
  constexpr int E4 = kPaSub * Q4;
#pragma unroll 1
  for (int64_t u0 = a0; u0 < a1; u0 += kPaSub) {
    const int ns = static_cast<int>(min(static_cast<int64_t>(kPaSub), a1 - u0));
    __syncthreads();
    const int ty = lane < ns ? clamp_type(a.tsort[u0 + lane], a.T) : 0;  // row 0 past the run
    if (lane < ns) {
      const double4 p = a.xyz[u0 + lane];
      sj[lane] = make_double4(p.x - cx, p.y - cy, p.z - cz, 0.0);
    }
    for (int e = lane; e < E4; e += kWave) {
      const int r = e / Q4;
      const int cc = e - r * Q4;
      const int tr = __shfl(ty, r, kWave);
      reinterpret_cast<float4*>(&fj[0][0])[e] =
          *reinterpret_cast<const float4*>(a.tabp + static_cast<int64_t>(tr) * a.ldt + ch.m0 + 4 * cc);
    }
    __syncthreads();
    float sre[QO], sim[QO];
#pragma unroll
    for (int m = 0; m < QO; ++m) sre[m] = sim[m] = 0.f;
#pragma unroll 1
    for (int jl = 0; jl < ns; ++jl) {
      asm volatile("" ::: "memory");
      const double4 p = sj[jl];
      const double pd = fma(uz, p.z, fma(uy, p.y, ux * p.x));
      const float* f = fj[jl];
      if constexpr (ROT) {
        // The start exp(i q_m0 p) in FP64: an FP32 polynomial's error has a
        // mean common to all atoms, and the walk would turn that constant
        // into a copy of the amplitude at q = m dq, large at low q.
        const SinCos z0 = sincos_any(qs[0] * pd);
        const StepInc d = step_increment(a.dq * pd);
        const float dr = static_cast<float>(d.cm1), di = static_cast<float>(d.s);
        float zr = static_cast<float>(z0.c), zi = static_cast<float>(z0.s);
#pragma unroll
        for (int m = 0; m < QO; ++m) {
          sre[m] = fmaf(f[m], zr, sre[m]);
          sim[m] = fmaf(f[m], zi, sim[m]);
          if (m + 1 < QO) {
            const float nr = fmaf(zr, dr, fmaf(-zi, di, zr));
            const float ni = fmaf(zr, di, fmaf(zi, dr, zi));
            zr = nr;
            zi = ni;
          }
        }
      } else {
        const double rp = pd * kOneOverPi;
#pragma unroll
        for (int m = 0; m < QO; ++m) {
          const SinCosF e = sincos_qr(qs[m], rp);
          sre[m] = fmaf(f[m], e.c, sre[m]);
          sim[m] = fmaf(f[m], e.s, sim[m]);
        }
      }
    }
#pragma unroll
    for (int m = 0; m < QO; ++m) {
      re[m] += static_cast<double>(sre[m]);
      im[m] += static_cast<double>(sim[m]);
    }
  }
  if (valid) {
    double2* out = a.apart + ch.a_off + (static_cast<int64_t>(part) * ndir + kdir) * QO;
#pragma unroll
    for (int m = 0; m < QO; ++m) out[m] = make_double2(re[m], im[m]);
  }
}

// First pass of sum_k w_k |sum over parts of A|^2: one work-group per (slice
// of a chunk's directions, chunk).  Thread t takes q value m = t % 16 of the
// chunk and every 16th direction of the slice from t / 16 on, so that the 64
// lanes of a wave read 64 consecutive amplitudes (four directions x 16 q);
// the 16 threads of each q value are then added in a fixed tree.  (One
// work-group per q value, walking all directions with 16-element strides,
// left most CUs idle and took 1.9 ms on the 50,000-atom globule.)
__global__ __launch_bounds__(256) void k_orient_reduce_slices(OrientArgs a) {
  __shared__ double red[256];
  const int s = blockIdx.x, c = blockIdx.y;
  const int t = threadIdx.x;
  const int m = t % kOrientQ, kk = t / kOrientQ;
  const OrientChunk ch = a.chunks[c];
  const int64_t ndir = static_cast<int64_t>(ch.nth) * ch.nph;
  const int64_t k0 = ndir * s / kOrientSlices, k1 = ndir * (s + 1) / kOrientSlices;
  double acc = 0.0;
  for (int64_t k = k0 + kk; k < k1; k += 256 / kOrientQ) {
    double xr = 0.0, xi = 0.0;
    for (int p = 0; p < a.parts; ++p) {
      const double2 v = a.apart[ch.a_off + (static_cast<int64_t>(p) * ndir + k) * kOrientQ + m];
      xr += v.x;
      xi += v.y;
    }
    const int ith = static_cast<int>(k / ch.nph);
    const double w = a.gl[2 * (ch.gl_off + ith) + 1] / (2.0 * ch.nph);
    acc = fma(w, fma(xr, xr, xi * xi), acc);
  }
  red[t] = acc;
  __syncthreads();
  for (int h = 256 / kOrientQ / 2; h >= 1; h >>= 1) {
    if (kk < h) red[t] += red[t + h * kOrientQ];
    __syncthreads();
  }
  if (kk == 0) a.ored[(static_cast<int64_t>(c) * kOrientSlices + s) * kOrientQ + m] = red[t];
}

// Second pass: I(q) of orientation q value mo = chunk * 16 + m, the slices'
// sums added in order.
__global__ __launch_bounds__(256) void k_orient_reduce_final(OrientArgs a, int32_t nq_o, double* __restrict__ I_out) {
  const int mo = blockIdx.x * blockDim.x + threadIdx.x;
  if (mo >= nq_o) return;
  const int c = mo / kOrientQ, m = mo - c * kOrientQ;
  const double* r = a.ored + static_cast<int64_t>(c) * kOrientSlices * kOrientQ + m;
  double sum = 0.0;
  for (int s = 0; s < kOrientSlices; ++s) sum += r[s * kOrientQ];
  I_out[mo] = sum;
}

// Copy columns [col0, col0 + ncols) of a [T][ld_src] table into [T][ldt],
// zero beyond ncols.
__global__ __launch_bounds__(256) void k_copy_cols(const float* __restrict__ src, int32_t T, int32_t ld_src,
                                                   int32_t col0, int32_t ncols, int32_t ldt, float* __restrict__ dst) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= static_cast<int64_t>(T) * ldt) return;
  const int64_t t = k / ldt;
  const int32_t m = static_cast<int32_t>(k - t * ldt);
  dst[k] = m < ncols ? src[t * ld_src + col0 + m] : 0.f;
}

hipError_t launch_geometry(const double4* xyz, int64_t n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_geometry, dim3(1), dim3(1024), 0, st, xyz, n, out);
  return hipGetLastError();
}

hipError_t launch_orient(const OrientArgs& a, int64_t total_blocks, int32_t nq_o, double* I_out, hipStream_t st) {
  if (total_blocks > 0 && nq_o > 0) {
    const dim3 grid(static_cast<uint32_t>(total_blocks), a.parts);
    if (a.rot)
      hipLaunchKernelGGL(k_orient_amp<true>, grid, dim3(kWave), 0, st, a);
    else
      hipLaunchKernelGGL(k_orient_amp<false>, grid, dim3(kWave), 0, st, a);
    hipLaunchKernelGGL(k_orient_reduce_slices, dim3(kOrientSlices, static_cast<uint32_t>(a.nchunks)), dim3(256), 0,
                       st, a);
    hipLaunchKernelGGL(k_orient_reduce_final, dim3(static_cast<uint32_t>(ceil_div(nq_o, 256))), dim3(256), 0, st, a,
                       nq_o, I_out);
  }
  return hipGetLastError();
}

int orient_wgs_per_cu(bool rot) {
  int k = 0;
  const hipError_t e = rot ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&k, k_orient_amp<true>, kWave, 0)
                           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&k, k_orient_amp<false>, kWave, 0);
  return e == hipSuccess && k > 0 ? k : 4 * 2;
}

hipError_t launch_copy_cols(const float* src, int32_t T, int32_t ld_src, int32_t col0, int32_t ncols, int32_t ldt,
                            float* dst, hipStream_t st) {
  const int64_t total = static_cast<int64_t>(T) * ldt;
  if (total > 0) {
    hipLaunchKernelGGL(k_copy_cols, dim3(static_cast<uint32_t>(ceil_div(total, 256))), dim3(256), 0, st, src, T,
                       ld_src, col0, ncols, ldt, dst);
  }
  return hipGetLastError();
}

}  // namespace sas
