// HIP kernels of the Debye summation for gfx950 (CDNA4).
//
// Pipeline of one profile evaluation (Implementation section: atoms spread
// over workers, blocks of atoms staged in fast local memory and swept by every
// worker, only pairs j > k evaluated, a local reduction per work-group and a
// final reduction of the work-group totals):
//
//   pack     stable counting sort of each structure's atoms by type, FP64
//            coordinates in the sorted order (so that every J block splits into
//            a few constant-type segments and f_a f_b factors out of the sum);
//   forward  (template in sas_forward_kernel.hpp) one 64-lane wave per
//            (I block, strip of J blocks, q chunk): each
//            lane owns one i atom, the J block is staged in LDS and swept by
//            all lanes; per pair a sin/cos set-up in FP64, then an FP32
//            second-order recurrence over the uniform q grid; per type segment
//            a transpose-reduction over the 64 lanes and an FP64 product with
//            the segment's form factor; one FP64 partial row per strip;
//   reduce   fixed-order FP64 sums of the partial rows (two levels), the
//            diagonal sum_a n_a f_a^2, the 2/q factor and the exact q = 0 value.
#include <hip/hip_runtime.h>

#include "sas_device.hpp"
#include "sas_forward.hpp"
#include "sas_forward_kernel.hpp"
#include "sas_kernels.hpp"
#include "sas_schedule.hpp"

namespace sas {

int64_t slices_of(int64_t n_strips) { return ceil_div(n_strips, kSliceTiles); }

// ---------------------------------------------------------------------------
// Pack: stable counting sort by type, per structure, in blocks of kPackBlock.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kPackBlock) void k_pack_count(const int32_t* __restrict__ types, DescView sd, int32_t T,
                                                           int32_t* __restrict__ bcount) {
  extern __shared__ int32_t cnt[];
  const int64_t b = blockIdx.x;
  const int s = find_struct_by_pack(sd, b);
  const StructDesc d = sd.get(s);
  for (int t = threadIdx.x; t < T; t += blockDim.x) cnt[t] = 0;
  __syncthreads();
  const int64_t a = (b - d.pack_off) * kPackBlock + threadIdx.x;
  if (a < d.n) atomicAdd(&cnt[clamp_type(types[d.atom_off + a], T)], 1);
  __syncthreads();
  for (int t = threadIdx.x; t < T; t += blockDim.x) bcount[b * T + t] = cnt[t];
}

// One work-group per structure.  Per type, an exclusive scan of its per-block
// counts (wave w takes types w, w + 4, ...; the 64 lanes scan 64 blocks at a
// time); then the type segments' absolute starts toff[s][0..T] in type
// order; then every block's destination base of every type is that start
// plus its exclusive count.
__global__ __launch_bounds__(256) void k_pack_scan(DescView sd, int32_t T, int32_t* __restrict__ bcount,
                                                   int32_t* __restrict__ toff) {
  extern __shared__ int32_t tot[];
  const int s = blockIdx.x;
  const StructDesc d = sd.get(s);
  const int64_t nb = ceil_div(d.n, kPackBlock);
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  for (int t = w; t < T; t += nw) {
    int32_t run = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kWave) {
      const int64_t lb = b0 + lane;
      int32_t* p = bcount + (d.pack_off + lb) * T + t;
      const int32_t c = lb < nb ? *p : 0;
      int32_t x = c;  // inclusive scan over the wave
      for (int off = 1; off < kWave; off <<= 1) {
        const int32_t y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
      }
      if (lb < nb) *p = run + x - c;
      run += __shfl(x, kWave - 1, kWave);
    }
    if (lane == 0) tot[t] = run;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = d.atom_off;
    int32_t* o = toff + static_cast<int64_t>(s) * (T + 1);
    for (int t = 0; t < T; ++t) {
      const int32_t c = tot[t];
      o[t] = static_cast<int32_t>(run);
      tot[t] = static_cast<int32_t>(run);
      run += c;
    }
    o[T] = static_cast<int32_t>(run);
  }
  __syncthreads();
  int32_t* base = bcount + static_cast<int64_t>(d.pack_off) * T;
  for (int64_t k = threadIdx.x; k < nb * T; k += blockDim.x) base[k] += tot[k % T];
}

__global__ __launch_bounds__(kPackBlock) void k_pack_scatter(const float* __restrict__ coords,
                                                             const int32_t* __restrict__ types, DescView sd,
                                                             int32_t T, const int32_t* __restrict__ bcount,
                                                             double4* __restrict__ xyz, int32_t* __restrict__ tsort,
                                                             int32_t* __restrict__ perm) {
  __shared__ int32_t ty[kPackBlock];
  const int64_t b = blockIdx.x;
  const int s = find_struct_by_pack(sd, b);
  const StructDesc d = sd.get(s);
  const int64_t first = (b - d.pack_off) * kPackBlock;
  const int64_t a = first + threadIdx.x;
  const bool live = a < d.n;
  const int t = live ? clamp_type(types[d.atom_off + a], T) : -1;
  ty[threadIdx.x] = t;
  __syncthreads();
  if (!live) return;
  int rank = 0;
  for (int p = 0; p < static_cast<int>(threadIdx.x); ++p) rank += (ty[p] == t);
  const int64_t dest = static_cast<int64_t>(bcount[b * T + t]) + rank;
  const int64_t src = d.atom_off + a;
  xyz[dest] = make_double4(coords[3 * src], coords[3 * src + 1], coords[3 * src + 2], 0.0);
  tsort[dest] = t;
  perm[dest] = static_cast<int32_t>(src);
}

// Copy the caller's [T][Nq] table into [T][ldt] with zeros in columns >= Nq.
__global__ __launch_bounds__(256) void k_pad_table(const float* __restrict__ table, int32_t T, int32_t Nq,
                                                   int32_t ldt, float* __restrict__ tabp,
                                                   unsigned long long* __restrict__ counter) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k == 0 && counter) *counter = 0ull;
  if (k >= static_cast<int64_t>(T) * ldt) return;
  const int64_t t = k / ldt;
  const int32_t m = static_cast<int32_t>(k - t * ldt);
  tabp[k] = m < Nq ? table[t * Nq + m] : 0.f;
}

// Input check of the debug mode: flags[0] and flags[1] count atoms with a
// type id outside [0, T) and atoms with a non-finite coordinate, flags[2] and
// flags[3] hold the first such atom (the host sets them to all ones).
__global__ __launch_bounds__(256) void k_validate(const float* __restrict__ coords, const int32_t* __restrict__ types,
                                                  int64_t n, int32_t T, unsigned long long* __restrict__ flags) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += stride) {
    const int32_t ty = types[k];
    const float x = coords[3 * k], y = coords[3 * k + 1], z = coords[3 * k + 2];
    if (ty < 0 || ty >= T) {
      atomicAdd(&flags[0], 1ull);
      atomicMin(&flags[2], static_cast<unsigned long long>(k));
    }
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
      atomicAdd(&flags[1], 1ull);
      atomicMin(&flags[3], static_cast<unsigned long long>(k));
    }
  }
}

hipError_t launch_validate(const float* coords, const int32_t* types, int64_t n, int32_t T, unsigned long long* flags,
                           hipStream_t st) {
  if (n > 0) {
    const int64_t blocks = std::min<int64_t>(ceil_div(n, int64_t(256)), 2048);
    hipLaunchKernelGGL(k_validate, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, st, coords, types, n, T, flags);
  }
  return hipGetLastError();
}

hipError_t launch_pad_table(const float* table, int32_t T, int32_t Nq, int32_t ldt, float* tabp, hipStream_t st,
                            unsigned long long* counter) {
  const int64_t total = static_cast<int64_t>(T) * ldt;
  hipLaunchKernelGGL(k_pad_table, dim3(static_cast<uint32_t>((total + 255) / 256)), dim3(256), 0, st, table, T, Nq,
                     ldt, tabp, counter);
  return hipGetLastError();
}

hipError_t launch_pack(const float* coords, const int32_t* types, const DescView& sd, int32_t S,
                       int64_t n_pack_blocks, int32_t T, int32_t* bcount, int32_t* toff, double4* xyz,
                       int32_t* tsort, int32_t* perm, hipStream_t st) {
  if (n_pack_blocks > 0) {
    hipLaunchKernelGGL(k_pack_count, dim3(static_cast<uint32_t>(n_pack_blocks)), dim3(kPackBlock),
                       sizeof(int32_t) * T, st, types, sd, T, bcount);
  }
  if (S > 0) {
    hipLaunchKernelGGL(k_pack_scan, dim3(S), dim3(256), sizeof(int32_t) * T, st, sd, T, bcount, toff);
  }
  if (n_pack_blocks > 0) {
    hipLaunchKernelGGL(k_pack_scatter, dim3(static_cast<uint32_t>(n_pack_blocks)), dim3(kPackBlock), 0, st, coords,
                       types, sd, T, bcount, xyz, tsort, perm);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Forward strips (recurrence and lane reductions: sas_forward.hpp).
// ---------------------------------------------------------------------------

bool forward_qc_supported(int32_t qc) {
  return qc == 16 || qc == 32 || qc == 50 || qc == 64 || qc == 100 || qc == 128 || qc == 150 || qc == 200;
}
bool forward_bj_supported(int32_t bj) { return bj == 64 || bj == 128 || bj == 256 || bj == 512; }

bool direct_qc_supported(int32_t qc) { return qc == 32; }

hipError_t launch_forward(const ForwardArgs& a, int64_t n_strips_total, int32_t qc_template, hipStream_t st) {
  if (n_strips_total <= 0) return hipSuccess;
  if (!geometry_ok(a.geo)) return hipErrorInvalidValue;
  const int nchunks = static_cast<int>(ceil_div(a.Nq, a.qc));
  const dim3 grid(static_cast<uint32_t>(n_strips_total), nchunks);
  if (a.counter) {
    // persistent launch (recurrence form only)
    if (a.qdev || a.n_work != n_strips_total * nchunks) return hipErrorInvalidValue;
    switch (qc_template) {
      case 16: return launch_forward_persist_qc<16>(a, st);
      case 32: return launch_forward_persist_qc<32>(a, st);
      case 50: return launch_forward_persist_qc<50>(a, st);
      case 64: return launch_forward_persist_qc<64>(a, st);
      case 100: return launch_forward_persist_qc<100>(a, st);
      case 128: return launch_forward_persist_qc<128>(a, st);
      case 150: return launch_forward_persist_qc<150>(a, st);
      case 200: return launch_forward_persist_qc<200>(a, st);
      default: return hipErrorInvalidValue;
    }
  }
  if (a.qdev) {
    switch (qc_template) {
      case 32: return launch_forward_qc<32, true, false>(a, grid, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (qc_template) {
    case 16: return launch_forward_qc<16, false, false>(a, grid, st);
    case 32: return launch_forward_qc<32, false, false>(a, grid, st);
    case 50: return launch_forward_qc<50, false, false>(a, grid, st);
    case 64: return launch_forward_qc<64, false, false>(a, grid, st);
    case 100: return launch_forward_qc<100, false, false>(a, grid, st);
    case 128: return launch_forward_qc<128, false, false>(a, grid, st);
    case 150: return launch_forward_qc<150, false, false>(a, grid, st);
    case 200: return launch_forward_qc<200, false, false>(a, grid, st);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Reduce.  Level 1: one work-group per (slice of kSliceTiles consecutive strip
// rows of one structure, 64 columns): wave w sums its quarter of the slice's
// rows in order, lane l one column, and the four wave sums are added in wave
// order.  Level 2: one work-group per (structure, 64 q values) sums the
// structure's slices the same way (wave w takes slices w, w+4, ...) and
// applies Eq. 2's diagonal and the 2/q factor.  Every order is fixed, so the
// results are deterministic.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce_slices(DescView sd, const double* __restrict__ partial, int32_t Nq,
                                                       double* __restrict__ slice_sums) {
  __shared__ double part[4][kWave];
  const int64_t sl = blockIdx.x;
  const int s = find_struct_by_slice(sd, sl);
  const StructDesc d = sd.get(s);
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int64_t first = d.strip_off + (sl - d.slice_off) * kSliceTiles;
  const int64_t last = min(first + kSliceTiles, d.strip_off + d.n_strips);
  constexpr int kQuarter = kSliceTiles / 4;
  const int64_t a = first + w * kQuarter, b = min(last, a + kQuarter);
  const int groups = static_cast<int>(ceil_div(Nq, kWave));
  for (int g = blockIdx.y; g < groups; g += gridDim.y) {  // (grid.y is capped at 65535)
    const int m = g * kWave + lane;
    double acc = 0.0;
    if (m < Nq)
      for (int64_t t = a; t < b; ++t) acc += partial[t * Nq + m];
    __syncthreads();
    part[w][lane] = acc;
    __syncthreads();
    if (w == 0 && m < Nq) slice_sums[sl * Nq + m] = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
  }
}

__global__ __launch_bounds__(256) void k_reduce_final(DescView sd, const double* __restrict__ slice_sums,
                                                      const int32_t* __restrict__ toff,
                                                      const double* __restrict__ asum,
                                                      const float* __restrict__ table, int32_t T, int32_t Nq,
                                                      double q0, double dq, const double* __restrict__ qdev,
                                                      double* __restrict__ I_out) {
  __shared__ double part[4][kWave];
  const int s = blockIdx.x;
  const StructDesc d = sd.get(s);
  const int32_t* o = toff ? toff + static_cast<int64_t>(s) * (T + 1) : nullptr;
  const int64_t nb = ceil_div(d.n, kPackBlock);
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int groups = static_cast<int>(ceil_div(Nq, kWave));
  for (int g = blockIdx.y; g < groups; g += gridDim.y) {  // (grid.y is capped at 65535)
    const int m = g * kWave + lane;
    const bool vm = m < Nq;
    const double qm = vm ? (qdev ? qdev[m] : q0 + m * dq) : 1.0;
    // the strip pair sums: wave w takes slices w, w + 4, ... in order
    double pairs = 0.0;
    if (vm && qm != 0.0)
      for (int64_t k = w; k < d.n_slices; k += 4) pairs += slice_sums[(d.slice_off + k) * Nq + m];
    __syncthreads();
    part[w][lane] = pairs;
    __syncthreads();
    if (w == 0 && vm) {
      double val;
      if (qm == 0.0) {
        double f = 0.0;
        if (asum) {
          for (int64_t k = 0; k < nb; ++k) f += asum[((d.pack_off + k) * 2 + 0) * Nq + m];
        } else {
          for (int t = 0; t < T; ++t)
            f += static_cast<double>(o[t + 1] - o[t]) * static_cast<double>(table[static_cast<int64_t>(t) * Nq + m]);
        }
        val = f * f;
      } else {
        const double psum = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
        double diag = 0.0;
        if (asum) {
          for (int64_t k = 0; k < nb; ++k) diag += asum[((d.pack_off + k) * 2 + 1) * Nq + m];
        } else {
          for (int t = 0; t < T; ++t) {
            const double f = table[static_cast<int64_t>(t) * Nq + m];
            diag += static_cast<double>(o[t + 1] - o[t]) * f * f;
          }
        }
        val = diag + (2.0 / qm) * psum;
      }
      I_out[static_cast<int64_t>(d.orig) * Nq + m] = val;
    }
  }
}

hipError_t launch_reduce_slices(const DescView& sd, int64_t n_slices_total, const double* partial, int32_t row,
                                double* slice_sums, hipStream_t st) {
  if (n_slices_total > 0) {
    const dim3 grid(static_cast<uint32_t>(n_slices_total), static_cast<uint32_t>(std::min<int64_t>(ceil_div(row, kWave), 65535)));
    hipLaunchKernelGGL(k_reduce_slices, grid, dim3(256), 0, st, sd, partial, row, slice_sums);
  }
  return hipGetLastError();
}

hipError_t launch_reduce(const DescView& sd, int32_t S, int64_t n_slices_total, const double* partial,
                         double* slice_sums, const int32_t* toff, const double* asum, const float* table, int32_t T,
                         int32_t Nq, double q0, double dq, const double* qdev, double* I_out, hipStream_t st) {
  const uint32_t qgroups = static_cast<uint32_t>(std::min<int64_t>(ceil_div(Nq, kWave), 65535));
  if (n_slices_total > 0) {
    hipLaunchKernelGGL(k_reduce_slices, dim3(static_cast<uint32_t>(n_slices_total), qgroups), dim3(256), 0, st, sd,
                       partial, Nq, slice_sums);
  }
  if (S > 0) {
    hipLaunchKernelGGL(k_reduce_final, dim3(S, qgroups), dim3(256), 0, st, sd, slice_sums, toff, asum, table, T, Nq,
                       q0, dq, qdev, I_out);
  }
  return hipGetLastError();
}

}  // namespace sas
