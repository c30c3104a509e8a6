// Derivative of the profile with respect to the form-factor table.
//
// At each q Eq. 2 is a quadratic form in the form factors, so
//     dI(q_m)/df_t(q_m) = 2 n_t f_t(q_m) + (2/q_m) G_t(q_m),
//     G_t = sum over pairs i < j of sin(q_m r_ij)/r_ij ([type i = t] f_{type j}
//           + [type j = t] f_{type i}),
// and at q_m = 0, dI/df_t = 2 n_t sum_b n_b f_b(0).  The forward pass with
// TG = true (sas_forward_kernel.hpp) accumulates G per strip beside the
// profile's partial rows; the strips are then summed in a fixed order and
// the final step forms w_m dI/df_t(q_m) for the caller's weights w.
//
// With many table rows (per-atom form factors) per-type sums in the forward
// pass would need T rows per strip.  That form instead takes, for every atom,
// S_i(q_m) = sum over all j of f_j(q_m) sinc(q_m r_ij) (the j = i term is
// f_i), since dI/df_t = 2 sum over atoms i of type t of S_i:
//   rows     the per-atom forward pass over the whole square of pairs
//            (k_forward_pa with ROWS), R_i = sum_{j != i} f_j sin(q r)/r per
//            J block, in FP32;
//   final    S_i = f_i + R_i / q_m (J blocks summed in FP64, in order); at q_m = 0,
//            S_i = sum_j f_j(0);
//   profile  I(q_m) = sum_i f_i S_i: sums over the final step's work-groups
//            (256 atoms each), then those sums in order, one wave per q;
//   by type  atoms sorted by type (stable radix sort, so each type's atoms
//            stay in index order), then one thread per (type, q) sums its
//            atoms' S_i in that order and writes 2 w_m times the sum.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include <algorithm>

#include "sas_forward_kernel.hpp"
#include "sas_kernels.hpp"
#include "sas_schedule.hpp"

namespace sas {

hipError_t launch_forward_tg(const ForwardArgs& a, int64_t n_strips_total, int32_t qc_template, hipStream_t st) {
  if (n_strips_total <= 0) return hipSuccess;
  if (!geometry_ok(a.geo)) return hipErrorInvalidValue;
  const int nchunks = static_cast<int>(ceil_div(a.Nq, a.qc));
  const dim3 grid(static_cast<uint32_t>(n_strips_total), nchunks);
  if (a.qdev) {
    switch (qc_template) {
      case 32: return launch_forward_qc<32, true, true>(a, grid, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (qc_template) {
    case 16: return launch_forward_qc<16, false, true>(a, grid, st);
    case 32: return launch_forward_qc<32, false, true>(a, grid, st);
    case 50: return launch_forward_qc<50, false, true>(a, grid, st);
    case 64: return launch_forward_qc<64, false, true>(a, grid, st);
    case 100: return launch_forward_qc<100, false, true>(a, grid, st);
    case 128: return launch_forward_qc<128, false, true>(a, grid, st);
    case 150: return launch_forward_qc<150, false, true>(a, grid, st);
    case 200: return launch_forward_qc<200, false, true>(a, grid, st);
    default: return hipErrorInvalidValue;
  }
}

// One thread per (type, q): the slices of G in order, then w_m dI/df_t(q_m).
__global__ __launch_bounds__(256) void k_table_grad_final(int64_t n_slices,
                                                          const double* __restrict__ gslices,
                                                          const int32_t* __restrict__ toff,
                                                          const float* __restrict__ table, int32_t T, int32_t Nq,
                                                          double q0, double dq, const double* __restrict__ qdev,
                                                          const double* __restrict__ w,
                                                          double* __restrict__ grad_table) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= static_cast<int64_t>(T) * Nq) return;
  const int t = static_cast<int>(k / Nq);
  const int m = static_cast<int>(k - static_cast<int64_t>(t) * Nq);
  const double qm = qdev ? qdev[m] : q0 + m * dq;
  const double nt = static_cast<double>(toff[t + 1] - toff[t]);
  double d_f;
  if (qm == 0.0) {
    double f1 = 0.0;
    for (int b = 0; b < T; ++b)
      f1 += static_cast<double>(toff[b + 1] - toff[b]) * static_cast<double>(table[static_cast<int64_t>(b) * Nq + m]);
    d_f = 2.0 * nt * f1;
  } else {
    double g = 0.0;
    for (int64_t sl = 0; sl < n_slices; ++sl) g += gslices[(sl * T + t) * static_cast<int64_t>(Nq) + m];
    d_f = 2.0 * nt * static_cast<double>(table[k]) + (2.0 / qm) * g;
  }
  grad_table[k] = w[m] * d_f;
}

hipError_t launch_table_grad_final(int64_t n_slices, const double* gslices, const int32_t* toff,
                                   const float* table, int32_t T, int32_t Nq, double q0, double dq, const double* qdev,
                                   const double* w, double* grad_table, hipStream_t st) {
  const int64_t total = static_cast<int64_t>(T) * Nq;
  hipLaunchKernelGGL(k_table_grad_final, dim3(static_cast<uint32_t>(ceil_div(total, 256))), dim3(256), 0, st,
                     n_slices, gslices, toff, table, T, Nq, q0, dq, qdev, w, grad_table);
  return hipGetLastError();
}

__global__ void k_rows_f0(const double* __restrict__ asum, int64_t n_pack, int32_t Nq, double* __restrict__ f0) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int64_t b = 0; b < n_pack; ++b) s += asum[(b * 2 + 0) * Nq];
  f0[0] = s;
}

hipError_t launch_rows_f0(const double* asum, int64_t n_pack, int32_t Nq, double* f0, hipStream_t st) {
  hipLaunchKernelGGL(k_rows_f0, dim3(1), dim3(64), 0, st, asum, n_pack, Nq, f0);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill_zero(double* __restrict__ p, int64_t count) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < count; k += stride) p[k] = 0.0;
}

// One thread per atom and four consecutive q (a work-group: 256 atoms by
// four q; blockIdx.y the q group): the atom's four form factors in one
// 16-byte read (ldt and the group start are multiples of 4), the J blocks
// summed in FP64 in order (unrolled, so that many loads are in flight), and
// the work-group's sums of f_i S_i per q written to part[m][blockIdx.x] for
// the profile.
__global__ __launch_bounds__(kRowsAtoms) void k_rows_final(const float* __restrict__ rows, int32_t nJ,
                                                           int32_t rows_ld, int32_t n, int32_t Nq,
                                                           const float* __restrict__ tabp, int32_t ldt,
                                                           const int32_t* __restrict__ tsort, double q0, double dq,
                                                           const double* __restrict__ qdev,
                                                           const double* __restrict__ f0, double* __restrict__ srow,
                                                           double* __restrict__ part) {
  __shared__ double red[4][kRowsAtoms];
  const int i = blockIdx.x * kRowsAtoms + threadIdx.x;
  const int m0 = blockIdx.y * 4;
  double fs[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < n) {
    const float4 f4 = *reinterpret_cast<const float4*>(tabp + static_cast<int64_t>(tsort[i]) * ldt + m0);
    const float f[4] = {f4.x, f4.y, f4.z, f4.w};
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    // (rows past the grid's end read the last row, in bounds, and are dropped)
    const float* col[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) col[g] = rows + static_cast<int64_t>(min(m0 + g, Nq - 1)) * n + i;
    const int64_t jstride = static_cast<int64_t>(rows_ld) * n;
#pragma unroll 4
    for (int J = 0; J < nJ; ++J) {
#pragma unroll
      for (int g = 0; g < 4; ++g) r[g] += static_cast<double>(col[g][J * jstride]);
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int m = m0 + g;
      if (m >= Nq) break;
      const double qm = qdev ? qdev[m] : q0 + m * dq;
      const double v = qm == 0.0 ? f0[0] : static_cast<double>(f[g]) + r[g] / qm;
      srow[static_cast<int64_t>(m) * n + i] = v;
      fs[g] = static_cast<double>(f[g]) * v;
    }
  }
#pragma unroll
  for (int g = 0; g < 4; ++g) red[g][threadIdx.x] = fs[g];
  __syncthreads();
  for (int h = kRowsAtoms / 2; h >= 1; h >>= 1) {
    if (static_cast<int>(threadIdx.x) < h) {
#pragma unroll
      for (int g = 0; g < 4; ++g) red[g][threadIdx.x] += red[g][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x < 4 && m0 + static_cast<int>(threadIdx.x) < Nq)
    part[static_cast<int64_t>(m0 + threadIdx.x) * gridDim.x + blockIdx.x] = red[threadIdx.x][0];
}

int64_t grid_stride_blocks(int64_t total) { return std::max<int64_t>(1, std::min<int64_t>(ceil_div(total, 256), 65536)); }

int32_t rows_final_blocks(int32_t n) { return static_cast<int32_t>(ceil_div(static_cast<int64_t>(n), kRowsAtoms)); }

hipError_t launch_rows_final(const float* rows, int32_t nJ, int32_t rows_ld, int32_t n, int32_t Nq, const float* tabp,
                             int32_t ldt, const int32_t* tsort, double q0, double dq, const double* qdev,
                             const double* f0, double* srow, double* part, hipStream_t st) {
  if (n <= 0 || Nq <= 0) return hipSuccess;
  if (ldt % 4 != 0 || ldt < (Nq + 3) / 4 * 4) return hipErrorInvalidValue;
  const dim3 grid(static_cast<uint32_t>(rows_final_blocks(n)), static_cast<uint32_t>((Nq + 3) / 4));
  hipLaunchKernelGGL(k_rows_final, grid, dim3(kRowsAtoms), 0, st, rows, nJ, rows_ld, n, Nq, tabp, ldt, tsort, q0, dq,
                     qdev, f0, srow, part);
  return hipGetLastError();
}

// I(q_m) = sum of the work-groups' parts of row m in order: one wave per q,
// lane k adding parts k, k + 64, ... in order, then a fixed shuffle tree.
__global__ __launch_bounds__(kWave) void k_rows_profile(const double* __restrict__ part, int32_t nparts,
                                                        double* __restrict__ I_out) {
  const int m = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nparts; b += kWave) acc += part[static_cast<int64_t>(m) * nparts + b];
  for (int h = kWave / 2; h >= 1; h >>= 1) acc += __shfl_down(acc, h, kWave);
  if (threadIdx.x == 0) I_out[m] = acc;
}

hipError_t launch_rows_profile(const double* part, int32_t n, int32_t Nq, double* I_out, hipStream_t st) {
  if (Nq <= 0) return hipSuccess;
  if (n <= 0) {
    hipLaunchKernelGGL(k_fill_zero, dim3(1), dim3(256), 0, st, I_out, static_cast<int64_t>(Nq));
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_rows_profile, dim3(static_cast<uint32_t>(Nq)), dim3(kWave), 0, st, part, rows_final_blocks(n),
                     I_out);
  return hipGetLastError();
}

hipError_t sort_atoms_by_type(void* tmp, size_t* tmp_bytes, const int32_t* keys_in, int32_t* keys_out,
                              const int32_t* vals_in, int32_t* vals_out, int32_t n, int32_t end_bit, hipStream_t st) {
  return hipcub::DeviceRadixSort::SortPairs(tmp, *tmp_bytes, keys_in, keys_out, vals_in, vals_out, n, 0, end_bit, st);
}

// Grid-stride over (q, sorted position k): the first atom of each type's run
// sums the run's S_i in order.  Rows of types no atom holds are zero.
__global__ __launch_bounds__(256) void k_rows_by_type(const int32_t* __restrict__ keys,
                                                      const int32_t* __restrict__ atoms, int32_t n,
                                                      const double* __restrict__ srow, int32_t Nq,
                                                      const double* __restrict__ w, double* __restrict__ grad_table) {
  const int64_t total = static_cast<int64_t>(n) * Nq;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < total; idx += stride) {
    const int m = static_cast<int>(idx / n);
    const int64_t k = idx - static_cast<int64_t>(m) * n;
    const int32_t t = keys[k];
    if (k > 0 && keys[k - 1] == t) continue;
    double s = 0.0;
    for (int64_t e = k; e < n && keys[e] == t; ++e) s += srow[static_cast<int64_t>(m) * n + atoms[e]];
    grad_table[static_cast<int64_t>(t) * Nq + m] = 2.0 * w[m] * s;
  }
}

hipError_t launch_rows_by_type(const int32_t* keys, const int32_t* atoms, int32_t n, const double* srow, int32_t T,
                               int32_t Nq, const double* w, double* grad_table, hipStream_t st) {
  const int64_t total = static_cast<int64_t>(T) * Nq;
  hipLaunchKernelGGL(k_fill_zero, dim3(static_cast<uint32_t>(grid_stride_blocks(total))), dim3(256), 0, st, grad_table,
                     total);
  if (n > 0) {
    const int64_t blocks = grid_stride_blocks(static_cast<int64_t>(n) * Nq);
    hipLaunchKernelGGL(k_rows_by_type, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, st, keys, atoms, n, srow, Nq,
                       w, grad_table);
  }
  return hipGetLastError();
}

}  // namespace sas
