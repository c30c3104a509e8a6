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
#include <hip/hip_runtime.h>

#include "sas_forward_kernel.hpp"
#include "sas_kernels.hpp"
#include "sas_schedule.hpp"

namespace sas {

hipError_t launch_forward_tg(const ForwardArgs& a, int64_t n_strips_total, int32_t qc_template, hipStream_t st) {
  if (n_strips_total <= 0) return hipSuccess;
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

}  // namespace sas
