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
//   forward  one 64-lane wave per (I block, strip of J blocks, q chunk): each
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
#include "sas_kernels.hpp"
#include "sas_schedule.hpp"

namespace sas {

int64_t strips_of(int64_t n, const Geometry& geo) {
  if (n < 2) return 0;
  const int64_t nI = ceil_div(n, geo.ib), nJ = ceil_div(n, geo.bj), c = geo.c, g = geo.g;
  const int64_t nsup = ceil_div(nI, c);
  const int64_t last_rows = nI - (nsup - 1) * c;
  return strips_before(nsup - 1, nJ, c, g) + last_rows * ceil_div(nJ - (nsup - 1), g);
}

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

// One work-group per structure: per type, exclusive prefix over the blocks;
// then the type segments' absolute starts toff[s][0..T] and the absolute
// destination base of every (block, type).
__global__ __launch_bounds__(256) void k_pack_scan(DescView sd, int32_t T, int32_t* __restrict__ bcount,
                                                   int32_t* __restrict__ toff) {
  extern __shared__ int32_t tot[];
  const int s = blockIdx.x;
  const StructDesc d = sd.get(s);
  const int64_t nb = ceil_div(d.n, kPackBlock);
  for (int t = threadIdx.x; t < T; t += blockDim.x) {
    int32_t run = 0;
    for (int64_t lb = 0; lb < nb; ++lb) {
      int32_t* p = bcount + (d.pack_off + lb) * T + t;
      const int32_t c = *p;
      *p = run;
      run += c;
    }
    tot[t] = run;
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
  for (int t = threadIdx.x; t < T; t += blockDim.x) {
    const int32_t base = tot[t];
    for (int64_t lb = 0; lb < nb; ++lb) bcount[(d.pack_off + lb) * T + t] += base;
  }
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
                                                   int32_t ldt, float* __restrict__ tabp) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= static_cast<int64_t>(T) * ldt) return;
  const int64_t t = k / ldt;
  const int32_t m = static_cast<int32_t>(k - t * ldt);
  tabp[k] = m < Nq ? table[t * Nq + m] : 0.f;
}

hipError_t launch_pad_table(const float* table, int32_t T, int32_t Nq, int32_t ldt, float* tabp, hipStream_t st) {
  const int64_t total = static_cast<int64_t>(T) * ldt;
  hipLaunchKernelGGL(k_pad_table, dim3(static_cast<uint32_t>((total + 255) / 256)), dim3(256), 0, st, table, T, Nq,
                     ldt, tabp);
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

template <int QC, int BJ, bool DIRECT>
__global__ __launch_bounds__(kWave, DIRECT ? (BJ >= 512 ? 2 : 5) : (QC > 128 ? 2 : 3)) void k_forward(ForwardArgs a) {
  constexpr int NG = QC / kWave;          // full groups of 64 q values
  constexpr int R = QC % kWave;           // values in the tail group
  constexpr int NT = NG + (R ? 1 : 0);    // q values owned per lane after the lane reduction
  __shared__ double4 sj[BJ];
  const int lane = threadIdx.x;
  const int64_t t = blockIdx.x;
  const int s = find_struct_by_strip(a.sd, t);
  const StructDesc d = a.sd.get(s);
  const StripPos sp = decode_strip(t - d.strip_off, d.n, a.geo);
  const int n = d.n;
  const int i = sp.I * kWave + lane;  // local sorted row of this lane's atom
  const bool vi = i < n;
  const int ic = vi ? i : n - 1;
  const double4 pi = a.xyz[d.atom_off + ic];
  const int ta = clamp_type(a.tsort[d.atom_off + ic], a.T);

  const int m0 = blockIdx.y * a.qc;
  const int nqc = min(a.qc, a.Nq - m0);   // <= QC; steps beyond nqc are computed and dropped
  // (the padded table tabp has ldt >= m0 + QC columns, zero beyond Nq, so no
  // per-step bounds test is needed)
  const double qs = a.q0 + m0 * a.dq;
  const double dq = a.dq;
  const float* fa_row = a.tabp + static_cast<int64_t>(ta) * a.ldt + m0;
  const int32_t* toff = a.toff + static_cast<int64_t>(s) * (a.T + 1);

  // FP64 strip totals, lane-major in LDS (kept out of VGPRs: the q
  // accumulators need nearly all of them)
  __shared__ double tot[NT][kWave];
#pragma unroll
  for (int k = 0; k < NT; ++k) tot[k][lane] = 0.0;
  // direct form: this chunk's q values (0 past the end of the grid)
  __shared__ double qv[DIRECT ? QC : 1];
  if constexpr (DIRECT) {
    for (int k = lane; k < QC; k += kWave) qv[k] = k < nqc ? a.qdev[m0 + k] : 0.0;
  }

#pragma unroll 1
  for (int J = sp.Ja; J < sp.Jb; ++J) {
    const int j0 = J * BJ;
    const int j1 = min(n, j0 + BJ);
    __syncthreads();
    for (int k = lane; k < j1 - j0; k += kWave) sj[k] = a.xyz[d.atom_off + j0 + k];
    __syncthreads();
    // first type segment that ends after j0 (toff holds absolute rows)
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
      float acc[QC];
#pragma unroll
      for (int m = 0; m < QC; ++m) acc[m] = 0.f;
      if constexpr (DIRECT) {
        // arbitrary q grid: sin(q_m r)/r evaluated for every q, one pair per
        // iteration (the q steps are independent of each other)
#pragma unroll 1
        for (int jl = sa; jl < sb; ++jl) {
          // (the q values are re-read from LDS for every pair rather than
          // held in 64 VGPRs: four waves per SIMD instead of three)
          asm volatile("" ::: "memory");
          const double4 pj = sj[jl - j0];
          const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
          const double r2 = fmax(fma(dz, dz, fma(dy, dy, dx * dx)), 1e-60);
          const double ir = rsqrt_f64(r2);
          const double rp = r2 * ir * kOneOverPi;
          const float w = (vi && jl > i) ? static_cast<float>(ir) : 0.f;
#pragma unroll
          for (int m = 0; m < QC; ++m) acc[m] = sin_qr_acc(qv[m], rp, w, acc[m]);
        }
      } else {
      // two atom pairs (j, j+1) per iteration: two independent recurrence
      // chains give the scheduler work to issue while either waits on its
      // previous result; an odd segment ends with a masked partner
#pragma unroll 1
      for (int jl = sa; jl < sb; jl += 2) {
        const int jb = jl + 1 < sb ? jl + 1 : jl;
        // (empty volatile asm: a scheduling boundary, so the two FP64 set-ups
        // run one after the other and their temporaries never coexist with
        // each other and the QC accumulators)
        const PairSeed A = pair_seed(pi, sj[jl - j0], vi && jl > i, dq, qs);
        asm volatile("" ::: "memory");
        const PairSeed B = pair_seed(pi, sj[jb - j0], vi && jb > i && jl + 1 < sb, dq, qs);
        asm volatile("" ::: "memory");
        float za = A.z, da = A.d, zb = B.z, db = B.d;
#pragma unroll
        for (int m = 0; m < QC; ++m) {
          if (m & 1) {
            acc[m] = fmaf(A.sg, za, acc[m]);
            acc[m] = fmaf(B.sg, zb, acc[m]);
          } else {
            acc[m] += za;
            acc[m] += zb;
          }
          za += da;
          zb += db;
          da = fmaf(A.nlam, za, da);
          db = fmaf(B.nlam, zb, db);
        }
      }
      }
      // weight by this lane's f_a(q_m), sum over lanes, weight by f_b(q_m) in FP64
      // (the row pointer is laundered so that the loads stay here instead of
      // being hoisted out of the j loops, where they would pin QC registers)
      const float* far = fa_row;
      asm volatile("" : "+v"(far));
#pragma unroll
      for (int m = 0; m < QC; ++m) acc[m] *= far[m];
      const float* fb_row = a.tabp + static_cast<int64_t>(tb) * a.ldt + m0;
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const float v = lane_transpose_reduce64(acc + g * kWave, lane);
        tot[g][lane] = fma(static_cast<double>(v), static_cast<double>(fb_row[g * kWave + lane]), tot[g][lane]);
      }
      if constexpr (R > 0) {
        const float v = lane_allreduce_tail<R>(acc + NG * kWave, lane);
        const float fb = lane < R ? fb_row[NG * kWave + lane] : 0.f;
        tot[NG][lane] = fma(static_cast<double>(v), static_cast<double>(fb), tot[NG][lane]);
      }
    }
  }
  double* out = a.partial + t * a.Nq + m0;
#pragma unroll
  for (int g = 0; g < NT; ++g) {
    const int m = g * kWave + lane;
    if (m < nqc) out[m] = tot[g][lane];
  }
}

bool forward_qc_supported(int32_t qc) {
  return qc == 16 || qc == 32 || qc == 50 || qc == 64 || qc == 100 || qc == 128 || qc == 150 || qc == 200;
}
bool forward_bj_supported(int32_t bj) { return bj == 64 || bj == 128 || bj == 256 || bj == 512; }

template <int QC, bool DIRECT>
static hipError_t launch_forward_qc(const ForwardArgs& a, dim3 grid, hipStream_t st) {
  switch (a.geo.bj) {
    case 64: hipLaunchKernelGGL((k_forward<QC, 64, DIRECT>), grid, dim3(kWave), 0, st, a); break;
    case 128: hipLaunchKernelGGL((k_forward<QC, 128, DIRECT>), grid, dim3(kWave), 0, st, a); break;
    case 256: hipLaunchKernelGGL((k_forward<QC, 256, DIRECT>), grid, dim3(kWave), 0, st, a); break;
    case 512: hipLaunchKernelGGL((k_forward<QC, 512, DIRECT>), grid, dim3(kWave), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

bool direct_qc_supported(int32_t qc) { return qc == 32; }

hipError_t launch_forward(const ForwardArgs& a, int64_t n_strips_total, int32_t qc_template, hipStream_t st) {
  if (n_strips_total <= 0) return hipSuccess;
  const int nchunks = static_cast<int>(ceil_div(a.Nq, a.qc));
  const dim3 grid(static_cast<uint32_t>(n_strips_total), nchunks);
  if (a.qdev) {
    switch (qc_template) {
      case 32: return launch_forward_qc<32, true>(a, grid, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (qc_template) {
    case 16: return launch_forward_qc<16, false>(a, grid, st);
    case 32: return launch_forward_qc<32, false>(a, grid, st);
    case 50: return launch_forward_qc<50, false>(a, grid, st);
    case 64: return launch_forward_qc<64, false>(a, grid, st);
    case 100: return launch_forward_qc<100, false>(a, grid, st);
    case 128: return launch_forward_qc<128, false>(a, grid, st);
    case 150: return launch_forward_qc<150, false>(a, grid, st);
    case 200: return launch_forward_qc<200, false>(a, grid, st);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Reduce.  Level 1: each work-group sums kSliceTiles consecutive strip rows of
// one structure, in order.  Level 2: one work-group per structure sums its
// slices in order and applies Eq. 2's diagonal and the 2/q factor.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce_slices(DescView sd, const double* __restrict__ partial, int32_t Nq,
                                                       double* __restrict__ slice_sums) {
  const int64_t sl = blockIdx.x;
  const int s = find_struct_by_slice(sd, sl);
  const StructDesc d = sd.get(s);
  const int64_t first = d.strip_off + (sl - d.slice_off) * kSliceTiles;
  const int64_t last = min(first + kSliceTiles, d.strip_off + d.n_strips);
  for (int m = threadIdx.x; m < Nq; m += blockDim.x) {
    double acc = 0.0;
    for (int64_t t = first; t < last; ++t) acc += partial[t * Nq + m];
    slice_sums[sl * Nq + m] = acc;
  }
}

__global__ __launch_bounds__(256) void k_reduce_final(DescView sd, const double* __restrict__ slice_sums,
                                                      const int32_t* __restrict__ toff,
                                                      const double* __restrict__ asum,
                                                      const float* __restrict__ table, int32_t T, int32_t Nq,
                                                      double q0, double dq, const double* __restrict__ qdev,
                                                      double* __restrict__ I_out) {
  const int s = blockIdx.x;
  const StructDesc d = sd.get(s);
  const int32_t* o = toff ? toff + static_cast<int64_t>(s) * (T + 1) : nullptr;
  const int64_t nb = ceil_div(d.n, kPackBlock);
  for (int m = threadIdx.x; m < Nq; m += blockDim.x) {
    const double qm = qdev ? qdev[m] : q0 + m * dq;
    double val;
    if (qm == 0.0) {
      double f = 0.0;
      if (asum) {
        for (int64_t k = 0; k < nb; ++k) f += asum[((d.pack_off + k) * 2 + 0) * Nq + m];
      } else {
        for (int t = 0; t < T; ++t) f += static_cast<double>(o[t + 1] - o[t]) * static_cast<double>(table[static_cast<int64_t>(t) * Nq + m]);
      }
      val = f * f;
    } else {
      double pairs = 0.0;
      for (int64_t k = 0; k < d.n_slices; ++k) pairs += slice_sums[(d.slice_off + k) * Nq + m];
      double diag = 0.0;
      if (asum) {
        for (int64_t k = 0; k < nb; ++k) diag += asum[((d.pack_off + k) * 2 + 1) * Nq + m];
      } else {
        for (int t = 0; t < T; ++t) {
          const double f = table[static_cast<int64_t>(t) * Nq + m];
          diag += static_cast<double>(o[t + 1] - o[t]) * f * f;
        }
      }
      val = diag + (2.0 / qm) * pairs;
    }
    I_out[static_cast<int64_t>(d.orig) * Nq + m] = val;
  }
}

hipError_t launch_reduce(const DescView& sd, int32_t S, int64_t n_slices_total, const double* partial,
                         double* slice_sums, const int32_t* toff, const double* asum, const float* table, int32_t T,
                         int32_t Nq, double q0, double dq, const double* qdev, double* I_out, hipStream_t st) {
  if (n_slices_total > 0) {
    hipLaunchKernelGGL(k_reduce_slices, dim3(static_cast<uint32_t>(n_slices_total)), dim3(256), 0, st, sd, partial,
                       Nq, slice_sums);
  }
  if (S > 0) {
    hipLaunchKernelGGL(k_reduce_final, dim3(S), dim3(256), 0, st, sd, slice_sums, toff, asum, table, T, Nq, q0, dq,
                       qdev, I_out);
  }
  return hipGetLastError();
}

}  // namespace sas
