// Per-atom form factors (the general case of Eq. 2, where f_j(q) cannot be
// grouped by element type: the text below Eq. 2 and the Implementation
// section, which stages each block's form factors in local memory beside its
// positions).
//
// The type-segment form factors f_a f_b out of the pair loop; when almost
// every atom has its own table row that factoring buys nothing and each
// segment's lane reduction would run once per pair.  This form instead
//   pack     copies the coordinates to FP64 in the caller's order (no sort);
//   sums     forms sum_i f_i(q) and sum_i f_i(q)^2 per structure (the q = 0
//            value and the diagonal of Eq. 2) in a fixed order;
//   forward  stages each run of kPaSub J atoms together with their table rows
//            for the chunk's q values in LDS and weights every pair term by
//            f_j(q_m) inside the q loop (one more FP32 instruction on odd
//            steps than the type-segment form); each J block's accumulators
//            are weighted by the lane's own f_i(q_m), reduced over the lanes
//            and added to FP64 strip totals.
// The strip schedule, the q recurrence (or the direct sine) and the reduce are
// the type-segment form's.
//
// With ROWS the same pair loop serves the derivative with respect to the
// form factors: each lane keeps its own atom's sum R_i(q_m) = sum over j != i
// of f_j(q_m) sin(q_m r_ij) / r_ij instead of reducing over the lanes.  The
// grid then covers the whole square of (I block, J block) pairs, one J block
// per work-group, and each lane stores its FP32 sums for the J block as one
// column of rows[J][q][atom] (atom index fastest, so the 64 lanes store 64
// consecutive values per q); the J blocks are added in FP64 afterwards.
#include <hip/hip_runtime.h>

#include "sas_device.hpp"
#include "sas_forward.hpp"
#include "sas_kernels.hpp"
#include "sas_schedule.hpp"

namespace sas {

__global__ __launch_bounds__(256) void k_pack_plain(const float* __restrict__ coords, const int32_t* __restrict__ types,
                                                    int64_t n_total, int32_t T, double4* __restrict__ xyz,
                                                    int32_t* __restrict__ tsort, int32_t* __restrict__ perm) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n_total) return;
  xyz[k] = make_double4(coords[3 * k], coords[3 * k + 1], coords[3 * k + 2], 0.0);
  tsort[k] = clamp_type(types[k], T);
  perm[k] = static_cast<int32_t>(k);
}

// One work-group per (pack block of kPackBlock atoms, 64 q values): wave w sums
// atoms [64w, 64w + 64) of the block for the lane's q, in order; the four
// waves are added in order.  asum[b][0][m] = sum f, asum[b][1][m] = sum f^2.
__global__ __launch_bounds__(256) void k_atom_sums(DescView sd, const int32_t* __restrict__ tsort,
                                                   const float* __restrict__ tabp, int32_t T, int32_t ldt, int32_t Nq,
                                                   double* __restrict__ asum) {
  __shared__ double part[kPackBlock / kWave][2][kWave];
  const int64_t b = blockIdx.x;
  const int s = find_struct_by_pack(sd, b);
  const StructDesc d = sd.get(s);
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int m = blockIdx.y * kWave + lane;
  const int64_t first = (b - d.pack_off) * kPackBlock + w * kWave;
  double f1 = 0.0, f2 = 0.0;
  if (m < Nq) {
    for (int k = 0; k < kWave && first + k < d.n; ++k) {
      const int t = clamp_type(tsort[d.atom_off + first + k], T);
      const double f = tabp[static_cast<int64_t>(t) * ldt + m];
      f1 += f;
      f2 = fma(f, f, f2);
    }
  }
  part[w][0][lane] = f1;
  part[w][1][lane] = f2;
  __syncthreads();
  if (w == 0 && m < Nq) {
    double s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < kPackBlock / kWave; ++k) {
      s1 += part[k][0][lane];
      s2 += part[k][1][lane];
    }
    asum[(b * 2 + 0) * Nq + m] = s1;
    asum[(b * 2 + 1) * Nq + m] = s2;
  }
}


template <int QC, bool DIRECT, bool ROWS>
__global__ __launch_bounds__(kWave, DIRECT ? 4 : (QC > 128 ? 2 : 3)) void k_forward_pa(ForwardArgs a) {
  constexpr int NG = QC / kWave;
  constexpr int R = QC % kWave;
  constexpr int NT = NG + (R ? 1 : 0);
  static_assert(QC % 4 == 0, "table rows are staged as float4");
  constexpr int Q4 = QC / 4;
  constexpr int E4 = kPaSub * Q4;  // float4 elements of one run's rows
  __shared__ double4 sj[kPaSub];
  __shared__ __align__(16) float fj[kPaSub][QC];
  __shared__ double tot[NT][kWave];
  const int lane = threadIdx.x;
  const int64_t t = blockIdx.x;
  const int s = ROWS ? 0 : find_struct_by_strip(a.sd, t);
  const StructDesc d = a.sd.get(s);
  StripPos sp;
  if constexpr (ROWS) {
    // square schedule: I block t / nJ with J block t % nJ
    const int nJ = static_cast<int>(ceil_div(d.n, a.geo.bj));
    sp.I = static_cast<int32_t>(t / nJ);
    sp.Ja = static_cast<int32_t>(t - static_cast<int64_t>(sp.I) * nJ);
    sp.Jb = sp.Ja + 1;
  } else {
    sp = decode_strip(t - d.strip_off, d.n, a.geo);
  }
  const int n = d.n;
  const int i = sp.I * kWave + lane;
  const bool vi = i < n;
  const int ic = vi ? i : n - 1;
  const double4 pi = a.xyz[d.atom_off + ic];
  const int ta = clamp_type(a.tsort[d.atom_off + ic], a.T);

  const int m0 = blockIdx.y * a.qc;
  const int nqc = min(a.qc, a.Nq - m0);
  const double qs = a.q0 + m0 * a.dq;
  const double dq = a.dq;
  const double hdq = 0.5 * dq;  // the pair set-up takes half the grid step
  const float* fa_row = a.tabp + static_cast<int64_t>(ta) * a.ldt + m0;
#pragma unroll
  for (int k = 0; k < NT; ++k) tot[k][lane] = 0.0;
  FracRange frange{0.0, 0.0, 0.0};  // from the chunk's smallest positive and largest q (the grid ascends)
  if constexpr (DIRECT) frange = frac_range(chunk_q_lo(a.qdev + m0, nqc), a.qdev[m0 + nqc - 1]);

  const int bj = a.geo.bj;
#pragma unroll 1
  for (int J = sp.Ja; J < sp.Jb; ++J) {
    const int j0 = J * bj;
    const int j1 = min(n, j0 + bj);
    float acc[QC];
#pragma unroll
    for (int m = 0; m < QC; ++m) acc[m] = 0.f;
#pragma unroll 1
    for (int u0 = j0; u0 < j1; u0 += kPaSub) {
      const int ns = min(kPaSub, j1 - u0);
      // stage the run's positions and its table rows for this q chunk (the
      // padded table has ldt >= m0 + QC columns, zero beyond Nq; ldt and m0
      // are multiples of 4).  Lane r < ns fetches row r's type; every lane
      // then issues its share of float4 loads at once.
      __syncthreads();
      const int ty = lane < ns ? clamp_type(a.tsort[d.atom_off + u0 + lane], a.T) : 0;  // row 0 past the run
      if (lane < ns) sj[lane] = a.xyz[d.atom_off + u0 + lane];
      constexpr int K4 = (E4 + kWave - 1) / kWave;  // float4 loads per lane
      constexpr int KG = 4;                          // issued together
      // (indices past the end repeat the last element, and rows past the run
      // read row 0's type: every lane loads a valid address and stores a
      // value some lane also stores)
#pragma unroll 1
      for (int k0 = 0; k0 < K4; k0 += KG) {
        float4 v[KG];
#pragma unroll
        for (int k = 0; k < KG; ++k) {
          const int e = min((k0 + k) * kWave + lane, E4 - 1);
          const int r = e / Q4;
          const int c = e - r * Q4;
          const int tr = __shfl(ty, r, kWave);
          v[k] = *reinterpret_cast<const float4*>(a.tabp + static_cast<int64_t>(tr) * a.ldt + m0 + 4 * c);
        }
#pragma unroll
        for (int k = 0; k < KG; ++k) {
          const int e = min((k0 + k) * kWave + lane, E4 - 1);
          reinterpret_cast<float4*>(&fj[0][0])[e] = v[k];
        }
      }
      __syncthreads();
      if constexpr (DIRECT) {
        // the one-FMA reduction for pairs whose lanes all admit it over the
        // chunk; the rest are listed, for the product form or the exact
        // reduction, and summed after the run (one accumulating path per
        // loop, as in the type form; q through the scalar cache as there)
        __shared__ int slow[DIRECT ? kPaSub : 1];
        __shared__ int near[DIRECT ? kPaSub : 1];
        int nslow = 0, nnear = 0;
        float kScale31 = 0x1p-31f;  // (held in a VGPR: see the one-FMA reduction)
        asm volatile("" : "+v"(kScale31));
        using ConstDouble = const __attribute__((address_space(4))) double;
        ConstDouble* qk = (ConstDouble*)(a.qdev + m0);
        double kMagicV = kHalfMagic, kRoundV = kRoundMagic;
        asm volatile("" : "+v"(kMagicV), "+v"(kRoundV));
        auto pair_setup = [&](int jl, double& rp, double& r2, float& w) {
          asm volatile("" ::: "memory");
          const double4 pj = sj[jl - u0];
          const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
          r2 = fmax(fma(dz, dz, fma(dy, dy, dx * dx)), 1e-60);
          const double ir = rsqrt_f64(r2);
          rp = r2 * ir * kOneOverPi;
          w = (vi && (ROWS ? jl != i : jl > i)) ? static_cast<float>(ir) : 0.f;
        };
        static_assert(QC % 4 == 0, "the direct form's q chunk holds groups of four");
        // (each group's q values loaded before the previous group's steps)
        auto over_q = [&](auto&& group) {
          double qn[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) qn[k] = qk[k];
#pragma unroll
          for (int m = 0; m < QC; m += 4) {
            const double qc[4] = {qn[0], qn[1], qn[2], qn[3]};
            if (m + 4 < QC) {
#pragma unroll
              for (int k = 0; k < 4; ++k) qn[k] = qk[m + 4 + k];
            }
            group(qc, m);
          }
        };
#pragma unroll 1
        for (int jl = u0; jl < u0 + ns; ++jl) {
          double rp, r2;
          float w;
          pair_setup(jl, rp, r2, w);
          if (__all(frac_reduction_ok(frange, r2, w))) {
            const float* fb = fj[jl - u0];
            const SinPiW wc = sinpi_weighted(w);
            over_q([&](const double(&qc)[4], int m) {
              sin_qr_acc4_frac_w<true>(qc, rp, wc, kScale31, kMagicV, acc + m, fb + m);
            });
          } else if (__all(small_t_ok(frange, r2, w))) {
            near[nnear] = jl;  // (every lane stores the same value)
            ++nnear;
          } else {
            slow[nslow] = jl;
            ++nslow;
          }
        }
#pragma unroll 1
        for (int k = 0; k < nnear; ++k) {
          const int jl = near[k];
          double rp, r2;
          float w;
          pair_setup(jl, rp, r2, w);
          const float* fb = fj[jl - u0];
          const SinPiW wc = sinpi_weighted(w);
          over_q([&](const double(&qc)[4], int m) { sin_qr_acc4_small_w<true>(qc, rp, wc, acc + m, fb + m); });
        }
#pragma unroll 1
        for (int k = 0; k < nslow; ++k) {
          const int jl = slow[k];
          double rp, r2;
          float w;
          pair_setup(jl, rp, r2, w);
          const float* fb = fj[jl - u0];
          const SinPiW wc = sinpi_weighted(w);
          over_q([&](const double(&qc)[4], int m) { sin_qr_acc4_exact_w<true>(qc, rp, wc, kRoundV, acc + m, fb + m); });
        }
      } else {
        // two pairs per iteration, as in the type-segment form; an odd run
        // ends with a masked partner
#pragma unroll 1
        for (int jl = u0; jl < u0 + ns; jl += 2) {
          const bool two = jl + 1 < u0 + ns;
          const int jb = two ? jl + 1 : jl;
          const PairSeed A = pair_seed(pi, sj[jl - u0], vi && (ROWS ? jl != i : jl > i), hdq, qs);
          asm volatile("" ::: "memory");
          const PairSeed B = pair_seed(pi, sj[jb - u0], vi && (ROWS ? jb != i : jb > i) && two, hdq, qs);
          asm volatile("" ::: "memory");
          const float4* fa4 = reinterpret_cast<const float4*>(fj[jl - u0]);
          const float4* fb4 = reinterpret_cast<const float4*>(fj[jb - u0]);
          float za = A.z, da = A.d, zb = B.z, db = B.d;
          float nla = A.nlam, nlb = B.nlam;  // laundered: see the type-segment form
          asm volatile("" : "+v"(nla), "+v"(nlb));
          // the rows' values for each 4 q steps are loaded one group ahead,
          // so the LDS latency overlaps the previous group's steps
          float4 ca = fa4[0], cb = fb4[0];
#pragma unroll
          for (int g4 = 0; g4 < QC / 4; ++g4) {
            float4 na = ca, nb = cb;
            if (g4 + 1 < QC / 4) {
              na = fa4[g4 + 1];
              nb = fb4[g4 + 1];
            }
            __builtin_amdgcn_sched_barrier(0);  // keep the loads issued here
            const float fav[4] = {ca.x, ca.y, ca.z, ca.w}, fbv[4] = {cb.x, cb.y, cb.z, cb.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int m = 4 * g4 + k;
              if (m & 1) {
                acc[m] = fmaf(fav[k] * A.sg, za, acc[m]);
                acc[m] = fmaf(fbv[k] * B.sg, zb, acc[m]);
              } else {
                acc[m] = fmaf(fav[k], za, acc[m]);
                acc[m] = fmaf(fbv[k], zb, acc[m]);
              }
              za += da;
              zb += db;
              da = fmaf(nla, za, da);
              db = fmaf(nlb, zb, db);
            }
            ca = na;
            cb = nb;
          }
        }
      }
    }
    if constexpr (ROWS) {
      // (only this chunk's nqc values: the steps past them belong to the next
      // chunk, which stores its own)
      if (vi) {
        float* p = a.rows + (static_cast<int64_t>(J) * a.rows_ld + m0) * n + i;
#pragma unroll
        for (int m = 0; m < QC; ++m) {
          if (m < nqc) *p = acc[m];
          p += n;
        }
      }
      continue;
    }
    // weight by this lane's f_i(q_m), sum over lanes, add in FP64 (the row
    // pointer is laundered so that the loads are not hoisted into registers)
    const float* far = fa_row;
    asm volatile("" : "+v"(far));
#pragma unroll
    for (int m = 0; m < QC; ++m) acc[m] *= far[m];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const float v = lane_transpose_reduce64(acc + g * kWave, lane);
      tot[g][lane] += static_cast<double>(v);
    }
    if constexpr (R > 0) {
      const float v = lane_allreduce_tail<R>(acc + NG * kWave, lane);
      tot[NG][lane] += static_cast<double>(v);
    }
  }
  if constexpr (!ROWS) {
    double* out = a.partial + t * a.Nq + m0;
#pragma unroll
    for (int g = 0; g < NT; ++g) {
      const int m = g * kWave + lane;
      if (m < nqc) out[m] = tot[g][lane];
    }
  }
}

bool pa_qc_supported(int32_t qc) {
  return qc == 16 || qc == 32 || qc == 64 || qc == 100 || qc == 128 || qc == 200;
}

hipError_t launch_pack_plain(const float* coords, const int32_t* types, int64_t n_total, int32_t T, double4* xyz,
                             int32_t* tsort, int32_t* perm, hipStream_t st) {
  if (n_total > 0) {
    hipLaunchKernelGGL(k_pack_plain, dim3(static_cast<uint32_t>(ceil_div(n_total, 256))), dim3(256), 0, st, coords,
                       types, n_total, T, xyz, tsort, perm);
  }
  return hipGetLastError();
}

hipError_t launch_atom_sums(const DescView& sd, int64_t n_pack_blocks, const int32_t* tsort, const float* tabp,
                            int32_t T, int32_t ldt, int32_t Nq, double* asum, hipStream_t st) {
  if (n_pack_blocks > 0) {
    const dim3 grid(static_cast<uint32_t>(n_pack_blocks), static_cast<uint32_t>(ceil_div(Nq, kWave)));
    hipLaunchKernelGGL(k_atom_sums, grid, dim3(256), 0, st, sd, tsort, tabp, T, ldt, Nq, asum);
  }
  return hipGetLastError();
}

template <bool ROWS>
hipError_t launch_forward_pa_t(const ForwardArgs& a, dim3 grid, int32_t qc_template, hipStream_t st) {
  if (!geometry_ok(a.geo)) return hipErrorInvalidValue;
  if (a.qdev) {
    if (qc_template != 32) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_forward_pa<32, true, ROWS>), grid, dim3(kWave), 0, st, a);
    return hipGetLastError();
  }
  switch (qc_template) {
    case 16: hipLaunchKernelGGL((k_forward_pa<16, false, ROWS>), grid, dim3(kWave), 0, st, a); break;
    case 32: hipLaunchKernelGGL((k_forward_pa<32, false, ROWS>), grid, dim3(kWave), 0, st, a); break;
    case 64: hipLaunchKernelGGL((k_forward_pa<64, false, ROWS>), grid, dim3(kWave), 0, st, a); break;
    case 100: hipLaunchKernelGGL((k_forward_pa<100, false, ROWS>), grid, dim3(kWave), 0, st, a); break;
    case 128: hipLaunchKernelGGL((k_forward_pa<128, false, ROWS>), grid, dim3(kWave), 0, st, a); break;
    case 200: hipLaunchKernelGGL((k_forward_pa<200, false, ROWS>), grid, dim3(kWave), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_forward_pa(const ForwardArgs& a, int64_t n_strips_total, int32_t qc_template, hipStream_t st) {
  if (n_strips_total <= 0) return hipSuccess;
  const int nchunks = static_cast<int>(ceil_div(a.Nq, a.qc));
  return launch_forward_pa_t<false>(a, dim3(static_cast<uint32_t>(n_strips_total), nchunks), qc_template, st);
}

hipError_t launch_forward_pa_rows(const ForwardArgs& a, int32_t qc_template, hipStream_t st) {
  const StructDesc d = a.sd.one;
  if (d.n <= 0) return hipSuccess;
  const int64_t blocks = ceil_div(d.n, kWave) * ceil_div(d.n, a.geo.bj);
  const int nchunks = static_cast<int>(ceil_div(a.Nq, a.qc));
  return launch_forward_pa_t<true>(a, dim3(static_cast<uint32_t>(blocks), nchunks), qc_template, st);
}

}  // namespace sas
