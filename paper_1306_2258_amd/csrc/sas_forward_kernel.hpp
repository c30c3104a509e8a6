// The forward pair kernel of the type-segment form, as a template shared by
// the profile (TG = false, sas_kernels.hip) and the table gradient (TG = true,
// sas_tablegrad.hip).
//
// One 64-lane wave per (I block, strip of J blocks, q chunk): each lane owns
// one i atom, the J block is staged in LDS and swept by all lanes; per pair a
// sin/cos set-up in FP64, then the FP32 recurrence over the q chunk (or, in
// the direct form, one sine per q); per type segment a reduction over the 64
// lanes and an FP64 product with the segment's form factor; one FP64 partial
// row per strip.  With TG the same strip also writes, per type, the sums that
// the derivative of Eq. 2 with respect to the table needs.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>

#include "sas_device.hpp"
#include "sas_forward.hpp"
#include "sas_kernels.hpp"
#include "sas_schedule.hpp"

namespace sas {

// Waves per SIMD the forward kernels are built for.
constexpr int forward_waves(int qc, int bj, bool direct) { return direct ? (bj >= 512 ? 2 : 4) : (qc > 128 ? 2 : 3); }

// One strip t (and q chunk) of the forward pass, by the one wave of a work-group.
template <int QC, int BJ, bool DIRECT, bool TG>
__device__ __forceinline__ void forward_strip(const ForwardArgs& a, int64_t t, int chunk, int lane) {
  constexpr int NG = QC / kWave;          // full groups of 64 q values
  constexpr int R = QC % kWave;           // values in the tail group
  constexpr int NT = NG + (R ? 1 : 0);    // q values owned per lane after the lane reduction
  __shared__ double4 sj[BJ];
  const int s = find_struct_by_strip(a.sd, t);
  const StructDesc d = a.sd.get(s);
  const StripPos sp = decode_strip(t - d.strip_off, d.n, a.geo);
  const int n = d.n;
  const int i = sp.I * kWave + lane;  // local sorted row of this lane's atom
  const bool vi = i < n;
  const int ic = vi ? i : n - 1;
  const double4 pi = a.xyz[d.atom_off + ic];
  const int ta = clamp_type(a.tsort[d.atom_off + ic], a.T);

  const int m0 = chunk * a.qc;
  const int nqc = min(a.qc, a.Nq - m0);   // <= QC; steps beyond nqc are computed and dropped
  // (the padded table tabp has ldt >= m0 + QC columns, zero beyond Nq, so no
  // per-step bounds test is needed)
  const double qs = a.q0 + m0 * a.dq;
  const double dq = a.dq;
  const double hdq = 0.5 * dq;  // the pair set-up takes half the grid step
  const float* fa_row = a.tabp + static_cast<int64_t>(ta) * a.ldt + m0;
  const int32_t* toff = a.toff + static_cast<int64_t>(s) * (a.T + 1);

  // table gradient (TG): this strip's rows [T][Nq] of the sums f_b v by lane
  // type and f_a v by segment type, zeroed by the lanes that later add to
  // them; the I block is "pure" when every valid lane holds one type
  double* grows = nullptr;
  int ta0 = ta;
  bool pure = true;
  if constexpr (TG) {
    grows = a.gpart + t * static_cast<int64_t>(a.T) * a.Nq + m0;
    for (int r = 0; r < a.T; ++r)
      for (int m = lane; m < nqc; m += kWave) grows[static_cast<int64_t>(r) * a.Nq + m] = 0.0;
    ta0 = __shfl(ta, 0, kWave);
    pure = __ballot(vi && ta != ta0) == 0;
  }

  // FP64 strip totals, lane-major in LDS (kept out of VGPRs: the q
  // accumulators need nearly all of them)
  __shared__ double tot[NT][kWave];
#pragma unroll
  for (int k = 0; k < NT; ++k) tot[k][lane] = 0.0;
  // direct form: the r^2 bounds of the reductions over this chunk's q values
  FracRange frange{0.0, 0.0, 0.0};  // from the chunk's smallest positive and largest q (the grid ascends)
  if constexpr (DIRECT) frange = frac_range(chunk_q_lo(a.qdev + m0, nqc), a.qdev[m0 + nqc - 1]);

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
      // TG on a block at a type boundary: one pass over the segment per lane
      // type present, the other lanes masked, so that each pass's lane sums
      // belong to one type (such blocks are at most T - 1 of a structure's)
      uint64_t rem = TG && !pure ? static_cast<uint64_t>(__ballot(vi)) : 0;
      int at = ta0;
      bool on = vi;
#pragma unroll 1
      do {
      if constexpr (TG) {
        if (!pure) {
          at = __shfl(ta, __ffsll(static_cast<unsigned long long>(rem)) - 1, kWave);
          on = vi && ta == at;
          rem &= ~static_cast<uint64_t>(__ballot(on));
        }
      }
      float acc[QC];
#pragma unroll
      for (int m = 0; m < QC; ++m) acc[m] = 0.f;
      if constexpr (DIRECT) {
        // arbitrary q grid: sin(q_m r)/r evaluated for every q, one pair per
        // iteration (the q steps are independent of each other).  A pair whose
        // lanes all admit the one-FMA reduction over the chunk is summed at
        // once; the others are listed, those whose lanes all have t <= 1/2
        // (near atoms at low q) for the product form and the rest (pairs
        // whose lanes straddle t = 1/4 or coincide) for the exact reduction,
        // and each list is summed after the segment, so that each loop has one
        // accumulating path (two paths in one loop make the compiler copy the
        // accumulators after every pair).
        __shared__ int slow[DIRECT ? BJ : 1];
        __shared__ int near[DIRECT ? BJ : 1];
        int nslow = 0, nnear = 0;
        float kScale31 = 0x1p-31f;  // (held in a VGPR: see the one-FMA reduction)
        asm volatile("" : "+v"(kScale31));
        // the q values come through the scalar cache into SGPRs (the same for
        // every pair; the uploaded grid is padded with zeros to the table's
        // row length, and the steps past its end are dropped), the FMAs'
        // constants from VGPR pairs
        using ConstDouble = const __attribute__((address_space(4))) double;
        ConstDouble* qk = (ConstDouble*)(a.qdev + m0);
        double kMagicV = kHalfMagic, kRoundV = kRoundMagic;
        asm volatile("" : "+v"(kMagicV), "+v"(kRoundV));
        auto pair_setup = [&](int jl, double& rp, double& r2, float& w) {
          asm volatile("" ::: "memory");
          const double4 pj = sj[jl - j0];
          const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
          r2 = fmax(fma(dz, dz, fma(dy, dy, dx * dx)), 1e-60);
          const double ir = rsqrt_f64(r2);
          rp = r2 * ir * kOneOverPi;
          w = (on && jl > i) ? static_cast<float>(ir) : 0.f;
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
            group(qc, acc + m);
          }
        };
#pragma unroll 1
        for (int jl = sa; jl < sb; ++jl) {
          double rp, r2;
          float w;
          pair_setup(jl, rp, r2, w);
          if (__all(frac_reduction_ok(frange, r2, w))) {
            const SinPiW wc = sinpi_weighted(w);
            over_q([&](const double(&qc)[4], float* ac) { sin_qr_acc4_frac_w(qc, rp, wc, kScale31, kMagicV, ac); });
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
          double rp, r2;
          float w;
          pair_setup(near[k], rp, r2, w);
          const SinPiW wc = sinpi_weighted(w);
          over_q([&](const double(&qc)[4], float* ac) { sin_qr_acc4_small_w(qc, rp, wc, ac); });
        }
#pragma unroll 1
        for (int k = 0; k < nslow; ++k) {
          double rp, r2;
          float w;
          pair_setup(slow[k], rp, r2, w);
          const SinPiW wc = sinpi_weighted(w);
          over_q([&](const double(&qc)[4], float* ac) { sin_qr_acc4_exact_w(qc, rp, wc, kRoundV, ac); });
        }
      } else {
      // two atom pairs (j, j+1) per iteration: two independent recurrence
      // chains give the scheduler work to issue while either waits on its
      // previous result; an odd segment ends with a masked partner
      // (the two-wave kernels, whose q steps leave registers free, load the
      // next two pairs' coordinates while the current pairs' steps run; the
      // three-wave kernels have none to spare and read them just before use)
      constexpr bool kAhead = QC > 128;
      double4 pja{}, pjb{};
      if constexpr (kAhead) {
        pja = sj[sa - j0];
        pjb = sj[(sa + 1 < sb ? sa + 1 : sa) - j0];
      }
#pragma unroll 1
      for (int jl = sa; jl < sb; jl += 2) {
        const int jb = jl + 1 < sb ? jl + 1 : jl;
        // (empty volatile asm: a scheduling boundary, so the two FP64 set-ups
        // run one after the other and their temporaries never coexist with
        // each other and the QC accumulators)
        PairSeed A, B;
        if constexpr (kAhead) {
          A = pair_seed(pi, pja, on && jl > i, hdq, qs);
          asm volatile("" ::: "memory");
          B = pair_seed(pi, pjb, on && jb > i && jl + 1 < sb, hdq, qs);
          asm volatile("" ::: "memory");
          const int jn = jl + 2 < sb ? jl + 2 : jl;
          const int jnb = jn + 1 < sb ? jn + 1 : jn;
          pja = sj[jn - j0];
          pjb = sj[jnb - j0];
          __builtin_amdgcn_sched_barrier(0);  // keep the loads issued here
        } else {
          A = pair_seed(pi, sj[jl - j0], on && jl > i, hdq, qs);
          asm volatile("" ::: "memory");
          B = pair_seed(pi, sj[jb - j0], on && jb > i && jl + 1 < sb, hdq, qs);
          asm volatile("" ::: "memory");
        }
        float za = A.z, da = A.d, zb = B.z, db = B.d;
        // (fixed registers, banks chosen so that no step instruction reads three
        // operands from one bank; the negated lambdas are plain register
        // operands, so the FMAs keep the 32-bit v_fmac encoding)
        constexpr int kPin = pin_base(QC > 128 ? 2 : 3, QC <= 32);
        // (four steps per asm block in the two-wave kernels: see rec_step8)
        constexpr int M4 = QC > 128 ? QC / 4 * 4 : 0;
#pragma unroll
        for (int m = 0; m < M4; m += 4)
          rec_step8<kPin>(acc[m], acc[m + 1], acc[m + 2], acc[m + 3], za, zb, da, db, A.sg, B.sg, A.nlam, B.nlam);
#pragma unroll
        for (int m = M4; m < QC; ++m) {
          if (m & 1)
            rec_step2<kPin, true>(acc[m], za, zb, da, db, A.sg, B.sg, A.nlam, B.nlam);
          else
            rec_step2<kPin, false>(acc[m], za, zb, da, db, A.sg, B.sg, A.nlam, B.nlam);
        }
      }
      }
      const float* fb_row = a.tabp + static_cast<int64_t>(tb) * a.ldt + m0;
      if constexpr (TG) {
        // lane sums v of the raw accumulators per lane type a give the
        // profile term f_a f_b v and the table-gradient terms f_b v (row a)
        // and f_a v (row b), all in FP64
        double* gb = grows + static_cast<int64_t>(tb) * a.Nq;
        auto add = [&](int g, float v, const float* fa_t, double* ga) {
          const int m = g * kWave + lane;
          const double fa = m < QC ? static_cast<double>(fa_t[m]) : 0.0;
          const double fb = m < QC ? static_cast<double>(fb_row[m]) : 0.0;
          const double vv = static_cast<double>(v);
          tot[g][lane] = fma(fa * fb, vv, tot[g][lane]);
          if (m < nqc) {
            ga[m] = fma(fb, vv, ga[m]);
            gb[m] = fma(fa, vv, gb[m]);
          }
        };
        // every contributing lane holds type `at` (this pass's type)
        const float* fat = a.tabp + static_cast<int64_t>(at) * a.ldt + m0;
        asm volatile("" : "+v"(fat));
        double* ga = grows + static_cast<int64_t>(at) * a.Nq;
#pragma unroll
        for (int g = 0; g < NG; ++g) add(g, lane_transpose_reduce64(acc + g * kWave, lane), fat, ga);
        if constexpr (R > 0) add(NG, lane_allreduce_tail<R>(acc + NG * kWave, lane), fat, ga);
      } else {
      // weight by this lane's f_a(q_m), sum over lanes, weight by f_b(q_m) in FP64
      // (the row pointer is laundered so that the loads stay here instead of
      // being hoisted out of the j loops, where they would pin QC registers)
      const float* far = fa_row;
      asm volatile("" : "+v"(far));
#pragma unroll
      for (int m = 0; m < QC; ++m) acc[m] *= far[m];
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
      } while (TG && rem);
    }
  }
  double* out = a.partial + t * a.Nq + m0;
#pragma unroll
  for (int g = 0; g < NT; ++g) {
    const int m = g * kWave + lane;
    if (m < nqc) out[m] = tot[g][lane];
  }
}

// One work-group per (strip, q chunk): blockIdx.x is the strip, blockIdx.y the chunk.
template <int QC, int BJ, bool DIRECT, bool TG>
__global__ __launch_bounds__(kWave, forward_waves(QC, BJ, DIRECT)) void k_forward(ForwardArgs a) {
  forward_strip<QC, BJ, DIRECT, TG>(a, blockIdx.x, blockIdx.y, threadIdx.x);
}

// Persistent form: as many work-groups as fit on the GPU at once, each taking
// the next (strip, chunk) item from a counter in device memory until all
// a.n_work items are taken (items in strip-major order, the order of the grid
// launch's work-groups).  The counter is zeroed by the table-padding kernel
// that precedes every forward launch.  Each item still writes its own partial
// row, so the result does not depend on which work-group took it.
template <int QC, int BJ>
__global__ __launch_bounds__(kWave, forward_waves(QC, BJ, false)) void k_forward_persist(ForwardArgs a) {
  const int nchunks = (a.Nq + a.qc - 1) / a.qc;
#pragma unroll 1
  for (;;) {
    unsigned long long w = 0;
    if (threadIdx.x == 0) w = atomicAdd(a.counter, 1ull);
    // broadcast from lane 0 as a wave-uniform (scalar) value, as blockIdx is
    // in the grid launch
    const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(w));
    const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(w >> 32));
    w = (static_cast<unsigned long long>(hi) << 32) | lo;
    if (w >= static_cast<unsigned long long>(a.n_work)) break;
    // (the lane index is made opaque in every iteration, so that nothing
    // derived from it is hoisted out of this loop and held across the strip's
    // q steps)
    int lane = threadIdx.x;
    asm volatile("" : "+v"(lane));
    forward_strip<QC, BJ, false, false>(a, static_cast<int64_t>(w / nchunks), static_cast<int>(w % nchunks), lane);
  }
}

// Work-groups of k_forward_persist<QC, BJ> resident on the current GPU (the
// occupancy query, cached per template and device).
template <int QC, int BJ>
int64_t persist_slots() {
  constexpr int kMaxDev = 64;
  static std::atomic<int64_t> cache[kMaxDev];  // 0: not queried yet
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 0;
  if (dev < kMaxDev) {
    const int64_t c = cache[dev].load(std::memory_order_relaxed);
    if (c > 0) return c;
  }
  int per_cu = 0;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_forward_persist<QC, BJ>, kWave, 0) != hipSuccess ||
      per_cu <= 0)
    return 0;
  const int64_t slots = static_cast<int64_t>(per_cu) * prop.multiProcessorCount;
  if (dev < kMaxDev) cache[dev].store(slots, std::memory_order_relaxed);
  return slots;
}

template <int QC>
hipError_t launch_forward_persist_qc(const ForwardArgs& a, hipStream_t st) {
  int64_t slots = 0;
  switch (a.geo.bj) {
    case 64: slots = persist_slots<QC, 64>(); break;
    case 128: slots = persist_slots<QC, 128>(); break;
    case 256: slots = persist_slots<QC, 256>(); break;
    case 512: slots = persist_slots<QC, 512>(); break;
    default: return hipErrorInvalidValue;
  }
  if (slots <= 0) return hipErrorInvalidValue;
  const dim3 grid(static_cast<uint32_t>(a.n_work < slots ? a.n_work : slots));
  switch (a.geo.bj) {
    case 64: hipLaunchKernelGGL((k_forward_persist<QC, 64>), grid, dim3(kWave), 0, st, a); break;
    case 128: hipLaunchKernelGGL((k_forward_persist<QC, 128>), grid, dim3(kWave), 0, st, a); break;
    case 256: hipLaunchKernelGGL((k_forward_persist<QC, 256>), grid, dim3(kWave), 0, st, a); break;
    case 512: hipLaunchKernelGGL((k_forward_persist<QC, 512>), grid, dim3(kWave), 0, st, a); break;
  }
  return hipGetLastError();
}

template <int QC, bool DIRECT, bool TG>
hipError_t launch_forward_qc(const ForwardArgs& a, dim3 grid, hipStream_t st) {
  switch (a.geo.bj) {
    case 64: hipLaunchKernelGGL((k_forward<QC, 64, DIRECT, TG>), grid, dim3(kWave), 0, st, a); break;
    case 128: hipLaunchKernelGGL((k_forward<QC, 128, DIRECT, TG>), grid, dim3(kWave), 0, st, a); break;
    case 256: hipLaunchKernelGGL((k_forward<QC, 256, DIRECT, TG>), grid, dim3(kWave), 0, st, a); break;
    case 512: hipLaunchKernelGGL((k_forward<QC, 512, DIRECT, TG>), grid, dim3(kWave), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sas
