// Internal interface between the C ABI (sas_api.hip) and the kernels
// (sas_kernels.hip).  Not part of the public header.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sas {

constexpr int kWave = 64;       // wavefront size on gfx950; one wave per forward work-group
constexpr int kPackBlock = 256; // atoms per block of the pack (type sort) kernels
constexpr int kSliceTiles = 256;  // strips summed by one first-level reduce work-group
constexpr int kPaSub = 16;      // J atoms staged with their table rows at a time (per-atom form)

// Per-structure schedule, in execution order (largest structure first).
struct StructDesc {
  int64_t atom_off;   // first row of this structure in the concatenated input
  int64_t strip_off;  // first strip of this structure
  int64_t slice_off;  // first first-level reduce slice of this structure
  int32_t n;          // atoms
  int32_t orig;       // index of the structure in the caller's order (row of I_out)
  int32_t pack_off;   // first pack block of this structure
  int32_t n_strips;   // strips of this structure
  int32_t n_slices;   // reduce slices of this structure
  int32_t pad;
};

// A view that carries one descriptor inline (plain call: no upload needed) or
// points at an array in device memory (batched call).
struct DescView {
  const StructDesc* arr;
  StructDesc one;
  int32_t S;
  __device__ __forceinline__ StructDesc get(int s) const { return S == 1 ? one : arr[s]; }
};

// Tile geometry for one launch: I blocks of ib atoms, J blocks of bj atoms,
// strips of up to g J blocks.
struct Geometry {
  int32_t bj;  // atoms per J block (multiple of ib)
  int32_t c;   // bj / ib
  int32_t g;   // J blocks per strip
  int32_t ib;  // atoms per I block (64 forward: one per lane; 128 adjoint: two per lane)
};

// The strip decode and the walks over a row and a column of strips assume J
// blocks made of whole I blocks (bj = c ib); a geometry that breaks this would
// send them past the strip rows, so the launchers refuse it.
inline bool geometry_ok(const Geometry& g) {
  return g.ib > 0 && g.bj > 0 && g.g > 0 && g.bj % g.ib == 0 && g.c == g.bj / g.ib;
}

struct ForwardArgs {
  DescView sd;
  Geometry geo;
  const double4* xyz;   // type-sorted FP64 coordinates (w unused)
  const int32_t* tsort; // type-sorted type ids
  const int32_t* toff;  // [S][T+1] absolute start of each type segment (sorted rows)
  const float* tabp;    // [T][ldt] form factors, zero in columns >= Nq
  double* partial;      // [strips][Nq]
  int32_t T, Nq;
  int32_t ldt;          // row stride of tabp: (chunks-1)*qc + QC
  int32_t qc;           // q values per chunk (grid.y = number of chunks)
  double q0, dq;        // uniform grid q_m = q0 + m dq (recurrence form)
  const double* qdev;   // non-null: arbitrary grid [Nq] on the device (direct form)
  double* gpart;        // table gradient only: [strips][T][Nq] per-type sums
  float* rows;          // per-atom table gradient: [J blocks][rows_ld][n] per-atom sums
  int32_t rows_ld;      // q stride of rows (>= Nq)
  unsigned long long* counter;  // persistent launch: next (strip, chunk) item; null for a grid launch
  int64_t n_work;               // persistent launch: strips x chunks
};

constexpr int kAdjQ = 512;  // q values per adjoint chunk (weights staged in LDS)
constexpr int kAdjPaBJ = 128; // J-block atoms of the per-atom adjoint

struct AdjArgs {
  DescView sd;          // one structure
  Geometry geo;         // adjoint strip geometry
  const double4* xyz;
  const int32_t* tsort;
  const int32_t* toff;  // [T+1]
  const float* tabp;    // [T][ldt]
  int32_t ldt;
  int32_t T, Nq;
  int32_t qa;           // q values per chunk (<= kAdjQ); grid.y = chunks
  const double* w;      // dL/dI [Nq]
  double* gI;           // [chunks][strips][ib][3] i-side partial sums
  double* gJ;           // [chunks][strips][g*bj][3] j-side partial sums
  int64_t n_strips;
  double q0, dq;
  const double* qdev;   // non-null: arbitrary grid [Nq] on the device (direct variant)
};

// Host-side helpers implemented in sas_kernels.hip / sas_adjoint.hip.
int64_t slices_of(int64_t n_strips);

hipError_t launch_pack(const float* coords, const int32_t* types, const DescView& sd, int32_t S,
                       int64_t n_pack_blocks, int32_t T, int32_t* bcount, int32_t* toff, double4* xyz,
                       int32_t* tsort, int32_t* perm, hipStream_t st);
// Also zeroes *counter (when non-null), the work counter of a persistent
// forward launch that follows on the same stream.
hipError_t launch_pad_table(const float* table, int32_t T, int32_t Nq, int32_t ldt, float* tabp, hipStream_t st,
                            unsigned long long* counter = nullptr);
hipError_t launch_validate(const float* coords, const int32_t* types, int64_t n, int32_t T, unsigned long long* flags,
                           hipStream_t st);
hipError_t launch_forward(const ForwardArgs& a, int64_t n_strips_total, int32_t qc_template, hipStream_t st);
// Diagonal and q = 0 terms come from the type counts toff (type-segment form)
// or, when asum is non-null, from the per-block sums of f and f^2 (per-atom
// form: asum[pack block][2][Nq]).
hipError_t launch_reduce(const DescView& sd, int32_t S, int64_t n_slices_total, const double* partial,
                         double* slice_sums, const int32_t* toff, const double* asum, const float* table, int32_t T,
                         int32_t Nq, double q0, double dq, const double* qdev, double* I_out, hipStream_t st);

// Sum rows of `row` values over each slice of kSliceTiles strips, in order.
hipError_t launch_reduce_slices(const DescView& sd, int64_t n_slices_total, const double* partial, int32_t row,
                                double* slice_sums, hipStream_t st);

// Table gradient (sas_tablegrad.hip): the forward pass that also writes the
// per-type sums, and the final step that forms w_m dI/df_t(q_m).
hipError_t launch_forward_tg(const ForwardArgs& a, int64_t n_strips_total, int32_t qc_template, hipStream_t st);
hipError_t launch_table_grad_final(int64_t n_slices, const double* gslices, const int32_t* toff,
                                   const float* table, int32_t T, int32_t Nq, double q0, double dq, const double* qdev,
                                   const double* w, double* grad_table, hipStream_t st);

// Orientation-averaged profile (sas_orient.hip).
constexpr int kOrientQ = 16;  // q values per orientation chunk (one quadrature per chunk)
constexpr int kOrientSlices = 32;  // direction slices per chunk in the first reduce pass

struct OrientChunk {
  int32_t m0, nq;    // first q (into the orientation q list) and count, m0 = chunk * kOrientQ
  int32_t nth, nph;  // Gauss-Legendre nodes in cos(theta), uniform nodes in phi
  int32_t gl_off;    // first node of this chunk in the node table
  int32_t pad;
  int64_t blk_off;   // first direction block (of 64) of this chunk
  int64_t a_off;     // first partial amplitude of this chunk: [parts][nth * nph][kOrientQ]
};

struct OrientArgs {
  const OrientChunk* chunks;
  int32_t nchunks;
  int32_t T;
  const double* gl;      // [nodes][2]: x, weight (weights of one rule sum to 2)
  const double4* xyz;    // FP64 coordinates of the structure
  const int32_t* tsort;  // their type ids
  const float* tabp;     // [T][ldt]: f_t at the orientation q values, zero beyond
  int32_t ldt;
  int32_t n;
  const double* qv;      // orientation q values
  const double* center;  // [3] (k_geometry output)
  int32_t parts;         // the atoms are split into parts (grid.y)
  int32_t atoms_per_part;
  double2* apart;        // partial amplitudes
  double* ored;          // [chunks][kOrientSlices][kOrientQ]: per-slice sums of the reduce
  int32_t rot;           // 1: uniform q, walk exp(i q p) from the chunk's first q
  double dq;             // the grid step (rot only)
};
// Largest phase step dq * r_max (radians) the rotation walk takes: its
// increment exp(i dq p) - 1 then has modulus below 0.5.
constexpr double kRotMaxStep = 0.5;

hipError_t launch_geometry(const double4* xyz, int64_t n, double* out, hipStream_t st);
hipError_t launch_orient(const OrientArgs& a, int64_t total_blocks, int32_t nq_o, double* I_out, hipStream_t st);
// Work-groups of the amplitude kernel that fit on one CU at once.
int orient_wgs_per_cu(bool rot);
hipError_t launch_copy_cols(const float* src, int32_t T, int32_t ld_src, int32_t col0, int32_t ncols, int32_t ldt,
                            float* dst, hipStream_t st);

// Per-atom form (sas_peratom.hip).
hipError_t launch_pack_plain(const float* coords, const int32_t* types, int64_t n_total, int32_t T, double4* xyz,
                             int32_t* tsort, int32_t* perm, hipStream_t st);
hipError_t launch_atom_sums(const DescView& sd, int64_t n_pack_blocks, const int32_t* tsort, const float* tabp,
                            int32_t T, int32_t ldt, int32_t Nq, double* asum, hipStream_t st);
hipError_t launch_forward_pa(const ForwardArgs& a, int64_t n_strips_total, int32_t qc_template, hipStream_t st);
// Per-atom sums over the whole square (one structure): ROWS variant above.
hipError_t launch_forward_pa_rows(const ForwardArgs& a, int32_t qc_template, hipStream_t st);
// Per-atom table gradient from the rows: sum of f(0) over all atoms; the
// per-atom sums S_i(q_m) = f_i + R_i / q_m ([Nq][n]); the profile from them;
// the stable sort of atoms by type (hipCUB radix sort; *tmp_bytes is the
// temporary size, queried with tmp = NULL); the per-type sums times 2 w_m.
hipError_t launch_rows_f0(const double* asum, int64_t n_pack, int32_t Nq, double* f0, hipStream_t st);
// (the final step also writes each work-group's sums of f_i S_i, [Nq] rows of
// rows_final_blocks(n) values in `part`, from which the profile is summed;
// ldt a multiple of 4)
constexpr int kRowsAtoms = 256;
int32_t rows_final_blocks(int32_t n);
hipError_t launch_rows_final(const float* rows, int32_t nJ, int32_t rows_ld, int32_t n, int32_t Nq, const float* tabp,
                             int32_t ldt, const int32_t* tsort, double q0, double dq, const double* qdev,
                             const double* f0, double* srow, double* part, hipStream_t st);
hipError_t launch_rows_profile(const double* part, int32_t n, int32_t Nq, double* I_out, hipStream_t st);
hipError_t sort_atoms_by_type(void* tmp, size_t* tmp_bytes, const int32_t* keys_in, int32_t* keys_out,
                              const int32_t* vals_in, int32_t* vals_out, int32_t n, int32_t end_bit, hipStream_t st);
hipError_t launch_rows_by_type(const int32_t* keys, const int32_t* atoms, int32_t n, const double* srow, int32_t T,
                               int32_t Nq, const double* w, double* grad_table, hipStream_t st);
bool pa_qc_supported(int32_t qc);

hipError_t launch_adjoint(const AdjArgs& a, int32_t nchunks, hipStream_t st);
// Per-atom form factors (no type sort): I blocks of 64 atoms (one per lane),
// J blocks of kAdjPaBJ, a.qa <= qa_template q values per chunk (templates 32,
// 64 and 100; the direct variant 64).
hipError_t launch_adjoint_pa(const AdjArgs& a, int32_t nchunks, int32_t qa_template, hipStream_t st);
hipError_t launch_grad_reduce(const AdjArgs& a, int64_t n, int32_t nchunks, const int32_t* perm, double* grad_out,
                              hipStream_t st);
bool adjoint_bj_supported(int32_t bj);
bool forward_qc_supported(int32_t qc);
bool direct_qc_supported(int32_t qc);
bool forward_bj_supported(int32_t bj);

}  // namespace sas
