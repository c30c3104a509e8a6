// Strip schedule shared by the forward and adjoint kernels (host and device).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sas_kernels.hpp"

namespace sas {

// ---------------------------------------------------------------------------
// Strip bookkeeping.  I blocks hold ib atoms, J blocks bj = c*ib atoms,
// both in the type-sorted order of one structure.  Row I needs J blocks
// J >= floor(I/c) (earlier blocks hold only j < i).  Rows are grouped into
// "super-rows" u = floor(I/c) of c rows with nJ-u J blocks each, cut into
// strips of g blocks.  F(V) = sum_{v=1..V} ceil(v/g) gives the strip count of
// all super-rows before u in closed form.
// ---------------------------------------------------------------------------
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

__host__ __device__ inline int64_t strip_F(int64_t V, int64_t g) {
  const int64_t a = V / g, b = V % g;
  return g * a * (a + 1) / 2 + b * (a + 1);
}

// Strips of all super-rows before u (all of them full: c rows).
__host__ __device__ inline int64_t strips_before(int64_t u, int64_t nJ, int64_t c, int64_t g) {
  return c * (strip_F(nJ, g) - strip_F(nJ - u, g));
}

// First strip of row I (rows of one super-row are consecutive).
__host__ __device__ inline int64_t row_first_strip(int64_t I, int64_t nJ, int64_t c, int64_t g) {
  const int64_t u = I / c;
  return strips_before(u, nJ, c, g) + (I - u * c) * ceil_div(nJ - u, g);
}

// Strips of row I (J blocks floor(I/c) .. nJ-1 in runs of g).
__host__ __device__ inline int64_t strips_in_row(int64_t I, int64_t nJ, int64_t c, int64_t g) {
  return ceil_div(nJ - I / c, g);
}

// The strip of row I that holds J block J (floor(I/c) <= J < nJ), and that
// strip's first J block in *ja.
__host__ __device__ inline int64_t strip_holding(int64_t I, int64_t J, int64_t nJ, int64_t c, int64_t g, int64_t* ja) {
  const int64_t u = I / c;
  const int64_t gi = (J - u) / g;
  *ja = u + gi * g;
  return row_first_strip(I, nJ, c, g) + gi;
}

// Strips of one structure of n atoms (none below two atoms).
__host__ __device__ inline int64_t strips_of(int64_t n, const Geometry& geo) {
  if (n < 2) return 0;
  const int64_t nI = ceil_div(n, geo.ib), nJ = ceil_div(n, geo.bj), c = geo.c, g = geo.g;
  const int64_t nsup = ceil_div(nI, c);
  const int64_t last_rows = nI - (nsup - 1) * c;
  return strips_before(nsup - 1, nJ, c, g) + last_rows * ceil_div(nJ - (nsup - 1), g);
}

struct StripPos {
  int32_t I, Ja, Jb;
};

// Row I, first J block Ja and end Jb of strip t (0 <= t < strips_of(n)).
__host__ __device__ inline StripPos decode_strip(int64_t t, int32_t n, const Geometry& geo) {
  const int64_t nI = ceil_div(n, geo.ib), nJ = ceil_div(n, geo.bj), c = geo.c, g = geo.g;
  const int64_t nsup = ceil_div(nI, c);
  // largest u in [0, nsup) with strips_before(u) <= t
  int64_t lo = 0, hi = nsup - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (strips_before(mid, nJ, c, g) <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int64_t u = lo;
  const int64_t r = t - strips_before(u, nJ, c, g);
  const int64_t spr = ceil_div(nJ - u, g);
  StripPos p;
  p.I = static_cast<int32_t>(u * c + r / spr);
  p.Ja = static_cast<int32_t>(u + (r % spr) * g);
  p.Jb = static_cast<int32_t>(p.Ja + g < nJ ? p.Ja + g : nJ);
  return p;
}

// Structure that owns global strip t (descriptors are sorted by strip_off).
__device__ inline int find_struct_by_strip(const DescView& sd, int64_t t) {
  if (sd.S == 1) return 0;
  int lo = 0, hi = sd.S - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sd.arr[mid].strip_off <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  // structures with zero strips share a strip_off with the next one: skip them
  while (lo + 1 < sd.S && sd.arr[lo + 1].strip_off <= t) ++lo;
  return lo;
}

__device__ inline int find_struct_by_slice(const DescView& sd, int64_t t) {
  if (sd.S == 1) return 0;
  int lo = 0, hi = sd.S - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sd.arr[mid].slice_off <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  while (lo + 1 < sd.S && sd.arr[lo + 1].slice_off <= t) ++lo;
  return lo;
}

__device__ inline int find_struct_by_pack(const DescView& sd, int64_t b) {
  if (sd.S == 1) return 0;
  int lo = 0, hi = sd.S - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sd.arr[mid].pack_off <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  while (lo + 1 < sd.S && sd.arr[lo + 1].pack_off <= b) ++lo;
  return lo;
}

__device__ __forceinline__ int clamp_type(int t, int T) { return t < 0 ? 0 : (t >= T ? T - 1 : t); }

}  // namespace sas
