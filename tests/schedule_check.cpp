// Host check of the strip schedule (paper_1306_2258_amd/csrc/sas_schedule.hpp)
// against brute-force enumeration, run on the CPU by tests/test_schedule_host.py.
//
// The forward and adjoint kernels cover the pairs j > i of one structure by
// strips: row I of ib atoms against a run of at most g J blocks of bj atoms.
// The brute force lists, row by row, every J block that holds some j > i of
// the row, cut into runs of g, and checks against it:
//   * strips_of (strip count), decode_strip (every strip), row_first_strip and
//     strips_in_row (every row);
//   * strip_holding, the walk of the gradient reduce over the strips of every
//     row that hold a J block: each visited strip has that row and holds the
//     block, and the visited set is exactly the set of strips holding it;
//   * pair coverage: every pair i < j lies in exactly one strip (small n);
//   * geometry_ok: accepts J blocks made of whole I blocks, refuses others.
// Prints "ok" and the number of cases, or the first mismatch (exit status 1).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <vector>

#include "../paper_1306_2258_amd/csrc/sas_schedule.hpp"

using sas::Geometry;

namespace {

struct Strip {
  int64_t I, Ja, Jb;
};

int failures = 0;

#define EXPECT(cond, ...)                                   \
  do {                                                      \
    if (!(cond)) {                                          \
      if (failures++ < 10) {                                \
        std::printf("mismatch: " __VA_ARGS__);              \
        std::printf("  [%s]\n", #cond);                     \
      }                                                     \
    }                                                       \
  } while (0)

std::vector<Strip> enumerate(int64_t n, const Geometry& g) {
  std::vector<Strip> out;
  if (n < 2) return out;
  const int64_t nI = (n + g.ib - 1) / g.ib, nJ = (n + g.bj - 1) / g.bj;
  for (int64_t I = 0; I < nI; ++I) {
    // first J block holding an atom j > the row's first atom i = I * ib
    int64_t first = 0;
    while ((first + 1) * g.bj - 1 <= I * g.ib) ++first;
    for (int64_t Ja = first; Ja < nJ; Ja += g.g) out.push_back({I, Ja, std::min(Ja + g.g, nJ)});
  }
  return out;
}

void check(int64_t n, const Geometry& g) {
  const std::vector<Strip> ref = enumerate(n, g);
  const int64_t ns = sas::strips_of(n, g);
  EXPECT(ns == static_cast<int64_t>(ref.size()), "n=%lld bj=%d ib=%d g=%d: %lld strips, expected %zu\n",
         (long long)n, g.bj, g.ib, g.g, (long long)ns, ref.size());
  if (ns != static_cast<int64_t>(ref.size())) return;
  for (int64_t t = 0; t < ns; ++t) {
    const sas::StripPos p = sas::decode_strip(t, static_cast<int32_t>(n), g);
    EXPECT(p.I == ref[t].I && p.Ja == ref[t].Ja && p.Jb == ref[t].Jb,
           "n=%lld bj=%d ib=%d g=%d strip %lld: (%d,%d,%d) expected (%lld,%lld,%lld)\n", (long long)n, g.bj, g.ib, g.g,
           (long long)t, p.I, p.Ja, p.Jb, (long long)ref[t].I, (long long)ref[t].Ja, (long long)ref[t].Jb);
  }
  if (n < 2) return;
  const int64_t nI = (n + g.ib - 1) / g.ib, nJ = (n + g.bj - 1) / g.bj;
  // rows: first strip and count
  std::vector<int64_t> first(nI, -1), count(nI, 0);
  for (int64_t t = 0; t < ns; ++t) {
    if (first[ref[t].I] < 0) first[ref[t].I] = t;
    ++count[ref[t].I];
  }
  for (int64_t I = 0; I < nI; ++I) {
    EXPECT(sas::row_first_strip(I, nJ, g.c, g.g) == first[I], "n=%lld bj=%d ib=%d g=%d row %lld first strip\n",
           (long long)n, g.bj, g.ib, g.g, (long long)I);
    EXPECT(sas::strips_in_row(I, nJ, g.c, g.g) == count[I], "n=%lld bj=%d ib=%d g=%d row %lld strip count\n",
           (long long)n, g.bj, g.ib, g.g, (long long)I);
  }
  // the gradient reduce's walk over the strips holding J block J
  for (int64_t J = 0; J < nJ; ++J) {
    std::set<int64_t> holding, visited;
    for (int64_t t = 0; t < ns; ++t)
      if (ref[t].Ja <= J && J < ref[t].Jb) holding.insert(t);
    const int64_t rows = std::min(nI, (J + 1) * g.c);
    for (int64_t Ip = 0; Ip < rows; ++Ip) {
      int64_t ja = -1;
      const int64_t s = sas::strip_holding(Ip, J, nJ, g.c, g.g, &ja);
      const bool in = s >= 0 && s < ns;
      EXPECT(in && ref[s].I == Ip && ref[s].Ja == ja && ja <= J && J < ref[s].Jb,
             "n=%lld bj=%d ib=%d g=%d: strip_holding(%lld, %lld) = %lld\n", (long long)n, g.bj, g.ib, g.g,
             (long long)Ip, (long long)J, (long long)s);
      EXPECT(visited.insert(s).second, "n=%lld: strip %lld visited twice for J block %lld\n", (long long)n,
             (long long)s, (long long)J);
    }
    EXPECT(visited == holding, "n=%lld bj=%d ib=%d g=%d: J block %lld walk misses or adds strips\n", (long long)n,
           g.bj, g.ib, g.g, (long long)J);
  }
  // every pair i < j in exactly one strip
  if (n <= 700) {
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = i + 1; j < n; ++j) {
        int hits = 0;
        for (const Strip& st : ref)
          if (st.I == i / g.ib && st.Ja <= j / g.bj && j / g.bj < st.Jb) ++hits;
        EXPECT(hits == 1, "n=%lld bj=%d ib=%d g=%d: pair (%lld, %lld) in %d strips\n", (long long)n, g.bj, g.ib, g.g,
               (long long)i, (long long)j, hits);
      }
  }
}

Geometry geo(int bj, int ib, int g) {
  Geometry x;
  x.bj = bj;
  x.ib = ib;
  x.c = ib > 0 ? bj / ib : 0;
  x.g = g;
  return x;
}

}  // namespace

int main() {
  const int64_t sizes[] = {0, 1, 2, 3, 63, 64, 65, 127, 128, 129, 191, 255, 256, 257, 511, 512, 513, 640, 700,
                           1000, 1023, 1024, 1025, 2047, 4097, 10000, 20000, 50000};
  int cases = 0;
  for (int ib : {64, 128})
    for (int bj : {64, 128, 256, 512})
      for (int g : {1, 2, 3, 4, 8, 1024}) {
        if (bj % ib) continue;
        const Geometry x = geo(bj, ib, g);
        EXPECT(sas::geometry_ok(x), "geometry bj=%d ib=%d g=%d refused\n", bj, ib, g);
        for (int64_t n : sizes) {
          if (n >= 20000 && (g > 8 || bj < 128)) continue;  // (keeps the run to seconds)
          check(n, x);
          ++cases;
        }
      }
  // pseudo-random sizes
  uint64_t st = 12345;
  for (int k = 0; k < 200; ++k) {
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    const int64_t n = static_cast<int64_t>((st >> 33) % 3000);
    const int ib = (st >> 20) & 1 ? 128 : 64;
    const int bj = ib << ((st >> 24) % (ib == 64 ? 4 : 3));
    const int g = 1 + static_cast<int>((st >> 40) % 5);
    check(n, geo(bj, ib, g));
    ++cases;
  }
  // J blocks that are not whole I blocks, and inconsistent fields, are refused
  EXPECT(!sas::geometry_ok(geo(64, 128, 1)), "bj=64 ib=128 accepted\n");
  EXPECT(!sas::geometry_ok(geo(192, 128, 1)), "bj=192 ib=128 accepted\n");
  Geometry bad = geo(256, 64, 1);
  bad.c = 2;
  EXPECT(!sas::geometry_ok(bad), "c != bj / ib accepted\n");
  EXPECT(!sas::geometry_ok(geo(256, 64, 0)), "g = 0 accepted\n");
  EXPECT(!sas::geometry_ok(geo(256, 0, 1)), "ib = 0 accepted\n");
  if (failures) {
    std::printf("%d mismatches\n", failures);
    return 1;
  }
  std::printf("ok %d cases\n", cases);
  return 0;
}
