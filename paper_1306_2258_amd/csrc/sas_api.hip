// C ABI of the Debye-summation library: argument checks, q-grid analysis,
// schedule and workspace layout, launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/sas_debye.h"
#include "sas_kernels.hpp"
#include "sas_schedule.hpp"

using sas::DescView;
using sas::Geometry;
using sas::StructDesc;

// Scratch memory of sas_debye_profile_noalloc: a fixed array in device memory,
// one copy per GPU the library runs on, held until the process ends.  In host
// code this name stands for a host-side shadow, not a device address, so it is
// never passed to a kernel or a copy: sas_create looks up each device's
// address once (hipGetSymbolAddress, that device current) and every use goes
// through that address.
static __device__ __align__(256) unsigned char scratch[SAS_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

sas_status fail(sas_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define SAS_HIP(call)                                                                           \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess) return fail(SAS_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

const int32_t kQcTemplates[] = {16, 32, 50, 64, 100, 128, 150, 200};
const int32_t kPaQcTemplates[] = {16, 32, 64, 100, 128, 200};

}  // namespace

struct sas_ctx {
  int device = 0;
  int cu_count = 0;
  int32_t force_bj = 0, force_qc = 0;
  bool force_direct = false;    // evaluate every grid by the direct form
  bool force_per_atom = false;  // per-atom form factors whatever T
  // pair-kernel launch of the recurrence's type form: 0 automatic (persistent
  // for one structure, the faster by timing in a plan, a grid for eager
  // batched calls), 1 persistent, 2 grid
  int launch = 0;
  bool last_direct = false, last_per_atom = false, last_persist = false;
  int32_t last_bj = 0, last_qc = 0;
  // pinned staging for the host-written blocks (descriptors of a batched
  // call, a non-uniform q grid, the orientation rule): a ring of slots, each
  // reused once the upload from it has completed
  static constexpr int kStageSlots = 4;
  struct Stage {
    void* buf = nullptr;
    size_t bytes = 0;
    hipEvent_t ev = nullptr;
    bool used = false;
  } stage[kStageSlots];
  int stage_next = 0;
  std::mutex mu;
  // tile shape (bj, qc) chosen by timing, per workload key; filled by plans
  struct Tile {
    int32_t bj = 0, qc = 0;  // 0: the schedule's default
    bool persist = false;
  };
  std::map<std::string, Tile> tuned;
  bool tune_log = false;  // SAS_TUNE_LOG: print every timed candidate to stderr
  // optional kernel timing: event pairs around pair-kernel launches
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_fwd, ev_adj;
  std::vector<hipEvent_t> ev_pool;
  // SAS_DEBUG_VALIDATE: check types and coordinates on the device before
  // each call (a synchronisation each); four counters on the device,
  // allocated when the context is created
  bool debug_validate = false;
  unsigned long long* dbg = nullptr;
  // this device's copy of the allocation-free call's scratch array
  void* scratch = nullptr;
  // hybrid profiles: a second stream (default priority) for the direct part,
  // which runs beside the orientation average, and the events that fork it
  // from and join it back into the caller's stream
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
};

namespace {

hipEvent_t take_event(sas_ctx* ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records an event pair around one kernel launch when timing is on.
struct LaunchTimer {
  sas_ctx* ctx;
  hipStream_t st;
  std::vector<std::pair<hipEvent_t, hipEvent_t>>* rec;
  hipEvent_t a = nullptr, b = nullptr;
  LaunchTimer(sas_ctx* c, hipStream_t s, bool adjoint) : ctx(c), st(s), rec(nullptr) {
    if (!c || !c->timing) return;
    rec = adjoint ? &c->ev_adj : &c->ev_fwd;
    a = take_event(c);
    b = take_event(c);
    if (a && b) (void)hipEventRecord(a, st);
  }
  ~LaunchTimer() {
    if (!rec || !a || !b) return;
    (void)hipEventRecord(b, st);
    rec->emplace_back(a, b);
  }
};

// RAII: make ctx's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

struct Schedule {
  Geometry geo{};
  bool direct = false;    // arbitrary q grid: per-q evaluation instead of the recurrence
  bool per_atom = false;  // f_j inside the pair loop, no type sort
  bool persist = false;   // persistent pair-kernel launch with a work counter
  int32_t tg_types = 0;   // > 0: the forward also writes per-type table-gradient rows
  int32_t qc = 0, qc_template = 0;
  int32_t nchunks = 0, ldt = 0;  // q chunks; row stride of the padded table
  // adjoint (gradient) schedule, single structure only
  bool grad = false;
  Geometry geo_adj{};
  int64_t n_strips_adj = 0;
  int32_t qa = 0, nchunks_adj = 0;
  int32_t qa_template = 0;  // per-atom adjoint kernel template (>= qa)
  int32_t S = 0;
  int64_t n_total = 0;
  int64_t n_pack = 0, n_strips = 0, n_slices = 0;
  std::vector<StructDesc> desc;  // execution order
};

struct Layout {
  size_t xyz = 0, tsort = 0, perm = 0, bcount = 0, toff = 0, tabp = 0, partial = 0, slices = 0;
  size_t gI = 0, gJ = 0, total = 0;
  size_t asum = 0;  // per-atom form: per pack block sums of f and f^2
  size_t gpart = 0, gslices = 0;  // table gradient: [strips][T][Nq], [slices][T][Nq]
  size_t counter = 0;             // persistent launch: the work counter
  // host-written block, uploaded in one copy: structure descriptors (S > 1)
  // followed by the q grid (direct form)
  size_t upload = 0, upload_bytes = 0, desc = 0, qdev = 0;
};

// A validated q grid: finite, >= 0, strictly increasing; uniform or not.
struct QGrid {
  const double* host = nullptr;
  int32_t nq = 0;
  double q0 = 0.0, dq = 0.0;
  bool uniform = false;
};

int32_t pick_qc_template(int32_t qc, bool per_atom) {
  if (per_atom) {
    for (int32_t t : kPaQcTemplates)
      if (t >= qc) return t;
    return 200;
  }
  for (int32_t t : kQcTemplates)
    if (t >= qc) return t;
  return 200;
}

// The per-atom form when the table cannot go through the type sort, or when
// the type segments would be short: with fewer than 16 atoms per type on
// average, the per-segment lane reductions cost more than weighting every
// pair term by f_j inside the q loop.
int64_t max_size(const std::vector<int64_t>& sizes) {
  int64_t m = 0;
  for (int64_t n : sizes) m = std::max(m, n);
  return m;
}

bool use_per_atom(const sas_ctx* ctx, int32_t T, int64_t max_n) {
  if (T > SAS_MAX_TYPES) return true;
  if (ctx && ctx->force_per_atom) return true;
  return T >= 64 && max_n < 16LL * T;
}

// J-block size by the largest structure (measured on MI355X with the current
// pair kernels: 256 atoms for the 50,000-atom rod, 128 for the 20,000-atom
// lattice and for 10,000 atoms; same-box A/B of whole calls against 512 and
// 256, 0.7% faster each): long enough to amortise the per-segment lane
// reduction, short enough to leave many strips.
int32_t default_bj(int64_t max_n) {
  if (max_n >= 40000) return 256;
  if (max_n >= 15000) return 128;
  if (max_n >= 2048) return 128;
  return 64;
}

// Build the schedule for structure sizes `sizes` (caller order).
Schedule make_schedule(const sas_ctx* ctx, const std::vector<int64_t>& sizes, int32_t T, int32_t Nq,
                       int32_t bj_override = 0, int32_t qc_override = 0, bool direct = false, bool per_atom = false,
                       int32_t tg_types = 0, int persist_override = -1) {
  Schedule sc;
  sc.direct = direct;
  sc.per_atom = per_atom;
  sc.tg_types = tg_types;
  // the persistent launch exists for the recurrence's type-form profile
  const int launch = ctx ? ctx->launch : 0;
  sc.persist = !direct && !per_atom && tg_types == 0 &&
               (persist_override >= 0 ? persist_override != 0 : (launch == 1 || (launch == 0 && sizes.size() == 1)));
  sc.S = static_cast<int32_t>(sizes.size());
  int64_t max_n = 0;
  for (int64_t n : sizes) {
    max_n = std::max(max_n, n);
    sc.n_total += n;
  }
  // q chunking: one chunk up to 200 values, else balanced chunks of <= 200
  int32_t qc = Nq;
  if (direct) {
    // per-q evaluation: balanced chunks of at most 32 q values
    const int32_t nch = (Nq + 31) / 32;
    qc = (Nq + nch - 1) / nch;
    sc.qc_template = 32;
  } else if (qc_override > 0 || (ctx && ctx->force_qc > 0)) {
    // a chunk of the template's length (a tuner candidate or sas_set_variant):
    // the shape sas_get_variant reports reproduces the same chunks
    const int32_t fq = qc_override > 0 ? qc_override : ctx->force_qc;
    qc = std::min(fq, Nq);
    sc.qc_template = per_atom ? pick_qc_template(fq, true) : fq;
  } else {
    const int32_t nch = (Nq + 199) / 200;
    qc = (Nq + nch - 1) / nch;
    sc.qc_template = pick_qc_template(qc, per_atom);
  }
  if (per_atom) {
    // the per-atom form stages table rows as float4: chunk starts at
    // multiples of 4 (every per-atom template is one)
    qc = (qc + 3) / 4 * 4;
    if (!direct) sc.qc_template = pick_qc_template(qc, true);
  }
  sc.qc = qc;
  sc.nchunks = (Nq + qc - 1) / qc;
  sc.ldt = ((sc.nchunks - 1) * qc + sc.qc_template + 3) / 4 * 4;
  // (the direct form's per-pair work is four times the recurrence's, so a
  // 128-atom J block already amortises the per-segment lane reduction)
  const int32_t auto_bj = direct ? std::min<int32_t>(default_bj(max_n), 128) : default_bj(max_n);
  int32_t bj = bj_override > 0 ? bj_override : (ctx && ctx->force_bj > 0 ? ctx->force_bj : auto_bj);
  sc.geo.bj = bj;
  sc.geo.ib = sas::kWave;
  sc.geo.c = bj / sas::kWave;
  // strips of g J blocks: g = 1 unless the partial rows (with the table
  // gradient's T rows per strip) would exceed 2 GiB (longer strips halve the
  // work-groups and lengthen the last round: the rod's table gradient ran 7%
  // slower with g = 2 under a 256 MiB bound)
  for (int32_t g = 1;; g *= 2) {
    sc.geo.g = g;
    int64_t strips = 0;
    for (int64_t n : sizes) strips += sas::strips_of(n, sc.geo);
    if (static_cast<double>(strips) * Nq * 8.0 * (1 + tg_types) <= 2048.0 * 1024 * 1024 || g >= 1024) break;
  }
  // execution order: largest structure first (longest-processing-time order)
  std::vector<int32_t> order(sc.S);
  for (int32_t s = 0; s < sc.S; ++s) order[s] = s;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return sizes[a] > sizes[b]; });
  // atom offsets in caller order
  std::vector<int64_t> off(sc.S + 1, 0);
  for (int32_t s = 0; s < sc.S; ++s) off[s + 1] = off[s] + sizes[s];
  sc.desc.resize(sc.S);
  int64_t strip = 0, slice = 0, pack = 0;
  for (int32_t k = 0; k < sc.S; ++k) {
    const int32_t s = order[k];
    StructDesc& d = sc.desc[k];
    std::memset(&d, 0, sizeof(d));
    d.atom_off = off[s];
    d.n = static_cast<int32_t>(sizes[s]);
    d.orig = s;
    d.strip_off = strip;
    d.n_strips = static_cast<int32_t>(sas::strips_of(sizes[s], sc.geo));
    d.slice_off = slice;
    d.n_slices = static_cast<int32_t>(sas::slices_of(d.n_strips));
    d.pack_off = static_cast<int32_t>(pack);
    strip += d.n_strips;
    slice += d.n_slices;
    pack += (sizes[s] + sas::kPackBlock - 1) / sas::kPackBlock;
  }
  sc.n_strips = strip;
  sc.n_slices = slice;
  sc.n_pack = pack;
  return sc;
}

// Tile shapes a plan may time: every J-block size, with the default q chunk
// and with half of it (more waves per SIMD, but each chunk repeats the
// per-pair FP64 set-up), each launched as a grid of one work-group per strip
// and as a persistent grid pulling strips from a counter (recurrence, type
// form only).  A forced variant (sas_set_variant, SAS_FORM_PERSISTENT) is the
// only candidate.
std::vector<sas_ctx::Tile> tile_candidates(const sas_ctx* ctx, int32_t Nq, bool direct, bool per_atom) {
  std::vector<sas_ctx::Tile> out;
  if (ctx && (ctx->force_bj > 0 || ctx->force_qc > 0)) {
    sas_ctx::Tile t;
    t.bj = ctx->force_bj;
    t.qc = ctx->force_qc;
    t.persist = ctx->launch != 2 && !direct && !per_atom;
    out.push_back(t);
    return out;
  }
  // the default chunk (make_schedule): balanced chunks of at most 200 q; the
  // other candidate is the shortest chunk template of at least half of it
  const int32_t def_qc = (Nq + (Nq + 199) / 200 - 1) / ((Nq + 199) / 200);
  std::vector<int32_t> qcs{0};
  if (!direct && def_qc >= 32) {
    const int32_t half = pick_qc_template((def_qc + 1) / 2, per_atom);
    if (half < def_qc) qcs.push_back(half);
  }
  for (int32_t bj : {64, 128, 256, 512})
    for (int32_t qc : qcs)
      for (bool persist : {false, true}) {
        if (persist && (direct || per_atom)) continue;
        if (ctx && ((ctx->launch == 1 && !persist) || (ctx->launch == 2 && persist))) continue;
        sas_ctx::Tile t;
        t.bj = bj;
        t.qc = qc;
        t.persist = persist;
        out.push_back(t);
      }
  return out;
}

std::string workload_key(const std::vector<int64_t>& sizes, int32_t T, int32_t Nq) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the sizes
  for (int64_t n : sizes) {
    h ^= static_cast<uint64_t>(n);
    h *= 1099511628211ull;
  }
  char buf[128];
  snprintf(buf, sizeof(buf), "S%zu:T%d:Q%d:%016llx", sizes.size(), T, Nq, static_cast<unsigned long long>(h));
  return buf;
}

// Adds the adjoint's strip geometry (J blocks of 128 atoms, one block per
// strip) and q chunks (<= kAdjQ values each) to a single-structure schedule.
void add_adjoint(Schedule* sc, int64_t n, int32_t Nq) {
  sc->grad = true;
  sc->geo_adj.bj = 128;
  sc->geo_adj.ib = 2 * sas::kWave;
  sc->geo_adj.c = 1;
  sc->geo_adj.g = 1;
  sc->n_strips_adj = sas::strips_of(n, sc->geo_adj);
  const int32_t nch = (Nq + sas::kAdjQ - 1) / sas::kAdjQ;
  int32_t qa = (Nq + nch - 1) / nch;
  qa = (qa + 7) / 8 * 8;
  sc->qa = std::min(qa, static_cast<int32_t>(sas::kAdjQ));
  sc->nchunks_adj = (Nq + sc->qa - 1) / sc->qa;
}

// The per-atom adjoint: I blocks of 64 atoms, J blocks of kAdjPaBJ; balanced
// chunks of at most 100 q values (64 in the direct variant), a multiple of 4
// each, run by the smallest kernel template that holds them; the padded
// table covers every chunk's template width.
void add_adjoint_pa(Schedule* sc, int64_t n, int32_t Nq) {
  sc->grad = true;
  sc->geo_adj.bj = sas::kAdjPaBJ;
  sc->geo_adj.ib = sas::kWave;
  sc->geo_adj.c = sas::kAdjPaBJ / sas::kWave;
  sc->geo_adj.g = 1;
  sc->n_strips_adj = sas::strips_of(n, sc->geo_adj);
  const int32_t cap = sc->direct ? 64 : 100;
  const int32_t nch = (Nq + cap - 1) / cap;
  const int32_t qa = std::min(cap, ((Nq + nch - 1) / nch + 3) / 4 * 4);
  sc->qa = qa;
  sc->qa_template = sc->direct ? 64 : (qa <= 32 ? 32 : (qa <= 64 ? 64 : 100));
  sc->nchunks_adj = (Nq + qa - 1) / qa;
  sc->ldt = std::max(sc->ldt, ((sc->nchunks_adj - 1) * qa + sc->qa_template + 3) / 4 * 4);
}

Layout make_layout(const Schedule& sc, int32_t T, int32_t Nq) {
  Layout L;
  size_t p = 0;
  auto take = [&](size_t bytes) {
    const size_t at = p;
    p = align_up(p + std::max<size_t>(bytes, 1));
    return at;
  };
  L.xyz = take(sizeof(double4) * sc.n_total);
  L.tsort = take(sizeof(int32_t) * sc.n_total);
  L.perm = take(sizeof(int32_t) * sc.n_total);
  if (sc.per_atom) {
    L.asum = take(sizeof(double) * 2 * sc.n_pack * static_cast<size_t>(Nq));
  } else {
    L.bcount = take(sizeof(int32_t) * sc.n_pack * T);
    L.toff = take(sizeof(int32_t) * static_cast<size_t>(sc.S) * (T + 1));
  }
  {
    const size_t dbytes = sc.S > 1 ? align_up(sizeof(StructDesc) * sc.S) : 0;
    // (the q grid is padded with zeros to the table's row length and at
    // least to a multiple of 8, so that the pair kernels read every chunk's
    // full q groups in bounds)
    const size_t qbytes = sc.direct ? sizeof(double) * static_cast<size_t>(std::max(sc.ldt, (Nq + 7) / 8 * 8)) : 0;
    L.upload_bytes = dbytes + qbytes;
    L.upload = take(L.upload_bytes);
    L.desc = L.upload;
    L.qdev = L.upload + dbytes;
  }
  L.tabp = take(sizeof(float) * static_cast<size_t>(T) * sc.ldt);
  // (the persistent launch's work counter; reserved for every schedule so that
  // the workspace queries do not depend on the launch form)
  L.counter = take(sizeof(unsigned long long));
  L.partial = take(sizeof(double) * sc.n_strips * Nq);
  L.slices = take(sizeof(double) * sc.n_slices * Nq);
  if (sc.tg_types > 0) {
    L.gpart = take(sizeof(double) * sc.n_strips * static_cast<size_t>(sc.tg_types) * Nq);
    L.gslices = take(sizeof(double) * sc.n_slices * static_cast<size_t>(sc.tg_types) * Nq);
  }
  if (sc.grad) {
    const size_t rows = static_cast<size_t>(sc.nchunks_adj) * sc.n_strips_adj;
    L.gI = take(sizeof(double) * 3 * rows * sc.geo_adj.ib);
    L.gJ = take(sizeof(double) * 3 * rows * sc.geo_adj.g * sc.geo_adj.bj);
  }
  L.total = p;
  return L;
}

sas_status check_sizes(int64_t n, int32_t T, int32_t Nq, int32_t max_types = SAS_MAX_TABLE_TYPES) {
  if (n < 0 || n > SAS_MAX_ATOMS) return fail(n < 0 ? SAS_ERR_INVALID_ARG : SAS_ERR_UNSUPPORTED, "atom count %lld outside [0, %lld]", (long long)n, (long long)SAS_MAX_ATOMS);
  if (T <= 0) return fail(SAS_ERR_INVALID_ARG, "type count %d must be >= 1", T);
  if (T > max_types) return fail(SAS_ERR_UNSUPPORTED, "type count %d above %d", T, max_types);
  if (Nq <= 0) return fail(SAS_ERR_INVALID_ARG, "q count %d must be >= 1", Nq);
  if (Nq > SAS_MAX_NQ) return fail(SAS_ERR_UNSUPPORTED, "q count %d above %d", Nq, SAS_MAX_NQ);
  return SAS_OK;
}

sas_status check_offsets(const int64_t* offsets, int32_t S, std::vector<int64_t>* sizes) {
  if (S < 0) return fail(SAS_ERR_INVALID_ARG, "S = %d must be >= 0", S);
  if (!offsets) return fail(SAS_ERR_INVALID_ARG, "offsets is NULL");
  if (offsets[0] != 0) return fail(SAS_ERR_INVALID_ARG, "offsets[0] = %lld, must be 0", (long long)offsets[0]);
  sizes->resize(S);
  for (int32_t s = 0; s < S; ++s) {
    const int64_t n = offsets[s + 1] - offsets[s];
    if (n < 0) return fail(SAS_ERR_INVALID_ARG, "offsets decrease at %d", s);
    if (n > SAS_MAX_ATOMS) return fail(SAS_ERR_UNSUPPORTED, "structure %d has %lld atoms", s, (long long)n);
    (*sizes)[s] = n;
  }
  if (offsets[S] > (int64_t)INT32_MAX) return fail(SAS_ERR_UNSUPPORTED, "more than 2^31-1 atoms in total");
  return SAS_OK;
}

DescView view_of(const Schedule& sc, const void* ws, const Layout& L) {
  DescView v;
  std::memset(&v, 0, sizeof(v));
  v.S = sc.S;
  if (sc.S == 1) v.one = sc.desc[0];
  v.arr = sc.S > 1 ? reinterpret_cast<const StructDesc*>(static_cast<const char*>(ws) + L.desc) : nullptr;
  return v;
}

// Debug mode (SAS_DEBUG_VALIDATE set and not "0" when the context was
// created): types in [0, T) and finite coordinates, checked on the device,
// then a synchronisation of the stream.  Without it an out-of-range type is
// clamped to the nearest valid row and non-finite coordinates give
// non-finite results.
sas_status refuse_capture(hipStream_t hs, const char* what);

sas_status debug_validate(sas_ctx* ctx, const float* coords, const int32_t* types, int64_t n, int32_t t,
                          hipStream_t hs) {
  if (!ctx->debug_validate || n <= 0) return SAS_OK;
  const sas_status cs = refuse_capture(hs, "debug mode (SAS_DEBUG_VALIDATE)");
  if (cs != SAS_OK) return cs;
  if (!ctx->dbg) return fail(SAS_ERR_HIP, "debug counters were not allocated");
  SAS_HIP(hipMemsetAsync(ctx->dbg, 0, 2 * sizeof(unsigned long long), hs));
  SAS_HIP(hipMemsetAsync(ctx->dbg + 2, 0xff, 2 * sizeof(unsigned long long), hs));
  SAS_HIP(sas::launch_validate(coords, types, n, t, ctx->dbg, hs));
  unsigned long long h[4] = {0, 0, 0, 0};
  SAS_HIP(hipMemcpyAsync(h, ctx->dbg, sizeof(h), hipMemcpyDeviceToHost, hs));
  SAS_HIP(hipStreamSynchronize(hs));
  if (h[0])
    return fail(SAS_ERR_INVALID_ARG, "%llu type ids outside [0, %d), the first at atom %llu", h[0], t, h[2]);
  if (h[1]) return fail(SAS_ERR_INVALID_ARG, "%llu atoms with a non-finite coordinate, the first at atom %llu", h[1], h[3]);
  return SAS_OK;
}

sas_status classify_q(const double* q, int32_t nq, QGrid* g) {
  if (!q) return fail(SAS_ERR_INVALID_ARG, "q is NULL");
  if (nq <= 0 || nq > SAS_MAX_NQ) return fail(SAS_ERR_INVALID_ARG, "q count %d outside [1, %d]", nq, SAS_MAX_NQ);
  for (int32_t m = 0; m < nq; ++m) {
    if (!std::isfinite(q[m])) return fail(SAS_ERR_Q_NOT_UNIFORM, "q[%d] is not finite", m);
    if (q[m] < 0.0) return fail(SAS_ERR_Q_NOT_UNIFORM, "q[%d] = %g is negative", m, q[m]);
    if (m > 0 && !(q[m] > q[m - 1])) return fail(SAS_ERR_Q_NOT_UNIFORM, "q is not strictly increasing at %d", m);
  }
  g->host = q;
  g->nq = nq;
  g->q0 = q[0];
  g->dq = nq > 1 ? (q[nq - 1] - q[0]) / (nq - 1) : 0.0;
  const double tol = 8.0 * (std::nextafter(q[nq - 1], INFINITY) - q[nq - 1]);
  g->uniform = true;
  for (int32_t m = 1; m + 1 < nq && g->uniform; ++m)
    if (std::fabs(q[m] - (g->q0 + m * g->dq)) > tol) g->uniform = false;
  return SAS_OK;
}

// The bytes of the upload block (descriptors, then the q grid) as the
// device expects them.
std::vector<char> upload_image(const Schedule& sc, const Layout& L, const QGrid& g) {
  std::vector<char> img(L.upload_bytes, 0);
  if (sc.S > 1) std::memcpy(img.data() + (L.desc - L.upload), sc.desc.data(), sizeof(StructDesc) * sc.S);
  if (sc.direct) std::memcpy(img.data() + (L.qdev - L.upload), g.host, sizeof(double) * g.nq);
  return img;
}

// Calls whose host-written block (descriptors, a non-uniform q grid) goes
// through the context's staging ring cannot be captured into a graph: the
// captured copy would keep reading a slot that later calls overwrite.  A plan
// (sas_plan_create_batched) is the capturable form of those calls.
sas_status refuse_capture(hipStream_t hs, const char* what) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  SAS_HIP(hipStreamIsCapturing(hs, &cs));
  if (cs != hipStreamCaptureStatusNone)
    return fail(SAS_ERR_UNSUPPORTED, "%s uploads host data through reused staging and cannot be captured; "
                "use a batched plan (or a uniform q grid for single structures)", what);
  return SAS_OK;
}

// Asynchronous upload through the next slot of the context's pinned staging
// ring.  The host waits only when that slot's previous upload is still in
// flight (kStageSlots uploads queued and unfinished).
sas_status stage_upload_to(sas_ctx* ctx, void* dst, const std::vector<char>& img, hipStream_t hs) {
  if (img.empty()) return SAS_OK;
  const sas_status cs = refuse_capture(hs, "this call");
  if (cs != SAS_OK) return cs;
  std::lock_guard<std::mutex> lock(ctx->mu);
  sas_ctx::Stage& sl = ctx->stage[ctx->stage_next];
  ctx->stage_next = (ctx->stage_next + 1) % sas_ctx::kStageSlots;
  if (sl.used) {
    hipError_t e = hipEventQuery(sl.ev);
    if (e == hipErrorNotReady) e = hipEventSynchronize(sl.ev);
    if (e != hipSuccess) return fail(SAS_ERR_HIP, "staging event: %s", hipGetErrorString(e));
  }
  if (sl.bytes < img.size()) {
    if (sl.buf) SAS_HIP(hipHostFree(sl.buf));
    sl.buf = nullptr;
    sl.bytes = 0;
    const size_t want = std::max<size_t>(img.size(), 4096);
    if (hipHostMalloc(&sl.buf, want, hipHostMallocDefault) != hipSuccess)
      return fail(SAS_ERR_OUT_OF_MEMORY, "pinned staging of %zu bytes failed", want);
    sl.bytes = want;
  }
  if (!sl.ev) SAS_HIP(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
  std::memcpy(sl.buf, img.data(), img.size());
  SAS_HIP(hipMemcpyAsync(dst, sl.buf, img.size(), hipMemcpyHostToDevice, hs));
  SAS_HIP(hipEventRecord(sl.ev, hs));
  sl.used = true;
  return SAS_OK;
}

sas_status stage_upload(sas_ctx* ctx, void* ws, const Layout& L, const std::vector<char>& img, hipStream_t hs) {
  return stage_upload_to(ctx, static_cast<char*>(ws) + L.upload, img, hs);
}

// Record the form and tile shape a profile call used (sas_get_form, sas_get_variant).
void note_last(sas_ctx* ctx, const Schedule& sc) {
  ctx->last_bj = sc.geo.bj;
  ctx->last_qc = sc.qc_template;
  ctx->last_direct = sc.direct;
  ctx->last_per_atom = sc.per_atom;
  ctx->last_persist = sc.persist;
}

// Enqueue pack -> forward -> reduce for a prepared schedule.  The upload
// block (descriptors when S > 1, the q grid in the direct form) must already
// be in the workspace.
sas_status enqueue_forward(sas_ctx* ctx, const Schedule& sc, const Layout& L, const float* coords,
                           const int32_t* types, const float* table, int32_t T, int32_t Nq, double q0, double dq,
                           double* I_out, void* ws, hipStream_t st) {
  const double* qdev = sc.direct ? reinterpret_cast<const double*>(static_cast<const char*>(ws) + L.qdev) : nullptr;
  char* w = static_cast<char*>(ws);
  DescView sd = view_of(sc, ws, L);
  auto* xyz = reinterpret_cast<double4*>(w + L.xyz);
  auto* tsort = reinterpret_cast<int32_t*>(w + L.tsort);
  auto* perm = reinterpret_cast<int32_t*>(w + L.perm);
  auto* bcount = reinterpret_cast<int32_t*>(w + L.bcount);
  auto* toff = reinterpret_cast<int32_t*>(w + L.toff);
  auto* partial = reinterpret_cast<double*>(w + L.partial);
  auto* slices = reinterpret_cast<double*>(w + L.slices);
  auto* tabp = reinterpret_cast<float*>(w + L.tabp);
  auto* asum = sc.per_atom ? reinterpret_cast<double*>(w + L.asum) : nullptr;
  auto* counter = sc.persist ? reinterpret_cast<unsigned long long*>(w + L.counter) : nullptr;
  SAS_HIP(sas::launch_pad_table(table, T, Nq, sc.ldt, tabp, st, counter));
  if (sc.per_atom) {
    SAS_HIP(sas::launch_pack_plain(coords, types, sc.n_total, T, xyz, tsort, perm, st));
    SAS_HIP(sas::launch_atom_sums(sd, sc.n_pack, tsort, tabp, T, sc.ldt, Nq, asum, st));
  } else {
    SAS_HIP(sas::launch_pack(coords, types, sd, sc.S, sc.n_pack, T, bcount, toff, xyz, tsort, perm, st));
  }
  sas::ForwardArgs a;
  std::memset(&a, 0, sizeof(a));
  a.sd = sd;
  a.geo = sc.geo;
  a.xyz = xyz;
  a.tsort = tsort;
  a.toff = sc.per_atom ? nullptr : toff;
  a.tabp = tabp;
  a.ldt = sc.ldt;
  a.partial = partial;
  a.T = T;
  a.Nq = Nq;
  a.qc = sc.qc;
  a.q0 = q0;
  a.dq = dq;
  a.qdev = qdev;
  a.gpart = sc.tg_types > 0 ? reinterpret_cast<double*>(w + L.gpart) : nullptr;
  a.counter = counter;
  a.n_work = sc.n_strips * sc.nchunks;
  {
    LaunchTimer timer(ctx, st, false);
    if (sc.per_atom)
      SAS_HIP(sas::launch_forward_pa(a, sc.n_strips, sc.qc_template, st));
    else if (sc.tg_types > 0)
      SAS_HIP(sas::launch_forward_tg(a, sc.n_strips, sc.qc_template, st));
    else
      SAS_HIP(sas::launch_forward(a, sc.n_strips, sc.qc_template, st));
  }
  if (I_out)
    SAS_HIP(sas::launch_reduce(sd, sc.S, sc.n_slices, partial, slices, sc.per_atom ? nullptr : toff, asum, table, T,
                               Nq, q0, dq, qdev, I_out, st));
  return SAS_OK;
}

// ---------------------------------------------------------------------------
// Table gradient with many table rows (per-atom form factors): per-atom sums
// over the whole square of pairs, then per type.
// ---------------------------------------------------------------------------
int64_t ceil_div64(int64_t a, int64_t b) { return (a + b - 1) / b; }

bool table_grad_by_atom(const sas_ctx* ctx, int32_t T) {
  return T > SAS_MAX_TABLE_GRAD_TYPES || (ctx && ctx->force_per_atom);
}

struct RowsLayout {
  Schedule sc;
  int32_t nJ = 0, end_bit = 1;
  size_t xyz = 0, tsort = 0, perm = 0, asum = 0, upload = 0, upload_bytes = 0, tabp = 0, rows = 0, srow = 0;
  size_t keys = 0, atoms = 0, f0 = 0, part = 0, tmp = 0, tmp_bytes = 0, total = 0;
};

// J blocks of at most 512 atoms (the FP32 sum of one block is exact enough,
// as in the forward), smaller for small structures so that the square still
// holds about 2048 work-groups.
RowsLayout rows_layout(const sas_ctx* ctx, int64_t n, int32_t T, int32_t Nq, bool direct) {
  RowsLayout R;
  R.sc = make_schedule(ctx, std::vector<int64_t>{n}, T, Nq, 0, 0, direct, true);
  const int64_t nI = std::max<int64_t>(1, ceil_div64(n, sas::kWave));
  int64_t bj = ceil_div64(n, std::max<int64_t>(1, ceil_div64(2048, nI)));
  bj = std::min<int64_t>(512, std::max<int64_t>(sas::kWave, ceil_div64(bj, sas::kWave) * sas::kWave));
  R.sc.geo.bj = static_cast<int32_t>(bj);
  R.sc.geo.c = R.sc.geo.bj / sas::kWave;
  R.sc.geo.g = 1;
  R.nJ = static_cast<int32_t>(std::max<int64_t>(1, ceil_div64(n, bj)));
  while (R.end_bit < 31 && (int64_t(1) << R.end_bit) < T) ++R.end_bit;
  size_t p = 0;
  auto take = [&](size_t bytes) {
    const size_t at = p;
    p = align_up(p + std::max<size_t>(bytes, 1));
    return at;
  };
  R.xyz = take(sizeof(double4) * n);
  R.tsort = take(sizeof(int32_t) * n);
  R.perm = take(sizeof(int32_t) * n);
  R.asum = take(sizeof(double) * 2 * R.sc.n_pack * static_cast<size_t>(Nq));
  // (padded with zeros to the table's row length, as in the profile's layout)
  R.upload_bytes = direct ? sizeof(double) * static_cast<size_t>(std::max(Nq, R.sc.ldt)) : 0;
  R.upload = take(R.upload_bytes);
  R.tabp = take(sizeof(float) * static_cast<size_t>(T) * R.sc.ldt);
  R.rows = take(sizeof(float) * static_cast<size_t>(R.nJ) * Nq * n);
  R.srow = take(sizeof(double) * static_cast<size_t>(Nq) * n);
  R.keys = take(sizeof(int32_t) * n);
  R.atoms = take(sizeof(int32_t) * n);
  R.f0 = take(sizeof(double));
  R.part = take(sizeof(double) * static_cast<size_t>(Nq) * sas::rows_final_blocks(static_cast<int32_t>(n)));
  size_t tb = 0;
  if (n > 0 && sas::sort_atoms_by_type(nullptr, &tb, nullptr, nullptr, nullptr, nullptr, static_cast<int32_t>(n),
                                       R.end_bit, nullptr) != hipSuccess)
    tb = 0;
  R.tmp_bytes = tb;
  R.tmp = take(tb);
  R.total = p;
  return R;
}

sas_status enqueue_table_grad_by_atom(sas_ctx* ctx, const RowsLayout& R, const float* coords, const int32_t* types,
                                      int64_t n, const float* table, int32_t T, int32_t Nq, const QGrid& grid,
                                      const double* w, double* grad_table, double* I_out, void* ws, hipStream_t st) {
  char* b = static_cast<char*>(ws);
  const Schedule& sc = R.sc;
  auto* xyz = reinterpret_cast<double4*>(b + R.xyz);
  auto* tsort = reinterpret_cast<int32_t*>(b + R.tsort);
  auto* perm = reinterpret_cast<int32_t*>(b + R.perm);
  auto* asum = reinterpret_cast<double*>(b + R.asum);
  auto* tabp = reinterpret_cast<float*>(b + R.tabp);
  auto* rows = reinterpret_cast<float*>(b + R.rows);
  auto* srow = reinterpret_cast<double*>(b + R.srow);
  auto* keys = reinterpret_cast<int32_t*>(b + R.keys);
  auto* atoms = reinterpret_cast<int32_t*>(b + R.atoms);
  auto* f0 = reinterpret_cast<double*>(b + R.f0);
  auto* part = reinterpret_cast<double*>(b + R.part);
  const double* qdev = sc.direct ? reinterpret_cast<const double*>(b + R.upload) : nullptr;
  if (sc.direct) {
    std::vector<char> img(R.upload_bytes, 0);
    std::memcpy(img.data(), grid.host, sizeof(double) * static_cast<size_t>(Nq));
    const sas_status s2 = stage_upload_to(ctx, b + R.upload, img, st);
    if (s2 != SAS_OK) return s2;
  }
  DescView sd;
  std::memset(&sd, 0, sizeof(sd));
  sd.S = 1;
  sd.one = sc.desc[0];
  SAS_HIP(sas::launch_pad_table(table, T, Nq, sc.ldt, tabp, st));
  SAS_HIP(sas::launch_pack_plain(coords, types, n, T, xyz, tsort, perm, st));
  SAS_HIP(sas::launch_atom_sums(sd, sc.n_pack, tsort, tabp, T, sc.ldt, Nq, asum, st));
  sas::ForwardArgs a;
  std::memset(&a, 0, sizeof(a));
  a.sd = sd;
  a.geo = sc.geo;
  a.xyz = xyz;
  a.tsort = tsort;
  a.tabp = tabp;
  a.ldt = sc.ldt;
  a.T = T;
  a.Nq = Nq;
  a.qc = sc.qc;
  a.q0 = grid.q0;
  a.dq = grid.dq;
  a.qdev = qdev;
  a.rows = rows;
  a.rows_ld = Nq;
  {
    LaunchTimer timer(ctx, st, false);
    SAS_HIP(sas::launch_forward_pa_rows(a, sc.qc_template, st));
  }
  SAS_HIP(sas::launch_rows_f0(asum, sc.n_pack, Nq, f0, st));
  SAS_HIP(sas::launch_rows_final(rows, R.nJ, Nq, static_cast<int32_t>(n), Nq, tabp, sc.ldt, tsort, grid.q0, grid.dq,
                                 qdev, f0, srow, part, st));
  if (I_out) SAS_HIP(sas::launch_rows_profile(part, static_cast<int32_t>(n), Nq, I_out, st));
  if (n > 0) {
    size_t tb = R.tmp_bytes;
    SAS_HIP(sas::sort_atoms_by_type(b + R.tmp, &tb, tsort, keys, perm, atoms, static_cast<int32_t>(n), R.end_bit, st));
  }
  SAS_HIP(sas::launch_rows_by_type(keys, atoms, static_cast<int32_t>(n), srow, T, Nq, w, grad_table, st));
  return SAS_OK;
}

}  // namespace

extern "C" {

int sas_version(void) { return 100; }

const char* sas_last_error(void) { return g_err.c_str(); }

const char* sas_status_string(sas_status s) {
  switch (s) {
    case SAS_OK: return "SAS_OK";
    case SAS_ERR_INVALID_ARG: return "SAS_ERR_INVALID_ARG";
    case SAS_ERR_Q_NOT_UNIFORM: return "SAS_ERR_Q_NOT_UNIFORM";
    case SAS_ERR_UNSUPPORTED: return "SAS_ERR_UNSUPPORTED";
    case SAS_ERR_WORKSPACE_TOO_SMALL: return "SAS_ERR_WORKSPACE_TOO_SMALL";
    case SAS_ERR_OUT_OF_MEMORY: return "SAS_ERR_OUT_OF_MEMORY";
    case SAS_ERR_HIP: return "SAS_ERR_HIP";
  }
  return "unknown status";
}

sas_status sas_q_grid_check(const double* q, int32_t nq, double* q0, double* dq) {
  QGrid g;
  const sas_status st = classify_q(q, nq, &g);
  if (st != SAS_OK) return st;
  if (!g.uniform) return fail(SAS_ERR_Q_NOT_UNIFORM, "q is not a uniform grid");
  if (q0) *q0 = g.q0;
  if (dq) *dq = g.dq;
  return SAS_OK;
}

namespace {

// Device address of `scratch` per device id, looked up once per device.
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_addr;

sas_status scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (static_cast<int>(g_scratch_addr.size()) <= device) g_scratch_addr.resize(device + 1, nullptr);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SAS_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    g_scratch_addr[device] = p;
  }
  *out = g_scratch_addr[device];
  return SAS_OK;
}

}  // namespace

sas_status sas_create(int device, sas_ctx** out) {
  if (!out) return fail(SAS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return fail(SAS_ERR_HIP, "hipGetDeviceCount: %s", hipGetErrorString(e));
  if (device < 0 || device >= count) return fail(SAS_ERR_INVALID_ARG, "device %d not in [0, %d)", device, count);
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return fail(SAS_ERR_HIP, "hipGetDeviceProperties: %s", hipGetErrorString(e));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(SAS_ERR_INVALID_ARG, "device %d is %s; this library is built for gfx950 only", device, prop.gcnArchName);
  sas_ctx* c = new (std::nothrow) sas_ctx();
  if (!c) return fail(SAS_ERR_OUT_OF_MEMORY, "context allocation failed");
  c->device = device;
  c->cu_count = prop.multiProcessorCount;
  const char* dv = std::getenv("SAS_DEBUG_VALIDATE");
  c->debug_validate = dv && dv[0] && std::strcmp(dv, "0") != 0;
  const char* tl = std::getenv("SAS_TUNE_LOG");
  c->tune_log = tl && tl[0] && std::strcmp(tl, "0") != 0;
  {
    DeviceGuard g(device);
    if (!g.ok) {
      delete c;
      return fail(SAS_ERR_HIP, "hipSetDevice(%d) failed", device);
    }
    sas_status st = scratch_address(device, &c->scratch);
    if (st == SAS_OK && c->debug_validate &&
        hipMalloc(reinterpret_cast<void**>(&c->dbg), 4 * sizeof(unsigned long long)) != hipSuccess)
      st = fail(SAS_ERR_OUT_OF_MEMORY, "debug counters: hipMalloc failed");
    if (st != SAS_OK) {
      delete c;
      return st;
    }
  }
  *out = c;
  return SAS_OK;
}

void sas_destroy(sas_ctx* ctx) {
  if (!ctx) return;
  {
    DeviceGuard g(ctx->device);
    for (auto* v : {&ctx->ev_fwd, &ctx->ev_adj})
      for (auto& p : *v) {
        (void)hipEventSynchronize(p.second);
        ctx->ev_pool.push_back(p.first);
        ctx->ev_pool.push_back(p.second);
      }
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    for (auto& sl : ctx->stage) {
      if (sl.ev) {
        (void)hipEventSynchronize(sl.ev);
        (void)hipEventDestroy(sl.ev);
      }
      if (sl.buf) (void)hipHostFree(sl.buf);
    }
    if (ctx->dbg) (void)hipFree(ctx->dbg);
    if (ctx->side) {
      (void)hipStreamSynchronize(ctx->side);
      (void)hipStreamDestroy(ctx->side);
    }
    if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
    if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
  }
  delete ctx;
}

sas_status sas_set_variant(sas_ctx* ctx, int32_t bj, int32_t qc) {
  if (!ctx) return fail(SAS_ERR_INVALID_ARG, "ctx is NULL");
  if (bj != 0 && !sas::forward_bj_supported(bj)) return fail(SAS_ERR_INVALID_ARG, "unsupported bj %d", bj);
  if (qc != 0 && !sas::forward_qc_supported(qc)) return fail(SAS_ERR_INVALID_ARG, "unsupported qc %d", qc);
  ctx->force_bj = bj;
  ctx->force_qc = qc;
  return SAS_OK;
}

sas_status sas_set_form(sas_ctx* ctx, int form) {
  if (!ctx) return fail(SAS_ERR_INVALID_ARG, "ctx is NULL");
  if (form & ~(SAS_FORM_DIRECT | SAS_FORM_PER_ATOM | SAS_FORM_PERSISTENT | SAS_FORM_GRID))
    return fail(SAS_ERR_INVALID_ARG, "unknown form %d", form);
  if ((form & SAS_FORM_PERSISTENT) && (form & SAS_FORM_GRID))
    return fail(SAS_ERR_INVALID_ARG, "SAS_FORM_PERSISTENT and SAS_FORM_GRID exclude each other");
  ctx->force_direct = (form & SAS_FORM_DIRECT) != 0;
  ctx->force_per_atom = (form & SAS_FORM_PER_ATOM) != 0;
  ctx->launch = (form & SAS_FORM_PERSISTENT) ? 1 : ((form & SAS_FORM_GRID) ? 2 : 0);
  return SAS_OK;
}

sas_status sas_get_form(const sas_ctx* ctx, int* form) {
  if (!ctx || !form) return fail(SAS_ERR_INVALID_ARG, "NULL argument");
  *form = (ctx->last_direct ? SAS_FORM_DIRECT : SAS_FORM_RECURRENCE) | (ctx->last_per_atom ? SAS_FORM_PER_ATOM : 0) |
          (ctx->last_persist ? SAS_FORM_PERSISTENT : 0);
  return SAS_OK;
}

sas_status sas_get_variant(const sas_ctx* ctx, int32_t* bj, int32_t* qc) {
  if (!ctx || !bj || !qc) return fail(SAS_ERR_INVALID_ARG, "NULL argument");
  *bj = ctx->last_bj;
  *qc = ctx->last_qc;
  return SAS_OK;
}

sas_status sas_enable_timing(sas_ctx* ctx, int on) {
  if (!ctx) return fail(SAS_ERR_INVALID_ARG, "ctx is NULL");
  ctx->timing = on != 0;
  return SAS_OK;
}

sas_status sas_read_timing(sas_ctx* ctx, double* forward_ms, int64_t* forward_launches, double* adjoint_ms,
                           int64_t* adjoint_launches) {
  if (!ctx) return fail(SAS_ERR_INVALID_ARG, "ctx is NULL");
  DeviceGuard g(ctx->device);
  double sums[2] = {0.0, 0.0};
  int64_t counts[2] = {0, 0};
  std::vector<std::pair<hipEvent_t, hipEvent_t>>* recs[2] = {&ctx->ev_fwd, &ctx->ev_adj};
  sas_status st = SAS_OK;
  for (int k = 0; k < 2; ++k) {
    for (auto& p : *recs[k]) {
      float ms = 0.f;
      if (st == SAS_OK) {
        hipError_t e = hipEventSynchronize(p.second);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.first, p.second);
        if (e != hipSuccess) st = fail(SAS_ERR_HIP, "event timing: %s", hipGetErrorString(e));
      }
      sums[k] += ms;
      counts[k] += 1;
      ctx->ev_pool.push_back(p.first);
      ctx->ev_pool.push_back(p.second);
    }
    recs[k]->clear();
  }
  if (forward_ms) *forward_ms = sums[0];
  if (forward_launches) *forward_launches = counts[0];
  if (adjoint_ms) *adjoint_ms = sums[1];
  if (adjoint_launches) *adjoint_launches = counts[1];
  return st;
}

size_t sas_debye_workspace_size(const sas_ctx* ctx, int64_t n, int32_t t, int32_t nq, int grad) {
  if (check_sizes(n, t, nq, SAS_MAX_TABLE_TYPES) != SAS_OK) return 0;
  const std::vector<int64_t> sizes{n};
  if (grad == 2) {
    size_t need = 0;
    for (bool direct : {false, true})
      need = std::max(need, table_grad_by_atom(ctx, t)
                                ? rows_layout(ctx, n, t, nq, direct).total
                                : make_layout(make_schedule(ctx, sizes, t, nq, 0, 0, direct, false, t), t, nq).total);
    return need;
  }
  if (grad) {
    // the type or the per-atom form; the recurrence or, for a non-uniform
    // grid, the direct variants
    const bool pa = use_per_atom(ctx, t, n);
    size_t need = 0;
    for (bool direct : {false, true}) {
      Schedule sc = make_schedule(ctx, sizes, t, nq, 0, 0, direct, pa);
      if (pa)
        add_adjoint_pa(&sc, n, nq);
      else
        add_adjoint(&sc, n, nq);
      need = std::max(need, make_layout(sc, t, nq).total);
    }
    return need;
  }
  // the grid is not known here: cover the recurrence and the direct form
  const bool pa = use_per_atom(ctx, t, n);
  size_t need = 0;
  for (bool direct : {false, true})
    need = std::max(need, make_layout(make_schedule(ctx, sizes, t, nq, 0, 0, direct, pa), t, nq).total);
  return need;
}

sas_status sas_debye_profile(sas_ctx* ctx, const float* coords, const int32_t* types, int64_t n, const float* table,
                             int32_t t, const double* q, int32_t nq, double* I_out, void* workspace, size_t ws_bytes,
                             void* stream) {
  if (!ctx) return fail(SAS_ERR_INVALID_ARG, "ctx is NULL");
  sas_status st = check_sizes(n, t, nq);
  if (st != SAS_OK) return st;
  if (n > 0 && (!coords || !types)) return fail(SAS_ERR_INVALID_ARG, "coords/types is NULL");
  if (!table || !I_out) return fail(SAS_ERR_INVALID_ARG, "table/I_out is NULL");
  QGrid grid;
  st = classify_q(q, nq, &grid);
  if (st != SAS_OK) return st;
  const Schedule sc = make_schedule(ctx, std::vector<int64_t>{n}, t, nq, 0, 0, !grid.uniform || ctx->force_direct,
                                    use_per_atom(ctx, t, n));
  const Layout L = make_layout(sc, t, nq);
  if (!workspace) return fail(SAS_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(SAS_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(SAS_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes, need %zu", ws_bytes, L.total);
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(SAS_ERR_HIP, "hipSetDevice(%d) failed", ctx->device);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  st = debug_validate(ctx, coords, types, n, t, hs);
  if (st != SAS_OK) return st;
  st = stage_upload(ctx, workspace, L, upload_image(sc, L, grid), hs);
  if (st != SAS_OK) return st;
  st = enqueue_forward(ctx, sc, L, coords, types, table, t, nq, grid.q0, grid.dq, I_out, workspace, hs);
  if (st == SAS_OK) note_last(ctx, sc);
  return st;
}

sas_status sas_debye_profile_noalloc(sas_ctx* ctx, const float* coords, const int32_t* types, int64_t n,
                                     const float* table, int32_t t, const double* q, int32_t nq, double* I_out,
                                     void* stream) {
  if (!ctx) return fail(SAS_ERR_INVALID_ARG, "ctx is NULL");
  sas_status st = check_sizes(n, t, nq);
  if (st != SAS_OK) return st;
  if (n > 0 && (!coords || !types)) return fail(SAS_ERR_INVALID_ARG, "coords/types is NULL");
  if (!table || !I_out) return fail(SAS_ERR_INVALID_ARG, "table/I_out is NULL");
  QGrid grid;
  st = classify_q(q, nq, &grid);
  if (st != SAS_OK) return st;
  // the direct form reads its q grid from device memory, which would need an
  // upload through the context's pinned staging
  if (!grid.uniform || ctx->force_direct)
    return fail(SAS_ERR_UNSUPPORTED, "the allocation-free call takes uniform q grids on the recurrence form only");
  const bool pa = use_per_atom(ctx, t, n);
  Schedule sc = make_schedule(ctx, std::vector<int64_t>{n}, t, nq, 0, 0, false, pa);
  Layout L = make_layout(sc, t, nq);
  // unless the caller forced a shape: when the strip rows do not fit, the
  // shortest longer J block whose rows do (each doubling halves the strips)
  for (int32_t bj = sc.geo.bj * 2; L.total > SAS_NOALLOC_SCRATCH_BYTES && ctx->force_bj == 0 && bj <= 512; bj *= 2) {
    sc = make_schedule(ctx, std::vector<int64_t>{n}, t, nq, bj, 0, false, pa);
    L = make_layout(sc, t, nq);
  }
  if (L.upload_bytes != 0) return fail(SAS_ERR_UNSUPPORTED, "this call would upload host data");
  if (L.total > SAS_NOALLOC_SCRATCH_BYTES)
    return fail(SAS_ERR_UNSUPPORTED, "n = %lld, t = %d, nq = %d needs %zu bytes of scratch; the allocation-free "
                "call has %zu (use sas_debye_profile with a workspace)", (long long)n, t, nq, L.total,
                (size_t)SAS_NOALLOC_SCRATCH_BYTES);
  if (!ctx->scratch) return fail(SAS_ERR_HIP, "no scratch address for device %d", ctx->device);
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(SAS_ERR_HIP, "hipSetDevice(%d) failed", ctx->device);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  st = debug_validate(ctx, coords, types, n, t, hs);
  if (st != SAS_OK) return st;
  // no kernel timing (its events are created on demand); every kernel of the
  // path writes the scratch regions it reads, so nothing is cleared first
  st = enqueue_forward(nullptr, sc, L, coords, types, table, t, nq, grid.q0, grid.dq, I_out, ctx->scratch, hs);
  if (st == SAS_OK) note_last(ctx, sc);
  return st;
}

size_t sas_debye_workspace_size_batched(const sas_ctx* ctx, const int64_t* offsets, int32_t S, int32_t t,
                                        int32_t nq) {
  std::vector<int64_t> sizes;
  if (check_offsets(offsets, S, &sizes) != SAS_OK) return 0;
  if (check_sizes(0, t, nq) != SAS_OK) return 0;
  // large enough for the automatic shape, every shape a plan may time, and
  // the direct form (the grid is not known here)
  const bool pa = use_per_atom(ctx, t, max_size(sizes));
  size_t need = make_layout(make_schedule(ctx, sizes, t, nq, 0, 0, false, pa), t, nq).total;
  for (bool direct : {false, true})
    for (const auto& c : tile_candidates(ctx, nq, direct, pa))
      need = std::max(need, make_layout(make_schedule(ctx, sizes, t, nq, c.bj, c.qc, direct, pa, 0, c.persist ? 1 : 0),
                                        t, nq).total);
  return need;
}

sas_status sas_debye_profile_batched(sas_ctx* ctx, const float* coords, const int32_t* types,
                                     const int64_t* offsets, int32_t S, const float* table, int32_t t,
                                     const double* q, int32_t nq, double* I_out, void* workspace, size_t ws_bytes,
                                     void* stream) {
  if (!ctx) return fail(SAS_ERR_INVALID_ARG, "ctx is NULL");
  std::vector<int64_t> sizes;
  sas_status st = check_offsets(offsets, S, &sizes);
  if (st != SAS_OK) return st;
  st = check_sizes(0, t, nq);
  if (st != SAS_OK) return st;
  if (offsets[S] > 0 && (!coords || !types)) return fail(SAS_ERR_INVALID_ARG, "coords/types is NULL");
  if (!table || (S > 0 && !I_out)) return fail(SAS_ERR_INVALID_ARG, "table/I_out is NULL");
  QGrid grid;
  st = classify_q(q, nq, &grid);
  if (st != SAS_OK) return st;
  if (S == 0) return SAS_OK;
  const Schedule sc = make_schedule(ctx, sizes, t, nq, 0, 0, !grid.uniform || ctx->force_direct,
                                    use_per_atom(ctx, t, max_size(sizes)));
  const Layout L = make_layout(sc, t, nq);
  if (!workspace) return fail(SAS_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(SAS_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(SAS_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes, need %zu", ws_bytes, L.total);
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(SAS_ERR_HIP, "hipSetDevice(%d) failed", ctx->device);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  st = debug_validate(ctx, coords, types, offsets[S], t, hs);
  if (st != SAS_OK) return st;
  st = stage_upload(ctx, workspace, L, upload_image(sc, L, grid), hs);
  if (st != SAS_OK) return st;
  st = enqueue_forward(ctx, sc, L, coords, types, table, t, nq, grid.q0, grid.dq, I_out, workspace, hs);
  if (st == SAS_OK) note_last(ctx, sc);
  return st;
}

}  // extern "C"

struct sas_plan {
  sas_ctx* ctx = nullptr;
  std::vector<int64_t> sizes;
  const float* coords = nullptr;
  const int32_t* types = nullptr;
  const float* table = nullptr;
  double* I_out = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int32_t T = 0, Nq = 0;
  std::vector<double> qh;  // the plan's own copy of the q grid
  QGrid grid;
  bool direct = false, per_atom = false;
  Schedule sc;
  Layout L;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool ready = false;
};

namespace {

// Synchronous upload of the host-written block (the plan's graph reads it
// from the workspace on every replay).
sas_status upload_sync(const Schedule& sc, const Layout& L, const QGrid& g, void* ws) {
  const std::vector<char> img = upload_image(sc, L, g);
  if (!img.empty())
    SAS_HIP(hipMemcpy(static_cast<char*>(ws) + L.upload, img.data(), img.size(), hipMemcpyHostToDevice));
  return SAS_OK;
}

// Times every candidate tile shape on the plan's own buffers (one warm-up and
// two timed evaluations each, HIP events on `st`) and returns the fastest.
sas_status tune_plan(sas_plan* p, hipStream_t st, sas_ctx::Tile* best_tile) {
  const auto cands = tile_candidates(p->ctx, p->Nq, p->direct, p->per_atom);
  float best = -1.f;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  SAS_HIP(hipEventCreate(&e0));
  SAS_HIP(hipEventCreate(&e1));
  sas_status status = SAS_OK;
  for (const auto& c : cands) {
    const Schedule sc =
        make_schedule(p->ctx, p->sizes, p->T, p->Nq, c.bj, c.qc, p->direct, p->per_atom, 0, c.persist ? 1 : 0);
    const Layout L = make_layout(sc, p->T, p->Nq);
    if (L.total > p->ws_bytes) continue;
    status = upload_sync(sc, L, p->grid, p->ws);
    if (status != SAS_OK) break;
    status = enqueue_forward(nullptr, sc, L, p->coords, p->types, p->table, p->T, p->Nq, p->grid.q0, p->grid.dq, p->I_out,
                             p->ws, st);
    if (status != SAS_OK) break;
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < 2 && status == SAS_OK; ++r)
      status = enqueue_forward(nullptr, sc, L, p->coords, p->types, p->table, p->T, p->Nq, p->grid.q0, p->grid.dq, p->I_out,
                               p->ws, st);
    (void)hipEventRecord(e1, st);
    if (status != SAS_OK) break;
    hipError_t e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      status = fail(SAS_ERR_HIP, "tuning timer: %s", hipGetErrorString(e));
      break;
    }
    if (p->ctx->tune_log)
      std::fprintf(stderr, "sas tune: bj %d qc %d (template %d) %s: %.4f ms per evaluation\n", sc.geo.bj, sc.qc,
                   sc.qc_template, sc.persist ? "persistent" : "grid", ms / 2);
    if (best < 0.f || ms < best) {
      best = ms;
      *best_tile = c;
      best_tile->bj = sc.geo.bj;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status == SAS_OK && best < 0.f) status = fail(SAS_ERR_WORKSPACE_TOO_SMALL, "no tile shape fits the workspace");
  return status;
}

}  // namespace

extern "C" {

sas_status sas_plan_create_batched(sas_ctx* ctx, const float* coords, const int32_t* types, const int64_t* offsets,
                                   int32_t S, const float* table, int32_t t, const double* q, int32_t nq,
                                   double* I_out, void* workspace, size_t ws_bytes, sas_plan** out) {
  if (!out) return fail(SAS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!ctx) return fail(SAS_ERR_INVALID_ARG, "ctx is NULL");
  std::vector<int64_t> sizes;
  sas_status st = check_offsets(offsets, S, &sizes);
  if (st != SAS_OK) return st;
  st = check_sizes(0, t, nq);
  if (st != SAS_OK) return st;
  if (S == 0) return fail(SAS_ERR_INVALID_ARG, "a plan needs at least one structure");
  if (offsets[S] > 0 && (!coords || !types)) return fail(SAS_ERR_INVALID_ARG, "coords/types is NULL");
  if (!table || !I_out) return fail(SAS_ERR_INVALID_ARG, "table/I_out is NULL");
  QGrid grid;
  st = classify_q(q, nq, &grid);
  if (st != SAS_OK) return st;
  if (!workspace) return fail(SAS_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(SAS_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  const bool direct = !grid.uniform || ctx->force_direct;
  const bool per_atom = use_per_atom(ctx, t, max_size(sizes));
  const Schedule sc0 = make_schedule(ctx, sizes, t, nq, 0, 0, direct, per_atom);
  const size_t need = make_layout(sc0, t, nq).total;
  if (ws_bytes < need) return fail(SAS_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes, need %zu", ws_bytes, need);
  sas_plan* p = new (std::nothrow) sas_plan();
  if (!p) return fail(SAS_ERR_OUT_OF_MEMORY, "plan allocation failed");
  p->ctx = ctx;
  p->sizes = sizes;
  p->coords = coords;
  p->types = types;
  p->table = table;
  p->I_out = I_out;
  p->ws = workspace;
  p->ws_bytes = ws_bytes;
  p->T = t;
  p->Nq = nq;
  p->qh.assign(q, q + nq);
  p->grid = grid;
  p->grid.host = p->qh.data();
  p->direct = direct;
  p->per_atom = per_atom;
  *out = p;
  return SAS_OK;
}

sas_status sas_plan_execute(sas_plan* p, void* stream) {
  if (!p) return fail(SAS_ERR_INVALID_ARG, "plan is NULL");
  DeviceGuard g(p->ctx->device);
  if (!g.ok) return fail(SAS_ERR_HIP, "hipSetDevice(%d) failed", p->ctx->device);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  {
    int64_t total = 0;
    for (int64_t v : p->sizes) total += v;
    const sas_status sv = debug_validate(p->ctx, p->coords, p->types, total, p->T, hs);
    if (sv != SAS_OK) return sv;
  }
  if (!p->ready) {
    // choose the tile shape: forced variant, cached choice, or timing
    sas_ctx::Tile tile;
    const std::string key = workload_key(p->sizes, p->T, p->Nq) + (p->direct ? "d" : "u") + (p->per_atom ? "a" : "t") +
                            (p->ctx->launch == 1 ? "p" : (p->ctx->launch == 2 ? "g" : ""));
    const bool forced = p->ctx->force_bj > 0 || p->ctx->force_qc > 0;
    auto it = p->ctx->tuned.find(key);
    if (forced) {
      tile.bj = p->ctx->force_bj;
      tile.persist = p->ctx->launch != 2 && !p->direct && !p->per_atom;
    } else if (it != p->ctx->tuned.end()) {
      tile = it->second;
    } else {
      sas_status st = tune_plan(p, hs, &tile);
      if (st != SAS_OK) return st;
      p->ctx->tuned[key] = tile;
    }
    p->sc = make_schedule(p->ctx, p->sizes, p->T, p->Nq, tile.bj, tile.qc, p->direct, p->per_atom, 0,
                          tile.persist ? 1 : 0);
    p->L = make_layout(p->sc, p->T, p->Nq);
    if (p->L.total > p->ws_bytes)
      return fail(SAS_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes, need %zu", p->ws_bytes, p->L.total);
    sas_status st = upload_sync(p->sc, p->L, p->grid, p->ws);
    if (st != SAS_OK) return st;
    // capture pack -> pair kernel -> reduce on a private stream
    if (!p->cap) SAS_HIP(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
    SAS_HIP(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    st = enqueue_forward(nullptr, p->sc, p->L, p->coords, p->types, p->table, p->T, p->Nq, p->grid.q0, p->grid.dq, p->I_out,
                         p->ws, p->cap);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(p->cap, &graph);
    if (st != SAS_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return fail(SAS_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    p->graph = graph;
    SAS_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    p->ready = true;
    note_last(p->ctx, p->sc);
  }
  SAS_HIP(hipGraphLaunch(p->exec, hs));
  return SAS_OK;
}

void sas_plan_destroy(sas_plan* p) {
  if (!p) return;
  {
    DeviceGuard g(p->ctx->device);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
  }
  delete p;
}

sas_status sas_debye_grad_table(sas_ctx* ctx, const float* coords, const int32_t* types, int64_t n,
                                const float* table, int32_t t, const double* q, int32_t nq, const double* dL_dI,
                                double* grad_table_out, double* I_out, void* workspace, size_t ws_bytes, void* stream) {
  if (!ctx) return fail(SAS_ERR_INVALID_ARG, "ctx is NULL");
  sas_status st = check_sizes(n, t, nq, SAS_MAX_TABLE_TYPES);
  if (st != SAS_OK) return st;
  if (n > 0 && (!coords || !types)) return fail(SAS_ERR_INVALID_ARG, "coords/types is NULL");
  if (!table || !dL_dI || !grad_table_out) return fail(SAS_ERR_INVALID_ARG, "table/dL_dI/grad_table_out is NULL");
  QGrid grid;
  st = classify_q(q, nq, &grid);
  if (st != SAS_OK) return st;
  if (table_grad_by_atom(ctx, t)) {
    const RowsLayout R = rows_layout(ctx, n, t, nq, !grid.uniform || ctx->force_direct);
    if (!workspace) return fail(SAS_ERR_INVALID_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
      return fail(SAS_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    if (ws_bytes < R.total) return fail(SAS_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes, need %zu", ws_bytes, R.total);
    if (n > 0 && R.tmp_bytes == 0) return fail(SAS_ERR_HIP, "radix sort size query failed");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(SAS_ERR_HIP, "hipSetDevice(%d) failed", ctx->device);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    st = debug_validate(ctx, coords, types, n, t, hs);
    if (st != SAS_OK) return st;
    st = enqueue_table_grad_by_atom(ctx, R, coords, types, n, table, t, nq, grid, dL_dI, grad_table_out, I_out,
                                    workspace, hs);
    if (st == SAS_OK) {
      ctx->last_direct = !grid.uniform || ctx->force_direct;
      ctx->last_per_atom = true;
      ctx->last_persist = false;
    }
    return st;
  }
  const Schedule sc = make_schedule(ctx, std::vector<int64_t>{n}, t, nq, 0, 0, !grid.uniform || ctx->force_direct,
                                    false, t);
  const Layout L = make_layout(sc, t, nq);
  if (!workspace) return fail(SAS_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(SAS_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(SAS_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes, need %zu", ws_bytes, L.total);
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(SAS_ERR_HIP, "hipSetDevice(%d) failed", ctx->device);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  st = debug_validate(ctx, coords, types, n, t, hs);
  if (st != SAS_OK) return st;
  char* w = static_cast<char*>(workspace);
  st = stage_upload(ctx, workspace, L, upload_image(sc, L, grid), hs);
  if (st != SAS_OK) return st;
  st = enqueue_forward(ctx, sc, L, coords, types, table, t, nq, grid.q0, grid.dq, I_out, workspace, hs);
  if (st != SAS_OK) return st;
  const double* qdev = sc.direct ? reinterpret_cast<const double*>(w + L.qdev) : nullptr;
  auto* gslices = reinterpret_cast<double*>(w + L.gslices);
  SAS_HIP(sas::launch_reduce_slices(view_of(sc, workspace, L), sc.n_slices, reinterpret_cast<const double*>(w + L.gpart),
                                    t * nq, gslices, hs));
  SAS_HIP(sas::launch_table_grad_final(sc.n_slices, gslices, reinterpret_cast<const int32_t*>(w + L.toff), table, t, nq,
                                       grid.q0, grid.dq, qdev, dL_dI, grad_table_out, hs));
  note_last(ctx, sc);
  return SAS_OK;
}

sas_status sas_debye_grad(sas_ctx* ctx, const float* coords, const int32_t* types, int64_t n, const float* table,
                          int32_t t, const double* q, int32_t nq, const double* dL_dI, double* grad_out,
                          double* I_out, void* workspace, size_t ws_bytes, void* stream) {
  if (!ctx) return fail(SAS_ERR_INVALID_ARG, "ctx is NULL");
  sas_status st = check_sizes(n, t, nq, SAS_MAX_TABLE_TYPES);
  if (st != SAS_OK) return st;
  if (n > 0 && (!coords || !types || !grad_out)) return fail(SAS_ERR_INVALID_ARG, "coords/types/grad_out is NULL");
  if (!table || !dL_dI) return fail(SAS_ERR_INVALID_ARG, "table/dL_dI is NULL");
  QGrid grid;
  st = classify_q(q, nq, &grid);
  if (st != SAS_OK) return st;
  const double q0 = grid.q0, dq = grid.dq;
  // a non-uniform grid (or a forced direct form) takes the direct variants
  // of the forward and the adjoint; many table rows (or a forced per-atom
  // form) the per-atom ones
  const bool pa = use_per_atom(ctx, t, n);
  Schedule sc = make_schedule(ctx, std::vector<int64_t>{n}, t, nq, 0, 0, !grid.uniform || ctx->force_direct, pa);
  if (pa)
    add_adjoint_pa(&sc, n, nq);
  else
    add_adjoint(&sc, n, nq);
  const Layout L = make_layout(sc, t, nq);
  if (!workspace) return fail(SAS_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(SAS_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(SAS_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes, need %zu", ws_bytes, L.total);
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(SAS_ERR_HIP, "hipSetDevice(%d) failed", ctx->device);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  st = debug_validate(ctx, coords, types, n, t, hs);
  if (st != SAS_OK) return st;
  char* w = static_cast<char*>(workspace);
  st = stage_upload(ctx, workspace, L, upload_image(sc, L, grid), hs);
  if (st != SAS_OK) return st;
  if (I_out) {
    st = enqueue_forward(ctx, sc, L, coords, types, table, t, nq, q0, dq, I_out, workspace, hs);
    if (st != SAS_OK) return st;
  } else {
    SAS_HIP(sas::launch_pad_table(table, t, nq, sc.ldt, reinterpret_cast<float*>(w + L.tabp), hs));
    if (pa)
      SAS_HIP(sas::launch_pack_plain(coords, types, n, t, reinterpret_cast<double4*>(w + L.xyz),
                                     reinterpret_cast<int32_t*>(w + L.tsort), reinterpret_cast<int32_t*>(w + L.perm),
                                     hs));
    else
      SAS_HIP(sas::launch_pack(coords, types, view_of(sc, workspace, L), sc.S, sc.n_pack, t,
                               reinterpret_cast<int32_t*>(w + L.bcount), reinterpret_cast<int32_t*>(w + L.toff),
                               reinterpret_cast<double4*>(w + L.xyz), reinterpret_cast<int32_t*>(w + L.tsort),
                               reinterpret_cast<int32_t*>(w + L.perm), hs));
  }
  if (n == 0) return SAS_OK;
  sas::AdjArgs a;
  std::memset(&a, 0, sizeof(a));
  a.sd = view_of(sc, workspace, L);
  a.geo = sc.geo_adj;
  a.xyz = reinterpret_cast<const double4*>(w + L.xyz);
  a.tsort = reinterpret_cast<const int32_t*>(w + L.tsort);
  a.toff = pa ? nullptr : reinterpret_cast<const int32_t*>(w + L.toff);
  a.tabp = reinterpret_cast<const float*>(w + L.tabp);
  a.ldt = sc.ldt;
  a.T = t;
  a.Nq = nq;
  a.qa = sc.qa;
  a.w = dL_dI;
  a.gI = reinterpret_cast<double*>(w + L.gI);
  a.gJ = reinterpret_cast<double*>(w + L.gJ);
  a.n_strips = sc.n_strips_adj;
  a.q0 = q0;
  a.dq = dq;
  a.qdev = sc.direct ? reinterpret_cast<const double*>(w + L.qdev) : nullptr;
  {
    LaunchTimer timer(ctx, hs, true);
    if (pa)
      SAS_HIP(sas::launch_adjoint_pa(a, sc.nchunks_adj, sc.qa_template, hs));
    else
      SAS_HIP(sas::launch_adjoint(a, sc.nchunks_adj, hs));
  }
  SAS_HIP(sas::launch_grad_reduce(a, n, sc.nchunks_adj, reinterpret_cast<const int32_t*>(w + L.perm), grad_out, hs));
  note_last(ctx, sc);
  return SAS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Orientation-averaged and hybrid profiles
// ---------------------------------------------------------------------------
namespace {

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
constexpr int64_t kOrientCapAll = int64_t(1) << 17;  // directions per chunk when every q is averaged
constexpr int64_t kOrientBlocksTarget = 16384;         // most work-groups the amplitude kernel takes
// Time per unit, in pair*q steps of the type-form recurrence (measured on
// MI355X): the per-pair set-up of the recurrence (about 66 steps), a step of
// the direct form (4.3) and its set-up (5), and an atom*direction*q of the
// orientation average with the rotation walk (6.5: whole calls on globules
// gave 6.2 at 50,000 atoms and 7.6 at 20,000) or with a sine and cosine per q
// (1.8x that, the kernels' ratio), plus a fixed cost of the averaged part
// (the radius read back and the host's quadrature plan, about 0.1 ms, 2.2e9
// steps), which keeps small molecules on the direct sum.
constexpr double kSetupRecurrence = 66.0, kStepDirect = 4.3, kSetupDirect = 5.0, kCostOrient = 11.7,
                 kCostOrientRot = 6.5, kCostOrientFixed = 2.2e9;

// The orientation kernel walks exp(i q p) over the leading nq_o q values when
// they form a uniform grid whose step *dq turns the farthest atom's phase by
// at most kRotMaxStep.
bool orient_rot(const double* q, int32_t nq_o, double r_max, double* dq) {
  QGrid g;
  if (nq_o <= 0 || classify_q(q, nq_o, &g) != SAS_OK || !g.uniform) return false;
  if (!(g.dq * r_max <= sas::kRotMaxStep)) return false;
  if (dq) *dq = g.dq;
  return true;
}

// Steps the forward kernel runs for nq q values (chunks padded to templates).
double direct_steps(int32_t nq, bool uniform) {
  if (nq <= 0) return 0.0;
  if (!uniform) return kSetupDirect + kStepDirect * 32.0 * ((nq + 31) / 32);
  const int32_t nch = (nq + 199) / 200;
  const int32_t qc = (nq + nch - 1) / nch;
  return kSetupRecurrence * nch + static_cast<double>(nch) * pick_qc_template(qc, false);
}

// Gauss-Legendre rule of n points on [-1, 1]: roots of P_n by Newton's method
// from cos(pi (i + 3/4) / (n + 1/2)), P_n and P_n' from the three-term
// recurrence, weights 2 / ((1 - x^2) P_n'(x)^2).
void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(3.14159265358979323846 * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) p0 = 1.0;
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) <= 1e-15 * std::fmax(1.0, std::fabs(z))) {
        // derivative at the converged root for the weight
        p0 = 1.0;
        p1 = z;
        for (int k = 2; k <= n; ++k) {
          const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        if (n == 1) p0 = 1.0;
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        break;
      }
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

int32_t orient_degree(double q, double r_max, double tol) {
  const double qr = q * r_max;
  const double d = std::min(15.0, std::max(4.0, -std::log10(tol)));
  return static_cast<int32_t>(std::ceil(qr + 0.25 * d * std::cbrt(qr) + 0.6 * d));
}

struct OrientPlan {
  int32_t nq_o = 0;  // leading q values averaged over orientations
  std::vector<sas::OrientChunk> chunks;
  std::vector<double> gl;  // node, weight pairs
  int64_t total_blocks = 0;
  int32_t parts = 1, atoms_per_part = 0;
  int64_t apart_elems = 0;  // double2 values
  int32_t ldo = 0;          // row stride of the orientation table
};

OrientPlan plan_orient(int64_t n, const double* q, int32_t nq_o, double r_max, double tol, int64_t slots) {
  OrientPlan p;
  p.nq_o = nq_o;
  if (nq_o <= 0) return p;
  const int32_t nch = (nq_o + sas::kOrientQ - 1) / sas::kOrientQ;
  p.ldo = nch * sas::kOrientQ;
  int64_t blk = 0;
  for (int32_t c = 0; c < nch; ++c) {
    sas::OrientChunk ch{};
    ch.m0 = c * sas::kOrientQ;
    ch.nq = std::min(sas::kOrientQ, nq_o - ch.m0);
    const int32_t L = orient_degree(q[ch.m0 + ch.nq - 1], r_max, tol);
    ch.nth = L + 1;
    ch.nph = 2 * L + 1;
    ch.gl_off = static_cast<int32_t>(p.gl.size() / 2);
    std::vector<double> x(ch.nth), w(ch.nth);
    gauss_legendre(ch.nth, x.data(), w.data());
    for (int32_t i = 0; i < ch.nth; ++i) {
      p.gl.push_back(x[i]);
      p.gl.push_back(w[i]);
    }
    ch.blk_off = blk;
    blk += cdiv(static_cast<int64_t>(ch.nth) * ch.nph, int64_t(sas::kWave));
    p.chunks.push_back(ch);
  }
  p.total_blocks = blk;
  // Every work-group does the same work (atoms_per_part atoms for 64
  // directions and 16 q), so the kernel takes about ceil(blk parts / slots)
  // rounds of 1/parts of the atoms each: choose the part count that makes
  // that smallest (the last round of a poor choice runs mostly empty), the
  // fewest parts among equals; at most kOrientBlocksTarget work-groups
  // (the workspace bound) and 256 atoms per part.
  const int64_t max_parts = std::max<int64_t>(
      1, std::min(cdiv(n, int64_t(256)), cdiv(kOrientBlocksTarget, std::max<int64_t>(blk, 1))));
  int64_t best = 1;
  double best_t = 1e300;
  for (int64_t parts = 1; parts <= max_parts; ++parts) {
    const double t = static_cast<double>(cdiv(blk * parts, std::max<int64_t>(slots, 1))) / static_cast<double>(parts);
    if (t < best_t * (1.0 - 1e-9)) {
      best_t = t;
      best = parts;
    }
  }
  p.parts = static_cast<int32_t>(best);
  p.atoms_per_part = static_cast<int32_t>(cdiv(cdiv(std::max<int64_t>(n, 1), int64_t(p.parts)),
                                                        int64_t(sas::kPaSub)) * sas::kPaSub);
  int64_t off = 0;
  for (auto& ch : p.chunks) {
    ch.a_off = off;
    off += static_cast<int64_t>(p.parts) * ch.nth * ch.nph * sas::kOrientQ;
  }
  p.apart_elems = off;
  return p;
}

// Workspace of the orientation part: upload block (chunks, rule, q values),
// geometry, padded table and partial amplitudes.
struct OrientLayout {
  size_t xyz = 0, tsort = 0, perm = 0, geom = 0;
  size_t upload = 0, upload_bytes = 0, chunks = 0, gl = 0, qv = 0;
  size_t tabo = 0, apart = 0, ored = 0, tabd = 0, direct = 0, total = 0;
};

OrientLayout orient_layout(int64_t n, int32_t T, const OrientPlan& p, int32_t nq_d, size_t direct_bytes) {
  OrientLayout L;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    const size_t o = at;
    at = align_up(at + std::max<size_t>(bytes, 1));
    return o;
  };
  L.xyz = take(sizeof(double4) * n);
  L.tsort = take(sizeof(int32_t) * n);
  L.perm = take(sizeof(int32_t) * n);
  L.geom = take(sizeof(double) * 4);
  const size_t cb = align_up(sizeof(sas::OrientChunk) * p.chunks.size());
  const size_t gb = align_up(sizeof(double) * p.gl.size());
  const size_t qb = sizeof(double) * p.nq_o;
  L.upload_bytes = cb + gb + qb;
  L.upload = take(L.upload_bytes);
  L.chunks = L.upload;
  L.gl = L.upload + cb;
  L.qv = L.upload + cb + gb;
  L.tabo = take(sizeof(float) * static_cast<size_t>(T) * p.ldo);
  L.apart = take(sizeof(double) * 2 * p.apart_elems);
  L.ored = take(sizeof(double) * p.chunks.size() * sas::kOrientSlices * sas::kOrientQ);
  L.tabd = take(sizeof(float) * static_cast<size_t>(T) * nq_d);
  L.direct = take(direct_bytes);
  L.total = at;
  return L;
}

size_t direct_part_bytes(const sas_ctx* ctx, int64_t n, int32_t t, int32_t nq_d) {
  if (nq_d <= 0) return 0;
  const std::vector<int64_t> sizes{n};
  const bool pa = use_per_atom(ctx, t, n);
  size_t need = 0;
  for (bool direct : {false, true})
    need = std::max(need, make_layout(make_schedule(ctx, sizes, t, nq_d, 0, 0, direct, pa), t, nq_d).total);
  return need;
}

// Bound on the orientation part's size: K directions per chunk at most cap.
size_t orient_bound_bytes(int64_t n, int32_t t, int32_t nq, int64_t cap) {
  const int64_t nch = cdiv(int64_t(nq), int64_t(sas::kOrientQ));
  const int64_t blocks = nch * cdiv(cap, int64_t(sas::kWave));
  const int64_t L = static_cast<int64_t>(std::sqrt(static_cast<double>(cap) / 2.0)) + 2;
  size_t b = 0;
  b += align_up(sizeof(double4) * n) + 2 * align_up(sizeof(int32_t) * n);
  b += 256 + align_up(sizeof(sas::OrientChunk) * nch) + align_up(sizeof(double) * 2 * nch * (L + 1)) +
       align_up(sizeof(double) * nq) + 256;
  b += align_up(sizeof(float) * t * nch * sas::kOrientQ);
  b += align_up(sizeof(double) * nch * sas::kOrientSlices * sas::kOrientQ);
  if (cap > 0) b += align_up(sizeof(double) * 2 * (kOrientBlocksTarget + blocks) * sas::kWave * sas::kOrientQ);
  b += align_up(sizeof(float) * t * static_cast<size_t>(nq));
  return b;
}

// Directions per chunk the automatic split can choose: an averaged q may cost
// up to 2.6 direct steps of the q it replaces (twice a step for padding, and
// 1.3 for the recurrence's set-up, which the direct sum spreads over its q
// values: without it the 50,000-atom globule's last chunks on [0, 1] would be
// refused although averaging every q is the faster choice there).  The
// workspace query bounds the averaged part by the same cap.
int64_t orient_cap(int64_t n, int32_t mode, bool uniform, bool rot) {
  if (mode == SAS_HYBRID_ORIENT_ALL) return kOrientCapAll;
  const double step = uniform ? 1.0 : kStepDirect;
  return std::max<int64_t>(1, static_cast<int64_t>(static_cast<double>(std::max<int64_t>(n - 1, 0)) * step * 1.3 /
                                                   (rot ? kCostOrientRot : kCostOrient)));
}

}  // namespace

extern "C" {

int32_t sas_orient_degree(double q, double r_max, double tol) {
  if (!(q >= 0.0) || !(r_max >= 0.0) || !(tol > 0.0) || !std::isfinite(q) || !std::isfinite(r_max)) return -1;
  return orient_degree(q, r_max, tol);
}

size_t sas_debye_workspace_size_hybrid(const sas_ctx* ctx, int64_t n, int32_t t, int32_t nq, int32_t mode) {
  if (check_sizes(n, t, nq, SAS_MAX_TABLE_TYPES) != SAS_OK) return 0;
  if (mode < SAS_HYBRID_AUTO || mode > SAS_HYBRID_DIRECT_ALL) return 0;
  const int64_t cap = std::max(orient_cap(n, mode, true, true), orient_cap(n, mode, false, true));
  // (the pack, geometry and table-copy regions precede the direct part in every mode)
  const size_t orient = orient_bound_bytes(n, t, nq, mode == SAS_HYBRID_DIRECT_ALL ? 0 : cap);
  size_t direct = 0;  // whichever number of q values is left to the direct sum
  for (int32_t nq_d = 1; nq_d <= nq; ++nq_d) direct = std::max(direct, direct_part_bytes(ctx, n, t, nq_d));
  return orient + direct + 4096;
}

sas_status sas_debye_profile_hybrid(sas_ctx* ctx, const float* coords, const int32_t* types, int64_t n,
                                    const float* table, int32_t t, const double* q, int32_t nq, double tol,
                                    int32_t mode, double* I_out, void* workspace, size_t ws_bytes, void* stream,
                                    int32_t* n_orient) {
  if (!ctx) return fail(SAS_ERR_INVALID_ARG, "ctx is NULL");
  sas_status st = check_sizes(n, t, nq, SAS_MAX_TABLE_TYPES);
  if (st != SAS_OK) return st;
  if (n > 0 && (!coords || !types)) return fail(SAS_ERR_INVALID_ARG, "coords/types is NULL");
  if (!table || !I_out) return fail(SAS_ERR_INVALID_ARG, "table/I_out is NULL");
  if (!(tol >= 1e-15 && tol <= 1e-2)) return fail(SAS_ERR_INVALID_ARG, "tol %g outside [1e-15, 1e-2]", tol);
  if (mode < SAS_HYBRID_AUTO || mode > SAS_HYBRID_DIRECT_ALL) return fail(SAS_ERR_INVALID_ARG, "unknown mode %d", mode);
  QGrid grid;
  st = classify_q(q, nq, &grid);
  if (st != SAS_OK) return st;
  if (!workspace) return fail(SAS_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(SAS_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(SAS_ERR_HIP, "hipSetDevice(%d) failed", ctx->device);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  st = refuse_capture(hs, "the hybrid profile (it reads the radius back)");
  if (st != SAS_OK) return st;
  st = debug_validate(ctx, coords, types, n, t, hs);
  if (st != SAS_OK) return st;
  char* w = static_cast<char*>(workspace);

  // 1. FP64 copy of the coordinates (caller order: the amplitude sums need no
  //    type sort, so any number of table rows works) and geometry; the radius
  //    decides the quadrature, so it is read back here (the one
  //    synchronisation of this call)
  OrientPlan none;
  OrientLayout L0 = orient_layout(n, t, none, 0, 0);
  if (ws_bytes < L0.total) return fail(SAS_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes, need %zu", ws_bytes, L0.total);
  double geom[4] = {0.0, 0.0, 0.0, 0.0};
  if (mode != SAS_HYBRID_DIRECT_ALL && n > 0) {
    SAS_HIP(sas::launch_pack_plain(coords, types, n, t, reinterpret_cast<double4*>(w + L0.xyz),
                                   reinterpret_cast<int32_t*>(w + L0.tsort), reinterpret_cast<int32_t*>(w + L0.perm),
                                   hs));
    SAS_HIP(sas::launch_geometry(reinterpret_cast<const double4*>(w + L0.xyz), n, reinterpret_cast<double*>(w + L0.geom),
                                 hs));
    SAS_HIP(hipMemcpyAsync(geom, w + L0.geom, sizeof(geom), hipMemcpyDeviceToHost, hs));
    SAS_HIP(hipStreamSynchronize(hs));
  }
  const double r_max = geom[3];

  // 2. the split: the leading q values whose orientation average costs less
  //    than the direct sum (directions grow with q, so it is a prefix)
  int32_t nq_o = 0;
  if (mode == SAS_HYBRID_ORIENT_ALL) {
    nq_o = nq;
  } else if (mode == SAS_HYBRID_AUTO && n > 1) {
    // the chunk-aligned split with the least estimated time, in pair steps:
    // averaged chunks cost K n kCostOrient per q against n(n-1)/2 pairs
    // running the direct kernel's steps (set-up, padding) over the rest
    const double pairs = 0.5 * static_cast<double>(n) * static_cast<double>(n - 1);
    double best = pairs * direct_steps(nq, grid.uniform), units = 0.0, orient = 0.0;
    for (int32_t m0 = 0; m0 < nq; m0 += sas::kOrientQ) {
      const int32_t m1 = std::min(nq, m0 + sas::kOrientQ);
      const int64_t L = orient_degree(q[m1 - 1], r_max, tol);
      units += static_cast<double>(L + 1) * (2 * L + 1) * (m1 - m0) * static_cast<double>(n);
      orient = kCostOrientFixed + units * (orient_rot(q, m1, r_max, nullptr) ? kCostOrientRot : kCostOrient);
      QGrid rest;
      const bool uni = m1 < nq && classify_q(q + m1, nq - m1, &rest) == SAS_OK && rest.uniform;
      const double total = orient + pairs * direct_steps(nq - m1, uni);
      if (total < best) {
        best = total;
        nq_o = m1;
      }
      if (orient >= best) break;
    }
  }
  const bool rot = orient_rot(q, nq_o, r_max, nullptr);
  const int64_t cap = orient_cap(n, mode, grid.uniform, rot);
  OrientPlan plan;
  OrientLayout L;
  for (;;) {
    plan = plan_orient(n, q, nq_o, r_max, tol,
                       static_cast<int64_t>(ctx->cu_count) * sas::orient_wgs_per_cu(orient_rot(q, nq_o, r_max, nullptr)));
    bool over = false;
    for (const auto& ch : plan.chunks) over = over || static_cast<int64_t>(ch.nth) * ch.nph > cap;
    const int32_t nq_d = nq - nq_o;
    L = orient_layout(n, t, plan, nq_d, direct_part_bytes(ctx, n, t, nq_d));
    if (!over && L.total <= ws_bytes) break;
    if (mode == SAS_HYBRID_ORIENT_ALL) {
      if (over) return fail(SAS_ERR_UNSUPPORTED, "orientation average needs more than %lld directions", (long long)cap);
      return fail(SAS_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes, need %zu", ws_bytes, L.total);
    }
    if (nq_o == 0) return fail(SAS_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes, need %zu", ws_bytes, L.total);
    nq_o = std::max(0, ((nq_o - 1) / sas::kOrientQ) * sas::kOrientQ);  // drop the last chunk
  }

  // the direct part runs on the context's second stream beside the
  // orientation average (disjoint q ranges, workspace regions and outputs),
  // forked from the caller's stream and joined back into it on every exit
  const int32_t nq_d = nq - nq_o;
  hipStream_t hd = hs;
  struct Join {
    hipStream_t from = nullptr, into = nullptr;
    hipEvent_t ev = nullptr;
    ~Join() {
      if (ev) {
        (void)hipEventRecord(ev, from);
        (void)hipStreamWaitEvent(into, ev, 0);
      }
    }
  } join;
  if (nq_o > 0 && nq_d > 0) {
    if (!ctx->side) SAS_HIP(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
    if (!ctx->fork_ev) SAS_HIP(hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming));
    if (!ctx->join_ev) SAS_HIP(hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming));
    hd = ctx->side;
    SAS_HIP(hipEventRecord(ctx->fork_ev, hs));
    SAS_HIP(hipStreamWaitEvent(hd, ctx->fork_ev, 0));
    join.from = hd;
    join.into = hs;
    join.ev = ctx->join_ev;
  }

  // 3. orientation average of the leading q values
  if (nq_o > 0) {
    std::vector<char> img(L.upload_bytes, 0);
    std::memcpy(img.data() + (L.chunks - L.upload), plan.chunks.data(), sizeof(sas::OrientChunk) * plan.chunks.size());
    std::memcpy(img.data() + (L.gl - L.upload), plan.gl.data(), sizeof(double) * plan.gl.size());
    std::memcpy(img.data() + (L.qv - L.upload), q, sizeof(double) * nq_o);
    st = stage_upload_to(ctx, w + L.upload, img, hs);
    if (st != SAS_OK) return st;
    SAS_HIP(sas::launch_copy_cols(table, t, nq, 0, nq_o, plan.ldo, reinterpret_cast<float*>(w + L.tabo), hs));
    sas::OrientArgs a;
    std::memset(&a, 0, sizeof(a));
    a.chunks = reinterpret_cast<const sas::OrientChunk*>(w + L.chunks);
    a.nchunks = static_cast<int32_t>(plan.chunks.size());
    a.T = t;
    a.gl = reinterpret_cast<const double*>(w + L.gl);
    a.xyz = reinterpret_cast<const double4*>(w + L0.xyz);
    a.tsort = reinterpret_cast<const int32_t*>(w + L0.tsort);
    a.tabp = reinterpret_cast<const float*>(w + L.tabo);
    a.ldt = plan.ldo;
    a.n = static_cast<int32_t>(n);
    a.qv = reinterpret_cast<const double*>(w + L.qv);
    a.center = reinterpret_cast<const double*>(w + L0.geom);
    a.parts = plan.parts;
    a.atoms_per_part = plan.atoms_per_part;
    a.apart = reinterpret_cast<double2*>(w + L.apart);
    a.ored = reinterpret_cast<double*>(w + L.ored);
    a.rot = orient_rot(q, nq_o, r_max, &a.dq) ? 1 : 0;
    SAS_HIP(sas::launch_orient(a, plan.total_blocks, nq_o, I_out, hs));
  }

  // 4. direct sum for the rest, on a compact copy of their table columns
  if (nq_d > 0) {
    QGrid gd;
    st = classify_q(q + nq_o, nq_d, &gd);
    if (st != SAS_OK) return st;
    float* tabd = reinterpret_cast<float*>(w + L.tabd);
    SAS_HIP(sas::launch_copy_cols(table, t, nq, nq_o, nq_d, nq_d, tabd, hd));
    const Schedule sd = make_schedule(ctx, std::vector<int64_t>{n}, t, nq_d, 0, 0, !gd.uniform || ctx->force_direct,
                                      use_per_atom(ctx, t, n));
    const Layout Ld = make_layout(sd, t, nq_d);
    void* wd = w + L.direct;
    st = stage_upload(ctx, wd, Ld, upload_image(sd, Ld, gd), hd);
    if (st != SAS_OK) return st;
    st = enqueue_forward(ctx, sd, Ld, coords, types, tabd, t, nq_d, gd.q0, gd.dq, I_out + nq_o, wd, hd);
    if (st != SAS_OK) return st;
  }
  if (n_orient) *n_orient = nq_o;
  return SAS_OK;
}

}  // extern "C"
