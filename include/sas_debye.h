/*
 * sas_debye.h -- C ABI of the MI355X (gfx950) Debye-summation library.
 *
 * The library evaluates the small-angle-scattering profile of a molecule by
 * direct summation over all atom pairs (Berlin, Gumerov, Duraiswami, Fushman,
 * "Performance of a GPU-based Direct Summation Algorithm for Computation of
 * Small Angle Scattering Profile", Background section, Eq. 2):
 *
 *     I(q) = sum_k sum_j f_k(q) f_j(q) sin(q r_jk) / (q r_jk),   sin(0)/0 := 1
 *
 * Form factors are given per atom *type*: f_k(q_m) = table[type_k * Nq + m].
 * One type per atom reproduces the paper's per-atom form factors (the text
 * below Eq. 2); a handful of element types is the common case.  With few
 * types the atoms are sorted by type and f_a f_b is applied once per run of
 * equal types; with many types (T > SAS_MAX_TYPES, or fewer than 16 atoms
 * per type on average and T >= 64) every pair term is weighted by its f_j
 * inside the q loop instead (the per-atom form), with the same accuracy.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Units: coordinates in Angstrom, q in 1/Angstrom, no 2pi or 4pi factors.
 *  - "dev" pointers are HIP device pointers on the context's device; "host"
 *    pointers are ordinary host memory and are only read before the call
 *    returns.  The caller owns every buffer; the library never frees caller
 *    memory.  It owns only sas_ctx and sas_plan objects.
 *  - Device work is enqueued asynchronously on `stream` (a hipStream_t passed
 *    as void*; NULL is the default stream).  Results are valid once the
 *    stream reaches the call.  No call synchronises the stream, except the
 *    hybrid profile and the debug mode (both below).  Host-written blocks
 *    that a call needs on the device (a batched call's descriptors, a
 *    non-uniform q grid) go through a ring of pinned staging buffers owned by
 *    the context; the host waits only if every slot's copy is still queued.
 *  - Graph capture: calls on a single structure with a uniform q grid upload
 *    nothing and may be captured into a caller's graph.  A call that would
 *    upload a host block, the hybrid profile and the debug mode refuse a
 *    capturing stream with SAS_ERR_UNSUPPORTED before enqueueing anything;
 *    a batched plan (sas_plan_*) is the capturable form of the batched call.
 *  - Scratch memory is the caller's `workspace` (dev, 256-byte aligned) of at
 *    least the size the matching *_workspace_size query returns.
 *  - The q grid is host double [nq], finite, q_0 >= 0 and strictly
 *    increasing.  A uniform grid (q_m = q_0 + m dq within 8 ulp of max q; the
 *    Results section evaluates profiles on such grids; Nq <= 2 always counts
 *    as uniform) takes the fast path: the pair kernel steps sin(q r) from one
 *    q to the next by a recurrence.  Any other grid is evaluated directly,
 *    one sine per pair and q, at a few times the cost per pair and q.  Every
 *    call accepts both.
 *  - Results are FP64.  Pair terms are evaluated in FP32 from FP64 per-pair
 *    set-up values; every cross-lane and cross-block sum beyond one 64-lane
 *    wave is FP64 and in a fixed order, so two identical calls give bitwise
 *    identical results.
 *  - Errors: a status code, plus a thread-local message from
 *    sas_last_error().  Host-detectable argument errors are reported before
 *    any device work is enqueued and leave the outputs untouched.  Device-side
 *    content errors (a type id outside [0,T), non-finite coordinates) are not
 *    checked by default: they give unspecified values, never an out-of-bounds
 *    access, because type ids are clamped when the table is read.
 *  - Debug mode: with the environment variable SAS_DEBUG_VALIDATE set to a
 *    non-empty value other than "0" when a context is created, every call on
 *    that context (and every sas_plan_execute of its plans) first checks on
 *    the device that each type id lies in [0,T) and each coordinate is
 *    finite, then synchronises the stream and reads the result back: such
 *    inputs give SAS_ERR_INVALID_ARG, naming the count and the first atom,
 *    before any output is written.  This mode synchronises (the exception to
 *    the rule above) and cannot be captured into a graph.
 *  - Thread safety: calls on distinct contexts, plans and workspaces may run
 *    concurrently.  Calls that share a workspace or plan must be ordered on
 *    one stream.
 */
#ifndef SAS_DEBYE_H
#define SAS_DEBYE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SAS_OK = 0,
  SAS_ERR_INVALID_ARG = 1,         /* null pointer, negative size, bad offsets, ...       */
  SAS_ERR_Q_NOT_UNIFORM = 2,       /* q not finite / non-negative / increasing (uniform where required) */
  SAS_ERR_UNSUPPORTED = 3,         /* a size beyond the documented limits                  */
  SAS_ERR_WORKSPACE_TOO_SMALL = 4, /* ws_bytes below the size the query returns            */
  SAS_ERR_OUT_OF_MEMORY = 5,       /* a host or device allocation of the library failed   */
  SAS_ERR_HIP = 6                  /* a HIP runtime call failed; see sas_last_error()      */
} sas_status;

/* Limits of this version. */
#define SAS_MAX_TYPES 4096          /* T up to which the type-sorted form can be used  */
#define SAS_MAX_TABLE_TYPES (1 << 24) /* T for the profile calls (per-atom form above SAS_MAX_TYPES) */
#define SAS_MAX_TABLE_GRAD_TYPES 64 /* T up to which sas_debye_grad_table keeps per-type sums */
#define SAS_MAX_NQ 65536            /* Nq                                          */
#define SAS_MAX_ATOMS 100000000LL   /* atoms per structure                         */

typedef struct sas_ctx sas_ctx;   /* device binding, tuning choices, staging buffers */
typedef struct sas_plan sas_plan; /* batched schedule bound to buffers + captured graph */

/* Library version as an integer MAJOR*10000 + MINOR*100 + PATCH. */
int sas_version(void);

/* Create a context on HIP device `device` (must be a gfx950 GPU).  *out is
 * set on success.  Errors: SAS_ERR_INVALID_ARG (out NULL, no such device,
 * not gfx950), SAS_ERR_HIP, SAS_ERR_OUT_OF_MEMORY. */
sas_status sas_create(int device, sas_ctx** out);
void sas_destroy(sas_ctx* ctx); /* NULL is ignored; waits for nothing */

/* Thread-local, human-readable detail of the last failed call on this thread. */
const char* sas_last_error(void);
const char* sas_status_string(sas_status s);

/* Host-only q-grid analysis (no device work, no context needed).
 * q: host [nq].  On SAS_OK writes q0 = q[0] and dq = (q[nq-1]-q[0])/(nq-1)
 * (dq = 0 when nq == 1).  Errors: SAS_ERR_INVALID_ARG (q NULL, nq <= 0 or
 * > SAS_MAX_NQ), SAS_ERR_Q_NOT_UNIFORM. */
sas_status sas_q_grid_check(const double* q, int32_t nq, double* q0, double* dq);

/* Workspace bytes needed by sas_debye_profile (grad = 0; enough for a
 * uniform or a non-uniform grid), sas_debye_grad (grad = 1) or
 * sas_debye_grad_table (grad = 2) for these sizes.  Returns 0 for invalid
 * sizes. */
size_t sas_debye_workspace_size(const sas_ctx* ctx, int64_t n, int32_t t, int32_t nq, int grad);

/*
 * Plain Debye profile (Eq. 2).
 *   coords  dev  float [n][3]     atom positions, Angstrom (AoS x,y,z)
 *   types   dev  int32 [n]        type id of each atom, in [0, t)
 *   n                             number of atoms, 0 <= n <= SAS_MAX_ATOMS
 *   table   dev  float [t][nq]    f_type(q_m), row-major
 *   t                             number of types, 1 <= t <= SAS_MAX_TABLE_TYPES
 *   q       host double [nq]      q grid, uniform or not (see conventions)
 *   nq                            1 <= nq <= SAS_MAX_NQ
 *   I_out   dev  double [nq]      written: I(q_m)
 *   workspace/ws_bytes            dev scratch, >= sas_debye_workspace_size(ctx,n,t,nq,0)
 *   stream                        hipStream_t as void*
 * n = 0 gives I = 0; n = 1 gives f(q)^2; q_m = 0 gives (sum_k f_k(0))^2.
 * Coincident distinct atoms contribute f_k f_j (the sinc limit).
 */
sas_status sas_debye_profile(sas_ctx* ctx, const float* coords, const int32_t* types, int64_t n,
                             const float* table, int32_t t, const double* q, int32_t nq, double* I_out,
                             void* workspace, size_t ws_bytes, void* stream);

/*
 * Allocation-free variant of sas_debye_profile, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, results and edge cases as
 * sas_debye_profile without the workspace: its scratch is a fixed array of
 * SAS_NOALLOC_SCRATCH_BYTES in device memory that the library holds, one per
 * GPU, from the first sas_create on that GPU until the process ends.  The call
 * allocates no device or pinned memory, uploads nothing, records no kernel
 * timing and never synchronises (except in the debug mode, as above); it may
 * be captured into a graph.
 *   - q must be a uniform grid and the context's form must not be
 *     SAS_FORM_DIRECT (the direct form needs its grid uploaded):
 *     SAS_ERR_UNSUPPORTED otherwise.
 *   - When the automatic tile shape's strip rows do not fit the array (and
 *     no shape was forced with sas_set_variant), the call takes the shortest
 *     longer J block whose rows fit, up to 512 atoms; its sums then run in
 *     another order than sas_debye_profile's, to the same accuracy.  Sizes
 *     that fit no shape give SAS_ERR_UNSUPPORTED with the bytes needed;
 *     64 MiB holds a 50,000-atom profile of 200 q with 5 types (J blocks of
 *     512 atoms).
 *   - Every call on one GPU, from any context or thread, shares that GPU's
 *     array: calls that overlap in time on one GPU (two streams, two threads,
 *     two contexts) race and give wrong results.  Order them on one stream.
 *     Each call rewrites every scratch region it reads, so no clearing is
 *     needed between calls.
 */
#define SAS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
sas_status sas_debye_profile_noalloc(sas_ctx* ctx, const float* coords, const int32_t* types, int64_t n,
                                     const float* table, int32_t t, const double* q, int32_t nq, double* I_out,
                                     void* stream);

/*
 * Batched profiles of S structures that share one table and one q grid (the
 * ensemble use the paper's introduction motivates: many conformations or
 * structures evaluated together).  Atoms of structure s are rows
 * [offsets[s], offsets[s+1]) of coords/types; offsets is a HOST int64 [S+1]
 * array with offsets[0] = 0, non-decreasing.  I_out is dev double [S][nq].
 * All structures run in one launch sequence; large structures are scheduled
 * first.  Same limits and edge cases as the plain call, per structure.
 */
size_t sas_debye_workspace_size_batched(const sas_ctx* ctx, const int64_t* offsets, int32_t S, int32_t t,
                                        int32_t nq);
sas_status sas_debye_profile_batched(sas_ctx* ctx, const float* coords, const int32_t* types,
                                     const int64_t* offsets, int32_t S, const float* table, int32_t t,
                                     const double* q, int32_t nq, double* I_out, void* workspace, size_t ws_bytes,
                                     void* stream);

/*
 * Batched plan: binds the device buffers above once, chooses the tile shape by
 * timing candidate variants on first execution (J blocks of 64, 128, 256 and
 * 512 atoms, the default q chunk and half of it, grid and persistent launch
 * of the pair kernel; the choice is cached in the context per workload shape;
 * with SAS_TUNE_LOG set in the environment when the context is created, every
 * timing is printed to stderr), captures the launch sequence in a hipGraph
 * and replays it on each execute.  The caller may rewrite coords/types/table in
 * place between executes; sizes, offsets and q are fixed at creation.
 * The plan must be destroyed before the context.
 */
sas_status sas_plan_create_batched(sas_ctx* ctx, const float* coords, const int32_t* types,
                                   const int64_t* offsets, int32_t S, const float* table, int32_t t,
                                   const double* q, int32_t nq, double* I_out, void* workspace, size_t ws_bytes,
                                   sas_plan** out);
sas_status sas_plan_execute(sas_plan* plan, void* stream);
void sas_plan_destroy(sas_plan* plan);

/*
 * Vector-Jacobian product of the profile w.r.t. the coordinates:
 *     grad_out[i][k] = sum_m dL_dI[m] * dI(q_m)/dx_ik
 *                    = sum_{j != i} 2 sum_m dL_dI[m] f_i f_j
 *                        (cos(q_m r)/r - sin(q_m r)/(q_m r^2)) (x_ik - x_jk)/r
 * (the derivative of Eq. 2; terms with q_m = 0 or r = 0 vanish).
 *   dL_dI    dev double [nq]    weights (e.g. dchi2/dI)
 *   grad_out dev double [n][3]  written, in the caller's atom order
 *   I_out    dev double [nq] or NULL: if given, the profile is written too
 * q follows the profile's conventions: a uniform grid takes the recurrence,
 * any other increasing grid the direct variant (sin and cos of q r evaluated
 * for every pair and q, about four times the cost).  The table form follows
 * the profile's choice: the type-sorted form, or with many rows (per-atom
 * form factors: t > SAS_MAX_TYPES, or t >= 64 with fewer than 16 atoms per
 * row) or SAS_FORM_PER_ATOM the per-atom form, whose pair weights
 * dL_dI[m] f_i(q_m) f_j(q_m) are formed inside the q loop.
 * 1 <= t <= SAS_MAX_TABLE_TYPES.
 * workspace >= sas_debye_workspace_size(ctx, n, t, nq, 1).
 */
sas_status sas_debye_grad(sas_ctx* ctx, const float* coords, const int32_t* types, int64_t n, const float* table,
                          int32_t t, const double* q, int32_t nq, const double* dL_dI, double* grad_out,
                          double* I_out, void* workspace, size_t ws_bytes, void* stream);

/*
 * Vector-Jacobian product of the profile w.r.t. the form-factor table.  At
 * each q Eq. 2 is a quadratic form in the form factors, so
 *     grad_table[t][m] = dL_dI[m] * dI(q_m)/df_t(q_m)
 *                      = dL_dI[m] * 2 sum_{i of type t} sum_j f_j(q_m) sinc(q_m r_ij)
 * (j over all atoms, i included).  It is what fitting form-factor or
 * solvent parameters needs (chain rule through the table).  Two forms:
 *  - t <= SAS_MAX_TABLE_GRAD_TYPES: one pass of the type-sorted forward
 *    kernel that also keeps per-type sums, about the cost of a profile;
 *  - more rows (per-atom form factors, the text below Eq. 2), or the context's
 *    form set to SAS_FORM_PER_ATOM: the per-atom sums
 *    S_i = sum_j f_j sinc(q r_ij) over the whole square of pairs (twice the
 *    profile's pairs), then added by type in atom order after a stable sort
 *    of the atoms by type.  Rows of types no atom holds are zero.  The
 *    workspace holds an FP32 [ceil(n/512)][nq][n] array of per-block sums
 *    (3.8 GiB for n = 50,000 and nq = 200).
 * Both are deterministic: identical calls give identical bits.
 *   dL_dI          dev double [nq]     weights
 *   grad_table_out dev double [t][nq]  written
 *   I_out          dev double [nq] or NULL: if given, the profile is written too
 * q: any increasing grid (uniform: recurrence; otherwise direct).
 * 1 <= t <= SAS_MAX_TABLE_TYPES.
 * workspace >= sas_debye_workspace_size(ctx, n, t, nq, 2).
 */
sas_status sas_debye_grad_table(sas_ctx* ctx, const float* coords, const int32_t* types, int64_t n,
                                const float* table, int32_t t, const double* q, int32_t nq, const double* dL_dI,
                                double* grad_table_out, double* I_out, void* workspace, size_t ws_bytes,
                                void* stream);

/*
 * Orientation-averaged and hybrid profiles (approximate at a stated
 * tolerance).  Eq. 1 averages |A(q,u)|^2, A = sum_j f_j exp(i q u.r_j), over
 * directions u; a product rule with L+1 Gauss-Legendre nodes in cos(theta)
 * and 2L+1 uniform nodes in phi averages it to relative accuracy about tol
 * when L >= q R + O((q R)^(1/3)) (R: largest distance from the centre), at
 * a cost of (L+1)(2L+1) N per q against N^2/2 for the direct sum: cheaper
 * at low q, as the Background section argues (O(q^2 D^2) directions).
 *
 * sas_orient_degree: the L used for q, R and tol (host only; -1 for invalid
 * arguments).
 *
 * sas_debye_profile_hybrid: mode SAS_HYBRID_AUTO averages the leading q values
 * for which (L+1)(2L+1) N costs less than the direct sum and sums the rest
 * directly (uniform rest: recurrence; otherwise direct form);
 * SAS_HYBRID_ORIENT_ALL averages every q (at most 2^17 directions per chunk
 * of 16 q, SAS_ERR_UNSUPPORTED beyond); SAS_HYBRID_DIRECT_ALL is the direct
 * sum.  tol in [1e-15, 1e-2].  *n_orient (host, may be NULL) receives the
 * number of leading q values that were averaged.  t <= SAS_MAX_TABLE_TYPES
 * (the amplitude sums take each atom's own row; no type sort).  This
 * call synchronises `stream` once (it reads the molecule's radius back to
 * choose L).  If the workspace is smaller than the query returns, fewer q
 * values are averaged (AUTO) or the call fails (ORIENT_ALL).  When both
 * parts are non-empty the direct part runs on a second stream owned by the
 * context, beside the averaged part; it is forked from `stream` and joined
 * back into it before the call returns, so work queued on `stream` after the
 * call sees the whole profile.  Two hybrid calls on one context must not
 * be made from different threads at the same time: they share that stream.
 */
#define SAS_HYBRID_AUTO 0
#define SAS_HYBRID_ORIENT_ALL 1
#define SAS_HYBRID_DIRECT_ALL 2
int32_t sas_orient_degree(double q, double r_max, double tol);
size_t sas_debye_workspace_size_hybrid(const sas_ctx* ctx, int64_t n, int32_t t, int32_t nq, int32_t mode);
sas_status sas_debye_profile_hybrid(sas_ctx* ctx, const float* coords, const int32_t* types, int64_t n,
                                    const float* table, int32_t t, const double* q, int32_t nq, double tol,
                                    int32_t mode, double* I_out, void* workspace, size_t ws_bytes, void* stream,
                                    int32_t* n_orient);

/*
 * Tuning controls (optional).  sas_set_variant forces the forward tile shape
 * for subsequent calls on ctx: bj = atoms per J block (64, 128, 256 or 512;
 * 0 = automatic) and qc = q values per chunk (one of 16, 32, 50, 64, 100,
 * 128, 150, 200: chunks of qc values, the last one shorter; 0 = automatic:
 * balanced chunks of at most 200; a non-uniform grid always uses chunks of
 * at most 32).  Returns SAS_ERR_INVALID_ARG for other values.
 * sas_get_variant reports the shape the last forward call (or plan) used;
 * passing it back to sas_set_variant reproduces that call's chunks, and so
 * its results bit for bit.
 */
sas_status sas_set_variant(sas_ctx* ctx, int32_t bj, int32_t qc);
sas_status sas_get_variant(const sas_ctx* ctx, int32_t* bj, int32_t* qc);

/*
 * Evaluation form of the profile calls on ctx, a combination of flags.
 * SAS_FORM_AUTO (0, the default) steps uniform grids by the recurrence,
 * evaluates other grids directly and picks the type-sorted or the per-atom
 * form from T and the atom counts.  SAS_FORM_DIRECT evaluates every grid
 * directly, one sine per pair and q as in the paper's per-q kernel
 * (Implementation section), which measures what the recurrence saves.
 * SAS_FORM_PER_ATOM weights every pair term by f_j inside the q loop even
 * for few types.  The pair kernel of the recurrence's type form has two
 * launches with bitwise the same results: a grid of one work-group per strip
 * of pair tiles, and a persistent grid (as many one-wave work-groups as the
 * GPU holds at once, each pulling the next strip from a counter in the
 * workspace).  By default calls on one structure use the persistent launch,
 * eager batched calls the grid, and a batched plan times both and keeps the
 * faster; SAS_FORM_PERSISTENT or SAS_FORM_GRID forces one (the other forms
 * ignore both).  sas_get_form reports the form the last profile or gradient
 * call (or plan) used: SAS_FORM_RECURRENCE or SAS_FORM_DIRECT, plus
 * SAS_FORM_PER_ATOM and SAS_FORM_PERSISTENT when they applied.
 * Errors: SAS_ERR_INVALID_ARG (NULL, unknown flags, both launch flags).
 * Both gradients (sas_debye_grad, sas_debye_grad_table) follow the same
 * flags: the direct variants on non-uniform grids or with SAS_FORM_DIRECT,
 * the per-atom variants with many table rows or SAS_FORM_PER_ATOM.
 */
#define SAS_FORM_AUTO 0
#define SAS_FORM_DIRECT 1
#define SAS_FORM_RECURRENCE 2
#define SAS_FORM_PER_ATOM 4
#define SAS_FORM_PERSISTENT 8
#define SAS_FORM_GRID 16
sas_status sas_set_form(sas_ctx* ctx, int form);
sas_status sas_get_form(const sas_ctx* ctx, int* form);

/*
 * Kernel timing (optional, for benchmarks).  While enabled, every forward and
 * adjoint pair-kernel launch on ctx is bracketed by two HIP events recorded on
 * the launch stream.  sas_read_timing waits for those events, writes the
 * summed device time of the forward (pair) kernels in ms and their launch
 * count (and the same for the adjoint kernels; either pointer may be NULL),
 * then clears the record.  Disabled by default; enabling costs two event
 * records per launch.
 */
sas_status sas_enable_timing(sas_ctx* ctx, int on);
sas_status sas_read_timing(sas_ctx* ctx, double* forward_ms, int64_t* forward_launches, double* adjoint_ms,
                           int64_t* adjoint_launches);

#ifdef __cplusplus
}
#endif

#endif /* SAS_DEBYE_H */
