/*
 * FP64 CPU oracle for the Debye summation -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load this file's library.  The HIP library shares no code with it.
 *
 * What is computed (Background section, Eq. 2, the Debye sum obtained by
 * integrating the orientational average of Eq. 1 analytically):
 *
 *     I(q) = sum_k sum_j f_k(q) f_j(q) sin(q r_jk) / (q r_jk)
 *
 * written out plainly:
 *   - every distance r_jk = |r_j - r_k| in FP64 from the given coordinates;
 *   - sin from the C library (libm), no recurrence, no type factoring, no
 *     tiling;
 *   - the j = k terms and any q r = 0 term use the limit sin(x)/x -> 1, so
 *     the diagonal gives f_k(q)^2 and I(0) = (sum_k f_k(0))^2;
 *   - because r_jk = r_kj the off-diagonal part is 2 * sum over j < k (the
 *     paper also evaluates only j <= k, Implementation section);
 *   - form factors come from a per-type table, f_k(q_m) = table[type_k][m];
 *     giving every atom its own type reproduces the paper's per-atom form
 *     factors exactly (Background section, below Eq. 2).
 *
 * Sums are Neumaier-compensated (Neumaier 1974).  Rows are cut into fixed
 * blocks of ORACLE_ROWS rows; each block is summed on its own and the block
 * totals are merged in block order, so the result does not depend on the
 * number of threads.
 *
 * A second output A(q) = sum_k sum_j |f_k f_j sinc(q r_jk)| measures how much
 * the sum cancels: kappa(q) = A(q) / I(q).
 *
 * Gradient (vector-Jacobian product of the profile w.r.t. coordinates):
 *     d/dx_i [ sin(q r)/(q r) ] = ( cos(q r)/r - sin(q r)/(q r^2) ) (x_i - x_j)/r
 * so for weights w_m (for instance dchi2/dI(q_m)):
 *     g_i = sum_{j != i} 2 sum_m w_m f_i f_j ( cos(q_m r)/r - sin(q_m r)/(q_m r^2) ) (x_i - x_j)/r
 * where a term with q_m = 0 or r = 0 is zero (the derivative of sin(x)/x is
 * zero at x = 0).  The loop is over all j != i, without symmetry.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_ROWS 64

typedef struct {
  double s, c;
} neu_t;

static inline void neu_add(neu_t* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}

static inline double neu_val(const neu_t* a) { return a->s + a->c; }

static inline double sinc(double x) { return x == 0.0 ? 1.0 : sin(x) / x; }

static int check_args(const double* coords, const int32_t* types, int64_t n, const double* table, int32_t t,
                      const double* q, int32_t nq) {
  if (n < 0 || t <= 0 || nq <= 0) return 1;
  if (n > 0 && (!coords || !types)) return 1;
  if (!table || !q) return 1;
  for (int64_t i = 0; i < n; ++i)
    if (types[i] < 0 || types[i] >= t) return 1;
  return 0;
}

/* I_out[m] and (optionally) A_out[m] for m in [0, nq).  Returns 0 on success. */
int oracle_debye_profile(const double* coords, const int32_t* types, int64_t n, const double* table, int32_t t,
                         const double* q, int32_t nq, double* I_out, double* A_out, int nthreads) {
  if (check_args(coords, types, n, table, t, q, nq) || !I_out) return 1;
  int64_t nblk = (n + ORACLE_ROWS - 1) / ORACLE_ROWS;
  neu_t* blkI = (neu_t*)calloc((size_t)(nblk > 0 ? nblk : 1) * (size_t)nq, sizeof(neu_t));
  neu_t* blkA = (neu_t*)calloc((size_t)(nblk > 0 ? nblk : 1) * (size_t)nq, sizeof(neu_t));
  if (!blkI || !blkA) {
    free(blkI);
    free(blkA);
    return 2;
  }
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  /* Off-diagonal pairs j < k, doubled; the block owns rows k in [k0, k1). */
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < nblk; ++b) {
    neu_t* sI = blkI + b * nq;
    neu_t* sA = blkA + b * nq;
    int64_t k0 = b * ORACLE_ROWS, k1 = k0 + ORACLE_ROWS < n ? k0 + ORACLE_ROWS : n;
    for (int64_t k = k0; k < k1; ++k) {
      const double xk = coords[3 * k], yk = coords[3 * k + 1], zk = coords[3 * k + 2];
      const double* fk = table + (int64_t)types[k] * nq;
      for (int64_t j = 0; j < k; ++j) {
        double dx = xk - coords[3 * j], dy = yk - coords[3 * j + 1], dz = zk - coords[3 * j + 2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        const double* fj = table + (int64_t)types[j] * nq;
        for (int32_t m = 0; m < nq; ++m) {
          double term = 2.0 * fk[m] * fj[m] * sinc(q[m] * r);
          neu_add(&sI[m], term);
          neu_add(&sA[m], fabs(term));
        }
      }
    }
  }
  for (int32_t m = 0; m < nq; ++m) {
    /* Diagonal j = k: sinc(0) = 1. */
    neu_t tot = {0.0, 0.0}, tabs = {0.0, 0.0};
    for (int64_t k = 0; k < n; ++k) {
      double f = table[(int64_t)types[k] * nq + m];
      neu_add(&tot, f * f);
      neu_add(&tabs, f * f);
    }
    for (int64_t b = 0; b < nblk; ++b) {
      neu_add(&tot, neu_val(&blkI[b * nq + m]));
      neu_add(&tabs, neu_val(&blkA[b * nq + m]));
    }
    I_out[m] = neu_val(&tot);
    if (A_out) A_out[m] = neu_val(&tabs);
  }
  free(blkI);
  free(blkA);
  return 0;
}

/* grad_out[a][0..2] = sum_m w[m] dI(q_m)/dx_{atoms[a]} for the listed atoms
 * (all atoms, in order, when atoms == NULL and n_atoms == n). */
int oracle_debye_grad(const double* coords, const int32_t* types, int64_t n, const double* table, int32_t t,
                      const double* q, int32_t nq, const double* w, const int64_t* atoms, int64_t n_atoms,
                      double* grad_out, int nthreads) {
  if (check_args(coords, types, n, table, t, q, nq) || !w || !grad_out || n_atoms < 0) return 1;
  if (!atoms && n_atoms != n) return 1;
  for (int64_t a = 0; atoms && a < n_atoms; ++a)
    if (atoms[a] < 0 || atoms[a] >= n) return 1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t a = 0; a < n_atoms; ++a) {
    int64_t i = atoms ? atoms[a] : a;
    const double xi = coords[3 * i], yi = coords[3 * i + 1], zi = coords[3 * i + 2];
    const double* fi = table + (int64_t)types[i] * nq;
    neu_t gx = {0, 0}, gy = {0, 0}, gz = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double dx = xi - coords[3 * j], dy = yi - coords[3 * j + 1], dz = zi - coords[3 * j + 2];
      double r = sqrt(dx * dx + dy * dy + dz * dz);
      if (r == 0.0) continue;
      const double* fj = table + (int64_t)types[j] * nq;
      neu_t dsum = {0, 0};
      for (int32_t m = 0; m < nq; ++m) {
        if (q[m] == 0.0) continue;
        double x = q[m] * r;
        double dsinc_dr = cos(x) / r - sin(x) / (q[m] * r * r);
        neu_add(&dsum, 2.0 * w[m] * fi[m] * fj[m] * dsinc_dr);
      }
      double g = neu_val(&dsum) / r;
      neu_add(&gx, g * dx);
      neu_add(&gy, g * dy);
      neu_add(&gz, g * dz);
    }
    grad_out[3 * a] = neu_val(&gx);
    grad_out[3 * a + 1] = neu_val(&gy);
    grad_out[3 * a + 2] = neu_val(&gz);
  }
  return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
