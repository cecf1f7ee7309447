/*
 * ORACLE -- plain, slow CPU reference for the 1-D Gauss transform.
 *
 * This file is test infrastructure.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it.  It shares no code, header,
 * table or helper with the GPU library, and the GPU library never calls it.
 *
 * Five computations, all in IEEE double precision (no fast-math):
 *
 *   O1  oracle_direct         the definition (1.1)-(1.2):
 *                             u_i = sum_j alpha_j exp(-(x_i - y_j)^2 / (4 delta)),
 *                             Neumaier-compensated, optionally restricted to
 *                             the sources where the Gaussian exceeds exp(-cutoff).
 *   O2  oracle_soe_recurrence the SOE algorithm of Section 4: sort, then for
 *                             every mode a forward sweep (4.5) and a backward
 *                             sweep (4.6) over the sorted targets, with source
 *                             contributions added as in the distinct-point
 *                             forward pass of Section 4 (Figure 6), and
 *                             u_i = sum_k Re(omega_k (h+_{k,i} + h-_{k,i})), (4.1).
 *   O3  oracle_soe_brute      the SOE sum written out, (1.3) inserted in (1.1):
 *                             u_i = sum_j alpha_j Re sum_k omega_k exp(-tau_k |x_i-y_j| / sqrt(delta)).
 *   O4  oracle_direct_field   the Gaussian's x- and delta-derivatives summed
 *                             directly (gradients of L = sum_i g_i u_i).
 *   O5  oracle_soe_deriv_brute the SOE's x-derivative summed pair by pair.
 *
 * The SOE table is an input: tau0_k (nodes at delta = 1) and omega_k, one
 * representative per conjugate pair with its weight already doubled
 * (Section 1, after (1.3)); S_n(x) = Re sum_k omega_k exp(-tau0_k |x|/sqrt(delta)).
 *
 * `plant` selects a deliberately wrong variant (0 = correct).  The tests use
 * it to show that the oracle's pins catch plausible mistakes; nothing else
 * passes a non-zero value.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  double v;
  int64_t i;
} vi_t;

static int cmp_vi(const void* a, const void* b) {
  const vi_t* p = (const vi_t*)a;
  const vi_t* q = (const vi_t*)b;
  if (p->v < q->v) return -1;
  if (p->v > q->v) return 1;
  return (p->i > q->i) - (p->i < q->i);
}

/* Values sorted ascending, ties kept in original index order. */
static vi_t* sorted_copy(const double* v, int64_t n) {
  vi_t* s = (vi_t*)malloc(sizeof(vi_t) * (size_t)(n > 0 ? n : 1));
  if (!s) return NULL;
  for (int64_t k = 0; k < n; ++k) {
    s[k].v = v[k];
    s[k].i = k;
  }
  qsort(s, (size_t)n, sizeof(vi_t), cmp_vi);
  return s;
}

static void set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Neumaier's improvement of Kahan summation. */
typedef struct {
  double s, c;
} nsum_t;

static inline void nsum_add(nsum_t* a, double t) {
  double s = a->s + t;
  if (fabs(a->s) >= fabs(t))
    a->c += (a->s - s) + t;
  else
    a->c += (t - s) + a->s;
  a->s = s;
}

/* ------------------------------------------------------------------------
 * O1: direct summation of (1.1) with the kernel (1.2).
 *
 * Targets are the K entries x[0..K-1].  Sources are sorted once; for each
 * target only sources with (x - y)^2 / (4 delta) <= cutoff are summed
 * (cutoff <= 0 sums all sources).  With cutoff = 69.1 every dropped term is
 * below 1e-30 |alpha_j|.
 * plant 1: kernel exp(-d^2/delta) (the 4 of (1.2) dropped).
 * plant 2: kernel exp(-d^2/(2 delta)).
 * ---------------------------------------------------------------------- */
int oracle_direct(const double* x, int64_t K, const double* y, const double* alpha, int64_t N,
                  double delta, double cutoff, double* u, int nthreads, int plant) {
  if (K < 0 || N < 0 || !(delta > 0)) return 1;
  if (K == 0) return 0;
  if (N == 0) {
    for (int64_t i = 0; i < K; ++i) u[i] = 0.0;
    return 0;
  }
  vi_t* ys = sorted_copy(y, N);
  double* beta = (double*)malloc(sizeof(double) * (size_t)N);
  if (!ys || !beta) {
    free(ys);
    free(beta);
    return 2;
  }
  for (int64_t j = 0; j < N; ++j) beta[j] = alpha[ys[j].i];
  double denom = 4.0 * delta;
  if (plant == 1) denom = delta;
  if (plant == 2) denom = 2.0 * delta;
  const double half_width = cutoff > 0 ? sqrt(denom * cutoff) : INFINITY;

  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < K; ++i) {
    const double xi = x[i];
    int64_t lo = 0, hi = N;
    if (isfinite(half_width)) {
      /* first source with y >= xi - half_width */
      int64_t a = 0, b = N;
      const double left = xi - half_width;
      while (a < b) {
        int64_t m = a + (b - a) / 2;
        if (ys[m].v < left) a = m + 1; else b = m;
      }
      lo = a;
      /* first source with y > xi + half_width */
      a = lo;
      b = N;
      const double right = xi + half_width;
      while (a < b) {
        int64_t m = a + (b - a) / 2;
        if (ys[m].v <= right) a = m + 1; else b = m;
      }
      hi = a;
    }
    nsum_t acc = {0.0, 0.0};
    for (int64_t j = lo; j < hi; ++j) {
      const double d = xi - ys[j].v;
      nsum_add(&acc, beta[j] * exp(-(d * d) / denom));
    }
    u[i] = acc.s + acc.c;
  }
  free(ys);
  free(beta);
  return 0;
}

/* ------------------------------------------------------------------------
 * O2: the SOE recurrences of Section 4.
 *
 * For mode k, tau = tau0_k / sqrt(delta).  With targets xs and sources ys
 * sorted ascending (beta = alpha aligned with ys):
 *
 *   forward  (4.4)-(4.5): h+_i = sum_{y_j <= xs_i} beta_j exp(-tau (xs_i - y_j)).
 *     Sweep targets left to right.  Sources below xs_i are added with their
 *     own exponential, sources equal to xs_i with weight 1 (Figure 6), then
 *     the value is carried to the next target with exp(-tau (xs_{i+1}-xs_i)).
 *     The sweep continues over the remaining targets once sources run out.
 *   backward (4.4),(4.6): h-_i = sum_{y_j > xs_i} beta_j exp(-tau (y_j - xs_i)),
 *     the mirror image: targets right to left, strictly larger sources only.
 *
 * Each (mode, direction) pair is independent (the parallel axis named in
 * Section 6) and writes Re(omega_k h) into its own row; rows are added in
 * a fixed order, then unsorted.
 *
 * plant 1: backward sweep also takes ties (y_j >= xs_i): double counting.
 * plant 2: conjugate partner not represented: omega_k / 2 used.
 * plant 3: forward carry without the decay factor.
 * plant 4: tau0 / delta instead of tau0 / sqrt(delta).
 * plant 5: forward sweep stops when the sources run out (the loop guard of
 *          the printed fragment taken literally).
 * plant 6: backward source term uses exp(-tau (xs_i - y_j)) (sign flipped).
 *
 * With deriv = 1 the same sweeps give the x-derivative of the SOE transform,
 * u'_i = sum_j alpha_j S'(x_i - y_j): a source left of x_i (h+) contributes
 * d/dx exp(-tau (x - y)) = -tau exp(...), one to the right (h-) +tau exp(...),
 * so the rows hold Re(-tau omega h+) and Re(+tau omega h-).  A source at x_i
 * itself counts with h+ (sign +1), as the sweeps order it.
 * plant 7 (deriv only): the h- rows keep the sign of the h+ rows.
 * ---------------------------------------------------------------------- */
/* Wall time of the last O2 call's sort (benchmark use only; no effect on results). */
static double g_last_sort_seconds = 0.0;
double oracle_last_sort_seconds(void) { return g_last_sort_seconds; }

int oracle_soe_recurrence_field(const double* x, int64_t M, const double* y, const double* alpha,
                                int64_t N, double delta, int n_modes, const double* tau_re,
                                const double* tau_im, const double* om_re, const double* om_im,
                                int deriv, double* u, int nthreads, int plant) {
  if (M < 0 || N < 0 || n_modes < 0 || !(delta > 0)) return 1;
  if (M == 0) return 0;
  const double t_sort0 = omp_get_wtime();
  vi_t* xs = sorted_copy(x, M);
  vi_t* ys = sorted_copy(y, N);
  g_last_sort_seconds = omp_get_wtime() - t_sort0;
  double* beta = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  const int64_t rows = 2 * (int64_t)n_modes;
  double* part = (double*)calloc((size_t)(rows > 0 ? rows : 1) * (size_t)M, sizeof(double));
  if (!xs || !ys || !beta || !part) {
    free(xs);
    free(ys);
    free(beta);
    free(part);
    return 2;
  }
  for (int64_t j = 0; j < N; ++j) beta[j] = alpha[ys[j].i];
  const double sd = (plant == 4) ? delta : sqrt(delta);

  set_threads(nthreads);
#pragma omp parallel for schedule(static, 1)
  for (int64_t r = 0; r < rows; ++r) {
    const int k = (int)(r / 2);
    const int backward = (int)(r % 2);
    const double complex tau = (tau_re[k] + I * tau_im[k]) / sd;
    double complex om = om_re[k] + I * om_im[k];
    if (plant == 2) om *= 0.5;
    if (deriv) om = (backward && plant != 7) ? tau * om : -tau * om;
    double* out = part + r * M;
    double complex h = 0.0;
    if (!backward) {
      int64_t i = 0, j = 0;
      while (i < M) {
        if (plant == 5 && j >= N) break;
        if (j < N && ys[j].v < xs[i].v) {
          h += beta[j] * cexp(-tau * (xs[i].v - ys[j].v));
          ++j;
        } else if (j < N && ys[j].v == xs[i].v) {
          h += beta[j];
          ++j;
        } else {
          out[i] = creal(om * h);
          if (i + 1 < M) {
            if (plant == 3)
              h = h;
            else
              h = cexp(-tau * (xs[i + 1].v - xs[i].v)) * h;
          }
          ++i;
        }
      }
    } else {
      int64_t i = M - 1, j = N - 1;
      while (i >= 0) {
        const int take = (plant == 1) ? (j >= 0 && ys[j].v >= xs[i].v) : (j >= 0 && ys[j].v > xs[i].v);
        if (take) {
          const double complex arg = (plant == 6) ? -tau * (xs[i].v - ys[j].v) : -tau * (ys[j].v - xs[i].v);
          h += beta[j] * cexp(arg);
          --j;
        } else {
          out[i] = creal(om * h);
          if (i > 0) h = cexp(-tau * (xs[i].v - xs[i - 1].v)) * h;
          --i;
        }
      }
    }
  }
  for (int64_t i = 0; i < M; ++i) {
    double s = 0.0;
    for (int64_t r = 0; r < rows; ++r) s += part[r * M + i];
    u[xs[i].i] = s;
  }
  free(xs);
  free(ys);
  free(beta);
  free(part);
  return 0;
}

int oracle_soe_recurrence(const double* x, int64_t M, const double* y, const double* alpha,
                          int64_t N, double delta, int n_modes, const double* tau_re,
                          const double* tau_im, const double* om_re, const double* om_im,
                          double* u, int nthreads, int plant) {
  return oracle_soe_recurrence_field(x, M, y, alpha, N, delta, n_modes, tau_re, tau_im, om_re,
                                     om_im, 0, u, nthreads, plant);
}

/* ------------------------------------------------------------------------
 * O3: the SOE transform summed pair by pair, O(M N n_modes).
 * ---------------------------------------------------------------------- */
int oracle_soe_brute(const double* x, int64_t M, const double* y, const double* alpha, int64_t N,
                     double delta, int n_modes, const double* tau_re, const double* tau_im,
                     const double* om_re, const double* om_im, double* u, int nthreads) {
  if (M < 0 || N < 0 || n_modes < 0 || !(delta > 0)) return 1;
  const double sd = sqrt(delta);
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < M; ++i) {
    nsum_t acc = {0.0, 0.0};
    for (int64_t j = 0; j < N; ++j) {
      const double d = fabs(x[i] - y[j]) / sd;
      double s = 0.0;
      for (int k = 0; k < n_modes; ++k) {
        const double complex tau = tau_re[k] + I * tau_im[k];
        const double complex om = om_re[k] + I * om_im[k];
        s += creal(om * cexp(-tau * d));
      }
      nsum_add(&acc, alpha[j] * s);
    }
    u[i] = acc.s + acc.c;
  }
  return 0;
}

/* ------------------------------------------------------------------------
 * Gradient oracle, direct definition.  With L = sum_i g_i u_i and u of (1.1):
 *   dL/dx_i = g_i sum_j alpha_j G'(x_i - y_j),  G'(r) = -(r / (2 delta)) G(r),
 *   dL/dy_j = alpha_j sum_i g_i G'(y_j - x_i),
 *   dL/dalpha_j = sum_i g_i G(x_i - y_j)          (oracle_direct with roles swapped),
 *   dL/ddelta = sum_i g_i sum_j alpha_j (r^2 / (4 delta^2)) G(r).
 * oracle_direct_field evaluates, at each entry of x,
 *   which = 1:  sum_j w_j G'(x - y_j),
 *   which = 2:  sum_j w_j (r^2 / (4 delta^2)) G(r),   r = x - y_j,
 * windowed like oracle_direct.
 * plant 1: G'(r) with the sign flipped.
 * plant 2: G'(r) = -(r / delta) G(r) (the 2 dropped).
 * plant 3: the delta-derivative factor r^2 / (4 delta) (one 1/delta dropped).
 * ---------------------------------------------------------------------- */
int oracle_direct_field(const double* x, int64_t K, const double* y, const double* w, int64_t N,
                        double delta, double cutoff, int which, double* out, int nthreads,
                        int plant) {
  if (K < 0 || N < 0 || !(delta > 0) || (which != 1 && which != 2)) return 1;
  if (K == 0) return 0;
  if (N == 0) {
    for (int64_t i = 0; i < K; ++i) out[i] = 0.0;
    return 0;
  }
  vi_t* ys = sorted_copy(y, N);
  double* ws = (double*)malloc(sizeof(double) * (size_t)N);
  if (!ys || !ws) {
    free(ys);
    free(ws);
    return 2;
  }
  for (int64_t j = 0; j < N; ++j) ws[j] = w[ys[j].i];
  const double denom = 4.0 * delta;
  const double half_width = cutoff > 0 ? sqrt(denom * cutoff) : INFINITY;
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < K; ++i) {
    const double xi = x[i];
    int64_t lo = 0, hi = N;
    if (isfinite(half_width)) {
      int64_t a = 0, b = N;
      while (a < b) {
        int64_t m = a + (b - a) / 2;
        if (ys[m].v < xi - half_width) a = m + 1; else b = m;
      }
      lo = a;
      a = lo;
      b = N;
      while (a < b) {
        int64_t m = a + (b - a) / 2;
        if (ys[m].v <= xi + half_width) a = m + 1; else b = m;
      }
      hi = a;
    }
    nsum_t acc = {0.0, 0.0};
    for (int64_t j = lo; j < hi; ++j) {
      const double r = xi - ys[j].v;
      const double gk = exp(-(r * r) / denom);
      double f;
      if (which == 1) {
        f = -(r / (2.0 * delta)) * gk;
        if (plant == 1) f = -f;
        if (plant == 2) f = -(r / delta) * gk;
      } else {
        f = (r * r) / (denom * delta) * gk;
        if (plant == 3) f = (r * r) / denom * gk;
      }
      nsum_add(&acc, ws[j] * f);
    }
    out[i] = acc.s + acc.c;
  }
  free(ys);
  free(ws);
  return 0;
}

/* ------------------------------------------------------------------------
 * Derivative of the SOE transform, pair by pair:
 *   out_i = sum_j w_j S'(x_i - y_j),
 *   S'(r) = Re sum_k omega_k (-tau_k) sign(r) exp(-tau_k |r|),  tau_k = tau0_k / sqrt(delta),
 * with sign(0) = 0 (the Gaussian's derivative vanishes at 0).
 * plant 1: sign(0) = +1 (a coincident source counted as one to the left).
 * plant 2: the sign factor dropped (derivative of exp(-tau r) without |r|).
 * ---------------------------------------------------------------------- */
int oracle_soe_deriv_brute(const double* x, int64_t M, const double* y, const double* w, int64_t N,
                           double delta, int n_modes, const double* tau_re, const double* tau_im,
                           const double* om_re, const double* om_im, double* out, int nthreads,
                           int plant) {
  if (M < 0 || N < 0 || n_modes < 0 || !(delta > 0)) return 1;
  const double sd = sqrt(delta);
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < M; ++i) {
    nsum_t acc = {0.0, 0.0};
    for (int64_t j = 0; j < N; ++j) {
      const double r = x[i] - y[j];
      if (r == 0.0 && plant != 1) continue;
      double sg = r >= 0 ? 1.0 : -1.0;
      if (plant == 2) sg = 1.0;
      double s = 0.0;
      for (int k = 0; k < n_modes; ++k) {
        const double complex tau = (tau_re[k] + I * tau_im[k]) / sd;
        const double complex om = om_re[k] + I * om_im[k];
        s += creal(-om * tau * cexp(-tau * fabs(r)));
      }
      nsum_add(&acc, w[j] * sg * s);
    }
    out[i] = acc.s + acc.c;
  }
  return 0;
}
