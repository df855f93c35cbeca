/*
 * Seeded synthetic test function for the HDMR / sparse-grid workloads.
 *
 * This file is part of the input generators: it defines the vector-valued
 * function f : [0,1]^d -> R^m that the builds approximate.  It contains none
 * of the approximation method's arithmetic (no hat basis, no grids, no
 * surpluses, no HDMR composition) and is shared as an *input* by the CPU
 * oracle and by the GPU library's build callback.
 *
 *   f_o(x) = c_o
 *          + sum_k   a_ok B(x_k) [sin(2 pi x_k + theta_ok) - sin(2 pi r_k + theta_ok)]
 *          + sum_p   b_op B(x_p1) B(x_p2) [e1(x_p1) - e1(r_p1)] [e2(x_p2) - e2(r_p2)]
 *          + kappa_o B(x_A) B(x_B) [K(x_A,x_B) - K(r_A,x_B) - K(x_A,r_B) + K(r_A,r_B)]
 *
 * with B(t) = 4 t (1 - t), e1(s) = exp(-(s - mu_op)^2 / 0.5),
 * e2(t) = exp(-(t - nu_op)^2 / 0.5), K(s,t) = max(0, s + t - 1), r the
 * reference point, p running over a chosen pair set and (A, B) the kink
 * pair.  Every term vanishes on the boundary of [0,1]^d and on the lines
 * through r, so f(r) = c and the order-two cut-HDMR decomposition of f
 * anchored at r is known in closed form (the individual terms).  f is smooth
 * except for the kink along x_A + x_B = 1.
 *
 * Rows that differ from the stored reference point in at most two
 * coordinates (the cut-HDMR evaluation pattern) take an incremental path:
 * f(ref) plus the change of every term that touches a changed coordinate.
 * Every row is evaluated independently of the others, so identical rows
 * always give bit-identical outputs regardless of the batch they sit in.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t d, m, npairs, kink_a, kink_b;
  const double *ref;      /* d   : reference point of the incremental path */
  const double *c;        /* m                                              */
  const double *a;        /* m*d (row o holds a_o.)                         */
  const double *theta;    /* m*d                                            */
  const int32_t *pairs;   /* npairs*2                                       */
  const double *b;        /* m*npairs                                       */
  const double *mu;       /* m*npairs                                       */
  const double *nu;       /* m*npairs                                       */
  const double *kappa;    /* m                                              */
  /* filled by tf_prepare */
  double *f_ref;          /* m                                              */
  int32_t *dp_off;        /* d+1 : CSR of pair ids per dimension            */
  int32_t *dp_idx;        /* 2*npairs                                       */
} tf_params;

static const double TF_PI = 3.14159265358979323846;

static inline double bump(double t) { return 4.0 * t * (1.0 - t); }

static inline double term1(const tf_params *P, int o, int k, double x) {
  double th = P->theta[(int64_t)o * P->d + k];
  return P->a[(int64_t)o * P->d + k] * bump(x) *
         (sin(2.0 * TF_PI * x + th) - sin(2.0 * TF_PI * P->ref[k] + th));
}

static inline double gauss(double s, double c) { double e = s - c; return exp(-(e * e) / 0.5); }

static inline double term2(const tf_params *P, int o, int p, double x1, double x2) {
  int64_t q = (int64_t)o * P->npairs + p;
  double r1 = P->ref[P->pairs[2 * p]], r2 = P->ref[P->pairs[2 * p + 1]];
  return P->b[q] * bump(x1) * bump(x2) * (gauss(x1, P->mu[q]) - gauss(r1, P->mu[q])) *
         (gauss(x2, P->nu[q]) - gauss(r2, P->nu[q]));
}

static inline double relu(double s) { return s > 0.0 ? s : 0.0; }

static inline double termk(const tf_params *P, int o, double xa, double xb) {
  double ra = P->ref[P->kink_a], rb = P->ref[P->kink_b];
  double mix = relu(xa + xb - 1.0) - relu(ra + xb - 1.0) - relu(xa + rb - 1.0) + relu(ra + rb - 1.0);
  return P->kappa[o] * bump(xa) * bump(xb) * mix;
}

static void eval_direct(const tf_params *P, const double *x, double *y) {
  for (int o = 0; o < P->m; ++o) {
    double s = P->c[o];
    for (int k = 0; k < P->d; ++k) s += term1(P, o, k, x[k]);
    for (int p = 0; p < P->npairs; ++p)
      s += term2(P, o, p, x[P->pairs[2 * p]], x[P->pairs[2 * p + 1]]);
    s += termk(P, o, x[P->kink_a], x[P->kink_b]);
    y[o] = s;
  }
}

/* Prepare the incremental path: f(ref) and the per-dimension pair lists. */
int tf_prepare(tf_params *P) {
  if (!P || P->d <= 0 || P->m <= 0 || P->npairs < 0) return -1;
  P->f_ref = (double *)malloc(sizeof(double) * P->m);
  P->dp_off = (int32_t *)calloc(P->d + 1, sizeof(int32_t));
  P->dp_idx = (int32_t *)malloc(sizeof(int32_t) * (2 * P->npairs + 1));
  if (!P->f_ref || !P->dp_off || !P->dp_idx) return -2;
  for (int p = 0; p < P->npairs; ++p) {
    P->dp_off[P->pairs[2 * p] + 1]++;
    P->dp_off[P->pairs[2 * p + 1] + 1]++;
  }
  for (int k = 0; k < P->d; ++k) P->dp_off[k + 1] += P->dp_off[k];
  int32_t *fill = (int32_t *)calloc(P->d, sizeof(int32_t));
  if (!fill) return -2;
  for (int p = 0; p < P->npairs; ++p) {
    int k1 = P->pairs[2 * p], k2 = P->pairs[2 * p + 1];
    P->dp_idx[P->dp_off[k1] + fill[k1]++] = p;
    P->dp_idx[P->dp_off[k2] + fill[k2]++] = p;
  }
  free(fill);
  eval_direct(P, P->ref, P->f_ref);
  return 0;
}

void tf_release(tf_params *P) {
  if (!P) return;
  free(P->f_ref); free(P->dp_off); free(P->dp_idx);
  P->f_ref = NULL; P->dp_off = NULL; P->dp_idx = NULL;
}

/* Incremental path for a row whose changed coordinates are ch[0..nc). */
static void eval_delta(const tf_params *P, const double *x, const int *ch, int nc, double *y) {
  const double *r = P->ref;
  for (int o = 0; o < P->m; ++o) {
    double s = P->f_ref[o];
    for (int t = 0; t < nc; ++t) {
      int k = ch[t];
      s += term1(P, o, k, x[k]) - term1(P, o, k, r[k]);
    }
    for (int t = 0; t < nc; ++t) {
      int k = ch[t];
      for (int q = P->dp_off[k]; q < P->dp_off[k + 1]; ++q) {
        int p = P->dp_idx[q];
        int k1 = P->pairs[2 * p], k2 = P->pairs[2 * p + 1];
        /* a pair touching two changed coordinates is counted once */
        int other = (k1 == k) ? k2 : k1;
        int dup = 0;
        for (int u = 0; u < t; ++u) dup |= (ch[u] == other);
        if (dup) continue;
        s += term2(P, o, p, x[k1], x[k2]) - term2(P, o, p, r[k1], r[k2]);
      }
    }
    int touch = 0;
    for (int t = 0; t < nc; ++t) touch |= (ch[t] == P->kink_a) | (ch[t] == P->kink_b);
    if (touch) s += termk(P, o, x[P->kink_a], x[P->kink_b]) - termk(P, o, r[P->kink_a], r[P->kink_b]);
    y[o] = s;
  }
}

/* Callback-compatible evaluator: X is n*d row-major, Y is n*m row-major.
 * Returns 0 on success, -1 on a shape mismatch. */
int tf_eval(const double *X, int64_t n, int32_t d, double *Y, int32_t m, void *user) {
  const tf_params *P = (const tf_params *)user;
  if (!P || d != P->d || m != P->m || !P->f_ref) return -1;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    const double *x = X + i * d;
    double *y = Y + i * m;
    int ch[3], nc = 0;
    for (int k = 0; k < d && nc < 3; ++k)
      if (!(x[k] == P->ref[k])) ch[nc++] = k;
    if (nc <= 2)
      eval_delta(P, x, ch, nc, y);
    else
      eval_direct(P, x, y);
  }
  return 0;
}

/* Direct evaluation only (no incremental path); used to check the
 * incremental path and to score approximation error at random points. */
int tf_eval_direct(const double *X, int64_t n, int32_t d, double *Y, int32_t m, void *user) {
  const tf_params *P = (const tf_params *)user;
  if (!P || d != P->d || m != P->m) return -1;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) eval_direct(P, X + i * d, Y + i * m);
  return 0;
}
