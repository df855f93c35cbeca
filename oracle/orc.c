/*
 * FP64 CPU oracle for cut-HDMR expansions whose component functions are
 * hierarchical (adaptive) sparse grids -- Eftekhari & Scheidegger,
 * "High-Dimensional Dynamic Stochastic Model Representation", arXiv 2202.06555.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the GPU library and does not include or call it.
 *
 * Conventions (readings of the paper, each stated where it is used):
 *   - 1-D basis: eq (3.1) with h_l = 2^-l, x_{l,i} = i h_l; index sets of
 *     eq (3.3): l >= 1, i odd, 0 < i < 2^l, zero boundary (Sec. 3.1).
 *   - tensor basis: eq (3.2); interpolant: eq (3.6) summed over the rows that
 *     a component stores.
 *   - the expansion evaluated is F(x) = c0 + sum_S w_S u_S(x_S) (eq (3.16)
 *     grouped per component; eq (4.2) when w_S = b_S).
 *   - a NaN coordinate anywhere in a point makes every output of that point NaN;
 *     points outside [0,1] see the zero extension that eq (3.1) gives.
 *   - all sums are Neumaier-compensated so oracle rounding stays far below the
 *     tolerances the GPU results are held to.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_KMAX 8

/* ------------------------------------------------------------------------ */
/* compensated summation                                                     */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } ksum;

static inline void ks_add(ksum *a, double t) {
  double s = a->s + t;
  if (fabs(a->s) >= fabs(t)) a->c += (a->s - s) + t;
  else a->c += (t - s) + a->s;
  a->s = s;
}
static inline double ks_val(const ksum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------------ */
/* eq (3.1): phi_{l,i}(x) = max(1 - |x - x_{l,i}| / h_l, 0)                  */
/* ------------------------------------------------------------------------ */
double orc_hat(int32_t l, int64_t i, double x) {
  double h = ldexp(1.0, -l);
  double xli = (double)i * h;
  double v = 1.0 - fabs(x - xli) / h;
  return v > 0.0 ? v : 0.0;
}

/* Derivative convention (the paper defines none): the right derivative of
 * eq (3.1) everywhere in [0,1), the left derivative at x = 1, zero outside
 * [0,1] where the zero extension is constant. */
double orc_dhat(int32_t l, int64_t i, double x) {
  double h = ldexp(1.0, -l);
  double xli = (double)i * h;
  if (!(x >= 0.0 && x <= 1.0)) return 0.0;
  if (x == 1.0) {
    if (x > xli && x <= xli + h) return -1.0 / h;
    if (x > xli - h && x <= xli) return 1.0 / h;
    return 0.0;
  }
  if (x >= xli - h && x < xli) return 1.0 / h;
  if (x >= xli && x < xli + h) return -1.0 / h;
  return 0.0;
}

/* The only odd index at level l whose support [x_{l,i}-h_l, x_{l,i}+h_l]
 * can hold x with a nonzero value or a nonzero one-sided derivative
 * (disjoint supports inside W_l, eq (3.3)).  Returns 0 for x outside [0,1]. */
static int64_t active_index(int32_t l, double x) {
  if (!(x >= 0.0 && x <= 1.0)) return 0;
  int64_t top = ((int64_t)1 << l) - 1;
  if (x == 1.0) return top;
  int64_t c = (int64_t)floor(ldexp(x, l - 1));
  int64_t i = 2 * c + 1;
  return i > top ? top : i;
}

/* ------------------------------------------------------------------------ */
/* model                                                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t d, m, ncomp, pad_;
  const double *c0;          /* m                                            */
  const int32_t *comp_off;   /* ncomp+1, offsets into comp_dims              */
  const int32_t *comp_dims;  /* sum_S |S|                                    */
  const int64_t *comp_npts;  /* ncomp                                        */
  const uint8_t *levels;     /* concatenated per component, N_S*|S|          */
  const uint32_t *indices;   /* concatenated per component, N_S*|S|          */
  const double *alpha;       /* concatenated per component, N_S*m            */
  const double *weights;     /* ncomp                                        */
} orc_model;

typedef struct {
  int32_t k;
  const int32_t *dims;
  int64_t n;
  const uint8_t *lv;
  const uint32_t *ix;
  const double *al;
  double w;
} comp_view;

static void comp_views(const orc_model *M, comp_view *cv) {
  int64_t lo = 0, ao = 0;
  for (int s = 0; s < M->ncomp; ++s) {
    cv[s].k = M->comp_off[s + 1] - M->comp_off[s];
    cv[s].dims = M->comp_dims + M->comp_off[s];
    cv[s].n = M->comp_npts[s];
    cv[s].lv = M->levels + lo;
    cv[s].ix = M->indices + lo;
    cv[s].al = M->alpha + ao;
    cv[s].w = M->weights[s];
    lo += cv[s].n * cv[s].k;
    ao += cv[s].n * M->m;
  }
}

static int point_has_nan(const double *x, int d) {
  for (int q = 0; q < d; ++q)
    if (isnan(x[q])) return 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* O1: brute force -- eq (3.6) summed over every stored row, eq (3.16)       */
/* grouped per component.  Yabs (optional) receives sum |terms|.             */
/* ------------------------------------------------------------------------ */
int orc_eval_brute(const orc_model *M, const double *X, int64_t n, double *Y, double *Yabs) {
  int d = M->d, m = M->m;
  comp_view *cv = (comp_view *)malloc(sizeof(comp_view) * (M->ncomp + 1));
  if (!cv) return -2;
  comp_views(M, cv);
#pragma omp parallel
  {
    ksum *u = (ksum *)malloc(sizeof(ksum) * m);
    ksum *tot = (ksum *)malloc(sizeof(ksum) * m);
    double *ab = (double *)malloc(sizeof(double) * m);
#pragma omp for schedule(dynamic, 1)
    for (int64_t p = 0; p < n; ++p) {
      const double *x = X + p * d;
      if (point_has_nan(x, d)) {
        for (int o = 0; o < m; ++o) { Y[p * m + o] = NAN; if (Yabs) Yabs[p * m + o] = NAN; }
        continue;
      }
      for (int o = 0; o < m; ++o) { tot[o].s = M->c0[o]; tot[o].c = 0; ab[o] = fabs(M->c0[o]); }
      for (int s = 0; s < M->ncomp; ++s) {
        const comp_view *c = &cv[s];
        for (int o = 0; o < m; ++o) { u[o].s = 0; u[o].c = 0; }
        for (int64_t j = 0; j < c->n; ++j) {
          double w = 1.0;
          for (int q = 0; q < c->k; ++q)
            w *= orc_hat(c->lv[j * c->k + q], c->ix[j * c->k + q], x[c->dims[q]]);
          if (w == 0.0) continue; /* a zero basis value adds nothing */
          for (int o = 0; o < m; ++o) {
            double t = w * c->al[j * m + o];
            ks_add(&u[o], t);
            ab[o] += fabs(c->w * t);
          }
        }
        for (int o = 0; o < m; ++o) ks_add(&tot[o], c->w * ks_val(&u[o]));
      }
      for (int o = 0; o < m; ++o) { Y[p * m + o] = ks_val(&tot[o]); if (Yabs) Yabs[p * m + o] = ab[o]; }
    }
    free(u); free(tot); free(ab);
  }
  free(cv);
  return 0;
}

/* Brute-force gradient: right partial derivatives (left at x_q = 1) of the
 * same sum.  G is n*d*m (point, input dimension, output). */
int orc_grad_brute(const orc_model *M, const double *X, int64_t n, double *Y, double *G) {
  int d = M->d, m = M->m;
  comp_view *cv = (comp_view *)malloc(sizeof(comp_view) * (M->ncomp + 1));
  if (!cv) return -2;
  comp_views(M, cv);
#pragma omp parallel
  {
    ksum *u = (ksum *)malloc(sizeof(ksum) * m * (ORC_KMAX + 1));
    ksum *tot = (ksum *)malloc(sizeof(ksum) * m);
    ksum *gt = (ksum *)malloc(sizeof(ksum) * (size_t)m * d);
#pragma omp for schedule(dynamic, 1)
    for (int64_t p = 0; p < n; ++p) {
      const double *x = X + p * d;
      if (point_has_nan(x, d)) {
        for (int o = 0; o < m; ++o) Y[p * m + o] = NAN;
        for (int64_t t = 0; t < (int64_t)d * m; ++t) G[p * d * m + t] = NAN;
        continue;
      }
      for (int o = 0; o < m; ++o) { tot[o].s = M->c0[o]; tot[o].c = 0; }
      memset(gt, 0, sizeof(ksum) * (size_t)m * d);
      for (int s = 0; s < M->ncomp; ++s) {
        const comp_view *c = &cv[s];
        int k = c->k;
        memset(u, 0, sizeof(ksum) * m * (k + 1));
        for (int64_t j = 0; j < c->n; ++j) {
          double ph[ORC_KMAX], dp[ORC_KMAX];
          for (int q = 0; q < k; ++q) {
            ph[q] = orc_hat(c->lv[j * k + q], c->ix[j * k + q], x[c->dims[q]]);
            dp[q] = orc_dhat(c->lv[j * k + q], c->ix[j * k + q], x[c->dims[q]]);
          }
          double w = 1.0;
          for (int q = 0; q < k; ++q) w *= ph[q];
          for (int o = 0; o < m; ++o) ks_add(&u[o], w * c->al[j * m + o]);
          for (int q = 0; q < k; ++q) {
            double g = dp[q];
            for (int r = 0; r < k; ++r)
              if (r != q) g *= ph[r];
            if (g == 0.0) continue;
            for (int o = 0; o < m; ++o) ks_add(&u[(q + 1) * m + o], g * c->al[j * m + o]);
          }
        }
        for (int o = 0; o < m; ++o) ks_add(&tot[o], c->w * ks_val(&u[o]));
        for (int q = 0; q < k; ++q)
          for (int o = 0; o < m; ++o)
            ks_add(&gt[(size_t)c->dims[q] * m + o], c->w * ks_val(&u[(q + 1) * m + o]));
      }
      for (int o = 0; o < m; ++o) Y[p * m + o] = ks_val(&tot[o]);
      for (int64_t t = 0; t < (int64_t)d * m; ++t) G[p * d * m + t] = ks_val(&gt[t]);
    }
    free(u); free(tot); free(gt);
  }
  free(cv);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* O2: level-wise evaluation.  Per level multi-index stored by a component  */
/* at most one row can be nonzero at x (disjoint supports, eq (3.3)): find  */
/* that row by binary search among the rows of the same level multi-index.  */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t k;
  int64_t ntup;
  int64_t *tup_start;  /* ntup+1 */
  int32_t *tup_lsum;   /* ntup   */
  int64_t *order;      /* n : row ids sorted by (levels, indices)       */
  const uint8_t *lv;
  const uint32_t *ix;
} comp_index;

static const uint8_t *g_sort_lv;
static const uint32_t *g_sort_ix;
static int g_sort_k;

static int cmp_rows(const void *pa, const void *pb) {
  int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
  int k = g_sort_k;
  for (int q = 0; q < k; ++q) {
    int la = g_sort_lv[a * k + q], lb = g_sort_lv[b * k + q];
    if (la != lb) return la < lb ? -1 : 1;
  }
  for (int q = 0; q < k; ++q) {
    uint32_t ia = g_sort_ix[a * k + q], ib = g_sort_ix[b * k + q];
    if (ia != ib) return ia < ib ? -1 : 1;
  }
  return (a > b) - (a < b);
}

static int build_index(int k, int64_t n, const uint8_t *lv, const uint32_t *ix, comp_index *ci) {
  ci->k = k; ci->lv = lv; ci->ix = ix;
  ci->order = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
  ci->tup_start = (int64_t *)malloc(sizeof(int64_t) * (n + 2));
  ci->tup_lsum = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
  if (!ci->order || !ci->tup_start || !ci->tup_lsum) return -2;
  for (int64_t j = 0; j < n; ++j) ci->order[j] = j;
#pragma omp critical(orc_sort)
  {
    g_sort_lv = lv; g_sort_ix = ix; g_sort_k = k;
    qsort(ci->order, n, sizeof(int64_t), cmp_rows);
  }
  ci->ntup = 0;
  for (int64_t t = 0; t < n; ++t) {
    int64_t j = ci->order[t];
    int newt = (t == 0);
    if (!newt) {
      int64_t jp = ci->order[t - 1];
      for (int q = 0; q < k; ++q)
        if (lv[j * k + q] != lv[jp * k + q]) newt = 1;
    }
    if (newt) {
      int s = 0;
      for (int q = 0; q < k; ++q) s += lv[j * k + q];
      ci->tup_lsum[ci->ntup] = s;
      ci->tup_start[ci->ntup++] = t;
    }
  }
  ci->tup_start[ci->ntup] = n;
  return 0;
}

static void free_index(comp_index *ci) {
  free(ci->order); free(ci->tup_start); free(ci->tup_lsum);
}

/* row with level multi-index of tuple t and index multi-index want[], or -1 */
static int64_t find_row(const comp_index *ci, int64_t t, const uint32_t *want) {
  int k = ci->k;
  int64_t lo = ci->tup_start[t], hi = ci->tup_start[t + 1] - 1;
  while (lo <= hi) {
    int64_t mid = lo + (hi - lo) / 2;
    int64_t j = ci->order[mid];
    int c = 0;
    for (int q = 0; q < k && c == 0; ++q) {
      uint32_t v = ci->ix[j * k + q];
      c = (v < want[q]) ? -1 : (v > want[q]) ? 1 : 0;
    }
    if (c == 0) return j;
    if (c < 0) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

/* Accumulate sum_j alpha_j phi_j(xs) (and, if du != NULL, its right partial
 * derivatives) over the tuples of a component whose level sum is < lsum_cap.
 * xs holds the component's own k coordinates. */
static void comp_sum(const comp_index *ci, const double *al, int m, const double *xs,
                     int32_t lsum_cap, ksum *u, ksum *du, double *abs_acc, double wabs) {
  int k = ci->k;
  for (int64_t t = 0; t < ci->ntup; ++t) {
    if (ci->tup_lsum[t] >= lsum_cap) continue;
    int64_t j0 = ci->order[ci->tup_start[t]];
    uint32_t want[ORC_KMAX];
    int ok = 1;
    for (int q = 0; q < k; ++q) {
      int64_t i = active_index(ci->lv[j0 * k + q], xs[q]);
      if (i == 0) { ok = 0; break; }
      want[q] = (uint32_t)i;
    }
    if (!ok) continue;
    int64_t j = find_row(ci, t, want);
    if (j < 0) continue;
    double ph[ORC_KMAX], w = 1.0;
    for (int q = 0; q < k; ++q) { ph[q] = orc_hat(ci->lv[j * k + q], want[q], xs[q]); w *= ph[q]; }
    if (w != 0.0)
      for (int o = 0; o < m; ++o) {
        double tt = w * al[j * m + o];
        ks_add(&u[o], tt);
        if (abs_acc) abs_acc[o] += wabs * fabs(tt);
      }
    if (du) {
      for (int q = 0; q < k; ++q) {
        double g = orc_dhat(ci->lv[j * k + q], want[q], xs[q]);
        for (int r = 0; r < k; ++r)
          if (r != q) g *= ph[r];
        if (g == 0.0) continue;
        for (int o = 0; o < m; ++o) ks_add(&du[q * m + o], g * al[j * m + o]);
      }
    }
  }
}

static int build_all_indices(const orc_model *M, const comp_view *cv, comp_index *ci) {
  int rc = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int s = 0; s < M->ncomp; ++s)
    if (build_index(cv[s].k, cv[s].n, cv[s].lv, cv[s].ix, &ci[s]) != 0) rc = -2;
  return rc;
}

/* Level-wise evaluation (O2).  With G != NULL also the gradient (n*d*m). */
int orc_eval_levelwise(const orc_model *M, const double *X, int64_t n, double *Y, double *Yabs,
                       double *G) {
  int d = M->d, m = M->m;
  comp_view *cv = (comp_view *)malloc(sizeof(comp_view) * (M->ncomp + 1));
  comp_index *ci = (comp_index *)calloc(M->ncomp + 1, sizeof(comp_index));
  if (!cv || !ci) return -2;
  comp_views(M, cv);
  int rc = build_all_indices(M, cv, ci);
  if (rc == 0) {
#pragma omp parallel
    {
      ksum *u = (ksum *)malloc(sizeof(ksum) * m);
      ksum *du = (ksum *)malloc(sizeof(ksum) * m * ORC_KMAX);
      ksum *tot = (ksum *)malloc(sizeof(ksum) * m);
      ksum *gt = G ? (ksum *)malloc(sizeof(ksum) * (size_t)m * d) : NULL;
      double *ab = (double *)malloc(sizeof(double) * m);
#pragma omp for schedule(dynamic, 16)
      for (int64_t p = 0; p < n; ++p) {
        const double *x = X + p * d;
        if (point_has_nan(x, d)) {
          for (int o = 0; o < m; ++o) { Y[p * m + o] = NAN; if (Yabs) Yabs[p * m + o] = NAN; }
          if (G) for (int64_t t = 0; t < (int64_t)d * m; ++t) G[p * d * m + t] = NAN;
          continue;
        }
        for (int o = 0; o < m; ++o) { tot[o].s = M->c0[o]; tot[o].c = 0; ab[o] = fabs(M->c0[o]); }
        if (gt) memset(gt, 0, sizeof(ksum) * (size_t)m * d);
        for (int s = 0; s < M->ncomp; ++s) {
          const comp_view *c = &cv[s];
          double xs[ORC_KMAX];
          for (int q = 0; q < c->k; ++q) xs[q] = x[c->dims[q]];
          memset(u, 0, sizeof(ksum) * m);
          if (gt) memset(du, 0, sizeof(ksum) * m * c->k);
          comp_sum(&ci[s], c->al, m, xs, 1 << 30, u, gt ? du : NULL, ab, fabs(c->w));
          for (int o = 0; o < m; ++o) ks_add(&tot[o], c->w * ks_val(&u[o]));
          if (gt)
            for (int q = 0; q < c->k; ++q)
              for (int o = 0; o < m; ++o)
                ks_add(&gt[(size_t)c->dims[q] * m + o], c->w * ks_val(&du[q * m + o]));
        }
        for (int o = 0; o < m; ++o) { Y[p * m + o] = ks_val(&tot[o]); if (Yabs) Yabs[p * m + o] = ab[o]; }
        if (G) for (int64_t t = 0; t < (int64_t)d * m; ++t) G[p * d * m + t] = ks_val(&gt[t]);
      }
      free(u); free(du); free(tot); free(gt); free(ab);
    }
  }
  for (int s = 0; s < M->ncomp; ++s) free_index(&ci[s]);
  free(ci); free(cv);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* grids                                                                    */
/* ------------------------------------------------------------------------ */

/* eq (3.5) (rule 1: |l|_1 <= ell + k - 1) or the full grid of eq (3.4)
 * (rule 0: every l_q <= ell).  Order: |l|_1, then l lexicographically, then
 * i lexicographically.  Writes at most cap rows (NULL outputs: count only);
 * returns the number of points. */
int64_t orc_regular_grid(int32_t k, int32_t ell, int32_t rule, uint8_t *lv, uint32_t *ix, int64_t cap) {
  if (k < 1 || k > ORC_KMAX || ell < 1) return -1;
  int32_t smax = (rule == 1) ? ell + k - 1 : ell * k;
  int64_t cnt = 0;
  for (int32_t s = k; s <= smax; ++s) {
    int32_t l[ORC_KMAX];
    for (int q = 0; q < k; ++q) l[q] = 1;
    /* enumerate all l with entries >= 1 (and <= ell for rule 0) in lexicographic order */
    for (;;) {
      int32_t sum = 0, okl = 1;
      for (int q = 0; q < k; ++q) { sum += l[q]; if (rule == 0 && l[q] > ell) okl = 0; }
      if (sum == s && okl) {
        uint32_t i[ORC_KMAX];
        for (int q = 0; q < k; ++q) i[q] = 1;
        for (;;) {
          if (lv && cnt < cap)
            for (int q = 0; q < k; ++q) { lv[cnt * k + q] = (uint8_t)l[q]; ix[cnt * k + q] = i[q]; }
          ++cnt;
          int q = k - 1;
          while (q >= 0) {
            i[q] += 2;
            if (i[q] < ((uint32_t)1 << l[q])) break;
            i[q] = 1;
            --q;
          }
          if (q < 0) break;
        }
      }
      int q = k - 1;
      while (q >= 0) {
        l[q] += 1;
        if (l[q] <= s) break;
        l[q] = 1;
        --q;
      }
      if (q < 0) break;
    }
  }
  return cnt;
}

/* Hierarchisation by the defining equations: the interpolant must equal the
 * nodal values Y at every grid node (eq (3.6) at x = x_{l,i}).  Finer hats
 * vanish at coarser nodes and hats of one level have disjoint supports, so
 * alpha_j = y_j - sum over rows of strictly smaller |l|_1 of alpha_j' phi_j'(x_j),
 * processed in increasing |l|_1. */
int orc_hierarchize(int32_t k, int64_t n, const uint8_t *lv, const uint32_t *ix, const double *Yv,
                    int32_t m, double *alpha) {
  if (k < 1 || k > ORC_KMAX) return -1;
  comp_index ci;
  if (build_index(k, n, lv, ix, &ci) != 0) return -2;
  int32_t smax = 0;
  for (int64_t t = 0; t < ci.ntup; ++t) if (ci.tup_lsum[t] > smax) smax = ci.tup_lsum[t];
  ksum *u = (ksum *)malloc(sizeof(ksum) * m);
  for (int32_t s = k; s <= smax; ++s) {
    for (int64_t j = 0; j < n; ++j) {
      int ls = 0;
      for (int q = 0; q < k; ++q) ls += lv[j * k + q];
      if (ls != s) continue;
      double xs[ORC_KMAX];
      for (int q = 0; q < k; ++q) xs[q] = ldexp((double)ix[j * k + q], -(int)lv[j * k + q]);
      for (int o = 0; o < m; ++o) { u[o].s = 0; u[o].c = 0; }
      comp_sum(&ci, alpha, m, xs, s, u, NULL, NULL, 0.0);
      for (int o = 0; o < m; ++o) alpha[j * m + o] = Yv[j * m + o] - ks_val(&u[o]);
    }
  }
  free(u);
  free_index(&ci);
  return 0;
}

/* Cross-check route for grids that hold every hierarchical ancestor: the
 * classical dimension-by-dimension stencil alpha = v(x) - (v(x-h) + v(x+h))/2
 * with zero boundary values, applied per dimension from the finest level
 * down.  Returns -3 if an ancestor is missing. */
int orc_hierarchize_stencil(int32_t k, int64_t n, const uint8_t *lv, const uint32_t *ix,
                            const double *Yv, int32_t m, double *alpha) {
  if (k < 1 || k > ORC_KMAX) return -1;
  comp_index ci;
  if (build_index(k, n, lv, ix, &ci) != 0) return -2;
  memcpy(alpha, Yv, sizeof(double) * n * m);
  int rc = 0;
  int lmax = 0;
  for (int64_t j = 0; j < n * k; ++j) if (lv[j] > lmax) lmax = lv[j];
  for (int q = 0; q < k && rc == 0; ++q) {
    for (int l = lmax; l >= 2 && rc == 0; --l) {
      for (int64_t j = 0; j < n && rc == 0; ++j) {
        if (lv[j * k + q] != l) continue;
        for (int side = -1; side <= 1; side += 2) {
          int64_t pos = (int64_t)ix[j * k + q] + side;
          int pl = l;
          while (pos > 0 && (pos % 2) == 0) { pos /= 2; pl -= 1; }
          if (pos == 0 || pos == ((int64_t)1 << pl)) continue; /* boundary value 0 */
          /* neighbour: same multi-index except dimension q -> (pl, pos) */
          uint8_t nl[ORC_KMAX]; uint32_t ni[ORC_KMAX];
          for (int r = 0; r < k; ++r) { nl[r] = lv[j * k + r]; ni[r] = ix[j * k + r]; }
          nl[q] = (uint8_t)pl; ni[q] = (uint32_t)pos;
          int64_t found = -1;
          for (int64_t t = 0; t < ci.ntup && found < 0; ++t) {
            int64_t j0 = ci.order[ci.tup_start[t]];
            int same = 1;
            for (int r = 0; r < k; ++r) if (lv[j0 * k + r] != nl[r]) same = 0;
            if (same) found = find_row(&ci, t, ni);
          }
          if (found < 0) { rc = -3; break; }
          for (int o = 0; o < m; ++o) alpha[j * m + o] -= 0.5 * alpha[found * m + o];
        }
      }
    }
  }
  free_index(&ci);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* adaptive build of one cut-HDMR component (Sec. 3.1 refinement, eq (3.8); */
/* cut functions and components from eq (2.2.6); Alg. 2 refines the cut   */
/* function f(xbar \ x_S)).                                                 */
/* ------------------------------------------------------------------------ */
typedef int (*orc_fn)(const double *X, int64_t n, int32_t d, double *Y, int32_t m, void *user);

typedef struct {
  int32_t k, d, m, max_level;
  int32_t level_rule;   /* 0: every l_q <= max_level; 1: |l|_1 <= max_level + k - 1 */
  int32_t refine_rule;  /* 0: all parents accepted;   1: any parent accepted      */
  double eps_gamma;     /* < 0: accept every point (regular grid of the level rule) */
  const int32_t *dims;  /* k */
  const double *anchor; /* d */
} orc_build_args;

typedef struct {
  int64_t n, cap;
  uint8_t *lv;
  uint32_t *ix;
  double *ag, *au;   /* surpluses of the cut function g_S and of the component u_S */
  uint8_t *acc;
} orc_grid;

/* --- open-addressing map from (l, i) multi-indices to rows ---------------- */
typedef struct { int64_t cap; int64_t *slot; } rmap;

static uint64_t key_hash(int k, const uint8_t *l, const uint32_t *i) {
  uint64_t h = 1469598103934665603ULL;
  for (int q = 0; q < k; ++q) {
    h ^= (uint64_t)l[q] * 0x9E3779B97F4A7C15ULL + i[q];
    h *= 1099511628211ULL;
    h ^= h >> 29;
  }
  return h;
}

static int rmap_init(rmap *mp, int64_t cap) {
  mp->cap = 64;
  while (mp->cap < 2 * cap) mp->cap *= 2;
  mp->slot = (int64_t *)malloc(sizeof(int64_t) * mp->cap);
  if (!mp->slot) return -2;
  for (int64_t t = 0; t < mp->cap; ++t) mp->slot[t] = -1;
  return 0;
}

static int64_t rmap_find(const rmap *mp, int k, const uint8_t *lvs, const uint32_t *ixs,
                         const uint8_t *l, const uint32_t *i) {
  uint64_t h = key_hash(k, l, i) & (mp->cap - 1);
  for (;;) {
    int64_t r = mp->slot[h];
    if (r < 0) return -1;
    if (memcmp(lvs + r * k, l, k) == 0 && memcmp(ixs + r * k, i, sizeof(uint32_t) * k) == 0) return r;
    h = (h + 1) & (mp->cap - 1);
  }
}

static int rmap_insert(rmap *mp, int k, const uint8_t *lvs, const uint32_t *ixs, int64_t row, int64_t count) {
  if (2 * (count + 1) > mp->cap) {
    rmap nm;
    if (rmap_init(&nm, count + 1) != 0) return -2;
    for (int64_t r = 0; r < count; ++r) {
      uint64_t h = key_hash(k, lvs + r * k, ixs + r * k) & (nm.cap - 1);
      while (nm.slot[h] >= 0) h = (h + 1) & (nm.cap - 1);
      nm.slot[h] = r;
    }
    free(mp->slot);
    *mp = nm;
  }
  uint64_t h = key_hash(k, lvs + row * k, ixs + row * k) & (mp->cap - 1);
  while (mp->slot[h] >= 0) h = (h + 1) & (mp->cap - 1);
  mp->slot[h] = row;
  return 0;
}

static int grow(void **p, size_t elem, int64_t need, int64_t *cap) {
  if (need <= *cap) return 0;
  int64_t nc = *cap ? *cap : 256;
  while (nc < need) nc *= 2;
  void *q = realloc(*p, elem * nc);
  if (!q) return -2;
  *p = q;
  *cap = nc;
  return 0;
}

/* odd hierarchical parent index in 1-D: the odd one of (i-1)/2, (i+1)/2 */
static uint32_t parent_index(uint32_t i) {
  uint32_t a = (i - 1) / 2, b = (i + 1) / 2;
  return (a & 1u) ? a : b;
}

typedef struct { uint8_t l[ORC_KMAX]; uint32_t i[ORC_KMAX]; } cand_t;
static int g_cand_k;
static int cmp_cand(const void *pa, const void *pb) {
  const cand_t *a = (const cand_t *)pa, *b = (const cand_t *)pb;
  for (int q = 0; q < g_cand_k; ++q) if (a->l[q] != b->l[q]) return a->l[q] < b->l[q] ? -1 : 1;
  for (int q = 0; q < g_cand_k; ++q) if (a->i[q] != b->i[q]) return a->i[q] < b->i[q] ? -1 : 1;
  return 0;
}

int orc_build_component(const orc_build_args *A, orc_fn f, void *user, orc_grid *out) {
  int k = A->k, d = A->d, m = A->m;
  if (k < 1 || k > ORC_KMAX || A->max_level < 1 || A->max_level > 30) return -1;
  memset(out, 0, sizeof(*out));
  int64_t cap_lv = 0, cap_ix = 0, cap_ag = 0, cap_au = 0, cap_acc = 0;
  rmap mp;
  if (rmap_init(&mp, 256) != 0) return -2;
  int64_t ncur = 1, cap_cur = 1;
  cand_t *cur = (cand_t *)calloc(1, sizeof(cand_t));
  for (int q = 0; q < k; ++q) { cur[0].l[q] = 1; cur[0].i[q] = 1; }
  int nsub = 1 << k;
  int rc = 0;
  int32_t lsum_cap = (A->level_rule == 1) ? A->max_level + k - 1 : A->max_level * k;
  ksum *acc = (ksum *)malloc(sizeof(ksum) * 2 * m);
  int32_t s = k;
  while (ncur > 0 && rc == 0) {
    int64_t base = out->n;
    int64_t nn = base + ncur;
    if (grow((void **)&out->lv, 1, nn * k, &cap_lv) || grow((void **)&out->ix, 4, nn * k, &cap_ix) ||
        grow((void **)&out->ag, 8, nn * m, &cap_ag) || grow((void **)&out->au, 8, nn * m, &cap_au) ||
        grow((void **)&out->acc, 1, nn, &cap_acc)) { rc = -2; break; }
    for (int64_t c = 0; c < ncur; ++c)
      for (int q = 0; q < k; ++q) {
        out->lv[(base + c) * k + q] = cur[c].l[q];
        out->ix[(base + c) * k + q] = cur[c].i[q];
      }
    /* nodal values: f at xbar \ x_v for every v subset of S (eq (2.2.6)) */
    double *Xe = (double *)malloc(sizeof(double) * ncur * nsub * d);
    double *Ye = (double *)malloc(sizeof(double) * ncur * nsub * m);
    if (!Xe || !Ye) { free(Xe); free(Ye); rc = -2; break; }
    for (int64_t c = 0; c < ncur; ++c)
      for (int v = 0; v < nsub; ++v) {
        double *row = Xe + (c * nsub + v) * d;
        memcpy(row, A->anchor, sizeof(double) * d);
        for (int q = 0; q < k; ++q)
          if (v & (1 << q)) row[A->dims[q]] = ldexp((double)cur[c].i[q], -(int)cur[c].l[q]);
      }
    if (f(Xe, ncur * nsub, d, Ye, m, user) != 0) { free(Xe); free(Ye); rc = -4; break; }
    /* g_S = f(xbar \ x_S); u_S = sum_v (-1)^{|S|-|v|} f(xbar \ x_v), summed as
     * nested differences over the dimensions of S so that a node on an anchor
     * line gives an exact zero (the identity the signed sum satisfies). */
    double *ub = (double *)malloc(sizeof(double) * nsub * m);
    for (int64_t c = 0; c < ncur; ++c) {
      memcpy(ub, Ye + c * nsub * m, sizeof(double) * nsub * m);
      for (int q = 0; q < k; ++q)
        for (int v = 0; v < nsub; ++v)
          if (v & (1 << q))
            for (int o = 0; o < m; ++o) ub[v * m + o] -= ub[(v ^ (1 << q)) * m + o];
      for (int o = 0; o < m; ++o) {
        out->ag[(base + c) * m + o] = Ye[(c * nsub + nsub - 1) * m + o];
        out->au[(base + c) * m + o] = ub[(nsub - 1) * m + o];
      }
    }
    free(ub); free(Xe); free(Ye);
    /* hierarchise the new rows against the rows of smaller level sum */
    if (base > 0) {
      comp_index ci;
      if (build_index(k, base, out->lv, out->ix, &ci) != 0) { rc = -2; break; }
      for (int64_t c = 0; c < ncur; ++c) {
        double xs[ORC_KMAX];
        for (int q = 0; q < k; ++q) xs[q] = ldexp((double)cur[c].i[q], -(int)cur[c].l[q]);
        for (int o = 0; o < 2 * m; ++o) { acc[o].s = 0; acc[o].c = 0; }
        comp_sum(&ci, out->ag, m, xs, s, acc, NULL, NULL, 0.0);
        comp_sum(&ci, out->au, m, xs, s, acc + m, NULL, NULL, 0.0);
        for (int o = 0; o < m; ++o) {
          out->ag[(base + c) * m + o] -= ks_val(&acc[o]);
          out->au[(base + c) * m + o] -= ks_val(&acc[m + o]);
        }
      }
      free_index(&ci);
    }
    /* refinement criterion eq (3.8): gamma = max_o |alpha_o| > eps_gamma */
    for (int64_t c = 0; c < ncur; ++c) {
      double g = 0.0;
      for (int o = 0; o < m; ++o) {
        double a = fabs(out->ag[(base + c) * m + o]);
        if (a > g || isnan(a)) g = a;
      }
      out->acc[base + c] = (A->eps_gamma < 0.0) ? 1 : (g > A->eps_gamma ? 1 : 0);
    }
    for (int64_t c = 0; c < ncur; ++c)
      if (rmap_insert(&mp, k, out->lv, out->ix, base + c, base + c) != 0) rc = -2;
    out->n = nn;
    /* children of accepted rows; a child whose support lies inside a rejected
     * point's support is excluded (Sec. 3.1): all parents must be accepted
     * (refine_rule 0) or at least one (refine_rule 1). */
    int64_t nnext = 0, cap_next = 0;
    cand_t *next = NULL;
    rmap cm;
    rmap_init(&cm, 256);
    uint8_t *clv = NULL; uint32_t *cix = NULL; int64_t cap_clv = 0, cap_cix = 0;
    for (int64_t c = 0; c < ncur && rc == 0; ++c) {
      int64_t r = base + c;
      if (!out->acc[r]) continue;
      int32_t ls = 0;
      for (int q = 0; q < k; ++q) ls += out->lv[r * k + q];
      if (ls + 1 > lsum_cap) continue;
      for (int q = 0; q < k; ++q) {
        if (A->level_rule == 0 && out->lv[r * k + q] + 1 > A->max_level) continue;
        for (int side = -1; side <= 1; side += 2) {
          cand_t ch;
          memset(&ch, 0, sizeof ch);
          for (int t = 0; t < k; ++t) { ch.l[t] = out->lv[r * k + t]; ch.i[t] = out->ix[r * k + t]; }
          ch.l[q] += 1;
          ch.i[q] = 2 * ch.i[q] + side;
          if (rmap_find(&cm, k, clv, cix, ch.l, ch.i) >= 0) continue;
          int nacc = 0, npar = 0;
          for (int t = 0; t < k; ++t) {
            if (ch.l[t] <= 1) continue;
            uint8_t pl[ORC_KMAX]; uint32_t pi[ORC_KMAX];
            memcpy(pl, ch.l, k); memcpy(pi, ch.i, sizeof(uint32_t) * k);
            pl[t] -= 1;
            pi[t] = parent_index(ch.i[t]);
            ++npar;
            int64_t pr = rmap_find(&mp, k, out->lv, out->ix, pl, pi);
            if (pr >= 0 && out->acc[pr]) ++nacc;
          }
          int admit = (A->refine_rule == 0) ? (nacc == npar) : (nacc > 0);
          if (!admit) continue;
          if (grow((void **)&next, sizeof(cand_t), nnext + 1, &cap_next) ||
              grow((void **)&clv, 1, (nnext + 1) * k, &cap_clv) ||
              grow((void **)&cix, 4, (nnext + 1) * k, &cap_cix)) { rc = -2; break; }
          next[nnext] = ch;
          memcpy(clv + nnext * k, ch.l, k);
          memcpy(cix + nnext * k, ch.i, sizeof(uint32_t) * k);
          rmap_insert(&cm, k, clv, cix, nnext, nnext);
          ++nnext;
        }
      }
    }
    free(cm.slot); free(clv); free(cix);
    if (nnext > 1) {
#pragma omp critical(orc_sort)
      {
        g_cand_k = k;
        qsort(next, nnext, sizeof(cand_t), cmp_cand);
      }
    }
    free(cur);
    cur = next;
    ncur = nnext;
    cap_cur = cap_next;
    ++s;
  }
  (void)cap_cur;
  free(cur);
  free(acc);
  free(mp.slot);
  return rc;
}

void orc_grid_free(orc_grid *g) {
  if (!g) return;
  free(g->lv); free(g->ix); free(g->ag); free(g->au); free(g->acc);
  memset(g, 0, sizeof(*g));
}

/* Build every component of a model (components are independent, Alg. 2
 * loops over them in parallel).  dims_off/dims list the index sets; grids
 * receives one orc_grid per component. */
int orc_build_components(int32_t ncomp, const int32_t *dims_off, const int32_t *dims,
                         const orc_build_args *common, orc_fn f, void *user, orc_grid *grids) {
  int rc = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int s = 0; s < ncomp; ++s) {
    orc_build_args a = *common;
    a.k = dims_off[s + 1] - dims_off[s];
    a.dims = dims + dims_off[s];
    int r = orc_build_component(&a, f, user, &grids[s]);
    if (r != 0) {
#pragma omp critical(orc_rc)
      rc = r;
    }
  }
  return rc;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Thread count of the parallel loops that follow (harness control for the
 * single-thread timing; no effect on results). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
