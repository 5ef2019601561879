/*
 * FP64 CPU oracle for sparse-support Wasserstein barycenters by the modified
 * Bregman ADMM (B-ADMM) and the D2-clustering assignment step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct
 * statement of what the GPU library computes.  Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code,
 * header or constant with the HIP library.
 *
 * Notation follows the paper (Ye, Wu, Wang, Li, "Fast Discrete Distribution
 * Clustering Using Wasserstein Barycenter with Sparse Support"):
 *   centroid P = {(w_i, x_i)}, i < m;   instance P^(k) = {(w^(k)_j, x^(k)_j)}
 *   C^(k)_ij = ||x_i - x^(k)_j||^2                        (Sec. 2, item 6)
 *   plan blocks Pi^(k) are m x m_k, stored column-major inside the
 *   concatenation Pi = (Pi^(1), ..., Pi^(N)) in R^{m x n}   (Sec. 2, items 8-9)
 *   so entry (i, j) of instance k lives at  m*off[k] + j*m + i.
 *
 * Every floating-point value is double; reductions run in a fixed order so
 * that results do not depend on the number of OpenMP threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_num_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/* Squared-Euclidean cost block C(x, x^(k)) (Sec. 2, item 6), column-major
 * m x mk: C[i + j*m] = sum_t (x[i,t] - y[j,t])^2, direct differences. */
void orc_cost_block(int m, int mk, int d, const double* x, const double* y,
                    double* C) {
  for (int j = 0; j < mk; ++j)
    for (int i = 0; i < m; ++i) {
      double s = 0.0;
      for (int t = 0; t < d; ++t) {
        double df = x[(int64_t)i * d + t] - y[(int64_t)j * d + t];
        s += df * df;
      }
      C[i + (int64_t)j * m] = s;
    }
}

/* Greedy pairwise merge of a member's support down to m points (Sec. 5,
 * Eq. (merge)): repeatedly merge the pair (a, b) minimising
 * w_a w_b ||x_a - x_b||^2 / (w_a + w_b) into (w_a + w_b, weighted mean).
 * Ties go to the lexicographically smallest (a, b); the merged point keeps
 * slot a and the points after b move down by one.  A pair of zero-weight
 * points has criterion 0 and merges onto x_a.
 * y: mk x d, wy: mk.  Outputs x: m x d, w: m.  Returns 0, or -1 if mk < m. */
int orc_ward_merge(int mk, int d, const double* y, const double* wy, int m,
                   double* x, double* w) {
  if (mk < m || m < 1) return -1;
  double* px = (double*)malloc(sizeof(double) * (size_t)mk * d);
  double* pw = (double*)malloc(sizeof(double) * (size_t)mk);
  memcpy(px, y, sizeof(double) * (size_t)mk * d);
  memcpy(pw, wy, sizeof(double) * (size_t)mk);
  int cnt = mk;
  while (cnt > m) {
    int ba = 0, bb = 1;
    double best = INFINITY;
    for (int a = 0; a < cnt; ++a)
      for (int b = a + 1; b < cnt; ++b) {
        double s = 0.0;
        for (int t = 0; t < d; ++t) {
          double df = px[a * d + t] - px[b * d + t];
          s += df * df;
        }
        double wsum = pw[a] + pw[b];
        double crit = wsum > 0.0 ? pw[a] * pw[b] * s / wsum : 0.0;
        if (crit < best) { best = crit; ba = a; bb = b; }
      }
    double wsum = pw[ba] + pw[bb];
    for (int t = 0; t < d; ++t) {
      double v = wsum > 0.0
                     ? (pw[ba] * px[ba * d + t] + pw[bb] * px[bb * d + t]) / wsum
                     : px[ba * d + t];
      px[ba * d + t] = v;
    }
    pw[ba] = wsum;
    for (int q = bb; q + 1 < cnt; ++q) {
      for (int t = 0; t < d; ++t) px[q * d + t] = px[(q + 1) * d + t];
      pw[q] = pw[q + 1];
    }
    --cnt;
  }
  memcpy(x, px, sizeof(double) * (size_t)m * d);
  memcpy(w, pw, sizeof(double) * (size_t)m);
  free(px);
  free(pw);
  return 0;
}

/*
 * Where the cost blocks of a run come from.  Euclidean (D == NULL): C^(k) =
 * C(x, X^(k)) of Sec. 2 item 6, x the current centroid support (updated in
 * place by the support step).  Symbolic (D != NULL, Sec. 5: support points
 * are symbols of a finite set with a given symbol-to-symbol dissimilarity):
 * C^(k)_ij = D[xsym[i] * S + ysym[off[k] + j]], the centroid's i-th symbol
 * against the instance's j-th; the support never moves.
 */
typedef struct {
  int d;
  const double* X;
  double* x;
  int S;
  const double* D;
  const int32_t* xsym;
  const int32_t* ysym;
} orc_costsrc;

static void member_cost(const orc_costsrc* cs, int64_t k, const int64_t* off,
                        int m, double* C) {
  int mk = (int)(off[k + 1] - off[k]);
  if (!cs->D) {
    orc_cost_block(m, mk, cs->d, cs->x, cs->X + off[k] * cs->d, C);
    return;
  }
  for (int j = 0; j < mk; ++j)
    for (int i = 0; i < m; ++i)
      C[i + (int64_t)j * m] =
          cs->D[(int64_t)cs->xsym[i] * cs->S + cs->ysym[off[k] + j]];
}

/*
 * B-ADMM barycenter of one cluster (Sec. 3.2, Algorithm "Centroid Update with
 * B-ADMM"; closed forms Eq. (badmmc0b), (badmmc0), (badmmc1b), (badmmc1);
 * weight rules Eq. (badmmw) = R1 and Eq. (badmmw2) = R2; dual step Eq.
 * (badmm2); support update Eq. (updatex); rho rule Eq. (rho)).
 *
 * Readings where the paper is loose:
 *  - rho = rho0 * mean over all (k, i, j) of C^(k)_ij, computed once from the
 *    initial x (the printed normaliser N n m counts N once too often);
 *  - both exponentials of an iteration use Lambda before its update; all
 *    Pi1 blocks, then w, then all Pi2 blocks and Lambda (Gauss-Seidel);
 *  - x is updated after iteration n whenever (n+1) % tau == 0, from Pi2
 *    (xplan 0) or Pi1 (xplan 1), with the plan's own row sums as the
 *    denominator (for Pi2 this is exactly N w_i); a row with total mass
 *    below 1e-300 keeps its point; the cost is then recomputed, rho is not.
 *    A symbolic run (Sec. 5) has no support step.
 *
 * Members are instance indices `mem` into the global ragged arrays
 * (off, X, W).  Plans P1, P2, L are global m x n arrays (see header); only
 * the members' blocks are touched.  On entry a member's P2 block is its
 * cached plan when warm[k] != 0 (warm may be NULL); otherwise Pi2^0 is the
 * product w_i w^(k)_j.  On exit P1, P2, L hold the last iterate, x and w the
 * new centroid, ftrace[n] = (1/N) sum_k <C^(k), Pi1^(k)> of iteration n with
 * the cost used in that iteration, rtrace[n] = (1/N) sum_k sum_ij
 * |Pi1_ij - Pi2_ij| (the residual of the splitting constraint Pi1 = Pi2
 * whose multiplier Eq. (badmm2) updates) after iteration n, and *rho_out the
 * rho used.  ftrace and rtrace may be NULL.
 */
static int badmm_cluster(int64_t nmem, const int64_t* mem, const int64_t* off,
                         const orc_costsrc* src, const double* W, int m,
                         double* w, const uint8_t* warm, double* P1,
                         double* P2, double* L, double rho0, int tau, int T,
                         double eps, int rule, int xplan, double* ftrace,
                         double* rtrace, double* rho_out) {
  if (nmem <= 0 || m < 1 || T < 0 || tau < 1) return -1;
  const int d = src->d;
  const double* X = src->X;
  double* x = src->x;
  /* local cost storage: member q's block starts at coff[q] */
  int64_t* coff = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nmem + 1));
  coff[0] = 0;
  int64_t ncols = 0;
  for (int64_t q = 0; q < nmem; ++q) {
    int64_t mk = off[mem[q] + 1] - off[mem[q]];
    coff[q + 1] = coff[q] + (int64_t)m * mk;
    ncols += mk;
  }
  double* C = (double*)malloc(sizeof(double) * (size_t)coff[nmem]);
  double* R = (double*)malloc(sizeof(double) * (size_t)nmem * m);  /* r^(k) */
  double* Wt = (double*)malloc(sizeof(double) * (size_t)nmem * m); /* w~^(k) */
  double* Fq = (double*)malloc(sizeof(double) * (size_t)nmem);
  double* Rq = (double*)malloc(sizeof(double) * (size_t)nmem);

  /* cost blocks at the initial support */
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < nmem; ++q) member_cost(src, mem[q], off, m, C + coff[q]);
  /* Eq. (rho), read as rho0 times the mean cost */
  double csum = 0.0;
  for (int64_t e = 0; e < coff[nmem]; ++e) csum += C[e];
  double rho = rho0 * csum / ((double)m * (double)ncols);
  if (rho_out) *rho_out = rho;

  /* Lambda := 0; Pi2^0 := cached plan or the product coupling (Sec. 5) */
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < nmem; ++q) {
    int64_t k = mem[q];
    int mk = (int)(off[k + 1] - off[k]);
    int64_t base = (int64_t)m * off[k];
    for (int j = 0; j < mk; ++j)
      for (int i = 0; i < m; ++i) {
        int64_t e = base + (int64_t)j * m + i;
        L[e] = 0.0;
        if (!(warm && warm[q])) P2[e] = w[i] * W[off[k] + j];
      }
  }

  for (int n = 0; n < T; ++n) {
    /* Pi1 by Eq. (badmmc0b)-(badmmc0), then Pi1~ by Eq. (badmmc1b) and the
     * normalised row sums w~^(k).  Pi1~ is kept in P2's storage: P2 is not
     * needed again until it is rebuilt from Pi1~ below. */
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < nmem; ++q) {
      int64_t k = mem[q];
      int mk = (int)(off[k + 1] - off[k]);
      int64_t base = (int64_t)m * off[k];
      const double* Cq = C + coff[q];
      double fq = 0.0;
      for (int j = 0; j < mk; ++j) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) {
          int64_t e = base + (int64_t)j * m + i;
          double a = P2[e] * exp(-(Cq[i + j * m] + L[e]) / rho) + eps;
          P1[e] = a;
          s += a;
        }
        double wj = W[off[k] + j];
        for (int i = 0; i < m; ++i) {
          int64_t e = base + (int64_t)j * m + i;
          P1[e] = P1[e] / s * wj;
          fq += Cq[i + j * m] * P1[e];
        }
      }
      Fq[q] = fq;
      double rsum = 0.0;
      for (int i = 0; i < m; ++i) {
        double r = 0.0;
        for (int j = 0; j < mk; ++j) {
          int64_t e = base + (int64_t)j * m + i;
          double b = P1[e] * exp(L[e] / rho) + eps;
          P2[e] = b; /* Pi1~ */
          r += b;
        }
        R[q * m + i] = r;
        rsum += r;
      }
      for (int i = 0; i < m; ++i) Wt[q * m + i] = R[q * m + i] / rsum;
    }

    /* barycenter weights: R1 Eq. (badmmw) or R2 Eq. (badmmw2) */
    double vsum = 0.0;
    for (int i = 0; i < m; ++i) {
      double v = 0.0;
      for (int64_t q = 0; q < nmem; ++q)
        v += (rule == 2) ? sqrt(Wt[q * m + i]) : Wt[q * m + i];
      v /= (double)nmem;
      w[i] = (rule == 2) ? v * v : v;
      vsum += w[i];
    }
    for (int i = 0; i < m; ++i) w[i] /= vsum;

    /* Pi2 by Eq. (badmmc1) and the dual step Eq. (badmm2) */
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < nmem; ++q) {
      int64_t k = mem[q];
      int mk = (int)(off[k + 1] - off[k]);
      int64_t base = (int64_t)m * off[k];
      double rq = 0.0;
      for (int j = 0; j < mk; ++j)
        for (int i = 0; i < m; ++i) {
          int64_t e = base + (int64_t)j * m + i;
          double p2 = P2[e] / R[q * m + i] * w[i];
          P2[e] = p2;
          L[e] += rho * (P1[e] - p2);
          rq += fabs(P1[e] - p2);
        }
      Rq[q] = rq;
    }

    if (ftrace) {
      double f = 0.0;
      for (int64_t q = 0; q < nmem; ++q) f += Fq[q];
      ftrace[n] = f / (double)nmem;
    }
    if (rtrace) {
      double r = 0.0;
      for (int64_t q = 0; q < nmem; ++q) r += Rq[q];
      rtrace[n] = r / (double)nmem;
    }

    /* support update, Eq. (updatex), every tau iterations */
    if (!src->D && (n + 1) % tau == 0) {
      const double* Pp = (xplan == 1) ? P1 : P2;
      for (int i = 0; i < m; ++i) {
        double den = 0.0;
        double* num = (double*)calloc((size_t)d, sizeof(double));
        for (int64_t q = 0; q < nmem; ++q) {
          int64_t k = mem[q];
          int mk = (int)(off[k + 1] - off[k]);
          int64_t base = (int64_t)m * off[k];
          for (int j = 0; j < mk; ++j) {
            double p = Pp[base + (int64_t)j * m + i];
            den += p;
            for (int t = 0; t < d; ++t) num[t] += p * X[(off[k] + j) * d + t];
          }
        }
        if (den > 1e-300)
          for (int t = 0; t < d; ++t) x[(int64_t)i * d + t] = num[t] / den;
        free(num);
      }
#pragma omp parallel for schedule(static)
      for (int64_t q = 0; q < nmem; ++q)
        member_cost(src, mem[q], off, m, C + coff[q]);
    }
  }
  free(coff);
  free(C);
  free(R);
  free(Wt);
  free(Fq);
  free(Rq);
  return 0;
}

/* Euclidean barycenter (see badmm_cluster).  Returns 0, or -1 on bad
 * arguments. */
int orc_barycenter(int64_t nmem, const int64_t* mem, const int64_t* off, int d,
                   const double* X, const double* W, int m, double* x,
                   double* w, const uint8_t* warm, double* P1, double* P2,
                   double* L, double rho0, int tau, int T, double eps, int rule,
                   int xplan, double* ftrace, double* rtrace,
                   double* rho_out) {
  if (d < 1) return -1;
  orc_costsrc src = {d, X, x, 0, NULL, NULL, NULL};
  return badmm_cluster(nmem, mem, off, &src, W, m, w, warm, P1, P2, L, rho0,
                       tau, T, eps, rule, xplan, ftrace, rtrace, rho_out);
}

/* Symbolic barycenter (Sec. 5): instance k's support points are the symbols
 * ysym[off[k] .. off[k+1]), the centroid's the m symbols xsym, the cost the
 * S x S table D (row: centroid symbol, column: instance symbol); only the
 * weights w are updated.  Returns 0, or -1 on bad arguments. */
int orc_barycenter_sym(int64_t nmem, const int64_t* mem, const int64_t* off,
                       const int32_t* ysym, const double* W, int m,
                       const int32_t* xsym, int S, const double* D, double* w,
                       const uint8_t* warm, double* P1, double* P2, double* L,
                       double rho0, int T, double eps, int rule,
                       double* ftrace, double* rtrace, double* rho_out) {
  if (S < 1 || !D) return -1;
  orc_costsrc src = {0, NULL, NULL, S, D, xsym, ysym};
  return badmm_cluster(nmem, mem, off, &src, W, m, w, warm, P1, P2, L, rho0,
                       1, T, eps, rule, 0, ftrace, rtrace, rho_out);
}

/*
 * B-ADMM for a single transport problem with both marginals fixed: the
 * updates of Eq. (badmmc0b)-(badmmc1) and Eq. (badmm2) with w held at the
 * centroid's weights (no consensus step).  Pi2^0 = w_i w'_j, Lambda = 0,
 * rho = rho0 * mean(C) for this pair.  Returns <C, Pi1> after T >= 1
 * iterations for the cost block C (column-major m x mk); Pi1, Pi2, Lambda
 * are written to p1, p2, lam when non-NULL (column-major m x mk).  This is
 * the assignment-step distance.
 */
double orc_ot_cost(int m, int mk, const double* C, const double* w,
                   const double* wy, double rho0, int T, double eps,
                   double* p1, double* p2, double* lam) {
  size_t E = (size_t)m * mk;
  double* A = (double*)malloc(sizeof(double) * E);
  double* B = (double*)malloc(sizeof(double) * E);
  double* P = (double*)malloc(sizeof(double) * E);
  double* L = (double*)malloc(sizeof(double) * E);
  double* r = (double*)malloc(sizeof(double) * (size_t)m);
  double csum = 0.0;
  for (size_t e = 0; e < E; ++e) csum += C[e];
  double rho = rho0 * csum / (double)E;
  for (int j = 0; j < mk; ++j)
    for (int i = 0; i < m; ++i) {
      P[i + j * m] = w[i] * wy[j];
      L[i + j * m] = 0.0;
    }
  for (int n = 0; n < T; ++n) {
    for (int j = 0; j < mk; ++j) {
      double s = 0.0;
      for (int i = 0; i < m; ++i) {
        int e = i + j * m;
        A[e] = P[e] * exp(-(C[e] + L[e]) / rho) + eps;
        s += A[e];
      }
      for (int i = 0; i < m; ++i) A[i + j * m] = A[i + j * m] / s * wy[j];
    }
    for (int i = 0; i < m; ++i) {
      double rr = 0.0;
      for (int j = 0; j < mk; ++j) {
        int e = i + j * m;
        B[e] = A[e] * exp(L[e] / rho) + eps;
        rr += B[e];
      }
      r[i] = rr;
    }
    for (int j = 0; j < mk; ++j)
      for (int i = 0; i < m; ++i) {
        int e = i + j * m;
        P[e] = B[e] / r[i] * w[i];
        L[e] += rho * (A[e] - P[e]);
      }
  }
  double v = 0.0;
  for (size_t e = 0; e < E; ++e) v += C[e] * A[e];
  if (p1) memcpy(p1, A, sizeof(double) * E);
  if (p2) memcpy(p2, P, sizeof(double) * E);
  if (lam) memcpy(lam, L, sizeof(double) * E);
  free(A); free(B); free(P); free(L); free(r);
  return v;
}

/* orc_ot_cost on the squared-Euclidean cost between x (m x d) and y. */
double orc_ot(int m, int mk, int d, const double* x, const double* w,
              const double* y, const double* wy, double rho0, int T,
              double eps, double* p1, double* p2, double* lam) {
  double* C = (double*)malloc(sizeof(double) * (size_t)m * mk);
  orc_cost_block(m, mk, d, x, y, C);
  double v = orc_ot_cost(m, mk, C, w, wy, rho0, T, eps, p1, p2, lam);
  free(C);
  return v;
}

/*
 * Assignment step of D2-clustering (Algorithm "D2 Clustering", assignment
 * loop): l^(k) = argmin_c D(Q^(c), P^(k)) with D the B-ADMM transport value
 * of orc_ot.  Ties go to the lowest centroid index.  Xc: K x m x d,
 * Wc: K x m.  dist (N x K, may be NULL) receives every D.
 */
void orc_assign(int64_t N, const int64_t* off, int d, const double* X,
                const double* W, int K, int m, const double* Xc,
                const double* Wc, double rho0, int T, double eps,
                int32_t* labels, double* best, double* dist) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < N; ++k) {
    int mk = (int)(off[k + 1] - off[k]);
    double bv = INFINITY;
    int bc = 0;
    for (int c = 0; c < K; ++c) {
      double v = orc_ot(m, mk, d, Xc + (int64_t)c * m * d, Wc + (int64_t)c * m,
                        X + off[k] * d, W + off[k], rho0, T, eps, NULL, NULL,
                        NULL);
      if (dist) dist[k * K + c] = v;
      if (v < bv) { bv = v; bc = c; }
    }
    labels[k] = bc;
    if (best) best[k] = bv;
  }
}

/*
 * Assignment step over symbolic supports (Sec. 5): as orc_assign with the
 * cost block of (centroid c, instance k) gathered from the S x S table D,
 * C_ij = D[xsym[c*m + i] * S + ysym[off[k] + j]].
 */
void orc_assign_sym(int64_t N, const int64_t* off, const int32_t* ysym,
                    const double* W, int K, int m, const int32_t* xsym,
                    const double* Wc, int S, const double* D, double rho0,
                    int T, double eps, int32_t* labels, double* best,
                    double* dist) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < N; ++k) {
    int mk = (int)(off[k + 1] - off[k]);
    double* C = (double*)malloc(sizeof(double) * (size_t)m * mk);
    double bv = INFINITY;
    int bc = 0;
    for (int c = 0; c < K; ++c) {
      for (int j = 0; j < mk; ++j)
        for (int i = 0; i < m; ++i)
          C[i + (int64_t)j * m] =
              D[(int64_t)xsym[(int64_t)c * m + i] * S + ysym[off[k] + j]];
      double v = orc_ot_cost(m, mk, C, Wc + (int64_t)c * m, W + off[k], rho0,
                             T, eps, NULL, NULL, NULL);
      if (dist) dist[k * K + c] = v;
      if (v < bv) { bv = v; bc = c; }
    }
    free(C);
    labels[k] = bc;
    if (best) best[k] = bv;
  }
}
