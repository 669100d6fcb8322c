/*
 * FP64 CPU oracle for the hybrid scattered-regular meshless hot path
 * (Jancic, Rot, Kosec, "Spatially-varying meshless approximation method for
 * enhanced computational efficiency").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * Build: gcc -O2 -ffp-contract=off (no fused multiply-add anywhere: every
 * product and sum below is one IEEE double rounding, in the order written).
 *
 * Contents, each following the passage cited:
 *   ora_knn          stencil selection: the n nearest nodes of the same
 *                    domain (Section 2, text before Eq. (1)), ordered by
 *                    (squared distance, node index), brute force.
 *   ora_classify     regular / scattered assignment (Section 2 and Fig. 1:
 *                    MON on regular nodes, RBF-FD on scattered ones), decided
 *                    by a complete axis cross at spacing h_r, brute force.
 *   ora_rbffd        RBF-FD weights: PHS r^3 plus all monomials of degree
 *                    <= m (Section 2, items (i) and the 3rd-order PHS choice;
 *                    Section 2.1, M w = l), dense LU with partial pivoting.
 *   ora_mon          MON weights: 2d+1 monomials {1, x_k, x_k^2} on the
 *                    2d+1 node cross (Section 2, footnote on the 5-term basis).
 *   ora_build        both of the above for a list of nodes.
 *   ora_apply        Eq. (1): sum_i w_i u(x_i), in stencil order.
 *   ora_step         explicit Euler Boussinesq step with Chorin projection
 *                    (Section 3, Eqs. (2)-(4)); pressure Poisson problem with
 *                    Neumann walls and zero mean (a border row and column
 *                    of 1/sqrt(N) per domain), solved by BiCGSTAB or by a
 *                    dense LU.
 *   ora_nusselt      Eq. (5), averaged over a node list.
 *   ora_dense_lu_*   dense LU with partial pivoting (used by the above).
 *
 * Error codes: 0 ok, -1 invalid argument, -2 singular local system,
 * -3 duplicate node, -4 Krylov solve not converged, -5 non-finite value.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_OK 0
#define ORA_E_INVALID -1
#define ORA_E_SINGULAR -2
#define ORA_E_DUPLICATE -3
#define ORA_E_NOT_CONVERGED -4
#define ORA_E_NONFINITE -5

/* relative pivot threshold below which a local system is declared singular */
#define ORA_PIVOT_REL 1e-14
/* cross-detection tolerance, in units of h_r */
#define ORA_CROSS_TAU 1e-6

static int64_t domain_of(int64_t i, const int64_t *off, int32_t nd) {
  int32_t lo = 0, hi = nd - 1;
  while (lo < hi) {
    int32_t mid = (lo + hi + 1) / 2;
    if (off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

/* squared distance: dx*dx + dy*dy (+ dz*dz), summed in axis order, no FMA */
static double dist2(int d, int64_t N, const double *x, int64_t i, int64_t j) {
  double s = 0.0;
  for (int a = 0; a < d; ++a) {
    double t = x[a * N + j] - x[a * N + i];
    double sq = t * t;
    s = (a == 0) ? sq : s + sq;
  }
  return s;
}

/* ------------------------------------------------------------------ kNN -- */
/* For each query i: the k nodes j of i's domain with the smallest key
 * (d2(i,j), j), ascending, so i itself comes first.  Candidates of an
 * interior query are all nodes of the domain; candidates of a boundary query
 * (kind[i] != 0) are i itself and the interior nodes of the domain, so that a
 * boundary stencil couples the boundary node to interior nodes only (kind ==
 * NULL: every node is a candidate).  out is row-major [nq][k].  Returns -3
 * and the lowest-index offending query if some candidate j != i has d2 == 0. */
int ora_knn(int d, int64_t N, const double *x, const uint8_t *kind, const int64_t *dom_off,
            int32_t n_dom, int64_t nq, const int64_t *queries, int k, int32_t *out, int64_t *bad_node) {
  if ((d != 2 && d != 3) || k < 1 || N < 0 || n_dom < 1 || dom_off[0] != 0 || dom_off[n_dom] != N)
    return ORA_E_INVALID;
  double *bd = malloc(sizeof(double) * k);
  int64_t *bj = malloc(sizeof(int64_t) * k);
  if (!bd || !bj) { free(bd); free(bj); return ORA_E_INVALID; }
  int rc = ORA_OK;
  if (bad_node) *bad_node = -1;
  for (int64_t q = 0; q < nq; ++q) {
    int64_t i = queries ? queries[q] : q;
    int64_t dm = domain_of(i, dom_off, n_dom);
    int64_t lo = dom_off[dm], hi = dom_off[dm + 1];
    const int bnd = kind && kind[i] != 0;
    int cnt = 0;
    for (int64_t j = lo; j < hi; ++j) {
      if (bnd && j != i && kind[j] != 0) continue;
      double s = dist2(d, N, x, i, j);
      if (s == 0.0 && j != i) {
        if (bad_node && (*bad_node < 0 || i < *bad_node)) *bad_node = i;
        rc = ORA_E_DUPLICATE;
      }
      /* insert (s, j) into the sorted list of the best k seen so far */
      if (cnt == k && !(s < bd[k - 1] || (s == bd[k - 1] && j < bj[k - 1]))) continue;
      int p = (cnt < k) ? cnt++ : k - 1;
      while (p > 0 && (s < bd[p - 1] || (s == bd[p - 1] && j < bj[p - 1]))) {
        bd[p] = bd[p - 1];
        bj[p] = bj[p - 1];
        --p;
      }
      bd[p] = s;
      bj[p] = j;
    }
    if (cnt < k) { rc = ORA_E_INVALID; break; }
    for (int t = 0; t < k; ++t) out[q * k + t] = (int32_t)bj[t];
  }
  free(bd);
  free(bj);
  return rc;
}

/* ------------------------------------------------------------ classify -- */
/* Interior node i is REGULAR (class 0) iff for every axis a and sign s there
 * is exactly one node j of its domain with
 *     | fl(x_j,a - x_i,a) - s*h |  <= tau*h   and   | fl(x_j,b - x_i,b) | <= tau*h  (b != a),
 * h = h_r of the domain, tau = 1e-6.  Boundary nodes are SCATTERED (class 1).
 * For regular nodes the cross is [i, -x, +x, -y, +y (, -z, +z)]. */
int ora_classify(int d, int64_t N, const double *x, const uint8_t *kind, const int64_t *dom_off,
                 int32_t n_dom, const double *h_dom, int64_t nq, const int64_t *queries,
                 uint8_t *cls, int32_t *cross) {
  if ((d != 2 && d != 3) || N < 0 || n_dom < 1 || dom_off[0] != 0 || dom_off[n_dom] != N)
    return ORA_E_INVALID;
  const int W = 2 * d + 1;
  for (int64_t q = 0; q < nq; ++q) {
    int64_t i = queries ? queries[q] : q;
    int64_t dm = domain_of(i, dom_off, n_dom);
    const double h = h_dom[dm];
    const double tol = ORA_CROSS_TAU * h;
    int32_t found[6];
    int count[6] = {0, 0, 0, 0, 0, 0};
    for (int t = 0; t < W; ++t) cross[q * W + t] = -1;
    if (kind[i] != 0) { cls[q] = 1; continue; }
    for (int64_t j = dom_off[dm]; j < dom_off[dm + 1]; ++j) {
      double t[3];
      for (int a = 0; a < d; ++a) t[a] = x[a * N + j] - x[a * N + i];
      for (int a = 0; a < d; ++a)
        for (int s = 0; s < 2; ++s) {
          double e = s ? t[a] - h : t[a] + h; /* sign -: x_i - h e_a ; sign +: x_i + h e_a */
          int ok = fabs(e) <= tol;
          for (int b = 0; b < d && ok; ++b)
            if (b != a && !(fabs(t[b]) <= tol)) ok = 0;
          if (ok) { found[2 * a + s] = (int32_t)j; count[2 * a + s]++; }
        }
    }
    int regular = 1;
    for (int c = 0; c < 2 * d; ++c) if (count[c] != 1) regular = 0;
    cls[q] = regular ? 0 : 1;
    if (regular) {
      cross[q * W] = (int32_t)i;
      for (int c = 0; c < 2 * d; ++c) cross[q * W + 1 + c] = found[c];
    }
  }
  return ORA_OK;
}

/* ---------------------------------------------------------- dense LU ---- */
/* LU with partial pivoting.  Column k: the pivot is the not-yet-used row r
 * with the largest |a_rk|; among equal magnitudes the lowest row number wins.
 * Rows are not moved; piv[k] records the row chosen for column k.  Every
 * remaining row r gets  l = a_rk / a_pk ;  a_rj = a_rj - l*a_pj  (j > k)  and
 * the same update of its right-hand sides.  Back substitution then runs
 * columns k = S-1 .. 0:  x_k = b_pk / a_pk,k ;  every row pivoted before
 * column k gets  b_r = b_r - a_rk * x_k.
 * a: row-major [S][S], b: row-major [S][nrhs] (overwritten), x: [S][nrhs].
 * Returns -2 if a pivot magnitude is <= ORA_PIVOT_REL * max|a|. */
int ora_dense_lu_solve(int S, double *a, int nrhs, double *b, double *x) {
  double amax = 0.0;
  for (int i = 0; i < S * S; ++i) if (fabs(a[i]) > amax) amax = fabs(a[i]);
  int *used = calloc(S, sizeof(int));
  int *piv = malloc(sizeof(int) * S);
  if (!used || !piv) { free(used); free(piv); return ORA_E_INVALID; }
  int rc = ORA_OK;
  for (int k = 0; k < S; ++k) {
    int p = -1;
    double best = -1.0;
    for (int r = 0; r < S; ++r)
      if (!used[r] && fabs(a[r * S + k]) > best) { best = fabs(a[r * S + k]); p = r; }
    if (!(best > ORA_PIVOT_REL * amax)) { rc = ORA_E_SINGULAR; break; }
    used[p] = 1;
    piv[k] = p;
    for (int r = 0; r < S; ++r) {
      if (used[r]) continue;
      double l = a[r * S + k] / a[p * S + k];
      for (int j = k + 1; j < S; ++j) a[r * S + j] = a[r * S + j] - l * a[p * S + j];
      for (int q = 0; q < nrhs; ++q) b[r * nrhs + q] = b[r * nrhs + q] - l * b[p * nrhs + q];
    }
  }
  if (rc == ORA_OK) {
    for (int k = S - 1; k >= 0; --k) {
      int p = piv[k];
      for (int q = 0; q < nrhs; ++q) x[k * nrhs + q] = b[p * nrhs + q] / a[p * S + k];
      for (int kk = 0; kk < k; ++kk) {
        int r = piv[kk];
        for (int q = 0; q < nrhs; ++q) b[r * nrhs + q] = b[r * nrhs + q] - a[r * S + k] * x[k * nrhs + q];
      }
    }
  }
  free(used);
  free(piv);
  return rc;
}

/* ------------------------------------------------------- monomials ------ */
/* Exponents of all monomials of degree <= m in d variables, graded, and
 * within one degree in descending power of x, then of y:
 *   2D m=2: 1, x, y, x^2, xy, y^2.   Returns the count Q = C(m+d, d). */
int ora_monomials(int d, int m, int *alpha /* [Q][3] */) {
  int q = 0;
  for (int deg = 0; deg <= m; ++deg) {
    if (d == 2) {
      for (int ax = deg; ax >= 0; --ax) {
        alpha[3 * q + 0] = ax; alpha[3 * q + 1] = deg - ax; alpha[3 * q + 2] = 0; ++q;
      }
    } else {
      for (int ax = deg; ax >= 0; --ax)
        for (int ay = deg - ax; ay >= 0; --ay) {
          alpha[3 * q + 0] = ax; alpha[3 * q + 1] = ay; alpha[3 * q + 2] = deg - ax - ay; ++q;
        }
    }
  }
  return q;
}

/* y^alpha as the left-to-right product 1*y_x*...*y_x*y_y*...*y_z */
static double mono_eval(int d, const int *al, const double *y) {
  double p = 1.0;
  for (int a = 0; a < d; ++a)
    for (int e = 0; e < al[a]; ++e) p = p * y[a];
  return p;
}

/* Local coordinates y_j = (x_j - x_c) / s, s = max_j |x_j - x_c|, with
 * |v| = sqrt(v_x*v_x + v_y*v_y (+ v_z*v_z)).  xs: row-major [n][d]. */
static double local_coords(int d, int n, const double *xs, double *y) {
  double s = 0.0;
  for (int j = 0; j < n; ++j) {
    double q = 0.0;
    for (int a = 0; a < d; ++a) {
      double t = xs[j * d + a] - xs[a];
      q = (a == 0) ? t * t : q + t * t;
    }
    double r = sqrt(q);
    if (r > s) s = r;
  }
  for (int j = 0; j < n; ++j)
    for (int a = 0; a < d; ++a) y[j * d + a] = (xs[j * d + a] - xs[a]) / s;
  return s;
}

static double norm_d(int d, const double *v) {
  double q = 0.0;
  for (int a = 0; a < d; ++a) q = (a == 0) ? v[a] * v[a] : q + v[a] * v[a];
  return sqrt(q);
}

/* ----------------------------------------------------------- RBF-FD ----- */
/* Weights of d/dx_a (a = 0..d-1) and of the Laplacian at the first stencil
 * node, from PHS phi(r) = r^3 augmented with all monomials of degree <= m.
 *   M = [[A, P], [P^T, 0]],  A_jl = |y_j - y_l|^3,  P_ja = y_j^alpha,
 *   rhs of d/dx_a: phi part  -3 |y_j| y_j,a ;  poly part 1 where alpha = e_a
 *   rhs of Lap   : phi part  3(d+1) |y_j|   ;  poly part 2 where alpha = 2 e_a
 * (derivatives of |y - y_j|^3 and of y^alpha, taken at y = 0).
 * Solved in the scaled coordinates; weights are then divided by s (first
 * derivatives) and by s*s (Laplacian).  xs: row-major [n][d], centre first.
 * w: row-major [d+1][n].  Returns -2 if the system is singular. */
int ora_rbffd(int d, int m, int n, const double *xs, double *w) {
  int alpha[3 * 64];
  if ((d != 2 && d != 3) || m < 0 || m > 6) return ORA_E_INVALID;
  const int Q = ora_monomials(d, m, alpha);
  const int S = n + Q;
  const int R = d + 1;
  if (n < 1 || S > 256) return ORA_E_INVALID;
  double *y = malloc(sizeof(double) * n * d);
  double *A = calloc((size_t)S * S, sizeof(double));
  double *b = calloc((size_t)S * R, sizeof(double));
  double *sol = malloc(sizeof(double) * S * R);
  if (!y || !A || !b || !sol) { free(y); free(A); free(b); free(sol); return ORA_E_INVALID; }
  double s = local_coords(d, n, xs, y);
  for (int j = 0; j < n; ++j) {
    for (int l = 0; l < n; ++l) {
      double dv[3];
      for (int a = 0; a < d; ++a) dv[a] = y[j * d + a] - y[l * d + a];
      double r = norm_d(d, dv);
      A[j * S + l] = r * r * r;
    }
    for (int q = 0; q < Q; ++q) {
      double p = mono_eval(d, alpha + 3 * q, y + j * d);
      A[j * S + n + q] = p;
      A[(n + q) * S + j] = p;
    }
    double rj = norm_d(d, y + j * d);
    for (int a = 0; a < d; ++a) b[j * R + a] = -((3.0 * rj) * y[j * d + a]);
    b[j * R + d] = (3.0 * (d + 1)) * rj;
  }
  for (int q = 0; q < Q; ++q) {
    const int *al = alpha + 3 * q;
    int deg = al[0] + al[1] + al[2];
    for (int a = 0; a < d; ++a) {
      if (deg == 1 && al[a] == 1) b[(n + q) * R + a] = 1.0;
      if (deg == 2 && al[a] == 2) b[(n + q) * R + d] = 2.0;
    }
  }
  int rc = ora_dense_lu_solve(S, A, R, b, sol);
  if (rc == ORA_OK) {
    double s2 = s * s;
    for (int j = 0; j < n; ++j) {
      for (int a = 0; a < d; ++a) w[a * n + j] = sol[j * R + a] / s;
      w[d * n + j] = sol[j * R + d] / s2;
    }
  }
  free(y); free(A); free(b); free(sol);
  return rc;
}

/* -------------------------------------------------------------- MON ----- */
/* Weights on the 2d+1 node cross from the basis {1, x, y, (z), x^2, y^2, (z^2)}
 * in the scaled local coordinates: rows of the system are basis functions,
 * columns stencil nodes:  sum_j p(y_j) w_j = (L p)(0).
 * xs: row-major [2d+1][d], centre first.  w: row-major [d+1][2d+1]. */
int ora_mon(int d, const double *xs, double *w) {
  if (d != 2 && d != 3) return ORA_E_INVALID;
  const int n = 2 * d + 1, R = d + 1;
  double y[7 * 3], A[7 * 7], b[7 * 4], sol[7 * 4];
  double s = local_coords(d, n, xs, y);
  for (int j = 0; j < n; ++j) {
    A[0 * n + j] = 1.0;
    for (int a = 0; a < d; ++a) {
      A[(1 + a) * n + j] = y[j * d + a];
      A[(1 + d + a) * n + j] = y[j * d + a] * y[j * d + a];
    }
  }
  for (int r = 0; r < n * R; ++r) b[r] = 0.0;
  for (int a = 0; a < d; ++a) {
    b[(1 + a) * R + a] = 1.0;       /* d/dx_a x_a = 1 */
    b[(1 + d + a) * R + d] = 2.0;   /* Lap x_a^2 = 2 */
  }
  int rc = ora_dense_lu_solve(n, A, R, b, sol);
  if (rc == ORA_OK) {
    double s2 = s * s;
    for (int j = 0; j < n; ++j) {
      for (int a = 0; a < d; ++a) w[a * n + j] = sol[j * R + a] / s;
      w[d * n + j] = sol[j * R + d] / s2;
    }
  }
  return rc;
}

/* ------------------------------------------------------------ build ----- */
/* Stencils and weights for a list of nodes (all nodes if queries == NULL).
 * mode 0 = hybrid (MON on regular nodes, RBF-FD elsewhere), 1 = all RBF-FD.
 * Per query q (row-major, padded to maxw columns):
 *   cls[q] 0/1, width[q], idx[q][maxw], w[q][d+1][maxw] and, for boundary
 *   nodes, wn[q][maxw] = sum_a n_a * w_a (normal derivative; 0 elsewhere).
 * Stencil width of scattered nodes: n_dom[dom] (RBF-FD), degree m_dom[dom]. */
int ora_build(int d, int64_t N, const double *x, const uint8_t *kind, const double *normal,
              const int64_t *dom_off, int32_t n_domains, const double *h_dom, const int32_t *m_dom,
              const int32_t *n_dom, int mode, int64_t nq, const int64_t *queries, int maxw,
              uint8_t *cls, int32_t *width, int32_t *idx, double *w, double *wn, int64_t *bad_node) {
  const int R = d + 1, W = 2 * d + 1;
  if (bad_node) *bad_node = -1;
  int32_t *cross = malloc(sizeof(int32_t) * W);
  double *xs = malloc(sizeof(double) * maxw * d);
  double *wl = malloc(sizeof(double) * maxw * R);
  int32_t *nb = malloc(sizeof(int32_t) * maxw);
  if (!cross || !xs || !wl || !nb) { free(cross); free(xs); free(wl); free(nb); return ORA_E_INVALID; }
  int rc = ORA_OK;
  for (int64_t q = 0; q < nq && rc == ORA_OK; ++q) {
    int64_t i = queries ? queries[q] : q;
    int64_t dm = domain_of(i, dom_off, n_domains);
    uint8_t c = 1;
    if (mode == 0) {
      rc = ora_classify(d, N, x, kind, dom_off, n_domains, h_dom, 1, &i, &c, cross);
      if (rc) break;
    }
    int wdt;
    if (c == 0) {
      wdt = W;
      for (int t = 0; t < W; ++t) nb[t] = cross[t];
    } else {
      wdt = n_dom[dm];
      if (wdt > maxw) { rc = ORA_E_INVALID; break; }
      int64_t bad = -1;
      rc = ora_knn(d, N, x, kind, dom_off, n_domains, 1, &i, wdt, nb, &bad);
      if (rc) { if (bad_node) *bad_node = i; break; }
    }
    for (int t = 0; t < wdt; ++t)
      for (int a = 0; a < d; ++a) xs[t * d + a] = x[a * N + nb[t]];
    rc = (c == 0) ? ora_mon(d, xs, wl) : ora_rbffd(d, m_dom[dm], wdt, xs, wl);
    if (rc == ORA_E_SINGULAR && c != 0 && kind[i] != 0 && m_dom[dm] >= 2) {
      /* A wall node's stencil of interior nodes can leave the degree-m
       * monomial block rank-deficient (for instance when all but the wall
       * node lie on two lattice planes, so x^2 and x agree on the stencil).
       * Walls only need first derivatives (the normal derivative), so the
       * node then takes PHS plus monomials of degree m-1 on the same nodes. */
      rc = ora_rbffd(d, m_dom[dm] - 1, wdt, xs, wl);
    }
    if (rc) { if (bad_node) *bad_node = i; break; }
    cls[q] = c;
    width[q] = wdt;
    for (int t = 0; t < maxw; ++t) {
      idx[q * maxw + t] = t < wdt ? nb[t] : -1;
      for (int r = 0; r < R; ++r) w[(q * R + r) * maxw + t] = t < wdt ? wl[r * wdt + t] : 0.0;
      double acc = 0.0;
      if (t < wdt && kind[i] != 0)
        for (int a = 0; a < d; ++a) {
          double v = normal[a * N + i] * wl[a * wdt + t];
          acc = (a == 0) ? v : acc + v;
        }
      wn[q * maxw + t] = acc;
    }
  }
  free(cross); free(xs); free(wl); free(nb);
  return rc;
}

/* Weights of given stencils (CSR: off[ns+1], idx, centre first) at the
 * nodes listed in `nodes`: the same local solves as ora_build (MON on the
 * axis cross where cls = 0, RBF-FD of degree m[q] otherwise, with the wall
 * fallback to degree m-1), without the neighbour search.  w: [d+1][nnz].
 * Used to time the local solves on their own. */
int ora_weights_csr(int d, int64_t N, const double *x, const uint8_t *kind, int64_t ns, const int64_t *nodes,
                    const int64_t *off, const int32_t *idx, const uint8_t *cls, const int32_t *m, double *w,
                    int64_t *bad_node) {
  const int R = d + 1;
  const int64_t nnz = off[ns];
  int maxw = 1;
  for (int64_t q = 0; q < ns; ++q)
    if (off[q + 1] - off[q] > maxw) maxw = (int)(off[q + 1] - off[q]);
  double *xs = malloc(sizeof(double) * maxw * d);
  double *wl = malloc(sizeof(double) * maxw * R);
  if (!xs || !wl) { free(xs); free(wl); return ORA_E_INVALID; }
  if (bad_node) *bad_node = -1;
  int rc = ORA_OK;
  for (int64_t q = 0; q < ns && rc == ORA_OK; ++q) {
    const int wdt = (int)(off[q + 1] - off[q]);
    for (int t = 0; t < wdt; ++t)
      for (int a = 0; a < d; ++a) xs[t * d + a] = x[a * N + idx[off[q] + t]];
    rc = (cls[q] == 0) ? ora_mon(d, xs, wl) : ora_rbffd(d, m[q], wdt, xs, wl);
    if (rc == ORA_E_SINGULAR && cls[q] != 0 && kind[nodes[q]] != 0 && m[q] >= 2) rc = ora_rbffd(d, m[q] - 1, wdt, xs, wl);
    if (rc) { if (bad_node) *bad_node = nodes[q]; break; }
    for (int r = 0; r < R; ++r)
      for (int t = 0; t < wdt; ++t) w[r * nnz + off[q] + t] = wl[r * wdt + t];
  }
  free(xs); free(wl);
  return rc;
}

/* ------------------------------------------------------------ apply ----- */
/* Eq. (1): out_i = sum_j w_ij u_{idx_ij}, accumulated in stencil order.
 * CSR stencils: off[N+1], idx[nnz], w[nnz]. */
void ora_apply(int64_t N, const int64_t *off, const int32_t *idx, const double *w,
               const double *u, double *out) {
  for (int64_t i = 0; i < N; ++i) {
    double acc = 0.0;
    for (int64_t t = off[i]; t < off[i + 1]; ++t) acc = acc + w[t] * u[idx[t]];
    out[i] = acc;
  }
}

/* ------------------------------------------------- pressure problem ----- */
/* The pressure operator: row i holds the Laplacian weights at interior nodes
 * and the normal-derivative weights at boundary nodes (dp/dn = 0 on no-slip
 * walls), each row divided by its centre weight.  Each domain k's zero-mean
 * condition is added as a border row and column scaled by c_k = 1/sqrt(N_k),
 * N_k the domain's node count (its multiplier lam_k at unknown N + k):
 *   sum_j a_ij p_j + c_k lam_k = b_i (i in k),   c_k sum_{i in k} p_i = 0.
 * With one domain: [[A, c 1], [c 1^T, 0]] [p; lam] = [b; 0].  The scale
 * leaves the constraint and p unchanged; it moves the eigenvalue pair that a
 * border of ones adds near +-sqrt(N_k) to near +-1 (reading R11). */
typedef struct {
  int64_t N, K;
  const int64_t *off;
  const int32_t *idx;
  const int32_t *dom; /* domain of each node */
  double *a;          /* scaled row weights, CSR */
  double *c;          /* [K] border scale 1/sqrt(N_k) */
} pop_t;

static double border_scale(const int64_t *dom_off, int64_t k) {
  return 1.0 / sqrt((double)(dom_off[k + 1] - dom_off[k]));
}

static void pop_matvec(const pop_t *P, const double *v, double *out) {
  const int64_t N = P->N;
  for (int64_t i = 0; i < N; ++i) {
    double acc = 0.0;
    for (int64_t t = P->off[i]; t < P->off[i + 1]; ++t) acc = acc + P->a[t] * v[P->idx[t]];
    out[i] = acc + P->c[P->dom[i]] * v[N + P->dom[i]];
  }
  for (int64_t k = 0; k < P->K; ++k) out[N + k] = 0.0;
  for (int64_t i = 0; i < N; ++i) out[N + P->dom[i]] = out[N + P->dom[i]] + v[i];
  for (int64_t k = 0; k < P->K; ++k) out[N + k] = P->c[k] * out[N + k];
}

static double dot(int64_t n, const double *a, const double *b) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s = s + a[i] * b[i];
  return s;
}

/* BiCGSTAB (van der Vorst 1992) on the bordered system, from the initial
 * guess in x[0..N+K), until ||r|| <= tol ||b||.  Returns iterations used, or
 * -1 if not converged within maxiter / on breakdown. */
static int bicgstab(const pop_t *P, const double *b, double *x, double tol, int maxiter, double *relres) {
  const int64_t n = P->N + P->K;
  double *r = malloc(sizeof(double) * n), *rh = malloc(sizeof(double) * n);
  double *p = calloc(n, sizeof(double)), *v = calloc(n, sizeof(double));
  double *s = malloc(sizeof(double) * n), *t = malloc(sizeof(double) * n);
  int it = -1;
  double bn = sqrt(dot(n, b, b));
  if (bn == 0.0) {
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    *relres = 0.0;
    free(r); free(rh); free(p); free(v); free(s); free(t);
    return 0;
  }
  pop_matvec(P, x, r);
  for (int64_t i = 0; i < n; ++i) { r[i] = b[i] - r[i]; rh[i] = r[i]; }
  double rho = 1.0, alpha = 1.0, omega = 1.0;
  double rn = sqrt(dot(n, r, r));
  if (rn <= tol * bn) { *relres = rn / bn; it = 0; goto done; }
  for (int k = 1; k <= maxiter; ++k) {
    double rho_new = dot(n, rh, r);
    if (rho_new == 0.0 || omega == 0.0) break;
    double beta = (rho_new / rho) * (alpha / omega);
    rho = rho_new;
    for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
    pop_matvec(P, p, v);
    double rv = dot(n, rh, v);
    if (rv == 0.0) break;
    alpha = rho / rv;
    for (int64_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
    double sn = sqrt(dot(n, s, s));
    if (sn <= tol * bn) {
      for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
      *relres = sn / bn;
      it = k;
      break;
    }
    pop_matvec(P, s, t);
    double tt = dot(n, t, t);
    if (tt == 0.0) break;
    omega = dot(n, t, s) / tt;
    for (int64_t i = 0; i < n; ++i) {
      x[i] = x[i] + alpha * p[i] + omega * s[i];
      r[i] = s[i] - omega * t[i];
    }
    rn = sqrt(dot(n, r, r));
    if (rn <= tol * bn) { *relres = rn / bn; it = k; break; }
  }
done:
  free(r); free(rh); free(p); free(v); free(s); free(t);
  return it;
}

/* Dense form of the same bordered pressure system, row-major [(N+K)^2], K
 * domains given by dom_off [K+1].  For small problems the oracle factorises
 * it once and solves exactly. */
int ora_pressure_dense(int64_t N, const int64_t *off, const int32_t *idx, const double *wlap,
                       const double *wn, const uint8_t *kind, int32_t K, const int64_t *dom_off, double *M) {
  const int64_t n = N + K;
  memset(M, 0, sizeof(double) * n * n);
  for (int64_t k = 0; k < K; ++k) {
    const double c = border_scale(dom_off, k);
    for (int64_t i = dom_off[k]; i < dom_off[k + 1]; ++i) {
      const double *wr = kind[i] ? wn : wlap;
      double dg = wr[off[i]];
      for (int64_t t = off[i]; t < off[i + 1]; ++t) M[i * n + idx[t]] += wr[t] / dg;
      M[i * n + N + k] = c;
      M[(N + k) * n + i] = c;
    }
  }
  return ORA_OK;
}

/* ------------------------------------------------------------- step ----- */
typedef struct {
  double Ra, Pr, dt, T_ref;
  double tol;
  int32_t maxiter;
  int32_t solver; /* 0: BiCGSTAB, 1: dense LU of the bordered system */
} ora_params;

/* State carried between steps by the caller: v [d][N], T [N], p [N+K]
 * (p[N+k] is domain k's border multiplier).  CSR stencils with weights wop[a] for
 * d/dx_a (a < d) and wop[d] for the Laplacian; wn holds normal-derivative
 * weights (read at boundary nodes only).  dense_lu: optional factorised
 * dense system (from ora_pressure_dense; may be NULL for BiCGSTAB).
 * One explicit Euler step, Section 3:
 *   1. v* = v + dt (-(v.grad)v + Pr Lap v + Ra Pr T_d e_up)  at interior nodes
 *      (T_d = T - T_ref; gravity points along -e_up, e_up = last axis);
 *      v* = 0 at boundary nodes (no slip).
 *   2. pressure: [scaled L_p, border] p = (div v* / dt) at interior nodes,
 *      0 at boundary nodes (dp/dn = 0); zero mean.
 *   3. v = v* - dt grad p at interior nodes, 0 at boundary nodes.
 *   4. T' = T + dt (-v.grad T + Lap T) at interior nodes, with the new v.
 *      Dirichlet nodes keep T.  Neumann node b:
 *      T'_b = -(sum_{j != b} wn_bj T~_j) / wn_bb, T~_j = T'_j at interior j
 *      and T_j at boundary j.
 * iters_out receives the Krylov iteration count. */
typedef struct {
  int d;
  int64_t N, K;
  int32_t *dom;
  const int64_t *off;
  const int32_t *idx;
  const double *wop[4];
  const double *wn;
  const uint8_t *kind;
  pop_t P;
  double *dense; /* LU-factorised rows, pivots and flags for solver 1 */
  int *dpiv;
  double *vs, *g0, *g1, *g2, *rhs, *Tn;
} ora_sim;

void *ora_sim_create(int d, int64_t N, const int64_t *off, const int32_t *idx, const double *const *wop,
                     const double *wn, const uint8_t *kind, int32_t K, const int64_t *dom_off, int solver) {
  if (K < 1 || dom_off[0] != 0 || dom_off[K] != N) return NULL;
  ora_sim *S = calloc(1, sizeof(ora_sim));
  if (!S) return NULL;
  S->d = d; S->N = N; S->K = K; S->off = off; S->idx = idx; S->wn = wn; S->kind = kind;
  S->dom = malloc(sizeof(int32_t) * (N > 0 ? N : 1));
  for (int64_t k = 0; k < K; ++k)
    for (int64_t i = dom_off[k]; i < dom_off[k + 1]; ++i) S->dom[i] = (int32_t)k;
  for (int a = 0; a <= d; ++a) S->wop[a] = wop[a];
  int64_t nnz = off[N];
  S->P.N = N; S->P.K = K; S->P.off = off; S->P.idx = idx; S->P.dom = S->dom;
  S->P.a = malloc(sizeof(double) * (nnz > 0 ? nnz : 1));
  S->P.c = malloc(sizeof(double) * K);
  for (int64_t k = 0; k < K; ++k) S->P.c[k] = border_scale(dom_off, k);
  for (int64_t i = 0; i < N; ++i) {
    const double *wr = kind[i] ? wn : wop[d];
    double dg = wr[off[i]];
    for (int64_t t = off[i]; t < off[i + 1]; ++t) S->P.a[t] = wr[t] / dg;
  }
  S->vs = malloc(sizeof(double) * d * N);
  S->g0 = malloc(sizeof(double) * N);
  S->g1 = malloc(sizeof(double) * N);
  S->g2 = malloc(sizeof(double) * N);
  S->rhs = malloc(sizeof(double) * (N + K));
  S->Tn = malloc(sizeof(double) * N);
  if (solver == 1) {
    const int64_t n = N + K;
    S->dense = malloc(sizeof(double) * n * n);
    S->dpiv = malloc(sizeof(int) * n);
    if (!S->dense || !S->dpiv) return S;
    ora_pressure_dense(N, off, idx, wop[d], wn, kind, K, dom_off, S->dense);
    /* factorise once: same pivoting rule as ora_dense_lu_solve, rows kept in place */
    int *used = calloc(n, sizeof(int));
    for (int64_t k = 0; k < n; ++k) {
      int64_t p = -1;
      double best = -1.0;
      for (int64_t r = 0; r < n; ++r)
        if (!used[r] && fabs(S->dense[r * n + k]) > best) { best = fabs(S->dense[r * n + k]); p = r; }
      used[p] = 1;
      S->dpiv[k] = (int)p;
      for (int64_t r = 0; r < n; ++r) {
        if (used[r]) continue;
        double l = S->dense[r * n + k] / S->dense[p * n + k];
        S->dense[r * n + k] = l; /* multiplier kept in the eliminated slot */
        if (l != 0.0)
          for (int64_t j = k + 1; j < n; ++j) S->dense[r * n + j] = S->dense[r * n + j] - l * S->dense[p * n + j];
      }
    }
    free(used);
  }
  return S;
}

void ora_sim_destroy(void *h) {
  ora_sim *S = (ora_sim *)h;
  if (!S) return;
  free(S->P.a); free(S->P.c); free(S->vs); free(S->g0); free(S->g1); free(S->g2); free(S->rhs); free(S->Tn); free(S->dom);
  free(S->dense); free(S->dpiv);
  free(S);
}

static void dense_solve(const ora_sim *S, double *b, double *x) {
  const int64_t n = S->N + S->K;
  /* forward: replay the elimination on b in pivot order */
  char *used = calloc(n, 1);
  for (int64_t k = 0; k < n; ++k) {
    int64_t p = S->dpiv[k];
    used[p] = 1;
    for (int64_t r = 0; r < n; ++r)
      if (!used[r]) b[r] = b[r] - S->dense[r * n + k] * b[p];
  }
  free(used);
  for (int64_t k = n - 1; k >= 0; --k) {
    int64_t p = S->dpiv[k];
    x[k] = b[p] / S->dense[p * n + k];
    for (int64_t kk = 0; kk < k; ++kk) {
      int64_t r = S->dpiv[kk];
      b[r] = b[r] - S->dense[r * n + k] * x[k];
    }
  }
}

/* Step 1 (momentum predictor): vs = v + dt (-(v.grad)v + Pr Lap v + Ra Pr (T - T_ref) e_up)
 * at interior nodes, 0 at boundary nodes. */
void ora_predict(void *h, const ora_params *prm, const double *v, const double *T, double *vs) {
  ora_sim *S = (ora_sim *)h;
  const int d = S->d;
  const int64_t N = S->N;
  for (int c = 0; c < d; ++c) {
    const double *vc = v + c * N;
    for (int64_t i = 0; i < N; ++i) {
      if (S->kind[i] != 0) { vs[c * N + i] = 0.0; continue; }
      double adv = 0.0;
      for (int a = 0; a < d; ++a) {
        double g = 0.0;
        for (int64_t t = S->off[i]; t < S->off[i + 1]; ++t) g = g + S->wop[a][t] * vc[S->idx[t]];
        double term = v[a * N + i] * g;
        adv = (a == 0) ? term : adv + term;
      }
      double lap = 0.0;
      for (int64_t t = S->off[i]; t < S->off[i + 1]; ++t) lap = lap + S->wop[d][t] * vc[S->idx[t]];
      double f = -adv + prm->Pr * lap;
      if (c == d - 1) f = f + (prm->Ra * prm->Pr) * (T[i] - prm->T_ref);
      vs[c * N + i] = vc[i] + prm->dt * f;
    }
  }
}

/* Step 2 (right-hand side of the pressure problem): div(vs) / dt at interior
 * nodes divided by the row's centre weight, 0 at boundary nodes, 0 in the borders. */
void ora_pressure_rhs(void *h, const ora_params *prm, const double *vs, double *rhs) {
  ora_sim *S = (ora_sim *)h;
  const int d = S->d;
  const int64_t N = S->N;
  for (int64_t i = 0; i < N; ++i) {
    if (S->kind[i] != 0) { rhs[i] = 0.0; continue; }
    double dv = 0.0;
    for (int a = 0; a < d; ++a) {
      double g = 0.0;
      for (int64_t t = S->off[i]; t < S->off[i + 1]; ++t) g = g + S->wop[a][t] * vs[a * N + S->idx[t]];
      dv = (a == 0) ? g : dv + g;
    }
    rhs[i] = (dv / prm->dt) / S->wop[d][S->off[i]];
  }
  for (int64_t k = 0; k < S->K; ++k) rhs[N + k] = 0.0;
}

/* Step 3 (projection): v = vs - dt grad p at interior nodes, 0 at boundary nodes. */
void ora_correct(void *h, const ora_params *prm, const double *vs, const double *p, double *v) {
  ora_sim *S = (ora_sim *)h;
  const int d = S->d;
  const int64_t N = S->N;
  for (int64_t i = 0; i < N; ++i) {
    for (int c = 0; c < d; ++c) {
      if (S->kind[i] != 0) { v[c * N + i] = 0.0; continue; }
      double g = 0.0;
      for (int64_t t = S->off[i]; t < S->off[i + 1]; ++t) g = g + S->wop[c][t] * p[S->idx[t]];
      v[c * N + i] = vs[c * N + i] - prm->dt * g;
    }
  }
}

/* Step 4 (heat transport): Tn = T + dt (-v.grad T + Lap T) at interior nodes
 * (v already projected); Dirichlet nodes keep T; Neumann node b takes the
 * value that zeroes its normal derivative:
 *   Tn_b = -(sum_{j != b} wn_bj T~_j) / wn_bb,  T~_j = Tn_j (interior j), T_j (boundary j). */
void ora_heat(void *h, const ora_params *prm, const double *v, const double *T, double *Tn) {
  ora_sim *S = (ora_sim *)h;
  const int d = S->d;
  const int64_t N = S->N;
  for (int64_t i = 0; i < N; ++i) {
    if (S->kind[i] != 0) { Tn[i] = T[i]; continue; }
    double adv = 0.0;
    for (int a = 0; a < d; ++a) {
      double g = 0.0;
      for (int64_t t = S->off[i]; t < S->off[i + 1]; ++t) g = g + S->wop[a][t] * T[S->idx[t]];
      double term = v[a * N + i] * g;
      adv = (a == 0) ? term : adv + term;
    }
    double lap = 0.0;
    for (int64_t t = S->off[i]; t < S->off[i + 1]; ++t) lap = lap + S->wop[d][t] * T[S->idx[t]];
    Tn[i] = T[i] + prm->dt * (-adv + lap);
  }
  for (int64_t i = 0; i < N; ++i) {
    if (S->kind[i] != 2) continue;
    double acc = 0.0;
    for (int64_t t = S->off[i] + 1; t < S->off[i + 1]; ++t) {
      int32_t j = S->idx[t];
      double tj = S->kind[j] != 0 ? T[j] : Tn[j];
      acc = acc + S->wn[t] * tj;
    }
    Tn[i] = -acc / S->wn[S->off[i]];
  }
}

int ora_sim_step(void *h, const ora_params *prm, int nsteps, double *v, double *T, double *p,
                 int32_t *iters_out) {
  ora_sim *S = (ora_sim *)h;
  const int d = S->d;
  const int64_t N = S->N;
  for (int st = 0; st < nsteps; ++st) {
    ora_predict(S, prm, v, T, S->vs);
    ora_pressure_rhs(S, prm, S->vs, S->rhs);
    int it = 0;
    if (S->dense) {
      dense_solve(S, S->rhs, p);
    } else {
      double rr = 0.0;
      it = bicgstab(&S->P, S->rhs, p, prm->tol, prm->maxiter, &rr);
      if (it < 0) { if (iters_out) iters_out[st] = prm->maxiter; return ORA_E_NOT_CONVERGED; }
    }
    if (iters_out) iters_out[st] = it;
    ora_correct(S, prm, S->vs, p, v);
    ora_heat(S, prm, v, T, S->Tn);
    int finite = 1;
    for (int64_t i = 0; i < N; ++i) {
      T[i] = S->Tn[i];
      if (!isfinite(T[i])) finite = 0;
      for (int c = 0; c < d; ++c) if (!isfinite(v[c * N + i])) finite = 0;
    }
    if (!finite) return ORA_E_NONFINITE;
  }
  return ORA_OK;
}

/* Eq. (5): Nu = L/(T_H - T_C) * mean over the listed nodes of |dT/dn|, with
 * dT/dn from the normal-derivative weights (CSR). */
double ora_nusselt(const int64_t *off, const int32_t *idx, const double *wn, const double *T,
                   int64_t nlist, const int64_t *nodes, double L, double dT) {
  double s = 0.0;
  for (int64_t q = 0; q < nlist; ++q) {
    int64_t i = nodes[q];
    double g = 0.0;
    for (int64_t t = off[i]; t < off[i + 1]; ++t) g = g + wn[t] * T[idx[t]];
    s = s + fabs(g);
  }
  return nlist ? (L / dT) * (s / (double)nlist) : 0.0;
}
