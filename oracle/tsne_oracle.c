/*
 * tsne_oracle.c -- plain FP64 CPU oracle for the exact t-SNE hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load or call this library.  It shares
 * no code, header, table or helper with the HIP library it checks, and the
 * product path never routes through it.
 *
 * The profiled paper names the stage (t-SNE of PCA scores: abstract; Table 1,
 * row 7) but defines none of its steps.  Each function below therefore writes
 * out the standard published definition it follows:
 *   [vdMH08] van der Maaten & Hinton, "Visualizing Data using t-SNE",
 *            JMLR 9 (2008): conditional P (eq. 1), perplexity (eq. 3),
 *            symmetric P (Sec. 3.1), Student-t Q (eq. 4), gradient (eq. 5),
 *            momentum and early exaggeration (Sec. 3.4, Algorithm 1).
 *   [vdM14]  van der Maaten, "Accelerating t-SNE using Tree-Based
 *            Algorithms", JMLR 15 (2014): sparse input similarities on the
 *            floor(3u) nearest neighbours (Sec. 4.1).
 *   [Jac88]  Jacobs, "Increased rates of convergence through learning rate
 *            adaptation", Neural Networks 1 (1988): the per-parameter gains.
 * Every floating-point step is IEEE double; inputs given as float are
 * widened exactly.  Reductions run in index order; Z uses Neumaier
 * compensated summation.  OpenMP splits work over rows only, so results do
 * not depend on the thread count.  Build with floating-point contraction off
 * so the arithmetic is exactly as written.
 *
 * All pointers are host pointers owned by the caller.  Every function
 * returns 0 on success and a negative value on invalid arguments.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Neumaier compensated sum.                                          */
typedef struct { double s, c; } nsum_t;
static void nsum_add(nsum_t* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static double nsum_get(const nsum_t* a) { return a->s + a->c; }

/* Lexicographic order on (distance, index): the neighbour order. */
static int key_less(double da, int64_t ja, double db, int64_t jb) {
  return da < db || (da == db && ja < jb);
}

/* Round a float to bfloat16, round-to-nearest-even, returned widened to
 * double.  bfloat16 keeps the top 16 bits of the IEEE single; RNE adds
 * 0x7FFF plus the lowest kept bit before truncating.  NaN stays NaN. */
static double bf16_rne(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) {
    return (double)f;
  }
  u += 0x7FFFu + ((u >> 16) & 1u);
  u &= 0xFFFF0000u;
  float r;
  memcpy(&r, &u, 4);
  return (double)r;
}

/* ------------------------------------------------------------------ */
/* Exact k nearest neighbours [vdM14 Sec. 4.1].
 * For query row q: d_qj = sum_c (x_qc - x_jc)^2 over all j != q (squared
 * Euclidean distance, the distance inside the Gaussian kernel of [vdMH08]
 * eq. 1).  The neighbours are the k smallest keys (d_qj, j) in
 * lexicographic order, listed ascending.  Self is excluded by index.
 * rows: optional list of n_rows query rows (NULL means rows 0..n-1, and
 * n_rows must equal n).  Output row r describes query rows[r].
 * bf16 != 0 rounds every coordinate to bfloat16 (RNE) first: the exact
 * result on the rounded points, i.e. what a BF16 candidate stage targets. */
static int knn_impl(const float* X, int64_t n, int32_t d, int32_t k, const int64_t* rows, int64_t n_rows,
                    int bf16, int32_t* nbr_idx, double* nbr_d2) {
  if (!X || !nbr_idx || !nbr_d2 || n < 2 || d < 1 || k < 1 || k >= n || n_rows < 0) return -1;
  if (!rows && n_rows != n) return -1;
  double* Xd = (double*)malloc(sizeof(double) * (size_t)n * (size_t)d);
  if (!Xd) return -2;
  for (int64_t t = 0; t < n * (int64_t)d; ++t) Xd[t] = bf16 ? bf16_rne(X[t]) : (double)X[t];
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t r = 0; r < n_rows; ++r) {
    int64_t q = rows ? rows[r] : r;
    if (q < 0 || q >= n) { bad = 1; continue; }
    int32_t* bj = nbr_idx + r * (int64_t)k;
    double* bd = nbr_d2 + r * (int64_t)k;
    int32_t cnt = 0;
    const double* xq = Xd + q * (int64_t)d;
    for (int64_t j = 0; j < n; ++j) {
      if (j == q) continue;
      const double* xj = Xd + j * (int64_t)d;
      double s = 0.0;
      for (int32_t c = 0; c < d; ++c) {
        double t = xq[c] - xj[c];
        s += t * t;
      }
      if (cnt == k && !key_less(s, j, bd[k - 1], bj[k - 1])) continue;
      /* insertion into the sorted list */
      int32_t p = cnt < k ? cnt : k - 1;
      while (p > 0 && key_less(s, j, bd[p - 1], bj[p - 1])) {
        bd[p] = bd[p - 1];
        bj[p] = bj[p - 1];
        --p;
      }
      bd[p] = s;
      bj[p] = (int32_t)j;
      if (cnt < k) ++cnt;
    }
  }
  free(Xd);
  return bad ? -1 : 0;
}

int oracle_knn(const float* X, int64_t n, int32_t d, int32_t k, const int64_t* rows, int64_t n_rows,
               int32_t* nbr_idx, double* nbr_d2) {
  return knn_impl(X, n, d, k, rows, n_rows, 0, nbr_idx, nbr_d2);
}

int oracle_knn_bf16_points(const float* X, int64_t n, int32_t d, int32_t k, const int64_t* rows, int64_t n_rows,
                           int32_t* nbr_idx, double* nbr_d2) {
  return knn_impl(X, n, d, k, rows, n_rows, 1, nbr_idx, nbr_d2);
}

/* Squared distances of given (query, candidate) pairs, FP64 direct
 * differences: out[t] = sum_c (x[qi[t]][c] - x[cj[t]][c])^2. */
int oracle_pair_d2(const float* X, int64_t n, int32_t d, const int64_t* qi, const int64_t* cj, int64_t m, double* out) {
  if (!X || !qi || !cj || !out || d < 1) return -1;
  int bad = 0;
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < m; ++t) {
    if (qi[t] < 0 || qi[t] >= n || cj[t] < 0 || cj[t] >= n) { bad = 1; continue; }
    const float* a = X + qi[t] * (int64_t)d;
    const float* b = X + cj[t] * (int64_t)d;
    double s = 0.0;
    for (int32_t c = 0; c < d; ++c) {
      double u = (double)a[c] - (double)b[c];
      s += u * u;
    }
    out[t] = s;
  }
  return bad ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* Perplexity calibration [vdMH08 eq. 1 and eq. 3], per row i over its k
 * neighbours.  With s_j = d_ij - min_l d_il (a shift that cancels in the
 * normalisation), p_j(beta) = exp(-beta s_j) / sum_l exp(-beta s_l), with
 * beta = 1/(2 sigma_i^2).  Its Shannon entropy in nats is
 *   H(beta) = ln sum_l exp(-beta s_l) + beta * sum_j p_j s_j,
 * and perplexity 2^{H_bits} = e^{H_nats}, so the target is H* = ln(perp).
 * H is non-increasing in beta, so beta is found by bisection: start at
 * beta = 1 with bracket (0, inf); when H > H* the kernel is too wide, so
 * raise the lower end and double beta (or bisect once the upper end is
 * finite); otherwise lower the upper end and bisect.  Stop when
 * |H - H*| < tol or after max_iter evaluations (converged = 0). */
int oracle_calibrate(const double* nbr_d2, int64_t n, int32_t k, double perplexity, double tol, int32_t max_iter,
                     double* P_cond, double* beta_out, uint8_t* converged, double* H_out) {
  if (!nbr_d2 || !P_cond || n < 1 || k < 1 || !(perplexity > 0) || !(tol > 0) || max_iter < 1) return -1;
  const double Hstar = log(perplexity);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    const double* d = nbr_d2 + i * (int64_t)k;
    double* p = P_cond + i * (int64_t)k;
    double dmin = d[0];
    for (int32_t j = 1; j < k; ++j)
      if (d[j] < dmin) dmin = d[j];
    double beta = 1.0, lo = 0.0, hi = INFINITY, H = 0.0;
    int ok = 0;
    for (int32_t it = 0; it < max_iter; ++it) {
      double S = 0.0, M = 0.0;
      for (int32_t j = 0; j < k; ++j) {
        double s = d[j] - dmin;
        double e = exp(-beta * s);
        p[j] = e;
        S += e;
        M += e * s;
      }
      H = log(S) + beta * M / S;
      for (int32_t j = 0; j < k; ++j) p[j] /= S;
      if (fabs(H - Hstar) < tol) { ok = 1; break; }
      if (it == max_iter - 1) break;
      if (H > Hstar) {
        lo = beta;
        beta = isinf(hi) ? beta * 2.0 : 0.5 * (beta + hi);
      } else {
        hi = beta;
        beta = 0.5 * (lo + beta);
      }
    }
    if (beta_out) beta_out[i] = beta;
    if (converged) converged[i] = (uint8_t)ok;
    if (H_out) H_out[i] = H;
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Symmetrisation [vdMH08 Sec. 3.1] on the kNN pattern [vdM14 Sec. 4.1]:
 * with C_ij = p_{j|i} for j in N(i) and 0 otherwise,
 *   P = (C + C^T) / (2n),
 * stored as CSR over the union pattern, columns ascending, no diagonal.
 * tpos[e] is the position of entry (j, i) for entry e = (i, j); it exists
 * because the pattern is symmetric.  Capacity of col/val/tpos: 2 n k.
 * Returns -3 if a neighbour list holds self, a repeat or an out-of-range
 * index. */
typedef struct { int32_t c; double v; } cv_t;
static int cv_cmp(const void* a, const void* b) {
  int32_t x = ((const cv_t*)a)->c, y = ((const cv_t*)b)->c;
  return (x > y) - (x < y);
}

int oracle_symmetrize(const int32_t* nbr_idx, const double* P_cond, int64_t n, int32_t k, int64_t* row_ptr,
                      int32_t* col, double* val, int32_t* tpos, int64_t* nnz_out) {
  if (!nbr_idx || !P_cond || !row_ptr || !col || !val || n < 2 || k < 1 || k >= n) return -1;
  int64_t nk = n * (int64_t)k;
  for (int64_t t = 0; t < nk; ++t)
    if (nbr_idx[t] < 0 || nbr_idx[t] >= n) return -3;
  /* transposed lists, filled sequentially in source order */
  int64_t* in_ptr = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  int64_t* fill = (int64_t*)calloc((size_t)n, sizeof(int64_t));
  cv_t* in = (cv_t*)malloc(sizeof(cv_t) * (size_t)nk);
  cv_t* uni = (cv_t*)malloc(sizeof(cv_t) * (size_t)(2 * nk));
  int64_t* ucnt = (int64_t*)calloc((size_t)n, sizeof(int64_t));
  if (!in_ptr || !fill || !in || !uni || !ucnt) {
    free(in_ptr); free(fill); free(in); free(uni); free(ucnt);
    return -2;
  }
  for (int64_t t = 0; t < nk; ++t) in_ptr[nbr_idx[t] + 1]++;
  for (int64_t i = 0; i < n; ++i) in_ptr[i + 1] += in_ptr[i];
  for (int64_t i = 0; i < n; ++i)
    for (int32_t a = 0; a < k; ++a) {
      int32_t j = nbr_idx[i * (int64_t)k + a];
      cv_t e = {(int32_t)i, P_cond[i * (int64_t)k + a]};
      in[in_ptr[j] + fill[j]++] = e;
    }
  int bad = 0;
  const double two_n = 2.0 * (double)n;
  /* union of out-list and in-list per row; row i's union lives at
   * uni[in_ptr[i] + i*k ...] which has room for k + indegree(i) entries */
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    cv_t* out = (cv_t*)malloc(sizeof(cv_t) * (size_t)k);
    if (!out) { bad = 2; continue; }
    for (int32_t a = 0; a < k; ++a) {
      out[a].c = nbr_idx[i * (int64_t)k + a];
      out[a].v = P_cond[i * (int64_t)k + a];
    }
    qsort(out, (size_t)k, sizeof(cv_t), cv_cmp);
    for (int32_t a = 0; a < k; ++a)
      if (out[a].c == i || (a > 0 && out[a].c == out[a - 1].c)) bad = 3;
    const cv_t* inl = in + in_ptr[i];
    int64_t m = in_ptr[i + 1] - in_ptr[i];
    cv_t* u = uni + in_ptr[i] + i * (int64_t)k;
    int64_t a = 0, b = 0, c = 0;
    while (a < k || b < m) {
      if (b == m || (a < k && out[a].c < inl[b].c)) {
        u[c].c = out[a].c; u[c].v = (out[a].v + 0.0) / two_n; ++a;
      } else if (a == k || inl[b].c < out[a].c) {
        u[c].c = inl[b].c; u[c].v = (0.0 + inl[b].v) / two_n; ++b;
      } else {
        u[c].c = out[a].c; u[c].v = (out[a].v + inl[b].v) / two_n; ++a; ++b;
      }
      ++c;
    }
    ucnt[i] = c;
    free(out);
  }
  if (bad) {
    free(in_ptr); free(fill); free(in); free(uni); free(ucnt);
    return bad == 3 ? -3 : -2;
  }
  row_ptr[0] = 0;
  for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + ucnt[i];
  for (int64_t i = 0; i < n; ++i) {
    const cv_t* u = uni + in_ptr[i] + i * (int64_t)k;
    for (int64_t c = 0; c < ucnt[i]; ++c) {
      col[row_ptr[i] + c] = u[c].c;
      val[row_ptr[i] + c] = u[c].v;
    }
  }
  if (tpos) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i)
      for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        int32_t j = col[e];
        int64_t lo = row_ptr[j], hi = row_ptr[j + 1];
        while (lo < hi) {
          int64_t mid = lo + (hi - lo) / 2;
          if (col[mid] < i) lo = mid + 1; else hi = mid;
        }
        tpos[e] = (int32_t)lo;
      }
  }
  if (nnz_out) *nnz_out = row_ptr[n];
  free(in_ptr); free(fill); free(in); free(uni); free(ucnt);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Student-t similarity in the 2-D map [vdMH08 eq. 4]:
 * w_ij = 1 / (1 + ||y_i - y_j||^2); q_ij = w_ij / Z with
 * Z = sum over ordered pairs i != j of w_ij. */
static double w_of(const double* Y, int64_t i, int64_t j) {
  double dx = Y[2 * i] - Y[2 * j];
  double dy = Y[2 * i + 1] - Y[2 * j + 1];
  return 1.0 / (1.0 + dx * dx + dy * dy);
}

static double Z_of(const double* Y, int64_t n, double* Zrow) {
  double* zr = Zrow ? Zrow : (double*)malloc(sizeof(double) * (size_t)n);
  if (!zr) return NAN;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    nsum_t a = {0, 0};
    for (int64_t j = 0; j < n; ++j)
      if (j != i) nsum_add(&a, w_of(Y, i, j));
    zr[i] = nsum_get(&a);
  }
  nsum_t z = {0, 0};
  for (int64_t i = 0; i < n; ++i) nsum_add(&z, zr[i]);
  if (!Zrow) free(zr);
  return nsum_get(&z);
}

/* The t-SNE gradient with early exaggeration alpha [vdMH08 eq. 5 and
 * Sec. 3.4]: for symmetric P,
 *   g_i = 4 sum_{j != i} (alpha p_ij - q_ij) w_ij (y_i - y_j),
 * with p_ij read from row i of the CSR (0 where not stored).  This is the
 * derivative of C_alpha = -alpha sum_e p_e ln w_e + ln Z, which for
 * alpha = 1 and sum P = 1 differs from KL(P||Q) by a constant.
 * Also returns Z and KL(P||Q) = sum_e p_e ln(p_e / q_e)
 *   = sum_e p_e ln p_e - sum_e p_e ln w_e + S ln Z,  S = sum_e p_e,
 * which always uses the stored, un-exaggerated P (0 ln 0 := 0).
 * Y is [n][2]; grad is [n][2]. */
int oracle_kl_grad(const double* Y, int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
                   double alpha, double* grad, double* Z_out, double* kl_out) {
  if (!Y || n < 2 || !row_ptr || !col || !val) return -1;
  double Z = Z_of(Y, n, NULL);
  if (grad) {
    int bad = 0;
#pragma omp parallel
    {
      double* prow = (double*)calloc((size_t)n, sizeof(double));
      if (!prow) bad = 1;
#pragma omp for schedule(dynamic, 16)
      for (int64_t i = 0; i < n; ++i) {
        if (!prow) continue;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) prow[col[e]] = val[e];
        double gx = 0.0, gy = 0.0;
        for (int64_t j = 0; j < n; ++j) {
          if (j == i) continue;
          double w = w_of(Y, i, j);
          double coef = (alpha * prow[j] - w / Z) * w;
          gx += coef * (Y[2 * i] - Y[2 * j]);
          gy += coef * (Y[2 * i + 1] - Y[2 * j + 1]);
        }
        grad[2 * i] = 4.0 * gx;
        grad[2 * i + 1] = 4.0 * gy;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) prow[col[e]] = 0.0;
      }
      free(prow);
    }
    if (bad) return -2;
  }
  if (kl_out) {
    nsum_t plogp = {0, 0}, plogw = {0, 0}, S = {0, 0};
    for (int64_t i = 0; i < n; ++i)
      for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        double p = val[e];
        if (p > 0) nsum_add(&plogp, p * log(p));
        nsum_add(&plogw, p * log(w_of(Y, i, col[e])));
        nsum_add(&S, p);
      }
    *kl_out = nsum_get(&plogp) - nsum_get(&plogw) + nsum_get(&S) * log(Z);
  }
  if (Z_out) *Z_out = Z;
  return 0;
}

/* Per-row parts of the gradient for a subset of rows, each O(n):
 *   Zrow[r] = sum_{j != i} w_ij,
 *   Rrow[r] = sum_{j != i} w_ij^2 (y_i - y_j)        (repulsion numerator),
 *   Arow[r] = sum_{e in row i} p_e w_e (y_i - y_col(e)) (attraction),
 * for i = rows[r].  Then g_i = 4 (alpha A_i - R_i / Z), Z = sum_i Z_i. */
int oracle_grad_rows(const double* Y, int64_t n, const int64_t* rows, int64_t n_rows, const int64_t* row_ptr,
                     const int32_t* col, const double* val, double* Zrow, double* Rrow, double* Arow) {
  if (!Y || n < 2 || !rows || n_rows < 0) return -1;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t r = 0; r < n_rows; ++r) {
    int64_t i = rows[r];
    if (i < 0 || i >= n) { bad = 1; continue; }
    nsum_t z = {0, 0};
    double rx = 0.0, ry = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double w = w_of(Y, i, j);
      nsum_add(&z, w);
      rx += w * w * (Y[2 * i] - Y[2 * j]);
      ry += w * w * (Y[2 * i + 1] - Y[2 * j + 1]);
    }
    if (Zrow) Zrow[r] = nsum_get(&z);
    if (Rrow) { Rrow[2 * r] = rx; Rrow[2 * r + 1] = ry; }
    if (Arow) {
      double ax = 0.0, ay = 0.0;
      if (row_ptr && col && val)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
          int64_t j = col[e];
          double pw = val[e] * w_of(Y, i, j);
          ax += pw * (Y[2 * i] - Y[2 * j]);
          ay += pw * (Y[2 * i + 1] - Y[2 * j + 1]);
        }
      Arow[2 * r] = ax;
      Arow[2 * r + 1] = ay;
    }
  }
  return bad ? -1 : 0;
}

/* Per-row, per-coordinate magnitude of the terms that make up the parts
 * above (the scale of their rounding error in any summation order), for
 * i = rows[r] and coordinate c in {x, y}:
 *   Rabs[r][c] = sum_{j != i} w_ij^2 |y_ic - y_jc|,
 *   Aabs[r][c] = sum_{e in row i} |p_e| w_e |y_ic - y_col(e),c|.
 * |R_i,c| <= Rabs[r][c] and |A_i,c| <= Aabs[r][c], with equality when every
 * term has the same sign. */
int oracle_grad_rows_scale(const double* Y, int64_t n, const int64_t* rows, int64_t n_rows, const int64_t* row_ptr,
                           const int32_t* col, const double* val, double* Rabs, double* Aabs) {
  if (!Y || n < 2 || !rows || n_rows < 0 || !Rabs || !Aabs) return -1;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t r = 0; r < n_rows; ++r) {
    int64_t i = rows[r];
    if (i < 0 || i >= n) { bad = 1; continue; }
    double rx = 0.0, ry = 0.0, ax = 0.0, ay = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double w = w_of(Y, i, j);
      rx += w * w * fabs(Y[2 * i] - Y[2 * j]);
      ry += w * w * fabs(Y[2 * i + 1] - Y[2 * j + 1]);
    }
    if (row_ptr && col && val)
      for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        int64_t j = col[e];
        double pw = fabs(val[e]) * w_of(Y, i, j);
        ax += pw * fabs(Y[2 * i] - Y[2 * j]);
        ay += pw * fabs(Y[2 * i + 1] - Y[2 * j + 1]);
      }
    Rabs[2 * r] = rx;
    Rabs[2 * r + 1] = ry;
    Aabs[2 * r] = ax;
    Aabs[2 * r + 1] = ay;
  }
  return bad ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* KL(P||Q) as a function of Y and of the stored values p_e, for the
 * differentiation form.  P need not be symmetric nor sum to one:
 *   C = sum_e p_e ln p_e - sum_e p_e ln w_e + S ln Z,  S = sum_e p_e.
 * Its exact derivatives:
 *   dC/dy_i = 2 sum_{e=(i,b)} p_e w_e (y_i - y_b) + 2 sum_{e=(a,i)} p_e w_e (y_i - y_a)
 *             - (4 S / Z) sum_{j != i} w_ij^2 (y_i - y_j),
 *   dC/dp_e = 1 + ln p_e - ln w_e + ln Z  (stored entries only).
 * The backward scales both by the incoming gradient gC. */
int oracle_kl(const double* Y, int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val, double* C_out,
              double* Z_out) {
  return oracle_kl_grad(Y, n, row_ptr, col, val, 1.0, NULL, Z_out, C_out);
}

int oracle_kl_backward(const double* Y, int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
                       double gC, double* dY, double* dP) {
  if (!Y || n < 2 || !row_ptr || !col || !val) return -1;
  double Z = Z_of(Y, n, NULL);
  nsum_t Sacc = {0, 0};
  int64_t nnz = row_ptr[n];
  for (int64_t e = 0; e < nnz; ++e) nsum_add(&Sacc, val[e]);
  double S = nsum_get(&Sacc);
  if (dY) {
    /* repulsion term per row */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
      double rx = 0.0, ry = 0.0;
      for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double w = w_of(Y, i, j);
        rx += w * w * (Y[2 * i] - Y[2 * j]);
        ry += w * w * (Y[2 * i + 1] - Y[2 * j + 1]);
      }
      dY[2 * i] = -(4.0 * S / Z) * rx;
      dY[2 * i + 1] = -(4.0 * S / Z) * ry;
    }
    /* attraction: each stored entry (a, b) pulls on both endpoints */
    for (int64_t a = 0; a < n; ++a)
      for (int64_t e = row_ptr[a]; e < row_ptr[a + 1]; ++e) {
        int64_t b = col[e];
        double pw2 = 2.0 * val[e] * w_of(Y, a, b);
        double dx = Y[2 * a] - Y[2 * b], dy = Y[2 * a + 1] - Y[2 * b + 1];
        dY[2 * a] += pw2 * dx;
        dY[2 * a + 1] += pw2 * dy;
        dY[2 * b] -= pw2 * dx;
        dY[2 * b + 1] -= pw2 * dy;
      }
    for (int64_t t = 0; t < 2 * n; ++t) dY[t] *= gC;
  }
  if (dP) {
    double lnZ = log(Z);
    for (int64_t a = 0; a < n; ++a)
      for (int64_t e = row_ptr[a]; e < row_ptr[a + 1]; ++e)
        dP[e] = gC * (1.0 + log(val[e]) - log(w_of(Y, a, col[e])) + lnZ);
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* One optimiser step: gradient descent with momentum [vdMH08 Algorithm 1]
 * and per-coordinate adaptive gains [Jac88], elementwise over the 2n
 * coordinates:
 *   gain <- gain + inc   if grad * update < 0   (the step keeps its sign)
 *   gain <- gain * dec   otherwise,
 *   gain <- max(gain, min_gain),
 *   update <- momentum * update - lr * gain * grad,
 *   y <- y + update. */
int oracle_step(double* Y, double* update, double* gains, const double* grad, int64_t n, double lr, double momentum,
                double gain_inc, double gain_dec, double min_gain) {
  if (!Y || !update || !gains || !grad || n < 1) return -1;
  for (int64_t t = 0; t < 2 * n; ++t) {
    double g = gains[t];
    if (grad[t] * update[t] < 0.0) g = g + gain_inc;
    else g = g * gain_dec;
    if (g < min_gain) g = min_gain;
    gains[t] = g;
    update[t] = momentum * update[t] - lr * g * grad[t];
    Y[t] = Y[t] + update[t];
  }
  return 0;
}
