/*
 * FP64 reference (oracle) for nonnegative Tucker + nonnegative CP of the core + lift,
 * i.e. the nnCANDELINC procedure "nnTD then nnCPD on the core" (Section 4.1, Algorithm 1).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call this code: it exists so
 * that tests, the smoke check and the benchmark's CPU baseline can compare the GPU library
 * against a plain, slow, obviously correct computation.  It shares no code with the GPU
 * library.
 *
 * Every quantity is computed from its definition with nested loops in double precision:
 *   - n-mode product (Appendix A, definition of n-mode multiplication):
 *       (X x_n M)[..., i, ...] = sum_l X[..., l, ...] * M[i, l],   M has dims[n] columns;
 *   - Tucker model G x_1 F1 x_2 F2 ... (Section 2, Tucker decomposition in matrix format);
 *   - CP model sum_rho outer(C1[:,rho], ..., Cd[:,rho]) (Section 2, CPD in matrix format);
 *   - relative error ||X - Xhat||_F / ||X||_F (Section 4.1, scoring);
 *   - the lift C_n = F_n B_n obtained by substituting a CPD of the core into the Tucker
 *     model (Section 2.1, proof of the rank/minimal-Tucker lemma; Section 2.2).
 * The multiplicative-update rules are not printed in the paper (it calls library solvers,
 * Section 4.1); the oracle uses Lee-Seung Frobenius multiplicative updates applied block by
 * block (factors 1..d in order, then the core), each block an NMF least-squares subproblem:
 *   factor n:  A_n <- A_n * num_n / max(den_n, eps)
 *       num_n = unfold_n(X x_{k!=n} A_k^T) unfold_n(G)^T
 *       den_n = A_n unfold_n(G x_{k!=n} (A_k^T A_k)) unfold_n(G)^T
 *   core:      G <- G * num_G / max(den_G, eps)
 *       num_G = X x_1 A_1^T ... x_d A_d^T,   den_G = G x_1 (A_1^T A_1) ... x_d (A_d^T A_d)
 *   nnCP of the core, factor n:  B_n <- B_n * M_n / max(B_n H_n, eps)
 *       M_n[i,rho] = sum over core entries with i_n = i of G[idx] prod_{k!=n} B_k[i_k,rho]
 *       H_n = Hadamard product over k!=n of B_k^T B_k
 * Each update is (x * num) / max(den, eps) evaluated in double precision.
 *
 * All tensors are row-major (last index fastest).  Reductions over many elements are
 * summed in fixed 4096-element chunks and then over chunks in order, so results do not
 * depend on the number of OpenMP threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_CHUNK 4096
#define ORC_MAXD 8

static int64_t prod_range(const int64_t *a, int lo, int hi) {
  int64_t p = 1;
  for (int k = lo; k < hi; ++k) p *= a[k];
  return p;
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* n-mode product by definition: out = X x_n M, M is rows x dims[n] (row-major).
 * out has the shape of X with dims[n] replaced by rows. */
void orc_nmode(int d, const int64_t *dims, const double *X, int n, const double *M,
               int64_t rows, double *out) {
  const int64_t pre = prod_range(dims, 0, n);
  const int64_t N = dims[n];
  const int64_t post = prod_range(dims, n + 1, d);
  if (post == 1) {
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < pre; ++p) {
      const double *x = X + p * N;
      for (int64_t i = 0; i < rows; ++i) {
        double s = 0.0;
        for (int64_t l = 0; l < N; ++l) s += x[l] * M[i * N + l];
        out[p * rows + i] = s;
      }
    }
    return;
  }
  const int64_t B = 256;
  const int64_t nb = (post + B - 1) / B;
#pragma omp parallel for collapse(2) schedule(static)
  for (int64_t p = 0; p < pre; ++p) {
    for (int64_t b = 0; b < nb; ++b) {
      const int64_t q0 = b * B;
      const int64_t q1 = q0 + B < post ? q0 + B : post;
      double *o = out + p * rows * post;
      for (int64_t i = 0; i < rows; ++i)
        for (int64_t q = q0; q < q1; ++q) o[i * post + q] = 0.0;
      /* each output element accumulates l = 0, 1, ..., N-1 in order */
      for (int64_t l = 0; l < N; ++l) {
        const double *x = X + (p * N + l) * post;
        for (int64_t i = 0; i < rows; ++i) {
          const double m = M[i * N + l];
          for (int64_t q = q0; q < q1; ++q) o[i * post + q] += x[q] * m;
        }
      }
    }
  }
}

static void transpose(const double *A, int64_t r, int64_t c, double *At) {
  for (int64_t i = 0; i < r; ++i)
    for (int64_t j = 0; j < c; ++j) At[j * r + i] = A[i * c + j];
}

/* X x_n A^T for a factor A (dims[n] x R): out[.., r, ..] = sum_l X[.., l, ..] A[l, r]. */
void orc_ttm_t(int d, const int64_t *dims, const double *X, int n, const double *A, int64_t R,
               double *out) {
  double *At = (double *)malloc(sizeof(double) * (size_t)(R * dims[n]));
  transpose(A, dims[n], R, At);
  orc_nmode(d, dims, X, n, At, R, out);
  free(At);
}

/* Chain of n-mode products with transposed factors over every mode k != skip, in order
 * k = 0, 1, ..., d-1 (skip = -1: all modes).  mats[k] is dims[k] x ranks[k].
 * Returns a malloc'd tensor; outdims receives its shape. */
static double *chain_ttm_t(int d, const int64_t *dims, const double *X, double *const *mats,
                           const int64_t *ranks, int skip, int64_t *outdims) {
  int64_t cur[ORC_MAXD];
  memcpy(cur, dims, sizeof(int64_t) * d);
  const double *src = X; /* not owned until the first product */
  double *owned = NULL;
  for (int k = 0; k < d; ++k) {
    if (k == skip) continue;
    int64_t nd[ORC_MAXD];
    memcpy(nd, cur, sizeof(int64_t) * d);
    nd[k] = ranks[k];
    double *dst = (double *)malloc(sizeof(double) * (size_t)prod_range(nd, 0, d));
    orc_ttm_t(d, cur, src, k, mats[k], ranks[k], dst);
    free(owned);
    owned = dst;
    src = dst;
    memcpy(cur, nd, sizeof(int64_t) * d);
  }
  if (!owned) { /* no mode contracted: return a copy */
    const int64_t n0 = prod_range(cur, 0, d);
    owned = (double *)malloc(sizeof(double) * (size_t)n0);
    memcpy(owned, X, sizeof(double) * (size_t)n0);
  }
  memcpy(outdims, cur, sizeof(int64_t) * d);
  return owned;
}

/* out[i, j] = sum over all indices except mode n of U[.., i, ..] V[.., j, ..].
 * U has shape udims, V has shape vdims; they agree except in mode n. */
void orc_contract_except(int d, const int64_t *udims, const double *U, const int64_t *vdims,
                         const double *V, int n, double *out) {
  const int64_t pre = prod_range(udims, 0, n);
  const int64_t post = prod_range(udims, n + 1, d);
  const int64_t I = udims[n], J = vdims[n];
#pragma omp parallel for collapse(2) schedule(static)
  for (int64_t i = 0; i < I; ++i) {
    for (int64_t j = 0; j < J; ++j) {
      double s = 0.0;
      for (int64_t p = 0; p < pre; ++p)
        for (int64_t q = 0; q < post; ++q)
          s += U[(p * I + i) * post + q] * V[(p * J + j) * post + q];
      out[i * J + j] = s;
    }
  }
}

/* Gram matrix S = A^T A of an N x R matrix. */
void orc_gram(const double *A, int64_t N, int64_t R, double *S) {
  for (int64_t r = 0; r < R; ++r)
    for (int64_t s = 0; s < R; ++s) {
      double acc = 0.0;
      for (int64_t i = 0; i < N; ++i) acc += A[i * R + r] * A[i * R + s];
      S[r * R + s] = acc;
    }
}

/* C = A B with A (n x k), B (k x m). */
void orc_matmul(const double *A, const double *B, int64_t n, int64_t k, int64_t m, double *C) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < m; ++j) {
      double s = 0.0;
      for (int64_t l = 0; l < k; ++l) s += A[i * k + l] * B[l * m + j];
      C[i * m + j] = s;
    }
}

/* sum of squares of a - b (b may be NULL: sum of squares of a), chunked for determinism. */
static double sumsq_diff(const double *a, const double *b, int64_t n) {
  const int64_t nc = (n + ORC_CHUNK - 1) / ORC_CHUNK;
  double *part = (double *)malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nc; ++c) {
    const int64_t lo = c * ORC_CHUNK, hi = lo + ORC_CHUNK < n ? lo + ORC_CHUNK : n;
    double s = 0.0;
    for (int64_t e = lo; e < hi; ++e) {
      const double t = b ? a[e] - b[e] : a[e];
      s += t * t;
    }
    part[c] = s;
  }
  double s = 0.0;
  for (int64_t c = 0; c < nc; ++c) s += part[c];
  free(part);
  return s;
}

/* Tucker reconstruction Xhat = G x_1 A_1 x_2 A_2 ... x_d A_d (A_n is dims[n] x ranks[n]). */
void orc_tucker_full(int d, const int64_t *dims, const int64_t *ranks, const double *G,
                     double *const *A, double *Xhat) {
  int64_t cur[ORC_MAXD];
  memcpy(cur, ranks, sizeof(int64_t) * d);
  double *src = (double *)malloc(sizeof(double) * (size_t)prod_range(cur, 0, d));
  memcpy(src, G, sizeof(double) * (size_t)prod_range(cur, 0, d));
  for (int k = 0; k < d; ++k) {
    int64_t nd[ORC_MAXD];
    memcpy(nd, cur, sizeof(int64_t) * d);
    nd[k] = dims[k];
    double *dst = (double *)malloc(sizeof(double) * (size_t)prod_range(nd, 0, d));
    orc_nmode(d, cur, src, k, A[k], dims[k], dst);
    free(src);
    src = dst;
    memcpy(cur, nd, sizeof(int64_t) * d);
  }
  memcpy(Xhat, src, sizeof(double) * (size_t)prod_range(dims, 0, d));
  free(src);
}

/* CP reconstruction xhat[idx] = sum_rho prod_n C_n[i_n, rho] (C_n is dims[n] x r). */
void orc_cp_full(int d, const int64_t *dims, int64_t r, double *const *C, double *Xhat) {
  const int64_t total = prod_range(dims, 0, d);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < total; ++e) {
    int64_t idx[ORC_MAXD];
    int64_t rem = e;
    for (int k = d - 1; k >= 0; --k) {
      idx[k] = rem % dims[k];
      rem /= dims[k];
    }
    double s = 0.0;
    for (int64_t rho = 0; rho < r; ++rho) {
      double p = 1.0;
      for (int k = 0; k < d; ++k) p *= C[k][idx[k] * r + rho];
      s += p;
    }
    Xhat[e] = s;
  }
}

double orc_sumsq(const double *X, int64_t n) { return sumsq_diff(X, NULL, n); }

/* ||X - G x {A}||_F^2 */
double orc_tucker_sq_residual(int d, const int64_t *dims, const double *X, const int64_t *ranks,
                              const double *G, double *const *A) {
  const int64_t total = prod_range(dims, 0, d);
  double *Xh = (double *)malloc(sizeof(double) * (size_t)total);
  orc_tucker_full(d, dims, ranks, G, A, Xh);
  const double s = sumsq_diff(X, Xh, total);
  free(Xh);
  return s;
}

/* ||X - cp(C)||_F^2 */
double orc_cp_sq_residual(int d, const int64_t *dims, const double *X, int64_t r, double *const *C) {
  const int64_t total = prod_range(dims, 0, d);
  double *Xh = (double *)malloc(sizeof(double) * (size_t)total);
  orc_cp_full(d, dims, r, C, Xh);
  const double s = sumsq_diff(X, Xh, total);
  free(Xh);
  return s;
}

/* One multiplicative-update block: x <- (x * num) / max(den, eps). Returns clip count. */
static long long mu_apply(double *x, const double *num, const double *den, int64_t n, double eps) {
  long long clips = 0;
  for (int64_t e = 0; e < n; ++e) {
    double dn = den[e];
    if (dn < eps) {
      dn = eps;
      ++clips;
    }
    x[e] = (x[e] * num[e]) / dn;
  }
  return clips;
}

/* Numerator and denominator of the factor-n block at the current point:
 *   num = unfold_n(X x_{k!=n} A_k^T) unfold_n(G)^T
 *   den = A_n unfold_n(G x_{k!=n} S_k) unfold_n(G)^T      (S_k = A_k^T A_k, symmetric)
 * num and den are dims[n] x R[n]. */
static void factor_numden(int d, const int64_t *dims, const double *X, const int64_t *R,
                          const double *G, double *const *A, double *const *S, int n,
                          double *num, double *den) {
  int64_t ydims[ORC_MAXD], hdims[ORC_MAXD];
  double *Y = chain_ttm_t(d, dims, X, A, R, n, ydims);
  orc_contract_except(d, ydims, Y, R, G, n, num);
  free(Y);
  double *H = chain_ttm_t(d, R, G, S, R, n, hdims);
  double *Mn = (double *)malloc(sizeof(double) * (size_t)(R[n] * R[n]));
  orc_contract_except(d, hdims, H, R, G, n, Mn);
  free(H);
  orc_matmul(A[n], Mn, dims[n], R[n], R[n], den);
  free(Mn);
}

/* Numerator and denominator of the core block: num_G = X x_k A_k^T, den_G = G x_k S_k. */
static void core_numden(int d, const int64_t *dims, const double *X, const int64_t *R,
                        const double *G, double *const *A, double *const *S, double *num,
                        double *den) {
  int64_t odims[ORC_MAXD];
  const int64_t gsz = prod_range(R, 0, d);
  double *a = chain_ttm_t(d, dims, X, A, R, -1, odims);
  double *b = chain_ttm_t(d, R, G, S, R, -1, odims);
  memcpy(num, a, sizeof(double) * (size_t)gsz);
  memcpy(den, b, sizeof(double) * (size_t)gsz);
  free(a);
  free(b);
}

/* All block numerators/denominators at one fixed point (no update).  Their differences
 * den - num are the gradient of 0.5 ||X - G x {A}||^2 with respect to each block. */
void orc_tucker_numden(int d, const int64_t *dims, const double *X, const int64_t *R,
                       const double *G, double *const *A, double *const *num,
                       double *const *den, double *numG, double *denG) {
  double *S[ORC_MAXD] = {0};
  for (int k = 0; k < d; ++k) {
    S[k] = (double *)malloc(sizeof(double) * (size_t)(R[k] * R[k]));
    orc_gram(A[k], dims[k], R[k], S[k]);
  }
  for (int n = 0; n < d; ++n) factor_numden(d, dims, X, R, G, A, S, n, num[n], den[n]);
  core_numden(d, dims, X, R, G, A, S, numG, denG);
  for (int k = 0; k < d; ++k) free(S[k]);
}

/* One nnTucker multiplicative-update sweep: factors 1..d in order, then the core. */
static long long nntucker_sweep(int d, const int64_t *dims, const double *X, const int64_t *R,
                                double eps, double *G, double *const *A) {
  long long clips = 0;
  double *S[ORC_MAXD] = {0};
  for (int k = 0; k < d; ++k) {
    S[k] = (double *)malloc(sizeof(double) * (size_t)(R[k] * R[k]));
    orc_gram(A[k], dims[k], R[k], S[k]);
  }
  for (int n = 0; n < d; ++n) {
    double *num = (double *)malloc(sizeof(double) * (size_t)(dims[n] * R[n]));
    double *den = (double *)malloc(sizeof(double) * (size_t)(dims[n] * R[n]));
    factor_numden(d, dims, X, R, G, A, S, n, num, den);
    clips += mu_apply(A[n], num, den, dims[n] * R[n], eps);
    free(num);
    free(den);
    orc_gram(A[n], dims[n], R[n], S[n]); /* Gauss-Seidel: later blocks see the new A_n */
  }
  const int64_t gsz = prod_range(R, 0, d);
  double *numG = (double *)malloc(sizeof(double) * (size_t)gsz);
  double *denG = (double *)malloc(sizeof(double) * (size_t)gsz);
  core_numden(d, dims, X, R, G, A, S, numG, denG);
  clips += mu_apply(G, numG, denG, gsz, eps);
  free(numG);
  free(denG);
  for (int k = 0; k < d; ++k) free(S[k]);
  return clips;
}

/* nnTucker by multiplicative updates for exactly `iters` sweeps, in place on G and A.
 * fhist (nullable) receives 0.5 ||X - G x {A}||^2 after each sweep. Returns clip count. */
long long orc_nntucker(int d, const int64_t *dims, const double *X, const int64_t *R, int iters,
                       double eps, double *G, double *const *A, double *fhist) {
  long long clips = 0;
  for (int t = 0; t < iters; ++t) {
    clips += nntucker_sweep(d, dims, X, R, eps, G, A);
    if (fhist) fhist[t] = 0.5 * orc_tucker_sq_residual(d, dims, X, R, G, A);
  }
  return clips;
}

/* MTTKRP by definition: M[i, rho] = sum_{idx: i_n = i} T[idx] prod_{k!=n} B_k[i_k, rho]. */
void orc_mttkrp(int d, const int64_t *tdims, const double *T, int n, int64_t r, double *const *B,
                double *M) {
  const int64_t total = prod_range(tdims, 0, d);
  memset(M, 0, sizeof(double) * (size_t)(tdims[n] * r));
  for (int64_t e = 0; e < total; ++e) {
    int64_t idx[ORC_MAXD];
    int64_t rem = e;
    for (int k = d - 1; k >= 0; --k) {
      idx[k] = rem % tdims[k];
      rem /= tdims[k];
    }
    for (int64_t rho = 0; rho < r; ++rho) {
      double p = T[e];
      for (int k = 0; k < d; ++k)
        if (k != n) p *= B[k][idx[k] * r + rho];
      M[idx[n] * r + rho] += p;
    }
  }
}

/* nnCP of a tensor T (here: the Tucker core) by multiplicative updates, in place on B. */
long long orc_nncp(int d, const int64_t *tdims, const double *T, int64_t r, int iters, double eps,
                   double *const *B, double *fhist) {
  long long clips = 0;
  double *W[ORC_MAXD] = {0};
  for (int k = 0; k < d; ++k) {
    W[k] = (double *)malloc(sizeof(double) * (size_t)(r * r));
    orc_gram(B[k], tdims[k], r, W[k]);
  }
  double *H = (double *)malloc(sizeof(double) * (size_t)(r * r));
  for (int t = 0; t < iters; ++t) {
    for (int n = 0; n < d; ++n) {
      double *M = (double *)malloc(sizeof(double) * (size_t)(tdims[n] * r));
      double *den = (double *)malloc(sizeof(double) * (size_t)(tdims[n] * r));
      orc_mttkrp(d, tdims, T, n, r, B, M);
      for (int64_t e = 0; e < r * r; ++e) {
        double h = 1.0;
        for (int k = 0; k < d; ++k)
          if (k != n) h *= W[k][e];
        H[e] = h;
      }
      orc_matmul(B[n], H, tdims[n], r, r, den);
      clips += mu_apply(B[n], M, den, tdims[n] * r, eps);
      orc_gram(B[n], tdims[n], r, W[n]);
      free(M);
      free(den);
    }
    if (fhist) fhist[t] = 0.5 * orc_cp_sq_residual(d, tdims, T, r, B);
  }
  free(H);
  for (int k = 0; k < d; ++k) free(W[k]);
  return clips;
}

/* Lift: C_n = A_n B_n for every mode (A_n: dims[n] x ranks[n], B_n: ranks[n] x r). */
void orc_lift(int d, const int64_t *dims, const int64_t *ranks, int64_t r, double *const *A,
              double *const *B, double *const *C) {
  for (int k = 0; k < d; ++k) orc_matmul(A[k], B[k], dims[k], ranks[k], r, C[k]);
}

/* Gradient of L = 0.5 ||X - G x {A}||^2 from the explicit residual E = X - Xhat:
 *   dL/dA_n = -unfold_n(E x_{k!=n} A_k^T) unfold_n(G)^T,   dL/dG = -E x_1 A_1^T ... x_d A_d^T.
 * Returns L. gA[n] is dims[n] x ranks[n]; gG has the core's shape. */
double orc_tucker_grad(int d, const int64_t *dims, const double *X, const int64_t *R,
                       const double *G, double *const *A, double *gG, double *const *gA) {
  const int64_t total = prod_range(dims, 0, d);
  double *E = (double *)malloc(sizeof(double) * (size_t)total);
  orc_tucker_full(d, dims, R, G, A, E);
  for (int64_t e = 0; e < total; ++e) E[e] = X[e] - E[e];
  const double L = 0.5 * sumsq_diff(E, NULL, total);
  for (int n = 0; n < d; ++n) {
    int64_t ydims[ORC_MAXD];
    double *Y = chain_ttm_t(d, dims, E, A, R, n, ydims);
    orc_contract_except(d, ydims, Y, R, G, n, gA[n]);
    for (int64_t e = 0; e < dims[n] * R[n]; ++e) gA[n][e] = -gA[n][e];
    free(Y);
  }
  int64_t odims[ORC_MAXD];
  double *Z = chain_ttm_t(d, dims, E, A, R, -1, odims);
  const int64_t gsz = prod_range(R, 0, d);
  for (int64_t e = 0; e < gsz; ++e) gG[e] = -Z[e];
  free(Z);
  free(E);
  return L;
}
