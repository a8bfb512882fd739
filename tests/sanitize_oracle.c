/* Driver for the sanitizer run of the FP64 oracle (tests/test_oracle_sanitize.py builds it
 * with oracle/oracle.c under AddressSanitizer and UndefinedBehaviorSanitizer).  It calls
 * every exported routine on small ragged shapes, 2- to 5-way, including a factor with a
 * zero column (the eps-guarded division) and more threads than some loops have work, and
 * checks a few identities so that the calls are not optimised away.  Test infrastructure:
 * nothing here is part of the library. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_set_threads(int n);
void orc_nmode(int d, const int64_t *dims, const double *X, int n, const double *M, int64_t rows,
               double *out);
void orc_ttm_t(int d, const int64_t *dims, const double *X, int n, const double *A, int64_t R,
               double *out);
void orc_contract_except(int d, const int64_t *udims, const double *U, const int64_t *vdims,
                         const double *V, int n, double *out);
void orc_gram(const double *A, int64_t N, int64_t R, double *S);
void orc_tucker_full(int d, const int64_t *dims, const int64_t *ranks, const double *G,
                     double *const *A, double *Xhat);
void orc_cp_full(int d, const int64_t *dims, int64_t r, double *const *C, double *Xhat);
double orc_sumsq(const double *X, int64_t n);
double orc_tucker_sq_residual(int d, const int64_t *dims, const double *X, const int64_t *ranks,
                              const double *G, double *const *A);
double orc_cp_sq_residual(int d, const int64_t *dims, const double *X, int64_t r, double *const *C);
long long orc_nntucker(int d, const int64_t *dims, const double *X, const int64_t *R, int iters,
                       double eps, double *G, double *const *A, double *fhist);
void orc_mttkrp(int d, const int64_t *tdims, const double *T, int n, int64_t r, double *const *B,
                double *M);
long long orc_nncp(int d, const int64_t *tdims, const double *T, int64_t r, int iters, double eps,
                   double *const *B, double *fhist);
void orc_lift(int d, const int64_t *dims, const int64_t *ranks, int64_t r, double *const *A,
              double *const *B, double *const *C);
double orc_tucker_grad(int d, const int64_t *dims, const double *X, const int64_t *R,
                       const double *G, double *const *A, double *gG, double *const *gA);

static uint64_t st = 88172645463325252ull;
static double urand(void) {  /* xorshift64, uniform in [0, 1) */
  st ^= st << 13;
  st ^= st >> 7;
  st ^= st << 17;
  return (double)(st >> 11) * (1.0 / 9007199254740992.0);
}
static double *vec(int64_t n) {
  double *v = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < n; ++i) v[i] = urand();
  return v;
}
static int64_t prod(const int64_t *a, int d) {
  int64_t p = 1;
  for (int k = 0; k < d; ++k) p *= a[k];
  return p;
}
static int fails = 0;
static void check(int ok, const char *what) {
  if (!ok) {
    printf("FAILED: %s\n", what);
    ++fails;
  }
}

static void one_case(int d, const int64_t *dims, const int64_t *R, int64_t r, int zero_col) {
  const int64_t size = prod(dims, d), gsize = prod(R, d);
  double *X = vec(size), *G = vec(gsize);
  double *A[8], *B[8], *C[8], *gA[8];
  for (int k = 0; k < d; ++k) {
    A[k] = vec(dims[k] * R[k]);
    B[k] = vec(R[k] * r);
    C[k] = vec(dims[k] * r);
    gA[k] = vec(dims[k] * R[k]);
  }
  if (zero_col)
    for (int64_t i = 0; i < dims[0]; ++i) A[0][i * R[0]] = 0.0;
  /* n-mode products: identity factor returns X; ttm_t against nmode with the transpose */
  for (int n = 0; n < d; ++n) {
    double *I = (double *)calloc((size_t)(dims[n] * dims[n]), sizeof(double));
    for (int64_t i = 0; i < dims[n]; ++i) I[i * dims[n] + i] = 1.0;
    double *out = vec(size);
    orc_nmode(d, dims, X, n, I, dims[n], out);
    double diff = 0.0;
    for (int64_t e = 0; e < size; ++e) diff += fabs(out[e] - X[e]);
    check(diff == 0.0, "identity n-mode product");
    int64_t odims[8];
    for (int k = 0; k < d; ++k) odims[k] = k == n ? R[n] : dims[k];
    double *t = vec(prod(odims, d));
    orc_ttm_t(d, dims, X, n, A[n], R[n], t);
    double *num = vec(dims[n] * dims[n]);
    orc_contract_except(d, dims, X, dims, X, n, num);  /* X_(n) X_(n)^T: exactly symmetric */
    int sym = 1;
    for (int64_t i = 0; i < dims[n]; ++i)
      for (int64_t j = 0; j < i; ++j) sym &= num[i * dims[n] + j] == num[j * dims[n] + i];
    check(sym, "contract_except symmetry");
    free(I);
    free(out);
    free(t);
    free(num);
  }
  double *S = vec(R[0] * R[0]);
  orc_gram(A[0], dims[0], R[0], S);
  check(S[0] >= 0.0, "gram");
  /* nnTucker: nonnegative iterates, monotone objective */
  double *fh = vec(4);
  long long clips = orc_nntucker(d, dims, X, R, 4, 1e-16, G, A, fh);
  for (int t = 1; t < 4; ++t) check(fh[t] <= fh[t - 1] * (1.0 + 1e-12), "monotone objective");
  check(zero_col ? clips > 0 : clips == 0, "clip count");
  for (int64_t e = 0; e < gsize; ++e) check(G[e] >= 0.0, "nonnegative core");
  const double tr = orc_tucker_sq_residual(d, dims, X, R, G, A);
  check(fabs(tr - 2.0 * fh[3]) <= 1e-9 * (1.0 + tr), "residual vs history");
  /* nnCP of the core, MTTKRP, lift, CP residual */
  double *ch = vec(3);
  orc_nncp(d, R, G, r, 3, 1e-16, B, ch);
  double *M = vec(R[d - 1] * r);
  orc_mttkrp(d, R, G, d - 1, r, B, M);
  orc_lift(d, dims, R, r, A, B, C);
  const double cr = orc_cp_sq_residual(d, dims, X, r, C);
  check(cr >= 0.0 && orc_sumsq(X, size) > 0.0, "cp residual");
  double *Xh = vec(size);
  orc_cp_full(d, dims, r, C, Xh);
  orc_tucker_full(d, dims, R, G, A, Xh);
  /* gradient */
  double *gG = vec(gsize);
  const double L = orc_tucker_grad(d, dims, X, R, G, A, gG, gA);
  check(fabs(L - 0.5 * tr) <= 1e-9 * (1.0 + L), "loss");
  free(X); free(G); free(S); free(fh); free(ch); free(M); free(Xh); free(gG);
  for (int k = 0; k < d; ++k) {
    free(A[k]); free(B[k]); free(C[k]); free(gA[k]);
  }
}

int main(void) {
  const int64_t d2[] = {7, 5}, r2[] = {3, 2};
  const int64_t d3[] = {9, 6, 5}, r3[] = {4, 3, 5};
  const int64_t d4[] = {5, 4, 6, 3}, r4[] = {2, 3, 2, 3};
  const int64_t d5[] = {3, 4, 2, 3, 4}, r5[] = {2, 2, 2, 3, 2};
  for (int threads = 1; threads <= 3; threads += 2) {
    orc_set_threads(threads);
    one_case(2, d2, r2, 2, 0);
    one_case(3, d3, r3, 3, 0);
    one_case(3, d3, r3, 3, 1);
    one_case(4, d4, r4, 2, 0);
    one_case(5, d5, r5, 2, 1);
  }
  if (fails) return 1;
  printf("sanitize driver ok\n");
  return 0;
}
