// Internal declarations shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "nncandelinc.h"

namespace nnc {

constexpr int kMaxDim = 8;

// a / b for 0 <= a < 2^22 and b >= 1 through the float reciprocal: (a + 0.5) / b lies at
// least 0.5 / b from the nearest integer, and the rounding of inv_b and of the product moves
// it by less than (a + 0.5) / b * 2^-23, which is smaller for such a.
static __device__ inline int qdiv(int a, float inv_b) { return (int)(((float)a + 0.5f) * inv_b); }

// Inverse of the r x r matrix in a (double, LDS) by Gauss-Jordan elimination without
// pivoting, ping-ponging between a and b with one barrier per pivot (every thread of the
// block takes part); returns the buffer that holds the inverse.  The pivots are those of the
// matrix's LDL^T factorization: all positive exactly when a symmetric matrix is positive
// definite (and, for a triangular matrix, its diagonal).  Thread 0 counts the pivots that are
// not positive in *bad.
static __device__ inline double *gj_inverse(double *a, double *b, int r, unsigned int *bad) {
  double *src = a, *dst = b;
  const int rr = r * r;
  for (int k = 0; k < r; ++k) {
    const double p = src[k * r + k];
    const double ip = 1.0 / p;
    for (int e0 = threadIdx.x; e0 < rr; e0 += 2 * blockDim.x) {
      // two entries per step, their LDS reads issued before any product
      const int e1 = e0 + blockDim.x;
      const bool has1 = e1 < rr;
      const int i0 = e0 / r, j0 = e0 - i0 * r;
      const int i1 = has1 ? e1 / r : i0, j1 = has1 ? e1 - i1 * r : j0;
      const double a0 = src[e0], rk0 = src[k * r + j0], ck0 = src[i0 * r + k];
      const double a1 = src[has1 ? e1 : e0], rk1 = src[k * r + j1], ck1 = src[i1 * r + k];
      double v0, v1;
      if (i0 == k)
        v0 = (j0 == k) ? ip : rk0 * ip;
      else
        v0 = (j0 == k) ? -ck0 * ip : a0 - ck0 * rk0 * ip;
      if (i1 == k)
        v1 = (j1 == k) ? ip : rk1 * ip;
      else
        v1 = (j1 == k) ? -ck1 * ip : a1 - ck1 * rk1 * ip;
      dst[e0] = v0;
      if (has1) dst[e1] = v1;
    }
    if (threadIdx.x == 0 && !(p > 0.0)) atomicAdd(bad, 1u);
    __syncthreads();
    double *x = src;
    src = dst;
    dst = x;
  }
  return src;
}

// Sets the thread-local error message and returns `st`.
nnc_status fail(nnc_status st, const char *fmt, ...);

// Checks the result of a HIP call; on failure records the message.
#define NNC_HIP(call)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::nnc::fail(NNC_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                         __FILE__, __LINE__);                                            \
  } while (0)

#define NNC_TRY(expr)                 \
  do {                                \
    nnc_status s_ = (expr);           \
    if (s_ != NNC_OK) return s_;      \
  } while (0)

// ------------------------------------------------------------------ launchers (kernels.hip)

// out[p][r][q] = sum_l F(l, r) * X[p][l][q], F(l, r) = F[l*ldl + r*ldr];
// X is [P][N][Q] of dtype xdt; out is [P][R][Q] float.  Chooses an MFMA kernel when the
// shape allows (allow_mfma) and a general kernel otherwise.
// reserve_cus > 0 keeps the X-streaming kernels off that many CUs, so that a kernel on
// another stream (the single-workgroup core step) finds a whole CU free while they run.
nnc_status launch_ttm(const void *X, nnc_dtype xdt, int64_t P, int64_t N, int64_t Q, const float *F,
                      int64_t ldl, int64_t ldr, int64_t R, float *out, hipStream_t s,
                      bool allow_mfma, const char **kernel_name = nullptr, int reserve_cus = 0);

// Software-pipelined X-streaming contractions (pass_kernels.hip).  Returns NNC_EUNSUPPORTED
// without recording an error when the shape does not suit them.
nnc_status launch_pass(const void *X, nnc_dtype xdt, int64_t P, int64_t N, int64_t Q, const float *F,
                       int64_t ldl, int64_t ldr, int64_t R, float *out, hipStream_t s,
                       const char **kernel_name, int reserve_cus);
// Compute units of the current device (queried once).
int device_cu_count();

// out[i][j] = sum_{p<pre, q<post} U[(p*I+i)*post+q] * V[(p*J+j)*post+q]
nnc_status launch_contract_except(const float *U, const float *V, int64_t pre, int64_t I, int64_t J,
                                  int64_t post, float *out, hipStream_t s);

// S = A^T A for A (N x R)
nnc_status launch_gram(const float *A, int64_t N, int64_t R, float *S, hipStream_t s);

// A <- A * num / max(A M, eps) row-wise (A: N x R, M: R x R); counts clips.
nnc_status launch_mu_factor(float *A, const float *num, const float *M, int64_t N, int64_t R,
                            double eps, unsigned long long *clips, hipStream_t s);

// x <- x * num / max(den, eps) elementwise.
nnc_status launch_mu_elem(float *x, const float *num, const float *den, int64_t n, double eps,
                          unsigned long long *clips, hipStream_t s);

// out = den - num elementwise (gradients).
nnc_status launch_sub(const float *den, const float *num, float *out, int64_t n, hipStream_t s);

// out = A M (A: N x R, M: R x C)
nnc_status launch_matmul_small(const float *A, const float *M, int64_t N, int64_t R, int64_t C,
                               float *out, hipStream_t s);

// Khatri-Rao rows W[m][rho] = prod_{k<d-1} C_k[i_k][rho] over the leading d-1 modes.
nnc_status launch_kr_rows(int d, const int64_t *dims, int64_t r, const float *const *C, float *W,
                          hipStream_t s);

// Squared-residual partial sums of X (M x K) against W (M x R) * Ad (K x R)^T; writes
// part[0..nblocks) pairs (sum (x-xhat)^2, sum x^2) and returns nblocks via *nblocks_out.
nnc_status launch_resid_stream(const void *X, nnc_dtype xdt, int64_t M, int64_t K, const float *W,
                               const float *Ad, int64_t R, double *part, int *nblocks_out,
                               hipStream_t s);
// out[0] = sum part[2i], out[1] = sum part[2i+1] in a fixed order.
nnc_status launch_reduce_pairs(const double *part, int n, double *out, hipStream_t s);
int resid_stream_max_blocks();

nnc_status launch_convert_bf16(const float *in, uint16_t *out, int64_t n, hipStream_t s);

// Counter-based SplitMix64 streams: key of (seed, stream id); element offset + i of the stream
// as a uniform double in [0, 1), written as float (RNE) to out32 or as double to out64.
uint64_t uniform_stream_key(uint64_t seed, uint64_t stream_id);
nnc_status launch_fill_uniform(uint64_t key, int64_t offset, int64_t n, float *out32, double *out64,
                               hipStream_t s);

// flag |= 1 if any of x[0..n) is not finite.
nnc_status launch_check_finite(const float *x, int64_t n, unsigned int *flag, hipStream_t s);

// x[0..n) = v (a kernel, so that it can sit inside a captured graph).
nnc_status launch_fill_u64(unsigned long long *x, int64_t n, unsigned long long v, hipStream_t s);
nnc_status launch_fill_f32(float *x, int64_t n, float v, hipStream_t s);

// ------------------------------------------------------------------ ls_kernels.hip
// Least-squares factor step of the real Tucker fit (two launches): A* = num K^{-1}, Cholesky
// QR A* = Q L^T, A <- Q (num and A distinct), T <- K^{-1} L^{-T} (R x R doubles),
// Lf <- L (R x R floats, for the core's G x_n L^T), S_out <- Q^T Q.  Pivots of K or of
// A*^T A* that are not positive are counted in *fails.  R <= 32.  K == nullptr: A* = num,
// the orthonormalization of a given factor alone.
nnc_status launch_ls_factor(const float *num, const float *K, int64_t N, int64_t R, float *A,
                            double *T, float *Lf, float *S_out, unsigned long long *fails, hipStream_t s);
// Sinv[k] = S[k]^{-1} for k < d (R[k] x R[k] floats, every R[k] <= 32), one launch.
nnc_status launch_ls_inverses(int d, const int64_t *R, float *const *S, float *const *Sinv,
                              unsigned long long *fails, hipStream_t s);

// ------------------------------------------------------------------ fused3_kernels.hip
// Side job of the fused three-way passes: blocks [0, nrows) each compute row blockIdx.x of
// M_n = unfold_n(G x_{k!=n} S_k) unfold_n(G)^T for the core G (R[0] x R[1] x R[2]).  S[k] are
// the stored Grams; with gram_part set, the Gram of mode gmode is summed from gram_parts
// row-block partials instead (block 0 stores it to S_store).
struct Side3 {
  int nrows;
  int n;
  int R[3];
  const float *G;
  const float *S[3];
  const float *gram_part;
  int gmode, gram_parts;
  float *S_store;
  float *M;
  unsigned int *ticket;  // zero before a launch, left zero (the side rows go to the first blocks done)
};
// Y0 = X x_2 A2^T x_1 A1^T (N0 x R1 x R2) without storing X x_2 A2^T.
bool pass1y_ok(nnc_dtype dt, int64_t N0, int64_t N1, int64_t N2, int64_t R0, int64_t R1, int64_t R2);
nnc_status launch_pass1y(const void *X, nnc_dtype dt, int64_t N0, int64_t N1, int64_t N2, const float *A2,
                         int64_t R2, const float *A1, int64_t R1, float *Y0, const Side3 &side, hipStream_t s);
// T = X x_0 A0^T (R0 x N1 x N2) and Y1 = T x_2 A2^T (R0 x N1 x R2).
bool pass2y_ok(nnc_dtype dt, int64_t N0, int64_t N1, int64_t N2, int64_t R0, int64_t R1, int64_t R2);
nnc_status launch_pass2y(const void *X, nnc_dtype dt, int64_t N0, int64_t N1, int64_t N2, const float *A0,
                         int64_t R0, const float *A2, int64_t R2, float *T, float *Y1, const Side3 &side,
                         hipStream_t s);

// ------------------------------------------------------------------ nnCP (cp_kernels.hip)
struct CpProblem {
  int d;
  int64_t dims[kMaxDim];
  int64_t size;  // prod dims
};

// One workgroup per fit.  Batched: fit b has rank d_ranks[b] <= max_rank and factor
// pointers d_factor_ptrs[b*d + n] (device tables).  Single fit: d_ranks == nullptr,
// nbatch == 1, rank max_rank and host array single_ptrs (passed by value).
// d_resid (nullable) receives each fit's relative residual.  zscratch: nbatch *
// nncp_zscratch_floats() floats, used when the contraction temporaries do not fit in LDS.
// als: least-squares updates B_n <- M_n H_n^{-1} (real CP) instead of the multiplicative
// ones; `clips` then counts pivots of H_n that were not positive.  t_global: the tensor is
// read from global memory even when it would fit in LDS (a tuner choice).
nnc_status launch_nncp(const float *T, const CpProblem &pb, int nbatch, const int *d_ranks,
                       int max_rank, float *const *d_factor_ptrs, float *const *single_ptrs,
                       int iters, double eps, double *d_resid, unsigned long long *clips,
                       float *zscratch, int threads, hipStream_t s, bool als = false,
                       bool t_global = false);
// Host-side check of a shape for launch_nncp (index ranges, rank, LDS); records the error.
nnc_status nncp_check_shape(const CpProblem &pb, int max_rank, int threads, bool als = false);
int64_t nncp_lds_bytes(const CpProblem &pb, int max_rank, int threads, bool als = false,
                       bool t_global = false);
int64_t nncp_zscratch_floats(const CpProblem &pb, int max_rank);
int nncp_default_threads(const CpProblem &pb, int max_rank);

nnc_status launch_lift(const float *A, const float *B, int64_t N, int64_t Rm, int64_t r, float *C,
                       hipStream_t s);

// ------------------------------------------------------------------ sweep_kernels.hip
// out[p][r][q] = sum_n F[n*ldl + r*ldr] * in[p][n][q] for FP32 partials, R <= 32.
nnc_status launch_ttm_small(const float *in, int64_t P, int64_t N, int64_t Q, const float *F,
                            int64_t ldl, int64_t ldr, int64_t R, float *out, hipStream_t s);

// Fused num/den/update of factor rows (R <= 32); see sweep_kernels.hip.
// npart (nullable; mu_rows_split_floats(Nn, R) floats): scratch that lets a long contracted
// index be split over blocks when the factor has few row blocks.
nnc_status launch_mu_rows(const float *Y, const float *G, float *A, const float *M, int64_t pre,
                          int64_t Nn, int64_t post, int64_t R, double eps, unsigned long long *clips,
                          float *gram, float *gpart, float *grad, hipStream_t s, float *npart = nullptr);
int64_t mu_rows_split_floats(int64_t Nn, int64_t R);
int64_t mu_rows_blocks(int64_t Nn);
// Per-block Gram partials of a factor, as mu_rows_k leaves them.
nnc_status launch_gram_parts(const float *A, int64_t Nn, int64_t R, float *gram, hipStream_t s);

struct CoreArgsHost {
  int d;
  int64_t R[kMaxDim];
  int64_t N[kMaxDim];
  const float *A[kMaxDim];
  float *S[kMaxDim];
  float *G;
  float *M;
  const float *gpart;
  int nparts;
  const float *gram;      // per-block Gram partials of factors gram_from.. (gram_stride apart)
  int gram_parts;
  int64_t gram_stride;
  float *t0, *t1, *numG;
  double eps;
  unsigned long long *clips;
  int gram_from, gram_to, do_core, next;
  float *u_out;  // launch_small_with_core: also U = G x_0 S_0 ... x_{d-2} S_{d-2} here (R_0 blocks)
};
nnc_status launch_core_step(const CoreArgsHost &h, hipStream_t s);
// dL/dG = G x_k S_k - h.numG into grad_out by the slice kernels (G unchanged); NNC_EUNSUPPORTED
// (no error recorded) for cores they do not take.
nnc_status launch_core_grad(const CoreArgsHost &h, float *grad_out, hipStream_t s);
// The core update in one launch (numerator from h.gpart, Gram of the last factor from its
// partials, den_G = U x_{d-1} S_{d-1} with U in h.t0, formed by launch_small_with_core).
nnc_status launch_core_last(const CoreArgsHost &h, hipStream_t s);
// launch_core_step(h) and launch_ttm_small(...) (independent of each other) in one launch
// when the core step only forms a Gram and M_next; two launches otherwise.
nnc_status launch_small_with_core(const float *in, int64_t P, int64_t N, int64_t Q, const float *F,
                                  int64_t ldl, int64_t ldr, int64_t R, float *out,
                                  const CoreArgsHost &h, hipStream_t s);
// out[e] = sum_{b < nparts} part[b][e] (fixed order)
// Nonnegative CP of the data tensor (cpx_kernels.hip).
nnc_status launch_diag(const float *Y, int rho_first, int64_t A, int64_t Nt, int64_t C, const float *WA,
                       const float *WC, int r, float *out, float *part, hipStream_t s);
int64_t diag_part_floats(int64_t A, int64_t Nt, int64_t C, int r);
nnc_status launch_cp_mu(float *B, const float *M, const float *S, int d, int n, int64_t N, int r,
                        double eps, unsigned long long *clips, hipStream_t s);
nnc_status launch_gram_block(const float *A, int64_t N, int r, float *S, hipStream_t s);
// S[k] = A[k]^T A[k] for k < d in one launch (one workgroup per factor, R[k] <= 32).
nnc_status launch_gram_set(int d, const float *const *A, const int64_t *N, const int64_t *R, float *const *S,
                           hipStream_t s);
bool nmf_block_fits(int rows, int cols, int m);
nnc_status launch_nmf_block(int n, const float *const *A, const int *rows, int cols, const int *m,
                            int iters, float *const *W, float *const *H, double eps,
                            unsigned long long *clips, double *red, hipStream_t s);
int64_t tiny_init_floats(int alg, const int *N, const int *M, int r);
nnc_status launch_tiny_candelinc(const float *X, const int *N, const int *M, int r, int alg, int nres,
                                 int outer, int inner, const float *inits, const float *const *truth,
                                 double eps, double *rel, double *cong, float *fout,
                                 unsigned long long *clips, hipStream_t s);
nnc_status launch_congruence(int d, const int64_t *dims, int r, const float *const *P, const float *const *Q,
                             double *out, hipStream_t s);
nnc_status launch_transpose(const float *in, int64_t rows, int64_t cols, float *out, hipStream_t s);
nnc_status launch_sum_parts(const float *part, int nparts, int64_t n, float *out, hipStream_t s);

}  // namespace nnc
