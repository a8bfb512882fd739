// Least-squares steps of the real-valued CANDELINC Tucker fit (Section 2.2: a Tucker
// decomposition of X, then a CPD of its core).  The X passes and the small contractions that
// feed these steps are the nonnegative sweep's kernels; what differs is the update of each
// block, done here in FP64:
//
//   factor n:  A* = num_n K_n^{-1}       (num_n = Y_(n) G_(n)^T, K_n = G_(n) (kron_{k!=n} S_k) G_(n)^T)
//              A* = Q L^T                 (Cholesky QR: L L^T = A*^T A*, Q = A* L^{-T})
//              A_n <- Q,  G <- G x_n L^T, S_n <- Q^T Q
//   core:      G <- (X x_1 A_1^T ... x_d A_d^T) x_1 S_1^{-1} ... x_d S_d^{-1}
//
// The factor step only needs R x R quantities besides two passes over the N x R rows:
//   Z = num^T num,  A*^T A* = K^{-1} Z K^{-1} = L L^T,  T = K^{-1} L^{-T},  Q = num T,
//   Q^T Q = T^T Z T;
// one workgroup forms Z and the R x R algebra (ls_small_k), a row kernel applies T
// (ls_rows_k), and the core's mode products with L^T and with the inverse Grams run on the
// small-contraction kernel of the sweep (launch_ttm_small).  R x R inverses come from Gauss-Jordan elimination without pivoting (one
// barrier per pivot): its pivots are those of the LDL^T factorization, positive exactly when
// the matrix is positive definite, so a pivot that is not positive marks a system that is not
// (counted in `fails`).  Every sum runs in a fixed order, so results are reproducible.
#include <algorithm>

#include "nnc_internal.h"

namespace nnc {

namespace {

constexpr int kLsThreads = 256;
constexpr int kLsChunk = 256;  // rows of num staged in LDS at a time (R <= 32: 32 KB)

// dst[e] = src[e] for e < n by the whole block, eight independent loads in flight per
// thread before their stores (a loop that stores each load before issuing the next waits a
// full memory round trip per element).
template <typename D>
__device__ inline void block_copy(const float *__restrict__ src, D *__restrict__ dst, int n) {
  for (int e0 = threadIdx.x; e0 < n; e0 += 8 * blockDim.x) {
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int e = e0 + k * blockDim.x;
      v[k] = e < n ? src[e] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int e = e0 + k * blockDim.x;
      if (e < n) dst[e] = (D)v[k];
    }
  }
}

// Cholesky factor L (lower, positive diagonal) of the SPD r x r matrix W, column by column,
// one barrier per column; every row of a column forms the column's diagonal itself.  L's
// upper triangle is written as zeros.  Non-positive diagonals are counted in *bad.
__device__ void cholesky(const double *W, double *L, int r, unsigned int *bad) {
  for (int t = threadIdx.x; t < r * r; t += blockDim.x) L[t] = 0.0;
  __syncthreads();
  for (int j = 0; j < r; ++j) {
    const int i = j + threadIdx.x;
    if (i < r) {
      double dj = W[j * r + j], v = W[i * r + j];
#pragma unroll 4
      for (int k = 0; k < j; ++k) {
        const double ljk = L[j * r + k];
        dj -= ljk * ljk;
        v -= L[i * r + k] * ljk;
      }
      if (i == j) {
        if (!(dj > 0.0)) atomicAdd(bad, 1u);
        L[j * r + j] = sqrt(dj);
      } else {
        L[i * r + j] = v / sqrt(dj);
      }
    }
    __syncthreads();
  }
}

// C = op(A) B for r x r double matrices in LDS (op = transpose when ta), then a barrier.
__device__ void small_mm(const double *A, bool ta, const double *B, double *C, int r) {
  for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
    const int i = e / r, j = e - (e / r) * r;
    double v = 0.0;
#pragma unroll 4
    for (int k = 0; k < r; ++k) v += (ta ? A[k * r + i] : A[i * r + k]) * B[k * r + j];
    C[e] = v;
  }
  __syncthreads();
}

// The R x R part of a factor step (see the top of the file), one workgroup.
//   num (N x R): the numerator rows; K (R x R): the system, or nullptr for the
//   orthonormalization of the factor given in num alone (K = I).
//   Writes T_out = K^{-1} L^{-T} (R x R doubles), L_out = L (R x R floats, upper triangle
//   zero) and S_out = T^T Z T (the Gram of the new factor).
__global__ __launch_bounds__(kLsThreads) void ls_small_k(const float *__restrict__ num,
                                                         const float *__restrict__ K, int N, int R,
                                                         double *__restrict__ T_out, float *__restrict__ L_out,
                                                         float *__restrict__ S_out, unsigned long long *fails) {
  extern __shared__ __attribute__((aligned(16))) double sd[];
  __shared__ unsigned int bad;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int P = R * R;
  double *Z = sd, *K0 = sd + P, *K1 = sd + 2 * P, *W = sd + 3 * P, *L = sd + 4 * P, *L0 = sd + 5 * P,
         *L1 = sd + 6 * P;
  float *rows = reinterpret_cast<float *>(sd + 7 * P);
  if (tid == 0) bad = 0;
  // Z = num^T num: thread t holds entries t, t + nt, ... (at most 4), rows in order
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i0 = 0; i0 < N; i0 += kLsChunk) {
    const int nr = min(kLsChunk, N - i0);
    block_copy(num + (int64_t)i0 * R, rows, nr * R);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + u * nt;
      if (e < P) {
        const int x = e / R, y = e - (e / R) * R;
        double a = acc[u];
#pragma unroll 4
        for (int i = 0; i < nr; ++i) a += (double)rows[i * R + x] * (double)rows[i * R + y];
        acc[u] = a;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (tid + u * nt < P) Z[tid + u * nt] = acc[u];
  if (K) {
    block_copy(K, K0, P);
  } else {
    for (int e = tid; e < P; e += nt) {
      const int i = e / R, j = e - (e / R) * R;
      K0[e] = i == j ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  const double *Kinv = K ? gj_inverse(K0, K1, R, &bad) : K0;
  double *Kfree = (Kinv == K0) ? K1 : K0;
  small_mm(Z, false, Kinv, Kfree, R);  // Z K^{-1}
  small_mm(Kinv, false, Kfree, W, R);  // K^{-1} Z K^{-1} = A*^T A*
  cholesky(W, L, R, &bad);
  for (int e = tid; e < P; e += nt) {
    L0[e] = L[e];
    L_out[e] = (float)L[e];
  }
  __syncthreads();
  const double *Linv = gj_inverse(L0, L1, R, &bad);
  // T = K^{-1} L^{-T}: T[s][c] = sum_{k <= c} Kinv[s][k] Linv[c][k]  (into W)
  for (int e = tid; e < P; e += nt) {
    const int s = e / R, c = e - (e / R) * R;
    double v = 0.0;
#pragma unroll 4
    for (int k = 0; k <= c; ++k) v += Kinv[s * R + k] * Linv[c * R + k];
    W[e] = v;
    T_out[e] = v;
  }
  __syncthreads();
  small_mm(Z, false, W, Kfree, R);  // Z T
  for (int e = tid; e < P; e += nt) {  // S = T^T (Z T)
    const int i = e / R, j = e - (e / R) * R;
    double v = 0.0;
#pragma unroll 4
    for (int k = 0; k < R; ++k) v += W[k * R + i] * Kfree[k * R + j];
    S_out[e] = (float)v;
  }
  if (tid == 0 && bad) atomicAdd(fails, (unsigned long long)bad);
}

// A[i][c] = sum_s num[i][s] T[s][c] (FP64 sums), one thread per entry.  num and A must not
// overlap.
__global__ __launch_bounds__(kLsThreads) void ls_rows_k(const float *__restrict__ num,
                                                        const double *__restrict__ T, int N, int R,
                                                        float *__restrict__ A) {
  __shared__ double Ts[32 * 32];
  for (int e0 = threadIdx.x; e0 < R * R; e0 += 4 * blockDim.x) {
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = e0 + k * (int)blockDim.x < R * R ? T[e0 + k * blockDim.x] : 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (e0 + k * (int)blockDim.x < R * R) Ts[e0 + k * blockDim.x] = v[k];
  }
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)N * R) return;
  const int64_t i = e / R;
  const int c = (int)(e - i * R);
  const float *x = num + i * R;
  double v = 0.0;
#pragma unroll 4
  for (int s = 0; s < R; ++s) v += (double)x[s] * Ts[s * R + c];
  A[e] = (float)v;
}

struct LsInvArgs {
  int d;
  int R[kMaxDim];
  const float *S[kMaxDim];
  float *Sinv[kMaxDim];
};

// Sinv[k] = S[k]^{-1} (as floats) for every mode, one workgroup, modes in turn.
__global__ __launch_bounds__(kLsThreads) void ls_inv_k(LsInvArgs a, unsigned long long *fails) {
  extern __shared__ __attribute__((aligned(16))) double sd[];
  __shared__ unsigned int bad;
  if (threadIdx.x == 0) bad = 0;
  for (int k = 0; k < a.d; ++k) {
    const int R = a.R[k];
    double *m0 = sd, *m1 = sd + R * R;
    block_copy(a.S[k], m0, R * R);
    __syncthreads();
    const double *inv = gj_inverse(m0, m1, R, &bad);
    for (int e = threadIdx.x; e < R * R; e += blockDim.x) a.Sinv[k][e] = (float)inv[e];
    __syncthreads();
  }
  if (threadIdx.x == 0 && bad) atomicAdd(fails, (unsigned long long)bad);
}

}  // namespace

nnc_status launch_ls_factor(const float *num, const float *K, int64_t N, int64_t R, float *A,
                            double *T, float *Lf, float *S_out, unsigned long long *fails, hipStream_t s) {
  if (R < 1 || R > 32) return fail(NNC_EUNSUPPORTED, "least-squares factor step: rank %lld outside 1..32", (long long)R);
  if (N < 1 || N * R > INT32_MAX) return fail(NNC_EUNSUPPORTED, "least-squares factor step: %lld rows", (long long)N);
  if (num == A) return fail(NNC_EINVAL, "least-squares factor step: num and A must differ");
  const size_t lds = sizeof(double) * 7 * R * R + sizeof(float) * kLsChunk * R;
  hipLaunchKernelGGL(ls_small_k, dim3(1), dim3(kLsThreads), lds, s, num, K, (int)N, (int)R, T, Lf, S_out, fails);
  const int64_t n = N * R;
  hipLaunchKernelGGL(ls_rows_k, dim3((unsigned)((n + kLsThreads - 1) / kLsThreads)), dim3(kLsThreads), 0, s, num,
                     T, (int)N, (int)R, A);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

nnc_status launch_ls_inverses(int d, const int64_t *R, float *const *S, float *const *Sinv,
                              unsigned long long *fails, hipStream_t s) {
  LsInvArgs a;
  a.d = d;
  int rmax = 1;
  for (int k = 0; k < kMaxDim; ++k) {
    a.R[k] = k < d ? (int)R[k] : 1;
    a.S[k] = k < d ? S[k] : nullptr;
    a.Sinv[k] = k < d ? Sinv[k] : nullptr;
    if (k < d) {
      if (R[k] < 1 || R[k] > 32)
        return fail(NNC_EUNSUPPORTED, "least-squares core step: rank %lld outside 1..32", (long long)R[k]);
      rmax = std::max(rmax, (int)R[k]);
    }
  }
  hipLaunchKernelGGL(ls_inv_k, dim3(1), dim3(kLsThreads), sizeof(double) * 2 * rmax * rmax, s, a, fails);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

}  // namespace nnc
