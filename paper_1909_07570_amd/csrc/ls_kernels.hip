// Least-squares steps of the real-valued CANDELINC Tucker fit (Section 2.2: a Tucker
// decomposition of X, then a CPD of its core).  The X passes and the small contractions that
// feed these steps are the nonnegative sweep's kernels; what differs is the update of each
// block, done here in FP64 inside one workgroup:
//
//   factor n:  A* = num_n K_n^{-1}       (num_n = Y_(n) G_(n)^T, K_n = G_(n) (kron_{k!=n} S_k) G_(n)^T)
//              A* = Q L^T                 (Cholesky QR: L L^T = A*^T A*, Q = A* L^{-T})
//              A_n <- Q,  G <- G x_n L^T, S_n <- Q^T Q
//   core:      G <- (X x_1 A_1^T ... x_d A_d^T) x_1 S_1^{-1} ... x_d S_d^{-1}
//
// R x R inverses come from Gauss-Jordan elimination without pivoting (one barrier per pivot):
// its pivots are those of the LDL^T factorization, positive exactly when the matrix is
// positive definite, so a pivot that is not positive marks a system that is not (counted in
// `fails`).  Every sum runs in a fixed order, so results are reproducible.
#include <algorithm>

#include "nnc_internal.h"

namespace nnc {

namespace {

constexpr int kLsThreads = 1024;
constexpr int kLsChunk = 64;  // factor rows staged in LDS at a time

// Cholesky factor L (lower, positive diagonal) of the SPD r x r matrix W, column by column,
// one barrier per column; every row of a column forms the column's diagonal itself.  L's
// upper triangle is written as zeros.  Non-positive diagonals are counted in *bad.
__device__ void cholesky(const double *W, double *L, int r, unsigned int *bad) {
  for (int t = threadIdx.x; t < r * r; t += blockDim.x) L[t] = 0.0;
  __syncthreads();
  for (int j = 0; j < r; ++j) {
    const int i = j + threadIdx.x;
    if (i < r) {
      double dj = W[j * r + j];
      for (int k = 0; k < j; ++k) dj -= L[j * r + k] * L[j * r + k];
      if (i == j) {
        if (!(dj > 0.0)) atomicAdd(bad, 1u);
        L[j * r + j] = sqrt(dj);
      } else {
        double v = W[i * r + j];
        for (int k = 0; k < j; ++k) v -= L[i * r + k] * L[j * r + k];
        L[i * r + j] = v / sqrt(dj);
      }
    }
    __syncthreads();
  }
}

// Gram partial sums of `rows` staged rows (stride RM) into the thread's accumulator: thread
// t < R*R*S takes entry (x, y) = (t % (R*R)) / R, % R and the rows i = split (mod S).
template <int RM>
__device__ inline double gram_chunk(const float *rowsbuf, int rows, int R, int S, double acc) {
  const int t = threadIdx.x, P = R * R;
  if (t < P * S) {
    const int pr = t % P, split = t / P;
    const int x = pr / R, y = pr - (pr / R) * R;
    for (int i = split; i < rows; i += S) acc += (double)rowsbuf[i * RM + x] * (double)rowsbuf[i * RM + y];
  }
  return acc;
}

// Sum the S split accumulators of every Gram entry in split order into out (double, R*R).
__device__ inline void gram_reduce(double acc, double *part, int R, int S, double *out) {
  const int t = threadIdx.x, P = R * R;
  if (t < P * S) part[t] = acc;
  __syncthreads();
  for (int e = t; e < P; e += blockDim.x) {
    double s = 0.0;
    for (int q = 0; q < S; ++q) s += part[q * P + e];
    out[e] = s;
  }
  __syncthreads();
}

// One factor's least-squares step, orthonormalization and core update (see the top of the
// file).  num: N x R, K: R x R, A: N x R (written), G: the core viewed as gpre x R x gpost
// (updated in place), S_out: R x R Gram of the new factor.  num == nullptr skips the
// least-squares step (A* = A): the orthonormalization of a given factor alone.
template <int RM>
__global__ __launch_bounds__(kLsThreads) void ls_factor_k(const float *__restrict__ num,
                                                          const float *__restrict__ K, int N, int R,
                                                          float *__restrict__ A, float *__restrict__ G,
                                                          int64_t gpre, int64_t gpost,
                                                          float *__restrict__ S_out,
                                                          unsigned long long *fails) {
  extern __shared__ __attribute__((aligned(16))) double sd[];
  __shared__ unsigned int bad;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int P = R * R;
  const int S = P >= nt ? 1 : nt / P;
  double *m0 = sd, *m1 = sd + P, *W = sd + 2 * P, *L = sd + 3 * P, *part = sd + 4 * P;
  float *c0 = reinterpret_cast<float *>(part + nt);  // staged rows: num, then Q
  float *c1 = c0 + kLsChunk * RM;                    // staged rows of A*
  if (tid == 0) bad = 0;
  const double *Kinv = nullptr;
  if (num) {
    for (int e = tid; e < P; e += nt) m0[e] = (double)K[e];
    __syncthreads();
    Kinv = gj_inverse(m0, m1, R, &bad);
  }

  // A* = num K^{-1}, written to A (num == nullptr: A* = A as given); Gram of A*'s floats
  double acc = 0.0;
  for (int i0 = 0; i0 < N; i0 += kLsChunk) {
    const int rows = min(kLsChunk, N - i0);
    if (num) {
      for (int e = tid; e < rows * R; e += nt) {
        const int i = e / R, c = e - (e / R) * R;
        c0[i * RM + c] = num[(int64_t)(i0 + i) * R + c];
      }
      __syncthreads();
      for (int e = tid; e < rows * R; e += nt) {
        const int i = e / R, c = e - (e / R) * R;
        double v = 0.0;
        for (int s = 0; s < R; ++s) v += (double)c0[i * RM + s] * Kinv[s * R + c];
        const float f = (float)v;
        c1[i * RM + c] = f;
        A[(int64_t)(i0 + i) * R + c] = f;
      }
    } else {
      for (int e = tid; e < rows * R; e += nt) {
        const int i = e / R, c = e - (e / R) * R;
        c1[i * RM + c] = A[(int64_t)(i0 + i) * R + c];
      }
    }
    __syncthreads();
    acc = gram_chunk<RM>(c1, rows, R, S, acc);
    __syncthreads();
  }
  gram_reduce(acc, part, R, S, W);
  cholesky(W, L, R, &bad);
  // L^{-1} (lower triangular) into m0/m1 (K^{-1} is no longer needed)
  for (int e = tid; e < P; e += nt) m0[e] = L[e];
  __syncthreads();
  const double *Linv = gj_inverse(m0, m1, R, &bad);

  // Q = A* L^{-T}: Q[i][c] = sum_{k <= c} A*[i][k] Linv[c][k]; Gram of Q's float values
  __threadfence_block();
  acc = 0.0;
  for (int i0 = 0; i0 < N; i0 += kLsChunk) {
    const int rows = min(kLsChunk, N - i0);
    for (int e = tid; e < rows * R; e += nt) {
      const int i = e / R, c = e - (e / R) * R;
      c1[i * RM + c] = A[(int64_t)(i0 + i) * R + c];
    }
    __syncthreads();
    for (int e = tid; e < rows * R; e += nt) {
      const int i = e / R, c = e - (e / R) * R;
      double v = 0.0;
      for (int k = 0; k <= c; ++k) v += (double)c1[i * RM + k] * Linv[c * R + k];
      const float f = (float)v;
      c0[i * RM + c] = f;
      A[(int64_t)(i0 + i) * R + c] = f;
    }
    __syncthreads();
    acc = gram_chunk<RM>(c0, rows, R, S, acc);
    __syncthreads();
  }
  gram_reduce(acc, part, R, S, W);
  for (int e = tid; e < P; e += nt) S_out[e] = (float)W[e];

  // G <- G x_n L^T: every mode-n fibre g becomes L^T g (one thread per fibre, in place)
  const int64_t nf = gpre * gpost;
  for (int64_t f = tid; f < nf; f += nt) {
    const int64_t p = f / gpost, q = f - (f / gpost) * gpost;
    float *g = G + p * R * gpost + q;
    float v[RM];
#pragma unroll
    for (int l = 0; l < RM; ++l) v[l] = l < R ? g[l * gpost] : 0.f;
#pragma unroll
    for (int i = 0; i < RM; ++i) {
      if (i < R) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < RM; ++l)
          if (l >= i && l < R) s += L[l * R + i] * (double)v[l];
        g[i * gpost] = (float)s;
      }
    }
  }
  if (tid == 0 && bad) atomicAdd(fails, (unsigned long long)bad);
}

struct LsCoreArgs {
  int d;
  int R[kMaxDim];
  const float *S[kMaxDim];
};

// G = numG x_1 S_1^{-1} ... x_d S_d^{-1}: per mode, the inverse of S_k, then every mode-k
// fibre replaced by S_k^{-1} fibre (one thread per fibre; the first mode reads numG).
template <int RM>
__global__ __launch_bounds__(kLsThreads) void ls_core_k(const float *__restrict__ numG, LsCoreArgs a,
                                                        float *__restrict__ G, unsigned long long *fails) {
  extern __shared__ __attribute__((aligned(16))) double sd[];
  __shared__ unsigned int bad;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) bad = 0;
  int64_t total = 1;
  for (int k = 0; k < a.d; ++k) total *= a.R[k];
  int64_t pre = 1;
  for (int k = 0; k < a.d; ++k) {
    const int R = a.R[k];
    const int64_t post = total / (pre * R);
    double *m0 = sd, *m1 = sd + R * R;
    for (int e = tid; e < R * R; e += nt) m0[e] = (double)a.S[k][e];
    __syncthreads();
    const double *Sinv = gj_inverse(m0, m1, R, &bad);
    const float *src = k == 0 ? numG : G;
    for (int64_t f = tid; f < pre * post; f += nt) {
      const int64_t p = f / post, q = f - (f / post) * post;
      const int64_t base = p * R * post + q;
      float v[RM];
#pragma unroll
      for (int l = 0; l < RM; ++l) v[l] = l < R ? src[base + l * post] : 0.f;
#pragma unroll
      for (int i = 0; i < RM; ++i) {
        if (i < R) {
          double s = 0.0;
#pragma unroll
          for (int l = 0; l < RM; ++l)
            if (l < R) s += Sinv[i * R + l] * (double)v[l];
          G[base + i * post] = (float)s;
        }
      }
    }
    __threadfence_block();
    __syncthreads();
    pre *= R;
  }
  if (tid == 0 && bad) atomicAdd(fails, (unsigned long long)bad);
}

int ls_rm(int R) { return R <= 8 ? 8 : (R <= 16 ? 16 : 32); }

}  // namespace

nnc_status launch_ls_factor(const float *num, const float *K, int64_t N, int64_t R, float *A, float *G,
                            int64_t gpre, int64_t gpost, float *S_out, unsigned long long *fails,
                            hipStream_t s) {
  if (R < 1 || R > 32) return fail(NNC_EUNSUPPORTED, "least-squares factor step: rank %lld outside 1..32", (long long)R);
  if (N < 1 || N > INT32_MAX) return fail(NNC_EUNSUPPORTED, "least-squares factor step: %lld rows", (long long)N);
  const int RM = ls_rm((int)R);
  const size_t lds = sizeof(double) * (4 * R * R + kLsThreads) + sizeof(float) * 2 * kLsChunk * RM;
#define NNC_LSF(RMV)                                                                                  \
  hipLaunchKernelGGL(ls_factor_k<RMV>, dim3(1), dim3(kLsThreads), lds, s, num, K, (int)N, (int)R, A, G, \
                     gpre, gpost, S_out, fails)
  if (RM == 8)
    NNC_LSF(8);
  else if (RM == 16)
    NNC_LSF(16);
  else
    NNC_LSF(32);
#undef NNC_LSF
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

nnc_status launch_ls_core(const float *numG, int d, const int64_t *R, float *const *S, float *G,
                          unsigned long long *fails, hipStream_t s) {
  LsCoreArgs a;
  a.d = d;
  int rmax = 1;
  for (int k = 0; k < kMaxDim; ++k) {
    a.R[k] = k < d ? (int)R[k] : 1;
    a.S[k] = k < d ? S[k] : nullptr;
    if (k < d) {
      if (R[k] < 1 || R[k] > 32)
        return fail(NNC_EUNSUPPORTED, "least-squares core step: rank %lld outside 1..32", (long long)R[k]);
      rmax = std::max(rmax, (int)R[k]);
    }
  }
  const int RM = ls_rm(rmax);
  const size_t lds = sizeof(double) * 2 * rmax * rmax;
#define NNC_LSC(RMV) hipLaunchKernelGGL(ls_core_k<RMV>, dim3(1), dim3(kLsThreads), lds, s, numG, a, G, fails)
  if (RM == 8)
    NNC_LSC(8);
  else if (RM == 16)
    NNC_LSC(16);
  else
    NNC_LSC(32);
#undef NNC_LSC
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

}  // namespace nnc
