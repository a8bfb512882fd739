// HIP kernels for gfx950 (CDNA4): the contraction dispatcher, multiplicative update steps,
// residual reductions and conversions.
//
// Contraction forms (n-mode product with a transposed factor, Appendix A):
//   X viewed as [P][N][Q] (N = the contracted mode, Q = product of the later modes):
//     out[p][r][q] = sum_n F(n, r) * X[p][n][q].
// The matrix-core X-streaming kernels (pass_kernels.hip) take every shape with rank <= 32,
// 16-byte aligned X and output and rows of a whole number of 16-byte chunks; the general
// kernel here takes the rest.
#include <stdarg.h>
#include <stdio.h>

#include <mutex>
#include <map>

#include <algorithm>

#include "nnc_internal.h"

namespace nnc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

static __device__ inline uint16_t f2bf_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
static __device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

static __device__ inline float load_x(const float *p) { return *p; }
static __device__ inline float load_x(const uint16_t *p) { return bf2f(*p); }

static __device__ inline bf8 as_bf8(u4 v) { return __builtin_bit_cast(bf8, v); }

static __device__ inline f4 mfma_bf16(u4 a, u4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(a), as_bf8(b), c, 0, 0, 0);
}

// =====================================================================================
// General contraction (any shape, any R): one thread per (p, 4 columns r, q), sequential
// sum over the contracted index.
// =====================================================================================
template <typename XT>
__global__ __launch_bounds__(256) void ttm_generic_k(const XT *__restrict__ X, int64_t P, int64_t N,
                                                     int64_t Q, const float *__restrict__ F,
                                                     int64_t ldl, int64_t ldr, int64_t R,
                                                     float *__restrict__ out) {
  const int64_t RC = (R + 3) >> 2;
  const int64_t total = P * RC * Q;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = idx % Q;
    const int64_t t = idx / Q;
    const int64_t rc = t % RC;
    const int64_t p = t / RC;
    const int64_t r0 = rc * 4;
    const int nr = (int)((R - r0) < 4 ? (R - r0) : 4);
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    const XT *x = X + p * N * Q + q;
    for (int64_t l = 0; l < N; ++l) {
      const float xv = load_x(x + l * Q);
      const float *f = F + l * ldl + r0 * ldr;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (j < nr) acc[j] = fmaf(f[j * ldr], xv, acc[j]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j < nr) out[(p * R + r0 + j) * Q + q] = acc[j];
  }
}

static int grid_for(int64_t work, int threads, int cap) {
  int64_t g = (work + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

static bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

nnc_status launch_ttm(const void *X, nnc_dtype xdt, int64_t P, int64_t N, int64_t Q, const float *F,
                      int64_t ldl, int64_t ldr, int64_t R, float *out, hipStream_t s,
                      bool allow_mfma, const char **kernel_name, int reserve_cus) {
  const char *name = "ttm_generic";
  const int64_t total_rows = P * N * Q;
  if (total_rows == 0 || R == 0) return NNC_OK;
  if (allow_mfma) {
    const nnc_status st = launch_pass(X, xdt, P, N, Q, F, ldl, ldr, R, out, s, kernel_name, reserve_cus);
    if (st != NNC_EUNSUPPORTED) return st;
  }
  // every other shape (rank above 32, unaligned pointers, rows of a length the matrix-core
  // kernels do not take): one thread per (p, 4 columns r, q)
  {
    const int64_t work = P * ((R + 3) / 4) * Q;
    const int grid = grid_for(work, 256, 65536);
    if (xdt == NNC_F32)
      hipLaunchKernelGGL(ttm_generic_k<float>, dim3(grid), dim3(256), 0, s, (const float *)X, P, N,
                         Q, F, ldl, ldr, R, out);
    else
      hipLaunchKernelGGL(ttm_generic_k<uint16_t>, dim3(grid), dim3(256), 0, s, (const uint16_t *)X,
                         P, N, Q, F, ldl, ldr, R, out);
  }
  if (kernel_name) *kernel_name = name;
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

// =====================================================================================
// Small dense steps of the multiplicative updates.
// =====================================================================================
__global__ void contract_except_k(const float *__restrict__ U, const float *__restrict__ V,
                                  int64_t pre, int64_t I, int64_t J, int64_t post,
                                  float *__restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= I * J) return;
  const int64_t i = idx / J, j = idx - (idx / J) * J;
  float acc = 0.f;
  for (int64_t p = 0; p < pre; ++p) {
    const float *u = U + (p * I + i) * post;
    const float *v = V + (p * J + j) * post;
    for (int64_t q = 0; q < post; ++q) acc = fmaf(u[q], v[q], acc);
  }
  out[idx] = acc;
}

// The same contraction for J <= JM (<= 32): one wave per output row i, its lanes striding
// over the flattened summation index t = p * post + q (lane l takes t = l, l + 64, ...) with
// JM partial sums each, then a butterfly over the wave.  V (pre x J x post) passes through
// LDS in chunks of the summation index that every wave of the block shares; U's loads are
// issued four steps ahead of their products.  Every sum runs in a fixed order.
constexpr int kCeVlds = 16384;  // floats of V staged in LDS per chunk (64 KB)

template <int JM>
__global__ __launch_bounds__(256) void contract_except_rows_k(const float *__restrict__ U,
                                                              const float *__restrict__ V, int pre,
                                                              int64_t I, int J, int post,
                                                              float *__restrict__ out) {
  __shared__ float Vs[kCeVlds];
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const bool active = i < I;  // every wave takes part in the staging barriers
  const int total = pre * post;
  const int tc = (kCeVlds / J) & ~63;  // chunk of the summation index, a multiple of 64
  float acc[JM];
#pragma unroll
  for (int j = 0; j < JM; ++j) acc[j] = 0.f;
  const int dp = 64 / post, dq = 64 - (64 / post) * post;
  for (int t0 = 0; t0 < total; t0 += tc) {
    const int tn = min(tc, total - t0);
    __syncthreads();  // the previous chunk has been consumed
    // thread per summation index tt: its J entries of V (stride post) loaded together
    for (int tt = threadIdx.x; tt < tn; tt += blockDim.x) {
      const int t = t0 + tt;
      const int p = t / post, q = t - (t / post) * post;
      const float *vb = V + (int64_t)p * J * post + q;
      float v[JM];
#pragma unroll
      for (int j = 0; j < JM; ++j) v[j] = j < J ? vb[(int64_t)j * post] : 0.f;
#pragma unroll
      for (int j = 0; j < JM; ++j)
        if (j < J) Vs[j * tc + tt] = v[j];
    }
    __syncthreads();
    if (!active) continue;
    int tt = lane;
    int p = (t0 + lane) / post, q = (t0 + lane) - ((t0 + lane) / post) * post;
    while (tt < tn) {
      float u[4];
      int vo[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bool ok = tt + 64 * k < tn;
        u[k] = ok ? U[((int64_t)p * I + i) * post + q] : 0.f;
        vo[k] = ok ? tt + 64 * k : 0;
        p += dp;
        q += dq;
        if (q >= post) {
          q -= post;
          ++p;
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int j = 0; j < JM; ++j)
          if (j < J) acc[j] = fmaf(u[k], Vs[j * tc + vo[k]], acc[j]);
      }
      tt += 256;
    }
  }
  if (!active) return;
#pragma unroll
  for (int j = 0; j < JM; ++j) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) acc[j] += __shfl_xor(acc[j], m, 64);
  }
  if (lane < J) {
    float v = 0.f;
#pragma unroll
    for (int j = 0; j < JM; ++j)
      if (j == lane) v = acc[j];
    out[i * J + lane] = v;
  }
}

// The same contraction for few output rows (I small, J <= JM <= 32): one block of kSplitWaves
// waves per row i, wave w summing the contiguous range w of the flattened summation index
// (lanes striding inside it), a butterfly per wave, then the waves' sums added in wave order
// through LDS.
constexpr int kSplitWaves = 16;

template <int JM>
__global__ __launch_bounds__(64 * kSplitWaves) void contract_except_split_k(const float *__restrict__ U,
                                                                           const float *__restrict__ V,
                                                                           int pre, int64_t I, int J,
                                                                           int post,
                                                                           float *__restrict__ out) {
  __shared__ float ws[kSplitWaves][JM];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = blockIdx.x;
  const int total = pre * post;
  const int per = (total + kSplitWaves - 1) / kSplitWaves;
  const int tb = w * per, te = min(total, tb + per);
  float acc[JM];
#pragma unroll
  for (int j = 0; j < JM; ++j) acc[j] = 0.f;
  for (int t0 = tb + lane; t0 < te; t0 += 256) {
    float u[4];
    int vo[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int t = t0 + 64 * k;
      const bool ok = t < te;
      const int tt = ok ? t : tb;
      const int p = tt / post, q = tt - (tt / post) * post;
      u[k] = ok ? U[((int64_t)p * I + i) * post + q] : 0.f;
      vo[k] = p * J * post + q;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
      for (int j = 0; j < JM; ++j)
        if (j < J) acc[j] = fmaf(u[k], V[vo[k] + j * post], acc[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < JM; ++j) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) acc[j] += __shfl_xor(acc[j], m, 64);
  }
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < JM; ++j) ws[w][j] = acc[j];
  }
  __syncthreads();
  if (threadIdx.x < J) {
    float sum = 0.f;
    for (int ww = 0; ww < kSplitWaves; ++ww) sum += ws[ww][threadIdx.x];
    out[i * J + threadIdx.x] = sum;
  }
}

nnc_status launch_contract_except(const float *U, const float *V, int64_t pre, int64_t I, int64_t J,
                                  int64_t post, float *out, hipStream_t s) {
  if (J <= 32 && I <= 64 && pre * post >= 64 * kSplitWaves && pre * J * post < INT32_MAX) {
    // few rows and a long sum: every row's sum split over a block of waves
#define NNC_CE_SPLIT(JM)                                                                        \
  hipLaunchKernelGGL(contract_except_split_k<JM>, dim3((unsigned)I), dim3(64 * kSplitWaves), 0, s, U, V, \
                     (int)pre, I, (int)J, (int)post, out)
    if (J <= 8)
      NNC_CE_SPLIT(8);
    else if (J <= 16)
      NNC_CE_SPLIT(16);
    else
      NNC_CE_SPLIT(32);
#undef NNC_CE_SPLIT
    NNC_HIP(hipGetLastError());
    return NNC_OK;
  }
  if (J <= 32 && pre * J * post < INT32_MAX && I < ((int64_t)1 << 31) / 64) {
    const int grid = (int)((I + 3) / 4);
#define NNC_CE_ROWS(JM)                                                                              \
  hipLaunchKernelGGL(contract_except_rows_k<JM>, dim3(grid), dim3(256), 0, s, U, V, (int)pre, I, (int)J, \
                     (int)post, out)
    if (J <= 8)
      NNC_CE_ROWS(8);
    else if (J <= 16)
      NNC_CE_ROWS(16);
    else
      NNC_CE_ROWS(32);
#undef NNC_CE_ROWS
    NNC_HIP(hipGetLastError());
    return NNC_OK;
  }
  const int64_t n = I * J;
  hipLaunchKernelGGL(contract_except_k, dim3(grid_for(n, 128, 1 << 30)), dim3(128), 0, s, U, V, pre,
                     I, J, post, out);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

__global__ void gram_k(const float *__restrict__ A, int64_t N, int64_t R, float *__restrict__ S) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= R * R) return;
  const int64_t r = idx / R, c = idx - (idx / R) * R;
  float acc = 0.f;
  for (int64_t i = 0; i < N; ++i) acc = fmaf(A[i * R + r], A[i * R + c], acc);
  S[idx] = acc;
}

nnc_status launch_gram(const float *A, int64_t N, int64_t R, float *S, hipStream_t s) {
  if (R <= 32) return launch_gram_block(A, N, (int)R, S, s);  // one workgroup, rows staged in LDS
  hipLaunchKernelGGL(gram_k, dim3(grid_for(R * R, 64, 1 << 30)), dim3(64), 0, s, A, N, R, S);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

static __device__ inline float mu_step(float x, float num, float den, double eps,
                                       unsigned long long *clips) {
  double dd = (double)den;
  if (dd < eps) {
    dd = eps;
    atomicAdd(clips, 1ull);
  }
  return (float)(((double)x * (double)num) / dd);
}

// Rows are owned by one block; every thread reads its row of A before the barrier and
// writes its entry after it.
__global__ void mu_factor_k(float *__restrict__ A, const float *__restrict__ num,
                            const float *__restrict__ M, int64_t N, int64_t R, double eps,
                            unsigned long long *clips) {
  const int64_t rpb = blockDim.x / R;
  const int64_t i = (int64_t)blockIdx.x * rpb + threadIdx.x / R;
  const int64_t r = threadIdx.x % R;
  const bool act = threadIdx.x < rpb * R && i < N;
  float nv = 0.f;
  if (act) {
    float den = 0.f;
    for (int64_t s = 0; s < R; ++s) den = fmaf(A[i * R + s], M[s * R + r], den);
    nv = mu_step(A[i * R + r], num[i * R + r], den, eps, clips);
  }
  __syncthreads();
  if (act) A[i * R + r] = nv;
}

nnc_status launch_mu_factor(float *A, const float *num, const float *M, int64_t N, int64_t R,
                            double eps, unsigned long long *clips, hipStream_t s) {
  const int threads = 256;
  if (R > threads) return fail(NNC_EUNSUPPORTED, "rank %lld above %d", (long long)R, threads);
  const int64_t rpb = threads / R;
  hipLaunchKernelGGL(mu_factor_k, dim3((unsigned)((N + rpb - 1) / rpb)), dim3(threads), 0, s, A, num,
                     M, N, R, eps, clips);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

__global__ void mu_elem_k(float *__restrict__ x, const float *__restrict__ num,
                          const float *__restrict__ den, int64_t n, double eps,
                          unsigned long long *clips) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = mu_step(x[i], num[i], den[i], eps, clips);
}

nnc_status launch_mu_elem(float *x, const float *num, const float *den, int64_t n, double eps,
                          unsigned long long *clips, hipStream_t s) {
  hipLaunchKernelGGL(mu_elem_k, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, x, num, den, n, eps,
                     clips);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

__global__ void sub_k(const float *__restrict__ a, const float *__restrict__ b, float *__restrict__ o,
                      int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    o[i] = a[i] - b[i];
}

nnc_status launch_sub(const float *den, const float *num, float *out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(sub_k, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, den, num, out, n);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

__global__ void matmul_small_k(const float *__restrict__ A, const float *__restrict__ M, int64_t N,
                               int64_t R, int64_t C, float *__restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * C) return;
  const int64_t i = idx / C, c = idx - (idx / C) * C;
  float acc = 0.f;
  for (int64_t s = 0; s < R; ++s) acc = fmaf(A[i * R + s], M[s * C + c], acc);
  out[idx] = acc;
}

nnc_status launch_matmul_small(const float *A, const float *M, int64_t N, int64_t R, int64_t C,
                               float *out, hipStream_t s) {
  hipLaunchKernelGGL(matmul_small_k, dim3(grid_for(N * C, 256, 1 << 30)), dim3(256), 0, s, A, M, N,
                     R, C, out);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

nnc_status launch_lift(const float *A, const float *B, int64_t N, int64_t Rm, int64_t r, float *C,
                       hipStream_t s) {
  return launch_matmul_small(A, B, N, Rm, r, C, s);
}

struct KrArgs {
  int d;
  int64_t dims[kMaxDim];
  const float *C[kMaxDim];
};

// W[m][rho] = prod_{k < d-1} C_k[i_k][rho] for the flattened leading index m.
__global__ void kr_rows_k(KrArgs a, int64_t lead, int64_t r, float *__restrict__ W) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < lead * r;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t rho = idx % r;
    int64_t m = idx / r;
    float p = 1.f;
    for (int k = a.d - 2; k >= 0; --k) {
      const int64_t ik = m % a.dims[k];
      m /= a.dims[k];
      p *= a.C[k][ik * r + rho];
    }
    W[idx] = p;
  }
}

nnc_status launch_kr_rows(int d, const int64_t *dims, int64_t r, const float *const *C, float *W,
                          hipStream_t s) {
  KrArgs a;
  a.d = d;
  int64_t lead = 1;
  for (int k = 0; k < d; ++k) {
    a.dims[k] = dims[k];
    a.C[k] = C[k];
    if (k < d - 1) lead *= dims[k];
  }
  hipLaunchKernelGGL(kr_rows_k, dim3(grid_for(lead * r, 256, 65536)), dim3(256), 0, s, a, lead, r, W);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

// =====================================================================================
// Residual: sum over X (M x K) of (x - W[m,:] . Ad[k,:])^2 and of x^2, accumulated per
// thread in double, then a fixed-shape tree per block.  The grid size depends only on
// the problem size, so the summation order (and the result) is reproducible.
// =====================================================================================
constexpr int kResidThreads = 256;
constexpr int kResidMaxBlocks = 2048;

int resid_stream_max_blocks() { return kResidMaxBlocks; }

// ||X - Xhat||^2 and ||X||^2 with Xhat[m][k] = sum_r W[m][r] Ad[k][r] (X viewed as M x K,
// W the expansion of every mode but the last, Ad the last factor).  A block takes tiles of
// kResidRows rows: the tile's W rows go to LDS, each thread keeps the factor rows of its
// columns k = t + 256 j (j < kResidCols) in registers and reads X along rows (coalesced).
// Each difference is formed and squared in FP64; sums are FP64 per thread, then per block.
// Rows past M are read clamped and left out of the sums by a predicate (not a loop exit), so
// the products of the tile's rows can interleave.
constexpr int kResidRows = 16;

template <typename XT, int RB, int kResidCols>  // columns per thread per chunk (1 when K <= 256)
__global__ __launch_bounds__(kResidThreads) void resid_stream_k(const XT *__restrict__ X, int64_t M,
                                                                int64_t K, const float *__restrict__ W,
                                                                const float *__restrict__ Ad,
                                                                int R, double *__restrict__ part) {
  __shared__ __attribute__((aligned(16))) float Ws[kResidRows][RB];
  __shared__ double s0[kResidThreads], s1[kResidThreads];
  const int t = threadIdx.x;
  double sr = 0.0, sx = 0.0;
  const int64_t ntile = (M + kResidRows - 1) / kResidRows;
  constexpr int64_t kChunk = (int64_t)kResidThreads * kResidCols;
  for (int64_t k0 = 0; k0 < K; k0 += kChunk) {
    float a[kResidCols][RB];
    int64_t kc[kResidCols];
    bool kv[kResidCols];
#pragma unroll
    for (int j = 0; j < kResidCols; ++j) {
      const int64_t k = k0 + t + (int64_t)j * kResidThreads;
      kv[j] = k < K;
      kc[j] = kv[j] ? k : K - 1;
#pragma unroll
      for (int r = 0; r < RB; ++r) a[j][r] = (kv[j] && r < R) ? Ad[kc[j] * R + r] : 0.f;
    }
    for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
      const int64_t m0 = tile * kResidRows;
      __syncthreads();  // the previous tile's W rows are no longer read
      for (int e = t; e < kResidRows * RB; e += kResidThreads) {
        const int row = e / RB, r = e - (e / RB) * RB;
        const int64_t m = m0 + row;
        Ws[row][r] = (m < M && r < R) ? W[m * R + r] : 0.f;
      }
      // the tile's X values, all loads in flight together
      float xv[kResidRows][kResidCols];
#pragma unroll
      for (int row = 0; row < kResidRows; ++row) {
        const int64_t m = (m0 + row) < M ? (m0 + row) : M - 1;
#pragma unroll
        for (int j = 0; j < kResidCols; ++j) xv[row][j] = load_x(X + m * K + kc[j]);
      }
      __syncthreads();
#pragma unroll
      for (int row = 0; row < kResidRows; ++row) {
        const bool rv = m0 + row < M;
        const float4 *w4 = reinterpret_cast<const float4 *>(&Ws[row][0]);
        float xh[kResidCols];
#pragma unroll
        for (int j = 0; j < kResidCols; ++j) xh[j] = 0.f;
#pragma unroll
        for (int r4 = 0; r4 < RB / 4; ++r4) {
          const float4 w = w4[r4];
#pragma unroll
          for (int j = 0; j < kResidCols; ++j) {
            xh[j] = fmaf(w.x, a[j][4 * r4 + 0], xh[j]);
            xh[j] = fmaf(w.y, a[j][4 * r4 + 1], xh[j]);
            xh[j] = fmaf(w.z, a[j][4 * r4 + 2], xh[j]);
            xh[j] = fmaf(w.w, a[j][4 * r4 + 3], xh[j]);
          }
        }
#pragma unroll
        for (int j = 0; j < kResidCols; ++j) {
          if (!kv[j] || !rv) continue;
          const double df = (double)xv[row][j] - (double)xh[j];
          sr += df * df;
          sx += (double)xv[row][j] * (double)xv[row][j];
        }
      }
    }
  }
  s0[t] = sr;
  s1[t] = sx;
  __syncthreads();
  for (int w = kResidThreads / 2; w > 0; w >>= 1) {
    if (t < w) {
      s0[t] += s0[t + w];
      s1[t] += s1[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[2 * blockIdx.x] = s0[0];
    part[2 * blockIdx.x + 1] = s1[0];
  }
}

// Any rank: one thread per element, the rank loop from global memory (L1/L2 hits).
template <typename XT>
__global__ __launch_bounds__(kResidThreads) void resid_any_k(const XT *__restrict__ X, int64_t M,
                                                             int64_t K, const float *__restrict__ W,
                                                             const float *__restrict__ Ad,
                                                             int64_t R, double *__restrict__ part) {
  __shared__ double s0[kResidThreads], s1[kResidThreads];
  double sr = 0.0, sx = 0.0;
  const int64_t total = M * K;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = e / K, k = e - (e / K) * K;
    const float *w = W + m * R;
    const float *a = Ad + k * R;
    float xh = 0.f;
    for (int64_t r = 0; r < R; ++r) xh = fmaf(w[r], a[r], xh);
    const float x = load_x(X + e);
    const double df = (double)x - (double)xh;
    sr += df * df;
    sx += (double)x * (double)x;
  }
  s0[threadIdx.x] = sr;
  s1[threadIdx.x] = sx;
  __syncthreads();
  for (int w = kResidThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s0[threadIdx.x] += s0[threadIdx.x + w];
      s1[threadIdx.x] += s1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s0[0];
    part[2 * blockIdx.x + 1] = s1[0];
  }
}

nnc_status launch_resid_stream(const void *X, nnc_dtype xdt, int64_t M, int64_t K, const float *W,
                               const float *Ad, int64_t R, double *part, int *nblocks_out,
                               hipStream_t s) {
  if (R < 1) return fail(NNC_EINVAL, "residual: rank %lld", (long long)R);
  if (R > 32) {
    const int grid = grid_for(M * K, kResidThreads, kResidMaxBlocks);
    if (xdt == NNC_F32)
      hipLaunchKernelGGL(resid_any_k<float>, dim3(grid), dim3(kResidThreads), 0, s,
                         (const float *)X, M, K, W, Ad, R, part);
    else
      hipLaunchKernelGGL(resid_any_k<uint16_t>, dim3(grid), dim3(kResidThreads), 0, s,
                         (const uint16_t *)X, M, K, W, Ad, R, part);
    *nblocks_out = grid;
    NNC_HIP(hipGetLastError());
    return NNC_OK;
  }
  const int64_t ntile = (M + kResidRows - 1) / kResidRows;
  const int grid = (int)std::min<int64_t>(std::max<int64_t>(ntile, 1), kResidMaxBlocks);
#define NNC_RES(XT, RBV)                                                                              \
  do {                                                                                                \
    if (K <= kResidThreads)                                                                           \
      hipLaunchKernelGGL((resid_stream_k<XT, RBV, 1>), dim3(grid), dim3(kResidThreads), 0, s,         \
                         (const XT *)X, M, K, W, Ad, (int)R, part);                                   \
    else                                                                                              \
      hipLaunchKernelGGL((resid_stream_k<XT, RBV, 2>), dim3(grid), dim3(kResidThreads), 0, s,         \
                         (const XT *)X, M, K, W, Ad, (int)R, part);                                   \
  } while (0)
#define NNC_RES2(XT)                    \
  do {                                  \
    if (R <= 8) NNC_RES(XT, 8);         \
    else if (R <= 16) NNC_RES(XT, 16);  \
    else if (R <= 24) NNC_RES(XT, 24);  \
    else NNC_RES(XT, 32);               \
  } while (0)
  if (xdt == NNC_F32)
    NNC_RES2(float);
  else
    NNC_RES2(uint16_t);
#undef NNC_RES2
#undef NNC_RES
  *nblocks_out = grid;
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

__global__ void reduce_pairs_k(const double *__restrict__ part, int n, double *__restrict__ out) {
  __shared__ double s0[256], s1[256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s0[threadIdx.x] += s0[threadIdx.x + w];
      s1[threadIdx.x] += s1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s0[0];
    out[1] = s1[0];
  }
}

nnc_status launch_reduce_pairs(const double *part, int n, double *out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_pairs_k, dim3(1), dim3(256), 0, s, part, n, out);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

__global__ void convert_bf16_k(const float *__restrict__ in, uint16_t *__restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = f2bf_rne(in[i]);
}

// =====================================================================================
// Counter-based SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): element i of a stream with
// key K is mix64(K + (i + 1) * GAMMA), mix64 being SplitMix64's finaliser; a uniform double
// in [0, 1) is its top 53 bits times 2^-53.  Each element depends only on (K, i), so any
// slice of a stream is generated on its own, in any order.
// =====================================================================================
constexpr uint64_t kSmGamma = 0x9E3779B97F4A7C15ull;

static __host__ __device__ inline uint64_t sm_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t uniform_stream_key(uint64_t seed, uint64_t stream_id) {
  return sm_mix64(sm_mix64(seed + kSmGamma) ^ (stream_id * 0xD1B54A32D192ED03ull));
}

__global__ void fill_uniform_k(uint64_t key, int64_t offset, int64_t n, float *__restrict__ out32,
                               double *__restrict__ out64) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t z = sm_mix64(key + (uint64_t)(offset + i + 1) * kSmGamma);
    const double u = (double)(z >> 11) * 0x1.0p-53;  // exact: 53-bit integer times 2^-53
    if (out32)
      out32[i] = (float)u;  // round to nearest even
    else
      out64[i] = u;
  }
}

nnc_status launch_fill_uniform(uint64_t key, int64_t offset, int64_t n, float *out32, double *out64,
                               hipStream_t s) {
  hipLaunchKernelGGL(fill_uniform_k, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, key, offset, n,
                     out32, out64);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

nnc_status launch_convert_bf16(const float *in, uint16_t *out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(convert_bf16_k, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, in, out, n);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

__global__ void check_finite_k(const float *__restrict__ x, int64_t n, unsigned int *flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) atomicOr(flag, 1u);
}

nnc_status launch_check_finite(const float *x, int64_t n, unsigned int *flag, hipStream_t s) {
  hipLaunchKernelGGL(check_finite_k, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, x, n, flag);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

__global__ void fill_u64_k(unsigned long long *x, int64_t n, unsigned long long v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

__global__ void fill_f32_k(float *x, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

nnc_status launch_fill_u64(unsigned long long *x, int64_t n, unsigned long long v, hipStream_t s) {
  hipLaunchKernelGGL(fill_u64_k, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, x, n, v);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

nnc_status launch_fill_f32(float *x, int64_t n, float v, hipStream_t s) {
  hipLaunchKernelGGL(fill_f32_k, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, x, n, v);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

}  // namespace nnc
