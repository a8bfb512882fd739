// Small steps of the nonnegative CP fit of the data tensor itself (the nnCPD step of
// Algorithm 2), around the two X-streaming contractions it shares with the Tucker sweep.
//
// With Z = X x_{d-1} B_{d-1}^T (rank index last) and T = X x_0 B_0^T (rank index first), the
// MTTKRP of every mode is a rank-wise ("diagonal") contraction of Z or T with the current
// factors of the remaining modes:
//   M_n[i][rho] = sum_{a, c} Y[a][i][c][rho] WA[a][rho] WC[c][rho]      (rank index last)
//   M_n[i][rho] = sum_{a, c} Y[rho][a][i][c] WA[a][rho] WC[c][rho]      (rank index first)
// where a runs over the modes of Y before mode n and c over those after it, and WA / WC are
// the Khatri-Rao rows of those modes' factors.  The multiplicative update then uses
// H_n = Hadamard product of the other factors' Grams (reading R1 applied to CP).
#include <string.h>

#include <algorithm>

#include "nnc_internal.h"

namespace nnc {

constexpr int kDiagThreads = 256;

struct DiagArgs {
  const float *Y;
  const float *WA, *WC;  // null: weight 1
  int64_t A, Nt, C;
  int r;
  int rho_first;
  float *out;    // [Nt][r] (one slice) or partials [slices][Nt][r]
  int slices;
};

static __device__ inline float diag_y(const DiagArgs &g, int64_t a, int64_t i, int64_t c, int rho) {
  const int64_t e = (a * g.Nt + i) * g.C + c;
  return g.rho_first ? g.Y[(int64_t)rho * g.A * g.Nt * g.C + e] : g.Y[e * g.r + rho];
}

static __device__ inline float diag_w(const DiagArgs &g, int64_t a, int64_t c, int rho) {
  float w = g.WA ? g.WA[a * g.r + rho] : 1.f;
  if (g.WC) w *= g.WC[c * g.r + rho];
  return w;
}

// C > 1: block (i, slice); the threads stride over the flattened (a, c) range of the slice
// (c fastest, contiguous in Y) and the partial sums are combined by a fixed pairwise tree.
template <int RM>
__global__ __launch_bounds__(kDiagThreads) void diag_inner_k(DiagArgs g) {
  __shared__ float red[kDiagThreads * RM];
  const int64_t i = blockIdx.x % g.Nt;
  const int s = (int)(blockIdx.x / g.Nt);
  const int64_t F = g.A * g.C;
  const int64_t f0 = F * s / g.slices, f1 = F * (s + 1) / g.slices;
  float acc[RM];
#pragma unroll
  for (int q = 0; q < RM; ++q) acc[q] = 0.f;
  int64_t f = f0 + threadIdx.x;
  int64_t a = f / g.C, c = f - a * g.C;  // advanced incrementally below
  for (; f < f1; f += kDiagThreads) {
#pragma unroll
    for (int q = 0; q < RM; ++q)
      if (q < g.r) acc[q] = fmaf(diag_y(g, a, i, c, q), diag_w(g, a, c, q), acc[q]);
    c += kDiagThreads;
    if (c >= g.C) {
      a += c / g.C;
      c %= g.C;
    }
  }
#pragma unroll
  for (int q = 0; q < RM; ++q) red[q * kDiagThreads + threadIdx.x] = acc[q];
  __syncthreads();
  for (int h = kDiagThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
#pragma unroll
      for (int q = 0; q < RM; ++q) red[q * kDiagThreads + threadIdx.x] += red[q * kDiagThreads + threadIdx.x + h];
    __syncthreads();
  }
  if ((int)threadIdx.x < g.r) g.out[((int64_t)s * g.Nt + i) * g.r + threadIdx.x] = red[threadIdx.x * kDiagThreads];
}

// C == 1: block (tile of 64 consecutive i, slice of a); lane <-> i (contiguous in Y), the
// four waves stride over a and their sums are added in wave order.
template <int RM>
__global__ __launch_bounds__(kDiagThreads) void diag_outer_k(DiagArgs g) {
  __shared__ float red[kDiagThreads * RM];
  const int64_t tiles = (g.Nt + 63) / 64;
  const int64_t tile = blockIdx.x % tiles;
  const int s = (int)(blockIdx.x / tiles);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = tile * 64 + lane;
  const bool live = i < g.Nt;
  const int64_t a0 = g.A * s / g.slices, a1 = g.A * (s + 1) / g.slices;
  float acc[RM];
#pragma unroll
  for (int q = 0; q < RM; ++q) acc[q] = 0.f;
  if (live)
    for (int64_t a = a0 + w; a < a1; a += kDiagThreads / 64) {
#pragma unroll
      for (int q = 0; q < RM; ++q)
        if (q < g.r) acc[q] = fmaf(diag_y(g, a, i, 0, q), diag_w(g, a, 0, q), acc[q]);
    }
#pragma unroll
  for (int q = 0; q < RM; ++q) red[(w * RM + q) * 64 + lane] = acc[q];
  __syncthreads();
  for (int idx = threadIdx.x; idx < RM * 64; idx += kDiagThreads) {
    const int q = idx >> 6, l = idx & 63;
    const int64_t ii = tile * 64 + l;
    if (q >= g.r || ii >= g.Nt) continue;
    float t = red[q * 64 + l];
    for (int ww = 1; ww < kDiagThreads / 64; ++ww) t += red[(ww * RM + q) * 64 + l];
    g.out[((int64_t)s * g.Nt + ii) * g.r + q] = t;
  }
}

// out[e] = sum_{s < slices} part[s][e], s in order.
__global__ void diag_sum_k(const float *__restrict__ part, int slices, int64_t n, float *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  float t = part[e];
  for (int s = 1; s < slices; ++s) t += part[(int64_t)s * n + e];
  out[e] = t;
}

int64_t diag_slices(int64_t A, int64_t Nt, int64_t C) {
  if (C > 1) {
    const int64_t per = std::max<int64_t>(1, 512 / Nt);
    return std::max<int64_t>(1, std::min<int64_t>(per, (A * C) / (kDiagThreads * 4)));
  }
  const int64_t tiles = (Nt + 63) / 64;
  const int64_t per = std::max<int64_t>(1, 512 / tiles);
  return std::max<int64_t>(1, std::min<int64_t>(per, A / 16));
}

nnc_status launch_diag(const float *Y, int rho_first, int64_t A, int64_t Nt, int64_t C, const float *WA,
                       const float *WC, int r, float *out, float *part, hipStream_t s) {
  if (r < 1 || r > 32) return fail(NNC_EUNSUPPORTED, "rank %d outside [1, 32]", r);
  const int64_t S = diag_slices(A, Nt, C);
  if (S > 1 && !part) return fail(NNC_EINVAL, "diag: partial buffer missing");
  DiagArgs g{Y, WA, WC, A, Nt, C, r, rho_first, S > 1 ? part : out, (int)S};
  const int64_t blocks = C > 1 ? Nt * S : ((Nt + 63) / 64) * S;
  if (blocks > 0x7fffffff) return fail(NNC_EUNSUPPORTED, "diag: grid too large");
  const int RM = r <= 8 ? 8 : (r <= 16 ? 16 : 32);
#define NNC_DIAG(KERN)                                                                         \
  do {                                                                                         \
    if (RM == 8) hipLaunchKernelGGL(KERN<8>, dim3((unsigned)blocks), dim3(kDiagThreads), 0, s, g);   \
    else if (RM == 16) hipLaunchKernelGGL(KERN<16>, dim3((unsigned)blocks), dim3(kDiagThreads), 0, s, g); \
    else hipLaunchKernelGGL(KERN<32>, dim3((unsigned)blocks), dim3(kDiagThreads), 0, s, g);          \
  } while (0)
  if (C > 1) NNC_DIAG(diag_inner_k);
  else NNC_DIAG(diag_outer_k);
#undef NNC_DIAG
  if (S > 1) {
    const int64_t n = Nt * r;
    hipLaunchKernelGGL(diag_sum_k, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, (int)S, n, out);
  }
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

int64_t diag_part_floats(int64_t A, int64_t Nt, int64_t C, int r) {
  const int64_t S = diag_slices(A, Nt, C);
  return S > 1 ? S * Nt * r : 0;
}

// B <- B * M / max(B H, eps) with H = prod_{k != n} S_k (entrywise, S packed [d][r][r]);
// FP64 division, clipped denominators counted.  Thread (row, rho), 256 / r rows per block.
__global__ __launch_bounds__(256) void cp_mu_k(float *__restrict__ B, const float *__restrict__ M,
                                               const float *__restrict__ S, int d, int n, int64_t N,
                                               int r, double eps, unsigned long long *clips) {
  __shared__ float H[32 * 32];
  __shared__ unsigned int nclip;
  const int tid = threadIdx.x;
  for (int e = tid; e < r * r; e += 256) {
    float h = 1.f;
    for (int k = 0; k < d; ++k)
      if (k != n) h *= S[(int64_t)k * r * r + e];
    H[e] = h;
  }
  if (tid == 0) nclip = 0;
  __syncthreads();
  const int rpb = 256 / r;
  const int64_t i = (int64_t)blockIdx.x * rpb + tid / r;
  const int q = tid % r;
  const bool act = tid < rpb * r && i < N;
  float nv = 0.f;
  unsigned int mine = 0;
  if (act) {
    float den = 0.f;
    for (int t = 0; t < r; ++t) den = fmaf(B[i * r + t], H[t * r + q], den);
    double dd = (double)den;
    if (dd < eps) {
      dd = eps;
      mine = 1;
    }
    nv = (float)(((double)B[i * r + q] * (double)M[i * r + q]) / dd);
  }
  if (mine) atomicAdd(&nclip, mine);
  __syncthreads();  // every row of the block is read before any is written
  if (act) B[i * r + q] = nv;
  if (tid == 0 && nclip) atomicAdd(clips, (unsigned long long)nclip);
}

nnc_status launch_cp_mu(float *B, const float *M, const float *S, int d, int n, int64_t N, int r,
                        double eps, unsigned long long *clips, hipStream_t s) {
  if (r < 1 || r > 32) return fail(NNC_EUNSUPPORTED, "rank %d outside [1, 32]", r);
  const int64_t rpb = 256 / r;
  hipLaunchKernelGGL(cp_mu_k, dim3((unsigned)((N + rpb - 1) / rpb)), dim3(256), 0, s, B, M, S, d, n, N,
                     r, eps, clips);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

// S = A^T A (A: N x r, r <= 32) in one workgroup: thread (entry, split) sums the rows of its
// split (rows j with j mod splits == split), the splits are added in order.
__global__ __launch_bounds__(1024) void gram_block_k(const float *__restrict__ A, int64_t N, int r,
                                                     float *__restrict__ S) {
  __shared__ float part[1024];
  const int tid = threadIdx.x;
  const int rr = r * r;
  const int splits = 1024 / rr;
  const int e = tid % rr, sp = tid / rr;
  float acc = 0.f;
  if (sp < splits) {
    const int a = e / r, b = e - (e / r) * r;
#pragma unroll 4
    for (int64_t j = sp; j < N; j += splits) acc = fmaf(A[j * r + a], A[j * r + b], acc);
  }
  part[tid] = acc;
  __syncthreads();
  if (tid < rr) {
    float t = part[tid];
    for (int k = 1; k < splits; ++k) t += part[k * rr + tid];
    S[tid] = t;
  }
}

nnc_status launch_gram_block(const float *A, int64_t N, int r, float *S, hipStream_t s) {
  if (r < 1 || r > 32) return fail(NNC_EUNSUPPORTED, "rank %d outside [1, 32]", r);
  hipLaunchKernelGGL(gram_block_k, dim3(1), dim3(1024), 0, s, A, N, r, S);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

// out[j][i] = in[i][j] (rows x cols -> cols x rows), small matrices.
__global__ void transpose_k(const float *__restrict__ in, int64_t rows, int64_t cols, float *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e / cols, j = e - (e / cols) * cols;
  out[j * rows + i] = in[e];
}

nnc_status launch_transpose(const float *in, int64_t rows, int64_t cols, float *out, hipStream_t s) {
  const int64_t n = rows * cols;
  if (n == 0) return NNC_OK;
  hipLaunchKernelGGL(transpose_k, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, rows, cols, out);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

}  // namespace nnc

namespace nnc {

// =====================================================================================
// NMF A ~ W H (Lee-Seung multiplicative sweeps, W first, then H) of up to kNmfMax
// independent problems with a common column count, one workgroup per problem with A, W, H
// and the small products in LDS:
//   G = H H^T;  W <- W * (A H^T) / max(W G, eps);
//   G = W^T W, P = W^T A (sums over the rows split in kNmfSplit ranges added in order);
//   H <- H * P / max(G H, eps).
// A is rows x cols, W rows x m, H m x cols; FP32 products, FP64 divisions, clipped
// denominators counted; ||A - W H||^2 and ||A||^2 in FP64 at the end.
// =====================================================================================
constexpr int kNmfMax = 8;
constexpr int kNmfThreads = 1024;
constexpr int kNmfSplit = 4;
constexpr int kNmfVals = 32;  // W entries per thread: rows * m <= kNmfThreads * kNmfVals
constexpr size_t kNmfLdsMax = 159 * 1024;  // dynamic LDS; the static part (counters) stays below 1 KiB

struct NmfArgs {
  const float *A[kNmfMax];
  float *W[kNmfMax];
  float *H[kNmfMax];
  int rows[kNmfMax], m[kNmfMax];
  int cols, iters;
  double eps;
  unsigned long long *clips;
  double *red;  // [problem][2] (||A - W H||^2, ||A||^2) or null
};

size_t nmf_lds_floats(int rows, int cols, int m) {
  const size_t pairs = (size_t)kNmfSplit * (m * m + m * cols);
  return (size_t)rows * cols + (size_t)rows * m + (size_t)m * cols + (size_t)m * m + (size_t)m * cols + pairs;
}

bool nmf_block_fits(int rows, int cols, int m) {
  return cols <= 32 && m <= 32 && (int64_t)rows * m <= (int64_t)kNmfThreads * kNmfVals &&
         m * cols <= kNmfThreads && nmf_lds_floats(rows, cols, m) * 4 <= kNmfLdsMax;
}

__global__ __launch_bounds__(kNmfThreads) void nmf_block_k(NmfArgs g) {
  extern __shared__ __attribute__((aligned(16))) float sm[];
  __shared__ unsigned int nclip;
  __shared__ double dred[2][kNmfThreads / 64];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int N = g.rows[b], m = g.m[b], r = g.cols;
  const float *__restrict__ Ag = g.A[b];
  float *__restrict__ Wg = g.W[b];
  float *__restrict__ Hg = g.H[b];
  float *A = sm, *W = A + N * r, *H = W + N * m, *G = H + m * r, *P = G + m * m, *part = P + m * r;
  for (int e = tid; e < N * r; e += kNmfThreads) A[e] = Ag[e];
  for (int e = tid; e < N * m; e += kNmfThreads) W[e] = Wg[e];
  for (int e = tid; e < m * r; e += kNmfThreads) H[e] = Hg[e];
  if (tid == 0) nclip = 0;
  __syncthreads();
  unsigned int mine = 0;
  const double eps = g.eps;
  auto mu = [&](float x, float num, float den) {
    double dd = (double)den;
    if (dd < eps) {
      dd = eps;
      ++mine;
    }
    return (float)(((double)x * (double)num) / dd);
  };
  const int O = m * m + m * r;  // outputs of the row reduction
  for (int it = 0; it < g.iters; ++it) {
    for (int e = tid; e < m * m; e += kNmfThreads) {  // G = H H^T
      const int j = e / m, k = e - (e / m) * m;
      float s = 0.f;
      for (int q = 0; q < r; ++q) s = fmaf(H[j * r + q], H[k * r + q], s);
      G[e] = s;
    }
    __syncthreads();
    float nv[kNmfVals];
#pragma unroll
    for (int u = 0; u < kNmfVals; ++u) {  // W <- W * (A H^T) / max(W G, eps)
      const int e = tid + u * kNmfThreads;
      if (e < N * m) {
        const int i = e / m, j = e - (e / m) * m;
        float num = 0.f, den = 0.f;
        for (int q = 0; q < r; ++q) num = fmaf(A[i * r + q], H[j * r + q], num);
        for (int k = 0; k < m; ++k) den = fmaf(W[i * m + k], G[k * m + j], den);
        nv[u] = mu(W[e], num, den);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kNmfVals; ++u) {
      const int e = tid + u * kNmfThreads;
      if (e < N * m) W[e] = nv[u];
    }
    __syncthreads();
    for (int pidx = tid; pidx < kNmfSplit * O; pidx += kNmfThreads) {  // W^T W and W^T A, split rows
      const int sp = pidx / O, o = pidx - (pidx / O) * O;
      const int i0 = N * sp / kNmfSplit, i1 = N * (sp + 1) / kNmfSplit;
      float s = 0.f;
      if (o < m * m) {
        const int j = o / m, k = o - (o / m) * m;
        for (int i = i0; i < i1; ++i) s = fmaf(W[i * m + j], W[i * m + k], s);
      } else {
        const int o2 = o - m * m, j = o2 / r, q = o2 - (o2 / r) * r;
        for (int i = i0; i < i1; ++i) s = fmaf(W[i * m + j], A[i * r + q], s);
      }
      part[pidx] = s;
    }
    __syncthreads();
    for (int o = tid; o < O; o += kNmfThreads) {
      float s = part[o];
      for (int sp = 1; sp < kNmfSplit; ++sp) s += part[sp * O + o];
      if (o < m * m) G[o] = s;
      else P[o - m * m] = s;
    }
    __syncthreads();
    float hv = 0.f;  // H <- H * (W^T A) / max(W^T W H, eps)
    if (tid < m * r) {
      const int j = tid / r, q = tid - (tid / r) * r;
      float den = 0.f;
      for (int k = 0; k < m; ++k) den = fmaf(G[j * m + k], H[k * r + q], den);
      hv = mu(H[tid], P[tid], den);
    }
    __syncthreads();
    if (tid < m * r) H[tid] = hv;
    __syncthreads();
  }
  for (int e = tid; e < N * m; e += kNmfThreads) Wg[e] = W[e];
  for (int e = tid; e < m * r; e += kNmfThreads) Hg[e] = H[e];
  if (mine) atomicAdd(&nclip, mine);
  if (g.red) {  // ||A - W H||^2 and ||A||^2, FP64
    double se = 0.0, sa = 0.0;
    for (int e = tid; e < N * r; e += kNmfThreads) {
      const int i = e / r, q = e - (e / r) * r;
      float x = 0.f;
      for (int k = 0; k < m; ++k) x = fmaf(W[i * m + k], H[k * r + q], x);
      const double dlt = (double)A[e] - (double)x;
      se += dlt * dlt;
      sa += (double)A[e] * (double)A[e];
    }
    for (int off = 32; off > 0; off >>= 1) {
      se += __shfl_down(se, off);
      sa += __shfl_down(sa, off);
    }
    if ((tid & 63) == 0) {
      dred[0][tid >> 6] = se;
      dred[1][tid >> 6] = sa;
    }
  }
  __syncthreads();
  if (tid == 0) {
    if (nclip) atomicAdd(g.clips, (unsigned long long)nclip);
    if (g.red) {
      double a = 0.0, c = 0.0;
      for (int w = 0; w < kNmfThreads / 64; ++w) {
        a += dred[0][w];
        c += dred[1][w];
      }
      g.red[2 * b] = a;
      g.red[2 * b + 1] = c;
    }
  }
}

nnc_status launch_nmf_block(int n, const float *const *A, const int *rows, int cols, const int *m,
                            int iters, float *const *W, float *const *H, double eps,
                            unsigned long long *clips, double *red, hipStream_t s) {
  if (n < 1 || n > kNmfMax) return fail(NNC_EUNSUPPORTED, "nmf: %d problems per launch", n);
  NmfArgs g;
  memset(&g, 0, sizeof g);
  size_t lds = 0;
  for (int b = 0; b < n; ++b) {
    if (!nmf_block_fits(rows[b], cols, m[b])) return NNC_EUNSUPPORTED;
    g.A[b] = A[b];
    g.W[b] = W[b];
    g.H[b] = H[b];
    g.rows[b] = rows[b];
    g.m[b] = m[b];
    lds = std::max(lds, nmf_lds_floats(rows[b], cols, m[b]) * 4);
  }
  g.cols = cols;
  g.iters = iters;
  g.eps = eps;
  g.clips = clips;
  g.red = red;
  static bool raised = false;
  if (!raised) {
    NNC_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(nmf_block_k),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kNmfLdsMax));
    raised = true;
  }
  hipLaunchKernelGGL(nmf_block_k, dim3(n), dim3(kNmfThreads), lds, s, g);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

}  // namespace nnc
