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
// (c fastest, contiguous in Y) and the partial sums are combined by a fixed pairwise tree
// (thread t adds thread t + h for h = 128, 64, ..., 1).  The tree's two cross-wave steps
// go through LDS; its steps inside wave 0 are shuffles that pair the same lanes.
template <int RM>
__global__ __launch_bounds__(kDiagThreads) void diag_inner_k(DiagArgs g) {
  static_assert(kDiagThreads == 256, "the tree below has two cross-wave steps");
  __shared__ float red[kDiagThreads * RM];
  const int t = threadIdx.x;
  const int64_t i = blockIdx.x % g.Nt;
  const int s = (int)(blockIdx.x / g.Nt);
  const int64_t F = g.A * g.C;
  const int64_t f0 = F * s / g.slices, f1 = F * (s + 1) / g.slices;
  float acc[RM];
#pragma unroll
  for (int q = 0; q < RM; ++q) acc[q] = 0.f;
  int64_t f = f0 + t;
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
  for (int q = 0; q < RM; ++q) red[q * kDiagThreads + t] = acc[q];
  __syncthreads();
  if (t < 128)
#pragma unroll
    for (int q = 0; q < RM; ++q) red[q * kDiagThreads + t] += red[q * kDiagThreads + t + 128];
  __syncthreads();
  if (t < 64) {
    float v[RM];
#pragma unroll
    for (int q = 0; q < RM; ++q) v[q] = red[q * kDiagThreads + t] + red[q * kDiagThreads + t + 64];
#pragma unroll
    for (int h = 32; h > 0; h >>= 1)
#pragma unroll
      for (int q = 0; q < RM; ++q) v[q] += __shfl_down(v[q], h, 64);
    if (t == 0)
#pragma unroll
      for (int q = 0; q < RM; ++q)
        if (q < g.r) g.out[((int64_t)s * g.Nt + i) * g.r + q] = v[q];
  }
}
// C == 1: block (tile of 64 consecutive i, slice of a); lane <-> i (contiguous in Y), the
// four waves stride over a and their sums are added in wave order.  A wave issues the loads
// of kU steps of a before their products (each accumulator still takes its terms in
// ascending a); the rank index of a load is clamped instead of guarded, so no load waits on
// a branch (accumulators past r are never stored), and lanes past Nt read row Nt - 1 and
// are not stored either.
template <int RM>
__global__ __launch_bounds__(kDiagThreads) void diag_outer_k(DiagArgs g) {
  __shared__ float red[kDiagThreads * RM];
  const int64_t tiles = (g.Nt + 63) / 64;
  const int64_t tile = blockIdx.x % tiles;
  const int s = (int)(blockIdx.x / tiles);
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t i = tile * 64 + lane;
  const int64_t ic = i < g.Nt ? i : g.Nt - 1;
  const int64_t a0 = g.A * s / g.slices, a1 = g.A * (s + 1) / g.slices;
  constexpr int kW = kDiagThreads / 64;
  constexpr int kU = RM <= 16 ? 4 : 2;
  // rank entry q of row a for this lane: Y[(a Nt + i) r + q] (rank last) or
  // Y[q A Nt + a Nt + i] (rank first)
  const int64_t qstride = g.rho_first ? g.A * g.Nt : 1;
  const int64_t astride = g.rho_first ? g.Nt : g.Nt * g.r;
  const float *ylane = g.Y + (g.rho_first ? ic : ic * g.r);
  float acc[RM];
#pragma unroll
  for (int q = 0; q < RM; ++q) acc[q] = 0.f;
  for (int64_t ab = a0 + w; ab < a1; ab += kU * kW) {
    float y[kU][RM], wt[kU][RM];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t a = ab + u * kW;
      const int64_t ac = a < a1 ? a : a1 - 1;
      const float *yr = ylane + ac * astride;
#pragma unroll
      for (int q = 0; q < RM; ++q) {
        const int qc = q < g.r ? q : g.r - 1;
        y[u][q] = yr[qc * qstride];
        wt[u][q] = diag_w(g, ac, 0, qc);
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const bool ok = ab + u * kW < a1;
#pragma unroll
      for (int q = 0; q < RM; ++q) {
        const float t = fmaf(y[u][q], wt[u][q], acc[q]);
        acc[q] = ok ? t : acc[q];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RM; ++q) red[(w * RM + q) * 64 + lane] = acc[q];
  __syncthreads();
  for (int idx = threadIdx.x; idx < RM * 64; idx += kDiagThreads) {
    const int q = idx >> 6, l = idx & 63;
    const int64_t ii = tile * 64 + l;
    if (q >= g.r || ii >= g.Nt) continue;
    float t = red[q * 64 + l];
    for (int ww = 1; ww < kW; ++ww) t += red[(ww * RM + q) * 64 + l];
    g.out[((int64_t)s * g.Nt + ii) * g.r + q] = t;
  }
}
// out[e] = sum_{s < slices} part[s][e], s in order.
__global__ void diag_sum_k(const float *__restrict__ part, int slices, int64_t n, float *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  // slices in order; the loads of a group of kB are all in flight before the adds
  constexpr int kB = 16;
  float t = part[e];
  int s = 1;
  for (; s + kB <= slices; s += kB) {
    float v[kB];
#pragma unroll
    for (int k = 0; k < kB; ++k) v[k] = part[(int64_t)(s + k) * n + e];
#pragma unroll
    for (int k = 0; k < kB; ++k) t += v[k];
  }
  for (; s < slices; ++s) t += part[(int64_t)s * n + e];
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
// split (rows j with j mod splits == split) in ascending order, the splits are added in
// order.  Rows come through LDS in chunks of a multiple of `splits` rows, each chunk one
// round of coalesced loads: read from global memory, the sum waited on one load latency per
// few rows.
constexpr int kGramLds = 8192;  // floats of A staged per chunk
static __device__ void gram_block_body(const float *__restrict__ A, int64_t N, int r, float *__restrict__ S) {
  __shared__ float part[1024];
  __shared__ float As[kGramLds];
  const int tid = threadIdx.x;
  const int rr = r * r;
  const int splits = 1024 / rr;
  const int e = tid % rr, sp = tid / rr;
  const int a = e / r, b = e - (e / r) * r;
  const int64_t crows = (int64_t)(kGramLds / r / splits) * splits;  // rows per chunk
  float acc = 0.f;
  for (int64_t c0 = 0; c0 < N; c0 += crows) {
    const int64_t nrow = N - c0 < crows ? N - c0 : crows;
    const int nv = (int)(nrow * r);
    __syncthreads();  // the previous chunk is consumed
    constexpr int kPer = kGramLds / 1024;
    float v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int i = tid + u * 1024;
      v[u] = A[c0 * r + (i < nv ? i : 0)];
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int i = tid + u * 1024;
      if (i < nv) As[i] = v[u];
    }
    __syncthreads();
    if (sp < splits) {
#pragma unroll 8
      for (int j = sp; j < nrow; j += splits) acc = fmaf(As[j * r + a], As[j * r + b], acc);
    }
  }
  part[tid] = acc;
  __syncthreads();
  if (tid < rr) {
    float t = part[tid];
    for (int k = 1; k < splits; ++k) t += part[k * rr + tid];
    S[tid] = t;
  }
}

__global__ __launch_bounds__(1024) void gram_block_k(const float *__restrict__ A, int64_t N, int r,
                                                     float *__restrict__ S) {
  gram_block_body(A, N, r, S);
}

// The Grams of several factors at once, block k taking factor k.
struct GramSet {
  const float *A[kMaxDim];
  float *S[kMaxDim];
  int64_t N[kMaxDim];
  int r[kMaxDim];
};
__global__ __launch_bounds__(1024) void gram_set_k(GramSet g) {
  const int k = blockIdx.x;
  const float *A = nullptr;
  float *S = nullptr;
  int64_t N = 0;
  int r = 1;
#pragma unroll
  for (int j = 0; j < kMaxDim; ++j)  // selects by unrolled compares: no dynamic argument indexing
    if (j == k) {
      A = g.A[j];
      S = g.S[j];
      N = g.N[j];
      r = g.r[j];
    }
  gram_block_body(A, N, r, S);
}

nnc_status launch_gram_block(const float *A, int64_t N, int r, float *S, hipStream_t s) {
  if (r < 1 || r > 32) return fail(NNC_EUNSUPPORTED, "rank %d outside [1, 32]", r);
  hipLaunchKernelGGL(gram_block_k, dim3(1), dim3(1024), 0, s, A, N, r, S);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

nnc_status launch_gram_set(int d, const float *const *A, const int64_t *N, const int64_t *R, float *const *S,
                           hipStream_t s) {
  GramSet g;
  memset(&g, 0, sizeof g);
  for (int k = 0; k < d; ++k) {
    if (R[k] < 1 || R[k] > 32) return NNC_EUNSUPPORTED;
    g.A[k] = A[k];
    g.S[k] = S[k];
    g.N[k] = N[k];
    g.r[k] = (int)R[k];
  }
  hipLaunchKernelGGL(gram_set_k, dim3(d), dim3(1024), 0, s, g);
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
//   G = H H^T;  W <- W * (A H^T) / max(W G, eps)          (a thread per row of W)
//   G = W^T W, P = W^T A                                    (a thread per (column j of W,
//                                                            row range), ranges added in order)
//   H <- H * P / max(G H, eps).
// A is rows x cols, W rows x m, H m x cols; FP32 products, FP64 divisions, clipped
// denominators counted; ||A - W H||^2 and ||A||^2 in FP64 at the end.  RC / MC bound cols / m
// (8, 16 or 32) so that a row of A, of W and its new values stay in registers.
// =====================================================================================
constexpr int kNmfMax = 8;
constexpr int kNmfThreads = 512;
constexpr int kNmfSplitMax = 32;
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

__host__ __device__ static inline int nmf_splits(int m) { return kNmfThreads / m < kNmfSplitMax ? kNmfThreads / m : kNmfSplitMax; }

static inline int pad4(int x) { return (x + 3) & ~3; }

// LDS floats: A [rows][rp] | W [rows][mp] | H [m][rp] | P [m][rp] | G [m][mp] |
// partial sums [splits][m][mp + rp]   (rp, mp: cols and m rounded up to 4, zero padding)
size_t nmf_lds_floats(int rows, int cols, int m) {
  const size_t rp = pad4(cols), mp = pad4(m);
  return (size_t)rows * (rp + mp) + 2 * (size_t)m * rp + (size_t)m * mp + (size_t)nmf_splits(m) * m * (mp + rp);
}

bool nmf_block_fits(int rows, int cols, int m) {
  return cols <= 32 && m <= 32 && nmf_lds_floats(rows, cols, m) * 4 <= kNmfLdsMax;
}

static __device__ inline float dot4(float4 a, float4 b, float s) {
  s = fmaf(a.x, b.x, s);
  s = fmaf(a.y, b.y, s);
  s = fmaf(a.z, b.z, s);
  return fmaf(a.w, b.w, s);
}

template <int RC, int MC>
__global__ __launch_bounds__(kNmfThreads) void nmf_block_k(NmfArgs g) {
  extern __shared__ __attribute__((aligned(16))) float sm[];
  __shared__ unsigned int nclip;
  __shared__ double dred[2][kNmfThreads / 64];
  constexpr int R4 = RC / 4, M4 = MC / 4;
  const int b = blockIdx.x, tid = threadIdx.x;
  const int N = g.rows[b], m = g.m[b], r = g.cols;
  const int rp = (r + 3) & ~3, mp = (m + 3) & ~3, rq = rp / 4, mq = mp / 4;
  const float *__restrict__ Ag = g.A[b];
  float *__restrict__ Wg = g.W[b];
  float *__restrict__ Hg = g.H[b];
  const int S = nmf_splits(m), O = mp + rp;
  float *A = sm, *W = A + N * rp, *H = W + N * mp, *P = H + m * rp, *G = P + m * rp, *part = G + m * mp;
  for (int e = tid; e < N * rp; e += kNmfThreads) {
    const int i = e / rp, q = e - (e / rp) * rp;
    A[e] = q < r ? Ag[i * r + q] : 0.f;
  }
  for (int e = tid; e < N * mp; e += kNmfThreads) {
    const int i = e / mp, k = e - (e / mp) * mp;
    W[e] = k < m ? Wg[i * m + k] : 0.f;
  }
  for (int e = tid; e < m * rp; e += kNmfThreads) {
    const int j = e / rp, q = e - (e / rp) * rp;
    H[e] = q < r ? Hg[j * r + q] : 0.f;
    P[e] = 0.f;
  }
  for (int e = tid; e < m * mp; e += kNmfThreads) G[e] = 0.f;  // the padding stays zero
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
  const float4 *A4 = reinterpret_cast<const float4 *>(A);
  const float4 *H4 = reinterpret_cast<const float4 *>(H);
  const float4 *G4 = reinterpret_cast<const float4 *>(G);
  const float4 *W4 = reinterpret_cast<const float4 *>(W);
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int it = 0; it < g.iters; ++it) {
    // Rows are read four entries at a time.  Loops run to the compile-time bounds RC / MC
    // with the group index clamped; a group past the row is multiplied by zeros (the
    // padded registers) or replaced by zeros, never guarded by a branch.
    for (int e = tid; e < m * m; e += kNmfThreads) {  // G = H H^T (symmetric)
      const int j = e / m, k = e - (e / m) * m;
      float sacc = 0.f;
#pragma unroll
      for (int q4 = 0; q4 < R4; ++q4) {
        const int qq = q4 < rq ? q4 : rq - 1;
        const float4 hj = H4[j * rq + qq];
        sacc = dot4(q4 < rq ? hj : z4, H4[k * rq + qq], sacc);
      }
      G[j * mp + k] = sacc;
    }
    __syncthreads();
#pragma unroll 1
    for (int i = tid; i < N; i += kNmfThreads) {  // row i of W
      float4 a[R4], w[M4];
#pragma unroll
      for (int q4 = 0; q4 < R4; ++q4) {
        const float4 v = A4[i * rq + (q4 < rq ? q4 : rq - 1)];
        a[q4] = q4 < rq ? v : z4;
      }
#pragma unroll
      for (int k4 = 0; k4 < M4; ++k4) {
        const float4 v = W4[i * mq + (k4 < mq ? k4 : mq - 1)];
        w[k4] = k4 < mq ? v : z4;
      }
#pragma unroll 1
      for (int j = 0; j < m; ++j) {
        float num = 0.f, den = 0.f;
#pragma unroll
        for (int q4 = 0; q4 < R4; ++q4) num = dot4(a[q4], H4[j * rq + (q4 < rq ? q4 : rq - 1)], num);
#pragma unroll
        for (int k4 = 0; k4 < M4; ++k4)  // G[k][j] = G[j][k]
          den = dot4(w[k4], G4[j * mq + (k4 < mq ? k4 : mq - 1)], den);
        // the row belongs to this thread alone: entry j still holds its old value
        W[i * mp + j] = mu(W[i * mp + j], num, den);
      }
    }
    __syncthreads();
    if (tid < S * m) {  // column j of W against rows [i0, i1) of W and A
      const int j = tid % m, sp = tid / m;
      const int i0 = N * sp / S, i1 = N * (sp + 1) / S;
      float4 acc[M4 + R4];
#pragma unroll
      for (int o = 0; o < M4 + R4; ++o) acc[o] = z4;
#pragma unroll 1
      for (int i = i0; i < i1; ++i) {  // accumulators past the row collect unused values
        const float wj = W[i * mp + j];
#pragma unroll
        for (int k4 = 0; k4 < M4; ++k4) {
          const float4 v = W4[i * mq + (k4 < mq ? k4 : mq - 1)];
          acc[k4].x = fmaf(wj, v.x, acc[k4].x);
          acc[k4].y = fmaf(wj, v.y, acc[k4].y);
          acc[k4].z = fmaf(wj, v.z, acc[k4].z);
          acc[k4].w = fmaf(wj, v.w, acc[k4].w);
        }
#pragma unroll
        for (int q4 = 0; q4 < R4; ++q4) {
          const float4 v = A4[i * rq + (q4 < rq ? q4 : rq - 1)];
          acc[M4 + q4].x = fmaf(wj, v.x, acc[M4 + q4].x);
          acc[M4 + q4].y = fmaf(wj, v.y, acc[M4 + q4].y);
          acc[M4 + q4].z = fmaf(wj, v.z, acc[M4 + q4].z);
          acc[M4 + q4].w = fmaf(wj, v.w, acc[M4 + q4].w);
        }
      }
      float4 *pp = reinterpret_cast<float4 *>(part + (sp * m + j) * O);
#pragma unroll
      for (int k4 = 0; k4 < M4; ++k4)
        if (k4 < mq) pp[k4] = acc[k4];
#pragma unroll
      for (int q4 = 0; q4 < R4; ++q4)
        if (q4 < rq) pp[mq + q4] = acc[M4 + q4];
    }
    __syncthreads();
    for (int e = tid; e < m * (m + r); e += kNmfThreads) {  // splits added in order
      const int j = e / (m + r), o = e - (e / (m + r)) * (m + r);
      const int col = o < m ? o : mp + (o - m);
      float t = part[j * O + col];
#pragma unroll
      for (int sp = 1; sp < kNmfSplitMax; ++sp) {  // adding 0 past S changes nothing
        const float v = part[((sp < S ? sp : S - 1) * m + j) * O + col];
        t += sp < S ? v : 0.f;
      }
      if (o < m) G[j * mp + o] = t;
      else P[j * rp + (o - m)] = t;
    }
    __syncthreads();
    // H <- H * (W^T A) / max(W^T W H, eps): m * cols <= 1024 entries, kHv per thread
    constexpr int kHv = (32 * 32 + kNmfThreads - 1) / kNmfThreads;
    float hv[kHv];
#pragma unroll
    for (int u = 0; u < kHv; ++u) {
      const int e = tid + u * kNmfThreads;
      hv[u] = 0.f;
      if (e < m * r) {
        const int j = e / r, q = e - (e / r) * r;
        float den = 0.f;
#pragma unroll
        for (int k = 0; k < MC; ++k) {
          const int kk = k < m ? k : m - 1;
          den = fmaf(k < m ? G[j * mp + kk] : 0.f, H[kk * rp + q], den);
        }
        hv[u] = mu(H[j * rp + q], P[j * rp + q], den);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kHv; ++u) {
      const int e = tid + u * kNmfThreads;
      if (e < m * r) H[(e / r) * rp + e % r] = hv[u];
    }
    __syncthreads();
  }
  for (int e = tid; e < N * m; e += kNmfThreads) Wg[e] = W[(e / m) * mp + e % m];
  for (int e = tid; e < m * r; e += kNmfThreads) Hg[e] = H[(e / r) * rp + e % r];
  if (mine) atomicAdd(&nclip, mine);
  if (g.red) {  // ||A - W H||^2 and ||A||^2, FP64
    double se = 0.0, sa = 0.0;
    for (int e = tid; e < N * r; e += kNmfThreads) {
      const int i = e / r, q = e - (e / r) * r;
      float x = 0.f;
      for (int k = 0; k < m; ++k) x = fmaf(W[i * mp + k], H[k * rp + q], x);
      const float av = A[i * rp + q];
      const double dlt = (double)av - (double)x;
      se += dlt * dlt;
      sa += (double)av * (double)av;
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
  int mmax = 1;
  for (int k = 0; k < n; ++k) mmax = std::max(mmax, m[k]);
  const int RC = cols <= 8 ? 8 : (cols <= 16 ? 16 : 32), MC = mmax <= 8 ? 8 : (mmax <= 16 ? 16 : 32);
#define NNC_NMF(RCV, MCV)                                                                         \
  do {                                                                                            \
    static bool raised = false;                                                                   \
    if (!raised) {                                                                                \
      NNC_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(nmf_block_k<RCV, MCV>),          \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kNmfLdsMax)); \
      raised = true;                                                                              \
    }                                                                                             \
    hipLaunchKernelGGL((nmf_block_k<RCV, MCV>), dim3(n), dim3(kNmfThreads), lds, s, g);           \
  } while (0)
#define NNC_NMF_M(RCV)                \
  do {                                \
    if (MC == 8) NNC_NMF(RCV, 8);     \
    else if (MC == 16) NNC_NMF(RCV, 16); \
    else NNC_NMF(RCV, 32);            \
  } while (0)
  if (RC == 8) NNC_NMF_M(8);
  else if (RC == 16) NNC_NMF_M(16);
  else NNC_NMF_M(32);
#undef NNC_NMF_M
#undef NNC_NMF
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

}  // namespace nnc
