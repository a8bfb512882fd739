// Core-space steps of a sweep spread over several workgroups (cores up to kSliceMax entries).
//
// With S_k = A_k^T A_k (R_k x R_k, symmetric), a sweep needs, between factor updates,
//   M_n   = unfold_n(G x_{k != n} S_k) unfold_n(G)^T          (R_n x R_n, used by mode n)
// and at its end the core update with den_G = G x_0 S_0 x_1 ... x_{d-1} S_{d-1}.
// Both split along one mode of the core:
//   mrows_k : block a builds H_a = G[.., a, ..] x_{k != n} S_k (the slice with mode n fixed
//             to a, contracted with the other Grams) and row a of M_n, M_n[a][b] = <H_a, G_b>;
//   denA_k  : block i builds T_i = G[i, ..] x_1 S_1 ... x_{d-1} S_{d-1} (mode-0 slices);
//   denB_k  : block i forms den[i] = sum_i' S_0[i'][i] T_i' and updates G[i] by the
//             multiplicative rule with the core numerator.
// A step that follows a factor update also needs that factor's new Gram: every block that
// uses it sums the factor's row-block partials (gram[b][R][R], Gram of rows [8b, 8b+8))
// itself, in one fixed order, and block 0 stores it.  The same order serves the start of a
// fit, so a fit resumed from its outputs continues bit for bit.
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "nnc_internal.h"

namespace nnc {

constexpr int kSliceThreads = 1024;  // four waves per SIMD: these steps are latency-bound
constexpr int kSliceMax = 16384;  // cores up to this many entries use these kernels

struct SliceArgs {
  int d;
  int R[kMaxDim];
  int gsize;
  const float *G;      // core (read)
  float *Gout;         // denB_k: updated core (same as G)
  float *S[kMaxDim];   // Grams (global), packed: S[k] = S[0] + soff[k]
  int soff[kMaxDim + 1];
  int gram;            // mode whose Gram is summed from partials here, or -1
  const float *gram_part;
  int gram_parts;
  int n;               // mrows_k: mode of M; denA/denB: unused
  float *M;            // mrows_k output (R_n x R_n)
  float *T;            // denA_k output / denB_k input (gsize floats)
  const float *numG;   // denB_k: core numerator
  float *gradG;        // denB_k: when set, gradG = den - numG instead of the update of G
  double eps;
  unsigned long long *clips;
};

// LDS layout (floats): Sl[d][RM*RM] | red[kSliceThreads*4] | G[gsize] (mrows) | H0 | H1
template <int RM>
struct SliceLds {
  static constexpr int kRed = kSliceThreads * 4;
  static size_t bytes(int d, int gsize, int slice, bool whole_core) {
    return sizeof(float) * ((size_t)d * RM * RM + kRed + (whole_core ? gsize : 0) + 2 * (size_t)slice);
  }
};

// Grams into LDS (row stride RM, zero padding); the gram mode's Gram is summed from the
// partials (entries in groups of 4 when R^2 is a multiple of 4, else one by one; each group
// by kSliceThreads / groups threads over contiguous ranges of partials, added in order).
// issue() starts every global read (the stored Grams and the first kPB partials of this
// thread); finish() consumes them, so a kernel can issue its own reads alongside and pay
// one round of memory latency.
template <int RM>
struct GramStage {
  static constexpr int SU = (kMaxDim * RM * RM + kSliceThreads - 1) / kSliceThreads;  // Gram entries
  static constexpr int GPT = (RM * RM + kSliceThreads - 1) / kSliceThreads;  // groups (nch == 1)
  static constexpr int kPB = 8;                                              // partials in flight
  float sv[SU];
  float4 pv[kPB];
  int W, ngrp, nch, ch, b0, b1, RR, Rk;
  bool vec;

  __device__ void issue(const SliceArgs &a) {
    const int tid = threadIdx.x;
    // every stored Gram, as one flat packed array (entries past the end read the last one)
    const int ns = a.soff[a.d];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int e = tid + u * kSliceThreads;
      sv[u] = a.S[0][e < ns ? e : ns - 1];
    }
    if (a.gram < 0) return;
    Rk = a.R[a.gram];
    RR = Rk * Rk;
    vec = (RR % 4) == 0;
    W = vec ? 4 : 1;
    ngrp = RR / W;
    nch = ngrp >= kSliceThreads ? 1 : kSliceThreads / ngrp;
    ch = nch > 1 ? tid / ngrp : 0;
    const int P = a.gram_parts;
    if (P < (1 << 21)) {  // P * nch < 2^31: the same bounds in 32-bit arithmetic
      b0 = (ch < nch) ? P * ch / nch : 0;
      b1 = (ch < nch) ? P * (ch + 1) / nch : 0;
    } else {
      b0 = (ch < nch) ? (int)((int64_t)P * ch / nch) : 0;
      b1 = (ch < nch) ? (int)((int64_t)P * (ch + 1) / nch) : 0;
    }
    // one group per thread: its first kPB partials now.  Only the float4 form is issued here
    // (single entries are read in finish()): with two load forms on two paths, the registers
    // of one path's loads are live-out of the other, and the wait that protects them stalls
    // every load above as well.
    if (nch > 1 && vec) {
      const int grp = tid % ngrp;
#pragma unroll
      for (int u = 0; u < kPB; ++u) {
        const int b = b0 + u < b1 ? b0 + u : (b1 > 0 ? b1 - 1 : 0);
        pv[u] = *reinterpret_cast<const float4 *>(a.gram_part + (int64_t)b * RR + grp * 4);
      }
    }
  }

  __device__ void finish(const SliceArgs &a, float *Sl, float *red) {
    const int tid = threadIdx.x;
    const int ns = a.soff[a.d];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int e = tid + u * kSliceThreads;
      if (e >= ns) continue;
      // the mode of entry e and its offset and size, by unrolled selects: an index that
      // differs between lanes would read the kernel arguments through vector memory
      int k = 0, base = 0, Rm = a.R[0];
#pragma unroll
      for (int j = 1; j < kMaxDim; ++j)
        if (j < a.d && e >= a.soff[j]) {
          k = j;
          base = a.soff[j];
          Rm = a.R[j];
        }
      if (k == a.gram) continue;  // formed below from the partials
      const int loc = e - base;
      const int l = loc / Rm, r = loc - (loc / Rm) * Rm;
      Sl[k * RM * RM + l * RM + r] = sv[u];
    }
    // zero padding of every mode (entries l >= R_k or r >= R_k; none of them is written above)
#pragma unroll
    for (int k = 0; k < kMaxDim; ++k)
      if (k < a.d)
        for (int e = tid; e < RM * RM; e += kSliceThreads)
          if (e / RM >= a.R[k] || e % RM >= a.R[k]) Sl[k * RM * RM + e] = 0.f;
    if (a.gram < 0) return;
    const int k = a.gram;
    float *Sg = Sl + k * RM * RM;
    auto load = [&](int b, int grp) {
      const float *src = a.gram_part + (int64_t)b * RR + grp * W;
      return vec ? *reinterpret_cast<const float4 *>(src) : make_float4(src[0], 0.f, 0.f, 0.f);
    };
    auto add = [](float4 &s4, float4 v) {
      s4.x += v.x;
      s4.y += v.y;
      s4.z += v.z;
      s4.w += v.w;
    };
    const float inv_rk = 1.0f / Rk;
    auto put = [&](int grp, float4 v) {
      const float vv[4] = {v.x, v.y, v.z, v.w};
      for (int w = 0; w < W; ++w) {
        const int e = grp * W + w;
        const int row = qdiv(e, inv_rk);
        Sg[row * RM + (e - row * Rk)] = vv[w];
        if (blockIdx.x == 0) a.S[k][e] = vv[w];
      }
    };
    if (nch > 1) {
      // The sum starts from an opaque zero: a constant start lets the compiler compute the
      // first addition right after its load is issued, which then waits for every load
      // issued before it.
      float z;
      asm volatile("v_mov_b32 %0, 0" : "=v"(z));
      float4 s4 = make_float4(z, z, z, z);
      if (ch < nch) {
        int bb = b0;
        if (vec) {
#pragma unroll
          for (int u = 0; u < kPB; ++u)
            if (b0 + u < b1) add(s4, pv[u]);
          bb = b0 + kPB;
        }
        for (; bb < b1; ++bb) add(s4, load(bb, tid % ngrp));
        reinterpret_cast<float4 *>(red)[tid] = s4;
      }
      __syncthreads();
      if (tid < ngrp) {
        float4 t4 = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 4
        for (int c = 0; c < nch; ++c) add(t4, reinterpret_cast<const float4 *>(red)[c * ngrp + tid]);
        put(tid, t4);
      }
    } else {
      for (int j = 0; j < GPT; ++j) {
        const int grp = tid + j * kSliceThreads;
        if (grp >= ngrp) break;
        float4 s4 = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int bb = 0; bb < a.gram_parts; ++bb) add(s4, load(bb, grp));
        put(grp, s4);
      }
    }
  }
};

// out[p][r][q] = sum_l S[l][r] in[p][l][q] on an LDS tensor whose mode of size Rk has pre
// entries before it and post after it; one output per thread and step.  The RM inputs of an
// output are loaded before the multiply-adds (rows l >= Rk read row Rk - 1, which the zero
// rows of S cancel), so each output costs one LDS round trip.  Kernels that keep many values
// in registers around it (coreL_k, small_mrows_k) use this form.
template <int RM>
static __device__ void slice_ttm(const float *in, float *out, int pre, int Rk, int post,
                                 const float *S) {
  const int total = pre * Rk * post;
  int off[RM];  // the same for every output; opaque so that it is not folded into multiplies
#pragma unroll
  for (int l = 0; l < RM; ++l) off[l] = __builtin_amdgcn_readfirstlane((l < Rk ? l : Rk - 1) * post);
  const float inv_post = 1.0f / post, inv_rk = 1.0f / Rk;
  for (int o = threadIdx.x; o < total; o += kSliceThreads) {  // total <= kSliceMax < 2^22
    const int pr = qdiv(o, inv_post), q = o - pr * post;
    const int p = qdiv(pr, inv_rk), r = pr - p * Rk;
    const float *src = in + p * Rk * post + q;
    float x[RM], sv[RM];
#pragma unroll
    for (int l = 0; l < RM; ++l) {
      x[l] = src[off[l]];
      sv[l] = S[l * RM + r];
    }
    float acc = 0.f;
#pragma unroll
    for (int l = 0; l < RM; ++l) acc = fmaf(sv[l], x[l], acc);
    out[o] = acc;
  }
}

// The same product with four outputs per thread, for RM <= 16 (at RM 24 and 32 the kernels
// that use it ran out of registers): a thread takes the four outputs r = 4g .. 4g + 3 of
// one (p, q): each input x[l] is read once for the four, and S[l][4g .. 4g + 3] is one
// 16-byte read (S rows are RM floats, zero past Rk).  The inputs are read in batches
// before their multiply-adds (rows l >= Rk read row Rk - 1, which the zero rows of S
// cancel); every output still takes its RM terms in l order.
template <int RM>
static __device__ void slice_ttm4(const float *in, float *out, int pre, int Rk, int post,
                                 const float *S) {
  const int RG = (Rk + 3) >> 2;
  const int total = pre * RG * post;
  int off[RM];  // the same for every output; opaque so that it is not folded into multiplies
#pragma unroll
  for (int l = 0; l < RM; ++l) off[l] = __builtin_amdgcn_readfirstlane((l < Rk ? l : Rk - 1) * post);
  const float inv_post = 1.0f / post, inv_rg = 1.0f / RG;
  for (int o = threadIdx.x; o < total; o += kSliceThreads) {  // total <= kSliceMax < 2^22
    const int pr = qdiv(o, inv_post), q = o - pr * post;
    const int p = qdiv(pr, inv_rg), g = pr - p * RG;
    const float *src = in + p * Rk * post + q;
    const float *sg = S + 4 * g;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    constexpr int LB = RM < 16 ? RM : 16;
#pragma unroll
    for (int l0 = 0; l0 < RM; l0 += LB) {
      float x[LB];
      float4 sv[LB];
#pragma unroll
      for (int l = 0; l < LB; ++l) {
        if (l0 + l < RM) {
          x[l] = src[off[l0 + l]];
          sv[l] = *reinterpret_cast<const float4 *>(sg + (l0 + l) * RM);
        }
      }
#pragma unroll
      for (int l = 0; l < LB; ++l) {
        if (l0 + l < RM) {
          acc[0] = fmaf(sv[l].x, x[l], acc[0]);
          acc[1] = fmaf(sv[l].y, x[l], acc[1]);
          acc[2] = fmaf(sv[l].z, x[l], acc[2]);
          acc[3] = fmaf(sv[l].w, x[l], acc[3]);
        }
      }
    }
    float *dst = out + (p * Rk + 4 * g) * post + q;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (4 * g + j < Rk) dst[j * post] = acc[j];
  }
}

// Contract the slice (modes of the core except `skip`, kept in order) with the Grams of its
// modes; returns the LDS buffer holding the result (H0 or H1).
template <int RM>
static __device__ float *contract_slice(const SliceArgs &a, int skip, const float *Sl, float *H0,
                                        float *H1) {
  int dims[kMaxDim], nd = 0;
  for (int k = 0; k < a.d; ++k)
    if (k != skip) dims[nd++] = a.R[k];
  float *cur = H0, *nxt = H1;
  int j = 0;
  for (int k = 0; k < a.d; ++k) {
    if (k == skip) continue;
    int pre = 1, post = 1;
    for (int t = 0; t < j; ++t) pre *= dims[t];
    for (int t = j + 1; t < nd; ++t) post *= dims[t];
    if constexpr (RM <= 16)
      slice_ttm4<RM>(cur, nxt, pre, dims[j], post, Sl + k * RM * RM);
    else
      slice_ttm<RM>(cur, nxt, pre, dims[j], post, Sl + k * RM * RM);
    __syncthreads();
    float *t2 = cur;
    cur = nxt;
    nxt = t2;
    ++j;
  }
  return cur;
}

// Row a = blockIdx.x of M_n (and, with a.gram >= 0, the new Gram of mode a.gram).  With
// a.n < 0 only the Gram is formed (one block).
template <int RM, bool BIG>
static __device__ void mrows_body(const SliceArgs &a, int ia) {
  extern __shared__ __attribute__((aligned(16))) float lds[];
  const int d = a.d, tid = threadIdx.x;
  float *Sl = lds;
  float *red = Sl + d * RM * RM;
  float *G = red + SliceLds<RM>::kRed;
  const int n = a.n;
  const int Rn = n >= 0 ? a.R[n] : 1;
  const int slice = a.gsize / Rn;
  float *H0 = G + a.gsize, *H1 = H0 + slice;
  // the whole core (for the dot products) and the Grams
  // every global read first (the core, the Grams, the Gram partials), then their use
  GramStage<RM> gs;
  constexpr int GPTH = (BIG ? kSliceMax : kSliceMax / 2) / kSliceThreads;  // core values per thread
  float gv[GPTH];
  if (n >= 0) {
#pragma unroll
    for (int u = 0; u < GPTH; ++u) {
      const int e = tid + u * kSliceThreads;
      gv[u] = a.G[e < a.gsize ? e : a.gsize - 1];
    }
  }
  gs.issue(a);
  __builtin_amdgcn_sched_barrier(0);  // every load above is issued before any is used
  if (n >= 0) {
#pragma unroll
    for (int u = 0; u < GPTH; ++u) {
      const int e = tid + u * kSliceThreads;
      if (e < a.gsize) G[e] = gv[u];
    }
  }
  gs.finish(a, Sl, red);
  __syncthreads();
  if (n < 0) return;
  int pre = 1, post = 1;
  for (int k = 0; k < n; ++k) pre *= a.R[k];
  for (int k = n + 1; k < d; ++k) post *= a.R[k];
  // slice with mode n fixed to ia, as [pre][post]
  for (int c = tid; c < slice; c += kSliceThreads) {
    const int pc = c / post, qc = c - (c / post) * post;
    H0[c] = G[(pc * Rn + ia) * post + qc];
  }
  __syncthreads();
  const float *H = contract_slice<RM>(a, n, Sl, H0, H1);
  // M[ia][b] = sum_c H[c] G[(pc * Rn + b) * post + qc]: half a wave per b (Rn <= 32 halves of
  // 32 lanes in the block); lane j adds c = j, j + 32, ... in order, and the 32 partial sums
  // meet in a fixed butterfly within the half.
  const int half = tid >> 5, l32 = tid & 31;
  if (half < Rn) {
    const int b = half;
    const float inv_post = 1.0f / post;
    float acc = 0.f;
#pragma unroll 4
    for (int c = l32; c < slice; c += 32) {
      const int pc = qdiv(c, inv_post), qc = c - pc * post;
      acc = fmaf(H[c], G[(pc * Rn + b) * post + qc], acc);
    }
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 32);
    if (l32 == 0) a.M[ia * Rn + b] = acc;
  }
}

template <int RM, bool BIG>
__global__ __launch_bounds__(kSliceThreads) void mrows_k(SliceArgs a) {
  mrows_body<RM, BIG>(a, blockIdx.x);
}

// Rows of M_n for cores larger than the whole-core kernels above take (slices of up to
// kSliceMax entries): block (a, g) stages the slice G_a and the slices G_b of its group,
// b in [g nb, g nb + nb), in LDS with one round of loads beside the Grams', forms
// H_a = G_a x_{k != n} S_k there, and writes M_n[a][b] = <H_a, G_b>.  Every group of row a
// forms H_a again (a few hundred multiply-adds per thread), which costs far less than the
// launches of a grid-wide chain.  Each dot product is split over Tb = kSliceThreads / nbp
// threads (nbp = nb rounded up to a power of two; thread j adds c = j, j + Tb, ... in
// order), reduced by a fixed butterfly within each wave (or half wave) and the partial sums
// added in thread order.
template <int RM>
__global__ __launch_bounds__(kSliceThreads) void mrows_big_k(SliceArgs a, int nb, int ngrp) {
  extern __shared__ __attribute__((aligned(16))) float lds[];
  const int d = a.d, tid = threadIdx.x, n = a.n;
  const int ia = blockIdx.x / ngrp, g = blockIdx.x - ia * ngrp;
  const int Rn = a.R[n];
  const int slice = a.gsize / Rn;
  const int b0 = g * nb, nbl = min(nb, Rn - b0);
  float *Sl = lds;
  float *red = Sl + d * RM * RM;
  float *H0 = red + SliceLds<RM>::kRed, *H1 = H0 + slice;  // the slices G_b follow H1
  int post = 1;
  for (int k = n + 1; k < d; ++k) post *= a.R[k];
  // staged entry e = s * slice + c (s = 0: G_a, s >= 1: G_{b0 + s - 1}; c = pc * post + qc)
  // holds G[(pc * Rn + row) * post + qc] and goes to H0[e] (s = 0) or H0[e + slice]
  const int total = (1 + nbl) * slice;  // < 2^22 (see big_slice_fits)
  const float inv_slice = 1.0f / (float)slice, inv_post = 1.0f / (float)post;
  GramStage<RM> gs;
  gs.issue(a);
  constexpr int kU = 16;  // staged values per thread and round
  for (int e0 = 0; e0 < total; e0 += kU * kSliceThreads) {
    float v[kU];
    int dst[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int e = min(e0 + tid + u * kSliceThreads, total - 1);  // past the end: the last again
      const int sx = qdiv(e, inv_slice), c = e - sx * slice;
      const int pc = qdiv(c, inv_post), qc = c - pc * post;
      const int row = sx == 0 ? ia : b0 + sx - 1;
      v[u] = a.G[((int64_t)pc * Rn + row) * post + qc];
      dst[u] = sx == 0 ? e : e + slice;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) H0[dst[u]] = v[u];
  }
  gs.finish(a, Sl, red);
  __syncthreads();
  const float *H = contract_slice<RM>(a, n, Sl, H0, H1);  // ends with a barrier
  const float *Gb = H1 + slice;
  int nbp = 1;
  while (nbp < nb) nbp <<= 1;
  const int Tb = kSliceThreads / nbp;  // >= 32 (nb <= 32)
  const int W = Tb < 64 ? Tb : 64;
  const int bi = tid / Tb, j = tid - bi * Tb;
  float acc = 0.f;
  if (bi < nbl) {
    const float *gp = Gb + bi * slice;
#pragma unroll 4
    for (int c = j; c < slice; c += Tb) acc = fmaf(H[c], gp[c], acc);
  }
  for (int off = W >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, W);
  if ((tid & (W - 1)) == 0) red[tid / W] = acc;
  __syncthreads();
  if (tid < nbl) {
    const int per = Tb / W;
    float m = 0.f;
    for (int w = 0; w < per; ++w) m += red[tid * per + w];
    a.M[(int64_t)ia * Rn + b0 + tid] = m;
  }
}

// T_i = G[i, ..] x_1 S_1 ... x_{d-1} S_{d-1} for slice i (and the new Gram of a.gram).
template <int RM, bool BIG>
static __device__ void denA_body(const SliceArgs &a, int i) {
  extern __shared__ __attribute__((aligned(16))) float lds[];
  const int d = a.d, tid = threadIdx.x;
  float *Sl = lds;
  float *red = Sl + d * RM * RM;
  const int slice = a.gsize / a.R[0];
  float *H0 = red + SliceLds<RM>::kRed, *H1 = H0 + slice;
  constexpr int SPT = (BIG ? kSliceMax : kSliceMax / 2) / kSliceThreads;  // slice values per thread
  float hv[SPT];
#pragma unroll
  for (int u = 0; u < SPT; ++u) {
    const int c = tid + u * kSliceThreads;
    hv[u] = a.G[(int64_t)i * slice + (c < slice ? c : slice - 1)];
  }
  GramStage<RM> gs;
  gs.issue(a);
  __builtin_amdgcn_sched_barrier(0);  // every load above is issued before any is used
#pragma unroll
  for (int u = 0; u < SPT; ++u) {
    const int c = tid + u * kSliceThreads;
    if (c < slice) H0[c] = hv[u];
  }
  gs.finish(a, Sl, red);
  __syncthreads();
  const float *T = contract_slice<RM>(a, 0, Sl, H0, H1);
  for (int c = tid; c < slice; c += kSliceThreads) a.T[(int64_t)i * slice + c] = T[c];
}

template <int RM, bool BIG>
__global__ __launch_bounds__(kSliceThreads) void denA_k(SliceArgs a) {
  denA_body<RM, BIG>(a, blockIdx.x);
}

// numG[e] = sum_{b < nparts} part[b][e] (the core numerator from the last mode's row-block
// partials), b in order from 0; the loads of a round of kSumB partials are all in flight
// (one round for factors up to 512 rows).
static __device__ void sum_body(const float *__restrict__ part, int nparts, int n,
                                float *__restrict__ out, int e) {
  if (e >= n) return;
  constexpr int kSumB = 64;
  float s2 = 0.f;
  for (int b0 = 0; b0 < nparts; b0 += kSumB) {
    float v[kSumB];
#pragma unroll
    for (int u = 0; u < kSumB; ++u) {
      const int b = b0 + u < nparts ? b0 + u : nparts - 1;
      v[u] = part[(int64_t)b * n + e];
    }
#pragma unroll
    for (int u = 0; u < kSumB; ++u)
      if (b0 + u < nparts) s2 += v[u];
  }
  out[e] = s2;
}

// denA_k's slices in blocks [0, na) and the core numerator's sum in the blocks after them:
// the two do not depend on each other and each alone leaves most CUs idle.
template <int RM, bool BIG>
__global__ __launch_bounds__(kSliceThreads) void denA_sum_k(SliceArgs a, const float *part,
                                                           int nparts, float *numG, int na) {
  if ((int)blockIdx.x < na)
    denA_body<RM, BIG>(a, blockIdx.x);
  else
    sum_body(part, nparts, a.gsize, numG, ((int)blockIdx.x - na) * kSliceThreads + threadIdx.x);
}

// den[i] = sum_i' S_0[i'][i] T_i' and G[i] <- G[i] * numG[i] / max(den[i], eps) (FP64
// division), for i = blockIdx.x; counts the clipped denominators.
__global__ __launch_bounds__(kSliceThreads) void denB_k(SliceArgs a) {
  __shared__ float s0[32];
  __shared__ unsigned int nclip;
  const int tid = threadIdx.x, i = blockIdx.x;
  const int R0 = a.R[0];
  const int slice = a.gsize / R0;
  // A slice that one pass of the block covers (the usual case) has every global read of its
  // entry issued before the barrier, beside S_0's: one memory round trip in all.  The R0
  // terms are unrolled to 32 with clamped rows and zero weights past R0, so the sum runs in
  // the same order as the general loop below.
  const bool one = slice <= kSliceThreads;
  float tv[32], gv = 0.f, nv = 0.f;
  if (one && tid < slice) {
#pragma unroll
    for (int ip = 0; ip < 32; ++ip) tv[ip] = a.T[(int64_t)(ip < R0 ? ip : R0 - 1) * slice + tid];
    gv = a.G[(int64_t)i * slice + tid];
    nv = a.numG[(int64_t)i * slice + tid];
  }
  if (tid < 32) s0[tid] = tid < R0 ? a.S[0][tid * R0 + i] : 0.f;  // S_0[i'][i], i' = tid
  if (tid == 0) nclip = 0;
  __syncthreads();
  unsigned int mine = 0;
  auto update = [&](int c, float den, float g, float num) {
    if (a.gradG) {  // the gradient of the loss with respect to G (reading R1): den - num
      a.gradG[(int64_t)i * slice + c] = den - num;
      return;
    }
    double dd = (double)den;
    if (dd < a.eps) {
      dd = a.eps;
      ++mine;
    }
    a.Gout[(int64_t)i * slice + c] = (float)(((double)g * (double)num) / dd);
  };
  if (one) {
    if (tid < slice) {
      float den = 0.f;
#pragma unroll
      for (int ip = 0; ip < 32; ++ip) den = fmaf(s0[ip], tv[ip], den);
      update(tid, den, gv, nv);
    }
  } else {
    for (int c = tid; c < slice; c += kSliceThreads) {
      float den = 0.f;
      for (int ip = 0; ip < R0; ++ip) den = fmaf(s0[ip], a.T[(int64_t)ip * slice + c], den);
      const int64_t e = (int64_t)i * slice + c;
      update(c, den, a.G[e], a.numG[e]);
    }
  }
  if (mine) atomicAdd(&nclip, mine);
  __syncthreads();
  if (tid == 0 && nclip) atomicAdd(a.clips, (unsigned long long)nclip);
}

// =====================================================================================
// out[p][r][q] = sum_n F[n*ldl + r*ldr] * in[p][n][q]   (R <= 32, FP32)
// A block owns 64 consecutive (p, q) pairs and W = ceil(N / 32) waves (at most 16), so that
// one round covers up to 512 rows of n with 32 rows per wave; each wave multiplies its rows
// on the FP32 matrix cores (the 64 pairs as four 16-row tiles of the product, the rank as one
// or two 16-column tiles) with every load of the round issued before the first product.
// Factor entries past R or N are zero, so rows past the end contribute nothing.  The wave
// partial sums are added in wave order through LDS.  Adding splits of n in a second
// pass or through a device-scope counter would give more blocks when P*Q is small, but
// the release fence such a counter needs writes back the whole L2 of the XCD, which has
// cost far more than the extra parallelism saves.
// =====================================================================================
constexpr int kSmallRows = 32;     // rows of n per wave and round
constexpr int kSmallMaxWaves = 16;

static int small_waves(int64_t N) {
  const int64_t w = (N + kSmallRows - 1) / kSmallRows;
  return (int)(w < 1 ? 1 : (w > kSmallMaxWaves ? kSmallMaxWaves : w));
}
// LDS of a block: the wave partial sums (W of RM rows of 64, kRedStride floats apart: with
// rows 64 floats apart every 16-row group of a wave's writes fell on the same banks).
constexpr int kRedStride = 68;
static size_t small_lds(int W, int RM) { return (size_t)W * kRedStride * RM * sizeof(float); }

struct SmallArgs {
  const float *in;
  int64_t P, N, Q;
  const float *F;
  int64_t ldl, ldr;
  int R;
  float *out;
  int W;  // waves that take rows (the block may hold more, which then only join barriers)
};

typedef float smf4 __attribute__((ext_vector_type(4)));

// Tile `tile` of the contraction; blockDim.x / 64 >= a.W.  The products run on the FP32
// matrix cores (v_mfma_f32_16x16x4_f32): in a wave, lane (li, lg) supplies the entry of the
// partial tensor in column 16 c + li (c = 0..3, the tile's 64 columns) and row 4 s + lg of its
// rows, and the factor entry of that row in rank column 16 t + li (t = 0, 1); its result
// holds columns 16 c + 4 lg + v (v = 0..3) of rank column 16 t + li.  The factor entries
// come from global memory (every block reads the same few kilobytes, held in L2) and are
// loaded before the rows of `in`, so that the products of step s wait only for step s's
// loads.
template <int RM>
static __device__ void small_body(const SmallArgs &a, int64_t tile) {
  extern __shared__ __attribute__((aligned(16))) float sm[];
  constexpr int RT = RM > 16 ? 2 : 1;
  const float *__restrict__ in = a.in;
  const float *__restrict__ F = a.F;
  float *__restrict__ out = a.out;
  const int64_t P = a.P, N = a.N, Q = a.Q, ldl = a.ldl, ldr = a.ldr;
  const int R = a.R, W = a.W;
  const int tid = threadIdx.x;
  const int lane = tid & 63, li = lane & 15, lg = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool active = w < W;
  const int64_t PQ = P * Q;
  const float *src[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {  // the lane's column of each 16-column group
    const int64_t e = tile * 64 + 16 * c + li;
    const int64_t ee = e < PQ ? e : 0;
    const int64_t p = ee / Q, q = ee - (ee / Q) * Q;
    src[c] = in + p * N * Q + q;
  }
  const int span = W * kSmallRows;  // rows of a round
  smf4 acc[4][RT];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[c][t] = smf4{0.f, 0.f, 0.f, 0.f};
  // Addresses: one 64-bit product per pointer and round; step st adds 4 st rows, a
  // wave-uniform offset, so the loads cost no per-load integer multiplies.
  const float *flast[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) flast[t] = F + (16 * t + li < R ? (16 * t + li) * ldr : 0);
  for (int64_t nb = 0; active && nb < N; nb += span) {
    constexpr int kSteps = kSmallRows / 4;
    const int64_t n0 = nb + w * kSmallRows + lg;  // the lane's row of step 0
    float fb[kSteps][RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const float *f0 = flast[t] + n0 * ldl;
#pragma unroll
      for (int st = 0; st < kSteps; ++st) {
        const bool ok = n0 + 4 * st < N && 16 * t + li < R;
        fb[st][t] = *(ok ? f0 + 4 * st * ldl : F);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    float xv[kSteps][4];
    const float *x0[4], *xl[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      x0[c] = src[c] + n0 * Q;
      xl[c] = src[c] + (N - 1) * Q;  // rows past N meet zero factor entries
    }
#pragma unroll
    for (int st = 0; st < kSteps; ++st) {
      const bool inside = n0 + 4 * st < N;
#pragma unroll
      for (int c = 0; c < 4; ++c) xv[st][c] = *(inside ? x0[c] + 4 * st * Q : xl[c]);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int st = 0; st < kSteps; ++st) {
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        // zero factor entries (past R or N) are selected here, where the values are awaited
        const int64_t n = nb + w * kSmallRows + 4 * st + lg;
        const float b = (n < N && 16 * t + li < R) ? fb[st][t] : 0.f;
#pragma unroll
        for (int c = 0; c < 4; ++c)
          acc[c][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv[st][c], b, acc[c][t], 0, 0, 0);
      }
    }
  }
  float *red = sm;  // red[w][r][kRedStride], columns 0 .. 63 used
  if (active) {
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int r = 16 * t + li;
      if (r < RM) {
#pragma unroll
        for (int c = 0; c < 4; ++c)  // columns 16 c + 4 lg .. + 3: one 16-byte write
          *reinterpret_cast<smf4 *>(red + (w * RM + r) * kRedStride + 16 * c + 4 * lg) = acc[c][t];
      }
    }
  }
  __syncthreads();
  for (int idx = tid; idx < RM * 64; idx += blockDim.x) {
    const int r = idx >> 6, l = idx & 63;
    const int64_t e2 = tile * 64 + l;
    if (r >= R || e2 >= PQ) continue;
    float s2 = red[r * kRedStride + l];
    for (int ww = 1; ww < W; ++ww) s2 += red[(ww * RM + r) * kRedStride + l];
    const int64_t p2 = e2 / Q, q2 = e2 - (e2 / Q) * Q;
    out[(p2 * R + r) * Q + q2] = s2;
  }
}

template <int RM>
__global__ __launch_bounds__(64 * kSmallMaxWaves) void ttm_small_k(SmallArgs a) {
  small_body<RM>(a, blockIdx.x);
}

static bool small_args(const float *in, int64_t P, int64_t N, int64_t Q, const float *F,
                       int64_t ldl, int64_t ldr, int64_t R, float *out, SmallArgs *a, int *RM,
                       int64_t *tiles) {
  if (R > 32 || R < 1 || N < 1) return false;
  *tiles = (P * Q + 63) / 64;
  if (*tiles > 0x7fffffff) return false;
  *a = SmallArgs{in, P, N, Q, F, ldl, ldr, (int)R, out, small_waves(N)};
  *RM = (int)((R + 3) / 4 * 4);
  return true;
}

// Partial tensors of at least this many floats (64 MiB) go to the X-streaming pass kernels
// when they take the shape (FP32 matrix cores, the factor in LDS, the tensor read once at
// near-HBM rate): 64^5 at multirank 8 ran 2.7 % faster, 128^4 at 16 0.8 %; below it this
// kernel's shorter launches win.
constexpr int64_t kStreamFloats = (int64_t)16 << 20;

nnc_status launch_ttm_small(const float *in, int64_t P, int64_t N, int64_t Q, const float *F,
                            int64_t ldl, int64_t ldr, int64_t R, float *out, hipStream_t s) {
  if (P * N * Q >= kStreamFloats) {
    const nnc_status st = launch_pass(in, NNC_F32, P, N, Q, F, ldl, ldr, R, out, s, nullptr, 0);
    if (st != NNC_EUNSUPPORTED) return st;
  }
  SmallArgs a;
  int RM;
  int64_t tiles;
  if (!small_args(in, P, N, Q, F, ldl, ldr, R, out, &a, &RM, &tiles))
    return fail(NNC_EUNSUPPORTED, "ttm_small: R %lld, N %lld or P*Q out of range", (long long)R,
                (long long)N);
  const size_t lds = small_lds(a.W, RM);
  const dim3 g((unsigned)tiles), b(64 * a.W);
#define NNC_SMALL(RMV) hipLaunchKernelGGL(ttm_small_k<RMV>, g, b, lds, s, a)
  switch (RM / 4) {
    case 1: NNC_SMALL(4); break;
    case 2: NNC_SMALL(8); break;
    case 3: NNC_SMALL(12); break;
    case 4: NNC_SMALL(16); break;
    case 5: NNC_SMALL(20); break;
    case 6: NNC_SMALL(24); break;
    case 7: NNC_SMALL(28); break;
    default: NNC_SMALL(32); break;
  }
#undef NNC_SMALL
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

static nnc_status allow_slice_lds(const void *kern, size_t bytes) {
  static std::mutex mu;
  static std::map<const void *, size_t> done;
  if (bytes <= 64 * 1024) return NNC_OK;
  std::lock_guard<std::mutex> lk(mu);
  auto it = done.find(kern);
  if (it != done.end() && it->second >= bytes) return NNC_OK;
  NNC_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  done[kern] = bytes;
  return NNC_OK;
}

static SliceArgs slice_args(const CoreArgsHost &h) {
  SliceArgs a;
  memset(&a, 0, sizeof a);
  a.d = h.d;
  a.gsize = 1;
  for (int k = 0; k < kMaxDim; ++k) {
    a.R[k] = k < h.d ? (int)h.R[k] : 1;
    a.S[k] = k < h.d ? h.S[k] : nullptr;
  }
  for (int k = 0; k < h.d; ++k) a.gsize *= a.R[k];
  a.soff[0] = 0;
  for (int k = 0; k < kMaxDim; ++k) a.soff[k + 1] = a.soff[k] + (k < h.d ? a.R[k] * a.R[k] : 0);
  a.G = h.G;
  a.gram = h.gram_to > h.gram_from ? h.gram_from : -1;
  a.gram_part = h.gram;
  a.gram_parts = h.gram_parts;
  a.eps = h.eps;
  a.clips = h.clips;
  return a;
}

template <int RM, bool BIG>
static nnc_status slice_step(const CoreArgsHost &h, hipStream_t s) {
  SliceArgs a = slice_args(h);
  if (h.do_core) {
    // T = G x_1 S_1 ... (the new Gram formed on the way), then the update
    a.T = h.t0;
    a.n = -1;
    const int slice0 = a.gsize / a.R[0];
    const size_t la = SliceLds<RM>::bytes(a.d, a.gsize, slice0, false);
    if (h.gpart && h.nparts > 0) {  // the numerator's sum rides along
      NNC_TRY(allow_slice_lds(reinterpret_cast<const void *>(denA_sum_k<RM, BIG>), la));
      const int nsum = (a.gsize + kSliceThreads - 1) / kSliceThreads;
      hipLaunchKernelGGL((denA_sum_k<RM, BIG>), dim3(a.R[0] + nsum), dim3(kSliceThreads), la, s, a,
                         h.gpart, h.nparts, h.numG, a.R[0]);
    } else {
      NNC_TRY(allow_slice_lds(reinterpret_cast<const void *>(denA_k<RM, BIG>), la));
      hipLaunchKernelGGL((denA_k<RM, BIG>), dim3(a.R[0]), dim3(kSliceThreads), la, s, a);
    }
    SliceArgs b = a;
    b.gram = -1;
    b.numG = h.numG;
    b.Gout = h.G;
    hipLaunchKernelGGL(denB_k, dim3(a.R[0]), dim3(kSliceThreads), 0, s, b);
    a.gram = -1;  // its Gram is stored now
  }
  if (h.next >= 0 || a.gram >= 0) {
    a.n = h.next;
    a.M = h.M;
    const int Rn = h.next >= 0 ? a.R[h.next] : 1;
    const size_t lm = SliceLds<RM>::bytes(a.d, a.gsize, a.gsize / Rn, h.next >= 0);
    NNC_TRY(allow_slice_lds(reinterpret_cast<const void *>(mrows_k<RM, BIG>), lm));
    hipLaunchKernelGGL((mrows_k<RM, BIG>), dim3(h.next >= 0 ? Rn : 1), dim3(kSliceThreads), lm, s, a);
  }
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

// Returns NNC_EUNSUPPORTED (no error recorded) when the core is too large for these kernels.
// Whether the slice kernels take this core; the Gram row stride RM and the core-size variant.
static bool slice_fits(const CoreArgsHost &h, int *RMo, bool *bigo) {
  int64_t gsize = 1;
  int maxr = 1;
  for (int k = 0; k < h.d; ++k) {
    gsize *= h.R[k];
    maxr = std::max(maxr, (int)h.R[k]);
  }
  if (gsize > kSliceMax || maxr > 32 || h.gram_to - h.gram_from > 1) return false;
  // the Grams must be packed one after another (the fit's workspace keeps them so)
  for (int64_t k = 1, off = h.R[0] * h.R[0]; k < h.d; off += h.R[k] * h.R[k], ++k)
    if (h.S[k] != h.S[0] + off) return false;
  // LDS of the largest launch (the whole core and two slices at worst)
  const int RM = maxr <= 8 ? 8 : (maxr <= 16 ? 16 : (maxr <= 24 ? 24 : 32));
  int64_t worst = 0;
  for (int k = 0; k < h.d; ++k) worst = std::max(worst, gsize / h.R[k]);
  const int64_t need = 4 * ((int64_t)h.d * RM * RM + 4 * kSliceThreads + gsize + 2 * worst);
  if (need > 160 * 1024) return false;
  *RMo = RM;
  *bigo = gsize > kSliceMax / 2;
  return true;
}

// Cores beyond kSliceMax entries whose mode slices the slice kernels can hold: the core
// update by denA_k / denB_k (which keep one slice, not the core, in LDS) and the rows of
// M_next by mrows_big_k.  LDS: the Grams, the reduction space and at least three slices.
// slices G_b per mrows_big_k block: enough that the R_n x ceil(R_n / nb) blocks fit the CUs
// in one round (R_n = 32: four), at least two (at 16^4 two measured faster than four, with
// more blocks and one round of loads, and the same as one), at most kBigSliceB
constexpr int kBigSliceB = 8;

static bool big_slice_fits(const CoreArgsHost &h, int *RMo) {
  int64_t gsize = 1;
  int maxr = 1;
  for (int k = 0; k < h.d; ++k) {
    gsize *= h.R[k];
    maxr = std::max(maxr, (int)h.R[k]);
  }
  if (gsize <= kSliceMax || maxr > 32 || h.gram_to - h.gram_from > 1) return false;
  // a Gram alone (no core update, no M_next) is left to the grid-wide steps
  if (!h.do_core && h.next < 0) return false;
  for (int64_t k = 1, off = h.R[0] * h.R[0]; k < h.d; off += h.R[k] * h.R[k], ++k)
    if (h.S[k] != h.S[0] + off) return false;
  const int RM = maxr <= 8 ? 8 : (maxr <= 16 ? 16 : (maxr <= 24 ? 24 : 32));
  int64_t worst = 0;
  for (int k = 0; k < h.d; ++k) worst = std::max(worst, gsize / h.R[k]);
  // staged entries of mrows_big_k ((1 + nb) slices) stay below 2^22 for the float-reciprocal
  // index divisions
  if (worst > kSliceMax || (1 + kBigSliceB) * worst >= ((int64_t)1 << 22)) return false;
  if (4 * ((int64_t)h.d * RM * RM + SliceLds<8>::kRed + 3 * worst) > 160 * 1024) return false;
  *RMo = RM;
  return true;
}

template <int RM>
static nnc_status big_slice_step(const CoreArgsHost &h, hipStream_t s) {
  SliceArgs a = slice_args(h);
  if (h.do_core) {
    a.T = h.t0;
    a.n = -1;
    const int slice0 = a.gsize / a.R[0];
    const size_t la = SliceLds<RM>::bytes(a.d, a.gsize, slice0, false);
    const bool bigs = slice0 > kSliceMax / 2;
    if (h.gpart && h.nparts > 0) {
      const int nsum = (a.gsize + kSliceThreads - 1) / kSliceThreads;
      if (bigs) {
        NNC_TRY(allow_slice_lds(reinterpret_cast<const void *>(denA_sum_k<RM, true>), la));
        hipLaunchKernelGGL((denA_sum_k<RM, true>), dim3(a.R[0] + nsum), dim3(kSliceThreads), la, s, a,
                           h.gpart, h.nparts, h.numG, a.R[0]);
      } else {
        NNC_TRY(allow_slice_lds(reinterpret_cast<const void *>(denA_sum_k<RM, false>), la));
        hipLaunchKernelGGL((denA_sum_k<RM, false>), dim3(a.R[0] + nsum), dim3(kSliceThreads), la, s, a,
                           h.gpart, h.nparts, h.numG, a.R[0]);
      }
    } else if (bigs) {
      NNC_TRY(allow_slice_lds(reinterpret_cast<const void *>(denA_k<RM, true>), la));
      hipLaunchKernelGGL((denA_k<RM, true>), dim3(a.R[0]), dim3(kSliceThreads), la, s, a);
    } else {
      NNC_TRY(allow_slice_lds(reinterpret_cast<const void *>(denA_k<RM, false>), la));
      hipLaunchKernelGGL((denA_k<RM, false>), dim3(a.R[0]), dim3(kSliceThreads), la, s, a);
    }
    SliceArgs b = a;
    b.gram = -1;
    b.numG = h.numG;
    b.Gout = h.G;
    hipLaunchKernelGGL(denB_k, dim3(a.R[0]), dim3(kSliceThreads), 0, s, b);
    a.gram = -1;  // its Gram is stored now
  }
  if (h.next >= 0) {
    a.n = h.next;
    a.M = h.M;
    const int Rn = a.R[h.next];
    const int slice = a.gsize / Rn;
    const int64_t room = (160 * 1024 / 4 - (int64_t)a.d * RM * RM - SliceLds<RM>::kRed) / slice - 2;
    const int64_t want = std::max<int64_t>(2, ((int64_t)Rn * Rn + device_cu_count() - 1) / device_cu_count());
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>({want, (int64_t)kBigSliceB, room, (int64_t)Rn}));
    const int ngrp = (Rn + nb - 1) / nb;
    const size_t lm = sizeof(float) * ((size_t)a.d * RM * RM + SliceLds<RM>::kRed + (size_t)(2 + nb) * slice);
    NNC_TRY(allow_slice_lds(reinterpret_cast<const void *>(mrows_big_k<RM>), lm));
    hipLaunchKernelGGL((mrows_big_k<RM>), dim3(Rn * ngrp), dim3(kSliceThreads), lm, s, a, nb, ngrp);
  }
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

// dL/dG = den_G - num_G (h.numG, the core numerator) with den_G = G x_k S_k, by the slice
// kernels (denA_k, then denB_k in its gradient form); G is left as it is.  NNC_EUNSUPPORTED
// (no error recorded) when they do not take the core.
template <int RM>
static nnc_status core_grad_step(const CoreArgsHost &h, float *grad_out, hipStream_t s) {
  SliceArgs a = slice_args(h);
  a.gram = -1;
  a.T = h.t0;
  a.n = -1;
  const int slice0 = a.gsize / a.R[0];
  const size_t la = SliceLds<RM>::bytes(a.d, a.gsize, slice0, false);
  if (slice0 > kSliceMax / 2) {
    NNC_TRY(allow_slice_lds(reinterpret_cast<const void *>(denA_k<RM, true>), la));
    hipLaunchKernelGGL((denA_k<RM, true>), dim3(a.R[0]), dim3(kSliceThreads), la, s, a);
  } else {
    NNC_TRY(allow_slice_lds(reinterpret_cast<const void *>(denA_k<RM, false>), la));
    hipLaunchKernelGGL((denA_k<RM, false>), dim3(a.R[0]), dim3(kSliceThreads), la, s, a);
  }
  SliceArgs b = a;
  b.numG = h.numG;
  b.Gout = h.G;
  b.gradG = grad_out;
  hipLaunchKernelGGL(denB_k, dim3(a.R[0]), dim3(kSliceThreads), 0, s, b);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

nnc_status launch_core_grad(const CoreArgsHost &h0, float *grad_out, hipStream_t s) {
  CoreArgsHost h = h0;
  h.gram_from = h.gram_to = 0;
  h.do_core = 1;
  h.next = -1;
  int RM;
  bool big;
  if (!grad_out || !h.numG || !h.t0) return NNC_EUNSUPPORTED;
  if (!slice_fits(h, &RM, &big) && !big_slice_fits(h, &RM)) return NNC_EUNSUPPORTED;
  if (RM == 8) return core_grad_step<8>(h, grad_out, s);
  if (RM == 16) return core_grad_step<16>(h, grad_out, s);
  if (RM == 24) return core_grad_step<24>(h, grad_out, s);
  return core_grad_step<32>(h, grad_out, s);
}

nnc_status launch_slice_step(const CoreArgsHost &h, hipStream_t s) {
  int RM;
  bool big;
  if (!slice_fits(h, &RM, &big)) {
    // NNC_NO_BIG_SLICES in the environment leaves large cores to the grid-wide steps (for
    // comparisons: the tests check that both give the same sweeps)
    if (getenv("NNC_NO_BIG_SLICES") || !big_slice_fits(h, &RM)) return NNC_EUNSUPPORTED;
    if (RM == 8) return big_slice_step<8>(h, s);
    if (RM == 16) return big_slice_step<16>(h, s);
    if (RM == 24) return big_slice_step<24>(h, s);
    return big_slice_step<32>(h, s);
  }
#define NNC_SLICE(RMV) return big ? slice_step<RMV, true>(h, s) : slice_step<RMV, false>(h, s)
  if (RM == 8) NNC_SLICE(8);
  if (RM == 16) NNC_SLICE(16);
  if (RM == 24) NNC_SLICE(24);
  NNC_SLICE(32);
#undef NNC_SLICE
}

// =====================================================================================
// The core update in one launch when the last mode's Gram is the only one still changing:
// with U = G x_0 S_0 x_1 S_1 ... x_{d-2} S_{d-2} formed beforehand (uslice_body, beside the
// last mode's small contraction), den_G = U x_{d-1} S_{d-1}, and block i only needs slice i
// of U, of G and of the numerator partials, so nothing crosses blocks:
//   num[i] = sum_b part[b][i]  (b in order),  den[i] = U[i] x_{last} S_{d-1},
//   G[i] <- G[i] * num[i] / max(den[i], eps)  (FP64 division, clips counted).
// S_{d-1} is summed from its row-block partials in every block (block 0 stores it).
// =====================================================================================
// Slice i of U = (sum_i' S_0[i][i'] G[i']) x_1 S_1 ... x_{d-2} S_{d-2}, into a.T (the Gram of
// a.gram, if any, summed on the way as in the other slice kernels).
template <int RM, bool BIG>
static __device__ void uslice_body(const SliceArgs &a, int i) {
  extern __shared__ __attribute__((aligned(16))) float lds[];
  const int d = a.d, tid = threadIdx.x;
  float *Sl = lds;
  float *red = Sl + d * RM * RM;
  float *G = red + SliceLds<RM>::kRed;
  const int R0 = a.R[0];
  const int slice = a.gsize / R0;
  float *H0 = G + a.gsize, *H1 = H0 + slice;
  GramStage<RM> gs;
  constexpr int GPTH = (BIG ? kSliceMax : kSliceMax / 2) / kSliceThreads;  // core values per thread
  float gv[GPTH];
#pragma unroll
  for (int u = 0; u < GPTH; ++u) {
    const int e = tid + u * kSliceThreads;
    gv[u] = a.G[e < a.gsize ? e : a.gsize - 1];
  }
  gs.issue(a);
  __builtin_amdgcn_sched_barrier(0);  // every load above is issued before any is used
#pragma unroll
  for (int u = 0; u < GPTH; ++u) {
    const int e = tid + u * kSliceThreads;
    if (e < a.gsize) G[e] = gv[u];
  }
  gs.finish(a, Sl, red);
  __syncthreads();
  for (int c = tid; c < slice; c += kSliceThreads) {  // mode 0 first: S_0 row i
    float acc = 0.f;
    for (int ip = 0; ip < R0; ++ip) acc = fmaf(Sl[i * RM + ip], G[ip * slice + c], acc);
    H0[c] = acc;
  }
  __syncthreads();
  float *cur = H0, *nxt = H1;
  for (int k = 1; k < d - 1; ++k) {  // then modes 1 .. d-2 of the slice (modes 1 .. d-1)
    int pre = 1, post = 1;
    for (int t = 1; t < k; ++t) pre *= a.R[t];
    for (int t = k + 1; t < d; ++t) post *= a.R[t];
    slice_ttm<RM>(cur, nxt, pre, a.R[k], post, Sl + k * RM * RM);
    __syncthreads();
    float *t2 = cur;
    cur = nxt;
    nxt = t2;
  }
  for (int c = tid; c < slice; c += kSliceThreads) a.T[(int64_t)i * slice + c] = cur[c];
}

template <int RM, bool BIG>
__global__ __launch_bounds__(kSliceThreads) void coreL_k(SliceArgs a, const float *__restrict__ part,
                                                        int nparts) {
  extern __shared__ __attribute__((aligned(16))) float lds[];
  __shared__ unsigned int nclip;
  const int d = a.d, tid = threadIdx.x, i = blockIdx.x;
  float *Sl = lds;
  float *red = Sl + d * RM * RM;
  const int slice = a.gsize / a.R[0];
  float *H0 = red + SliceLds<RM>::kRed, *H1 = H0 + slice;
  constexpr int SPT = (BIG ? kSliceMax : kSliceMax / 2) / kSliceThreads;  // slice values per thread
  constexpr int kNB = BIG ? 32 : 64;  // partials in flight (fewer beside a larger slice)
  float uv[SPT];
#pragma unroll
  for (int u = 0; u < SPT; ++u) {
    const int c = tid + u * kSliceThreads;
    uv[u] = a.T[(int64_t)i * slice + (c < slice ? c : slice - 1)];
  }
  // the numerator of the thread's first entry: its first kNB partials now
  const int c0 = tid < slice ? tid : slice - 1;
  float pv[kNB];
#pragma unroll
  for (int u = 0; u < kNB; ++u) pv[u] = part[(int64_t)(u < nparts ? u : nparts - 1) * a.gsize + (int64_t)i * slice + c0];
  GramStage<RM> gs;
  gs.issue(a);
  __builtin_amdgcn_sched_barrier(0);  // every load above is issued before any is used
  if (tid == 0) nclip = 0;
#pragma unroll
  for (int u = 0; u < SPT; ++u) {
    const int c = tid + u * kSliceThreads;
    if (c < slice) H0[c] = uv[u];
  }
  gs.finish(a, Sl, red);
  __syncthreads();
  const int Rl = a.R[d - 1];
  slice_ttm<RM>(H0, H1, slice / Rl, Rl, 1, Sl + (d - 1) * RM * RM);  // den = U[i] x_last S_last
  __syncthreads();
  unsigned int mine = 0;
  for (int c = tid; c < slice; c += kSliceThreads) {
    const int64_t e = (int64_t)i * slice + c;
    float num = 0.f;  // partials in order from 0, kNB loads in flight per round
    int b0 = 0;
    if (c == tid) {
#pragma unroll
      for (int u = 0; u < kNB; ++u)
        if (u < nparts) num += pv[u];
      b0 = kNB;
    }
    for (; b0 < nparts; b0 += kNB) {
      float v[kNB];
#pragma unroll
      for (int u = 0; u < kNB; ++u) v[u] = part[(int64_t)(b0 + u < nparts ? b0 + u : nparts - 1) * a.gsize + e];
#pragma unroll
      for (int u = 0; u < kNB; ++u)
        if (b0 + u < nparts) num += v[u];
    }
    double dd = (double)H1[c];
    if (dd < a.eps) {
      dd = a.eps;
      ++mine;
    }
    a.Gout[e] = (float)(((double)a.G[e] * (double)num) / dd);
  }
  if (mine) atomicAdd(&nclip, mine);
  __syncthreads();
  if (tid == 0 && nclip) atomicAdd(a.clips, (unsigned long long)nclip);
}

// =====================================================================================
// One launch for independent steps: blocks [0, nm) build the rows of M_next (with the new
// Gram of the factor just updated), blocks [nm, nm + tiles) contract a partial tensor
// (small_body) and, when h.u_out is set, the R_0 blocks after them form the slices of
// U = G x_0 S_0 ... x_{d-2} S_{d-2} for coreL_k.  Each step alone leaves most CUs idle for most of its time, and the two
// do not depend on each other, so sharing a launch runs them side by side without the
// cost of a second stream.
// =====================================================================================
template <int RMS, int RMC, bool BIG>
__global__ __launch_bounds__(kSliceThreads) void small_mrows_k(SmallArgs sa, SliceArgs ca, int nm,
                                                              int64_t tiles) {
  if ((int)blockIdx.x < nm)
    mrows_body<RMC, BIG>(ca, blockIdx.x);
  else if ((int64_t)blockIdx.x - nm < tiles)
    small_body<RMS>(sa, (int64_t)blockIdx.x - nm);
  else
    uslice_body<RMC, BIG>(ca, (int)((int64_t)blockIdx.x - nm - tiles));
}

nnc_status launch_small_with_core(const float *in, int64_t P, int64_t N, int64_t Q, const float *F,
                                  int64_t ldl, int64_t ldr, int64_t R, float *out,
                                  const CoreArgsHost &h, hipStream_t s) {
  SmallArgs sa;
  int RMS, RMC;
  int64_t tiles;
  bool big;
  // the shared launch covers a core step that only forms a Gram and M_next
  // the contraction's rank tile is padded up to RMC - 4 when smaller (rows past R are masked,
  // so the values are the same), which keeps the instantiations to two per core tile
  const bool ok = !h.do_core && h.next >= 0 && slice_fits(h, &RMC, &big) &&
                  small_args(in, P, N, Q, F, ldl, ldr, R, out, &sa, &RMS, &tiles) && RMS <= RMC &&
                  tiles + h.R[h.next] + h.R[0] <= 0x7fffffff;
  if (ok && RMS < RMC - 4) RMS = RMC - 4;
  if (!ok) {
    if (h.u_out) return fail(NNC_EUNSUPPORTED, "U slices need the shared small-contraction launch");
    NNC_TRY(launch_core_step(h, s));
    return launch_ttm_small(in, P, N, Q, F, ldl, ldr, R, out, s);
  }
  SliceArgs ca = slice_args(h);
  ca.n = h.next;
  ca.M = h.M;
  ca.T = h.u_out;
  const int nm = (int)h.R[h.next];
  const int nu = h.u_out ? (int)h.R[0] : 0;
  size_t lds = 0;
#define NNC_SM(RMSV, RMCV, BIGV)                                                                  \
  do {                                                                                            \
    lds = std::max(SliceLds<RMCV>::bytes(ca.d, ca.gsize, std::max(ca.gsize / nm, ca.gsize / ca.R[0]), true), \
                   small_lds(sa.W, RMSV));                                                        \
    NNC_TRY(allow_slice_lds(reinterpret_cast<const void *>(small_mrows_k<RMSV, RMCV, BIGV>), lds)); \
    hipLaunchKernelGGL((small_mrows_k<RMSV, RMCV, BIGV>), dim3((unsigned)(nm + tiles + nu)),       \
                       dim3(kSliceThreads), lds, s, sa, ca, nm, tiles);                           \
  } while (0)
#define NNC_SM2(RMCV)                                  \
  do {                                                 \
    if (RMS == RMCV && big) NNC_SM(RMCV, RMCV, true);  \
    else if (RMS == RMCV) NNC_SM(RMCV, RMCV, false);   \
    else if (big) NNC_SM(RMCV - 4, RMCV, true);        \
    else NNC_SM(RMCV - 4, RMCV, false);                \
  } while (0)
  if (RMC == 8) NNC_SM2(8);
  else if (RMC == 16) NNC_SM2(16);
  else if (RMC == 24) NNC_SM2(24);
  else NNC_SM2(32);
#undef NNC_SM2
#undef NNC_SM
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

nnc_status launch_core_last(const CoreArgsHost &h, hipStream_t s) {
  int RM;
  bool big;
  if (!h.do_core || h.gram_to != h.d || h.gram_from != h.d - 1 || !h.gpart || h.nparts < 1 || !h.t0 ||
      !slice_fits(h, &RM, &big))
    return fail(NNC_EUNSUPPORTED, "core update in one launch: unsupported arguments");
  SliceArgs a = slice_args(h);
  a.T = h.t0;
  a.Gout = h.G;
#define NNC_CL(RMV, BIGV)                                                                         \
  do {                                                                                            \
    const size_t lds = SliceLds<RMV>::bytes(a.d, a.gsize, a.gsize / a.R[0], false);               \
    NNC_TRY(allow_slice_lds(reinterpret_cast<const void *>(coreL_k<RMV, BIGV>), lds));            \
    hipLaunchKernelGGL((coreL_k<RMV, BIGV>), dim3(a.R[0]), dim3(kSliceThreads), lds, s, a, h.gpart, \
                       h.nparts);                                                                 \
  } while (0)
#define NNC_CL2(RMV)                  \
  do {                                \
    if (big) NNC_CL(RMV, true);       \
    else NNC_CL(RMV, false);          \
  } while (0)
  if (RM == 8) NNC_CL2(8);
  else if (RM == 16) NNC_CL2(16);
  else if (RM == 24) NNC_CL2(24);
  else NNC_CL2(32);
#undef NNC_CL2
#undef NNC_CL
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

}  // namespace nnc
