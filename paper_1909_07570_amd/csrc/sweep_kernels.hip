// Kernels for the small (non-X-streaming) steps of a multiplicative-update sweep:
//   mu_rows_k   : fused numerator, denominator and update of a block of factor rows
//   core_step_k : one workgroup doing the core-space work between mode updates
//                 (Gram of the new factor, the core update, the next mode's R x R matrix)
#include <string.h>

#include <algorithm>

#include "nnc_internal.h"

namespace nnc {

// =====================================================================================
// Fused multiplicative update of rows [i0, i0 + kRB) of factor A_n (N_n x R, R <= 32):
//   num[i][r] = sum_{c=(p,q)} Y[p][i][q] * G[p][r][q]        (unfold_n(Y) unfold_n(G)^T)
//   den[i][r] = sum_s A[i][s] * M[s][r]
//   A[i][r]  <- A[i][r] * num / max(den, eps)        (or grad[i][r] = den - num)
// Each block also leaves the Gram of its new rows in gram[block][R][R] (summed later in a
// fixed order) and, with gpart (last mode, q range 1), its share of the core numerator
// gpart[block][p][r] = sum_{i in block} Y[p][i] * Anew[i][r].
// =====================================================================================
constexpr int kRB = 8;
constexpr int kRowThreads = 512;
// dynamic LDS budget of one block (floats); with the static arrays below one block takes
// most of a CU's LDS when the core is large (fewer chunks of G: 128^4 at rank 16 ran 2.5 %
// faster than with a 56 KB budget), while small problems use only what their chunk needs
constexpr int kRowLdsFloats = 32 * 1024;
constexpr int kRowRed = 4096;             // partial sums of the contraction (floats)

// Contraction paths (chosen per launch from the shape):
//   kPathQ4: post % 4 == 0; a thread takes row i and columns r, r + 1 over a range of
//            column quads (4 adjacent q of one p): 3 float4 LDS reads per 8 FMAs
//   kPathP : post == 1, R % 4 == 0; a thread takes rows i, i + 1 and columns r .. r + 3
//            over a range of p: 2 reads and one float4 read per 8 FMAs
//   kPathS : anything else, one output per thread, scalar reads
enum { kPathQ4 = 0, kPathP = 1, kPathS = 2 };

// LDS (dynamic): the chunk of G and of the block's Y rows in their natural layouts, rows of
// qn values at a stride of qs floats,
//   Gs[(pl * R + r) * qs + qq] = G[p0 + pl][r][q0 + qq]
//   Ys[(pl * nr + i) * qs + qq] = Y[p0 + pl][i0 + i][q0 + qq]
// A chunk is pn whole slices p (qn = post) when they fit, else a quad-aligned q range of
// one slice.  Staging is a copy: consecutive threads read consecutive addresses.  In the
// quad path qs is an odd number of quads (qn, or qn + 4), so the rows that one wave's
// 16-byte reads touch start in different bank groups.  Elsewhere qs = qn.
// Index arithmetic is kept off the quarter-rate integer multiplier: divisions go through
// float reciprocals (qdiv), and the contraction walks LDS pointers with a fixed jump at the
// end of a slice.  The contraction issues the reads of kUn steps before their products, so
// one LDS latency covers kUn steps; each accumulator still takes its terms in c order.
constexpr int kUn = 4;
constexpr int kMuSplitMax = 16;  // parts of a split numerator at most (mu_fin_k takes up to 16 at once)

template <int PATH, bool SPLIT>
__global__ __launch_bounds__(kRowThreads) void mu_rows_k(const float *__restrict__ Y,
                                                         const float *__restrict__ G,
                                                         float *__restrict__ A,
                                                         const float *__restrict__ M, int pre,
                                                         int Nn, int post, int R, int PC, int QC,
                                                         double eps, unsigned long long *clips,
                                                         float *__restrict__ gram,
                                                         float *__restrict__ gpart,
                                                         float *__restrict__ grad,
                                                         int ksplit, float *__restrict__ npart) {
  extern __shared__ __attribute__((aligned(16))) float dynr[];
  // the block's rows of A_n and M_n transposed, zero past nr / R, rows of 36 floats (an odd
  // number of 16-byte quads) for the 16-byte reads of the denominator
  __shared__ __attribute__((aligned(16))) float As[kRB][36];
  __shared__ __attribute__((aligned(16))) float MsT[32][36];
  __shared__ __attribute__((aligned(16))) float red[kRowRed];
  __shared__ unsigned int nclip;
  const int tid = threadIdx.x;
  const int i0 = blockIdx.x * kRB;
  const int nr = (Nn - i0) < kRB ? (Nn - i0) : kRB;
  if (tid == 0) nclip = 0;
  const float inv_R = 1.0f / (float)R;
  // work items and splits of the contraction (every chunk uses the same assignment, so a
  // thread's partial sums carry across chunks)
  const int RH = (R + 1) / 2, RQ = R / 4, NH = (nr + 1) / 2;
  const int items = PATH == kPathQ4 ? nr * RH : (PATH == kPathP ? NH * RQ : nr * R);
  const float inv_items = 1.0f / (float)items;
  const int SPL = qdiv(kRowThreads, inv_items);  // >= 1: items <= 8 * 32
  const int sp = qdiv(tid, inv_items), item = tid - sp * items;
  const bool act = sp < SPL;
  const float inv_spl = 1.0f / (float)SPL;
  int ii, rr;  // first row / column of the item
  if (PATH == kPathQ4) { ii = qdiv(item, 1.0f / (float)RH); rr = 2 * (item - ii * RH); }
  else if (PATH == kPathP) { const int g = qdiv(item, 1.0f / (float)RQ); ii = 2 * g; rr = 4 * (item - g * RQ); }
  else { ii = qdiv(item, inv_R); rr = item - ii * R; }
  constexpr int NO = PATH == kPathQ4 ? 2 : (PATH == kPathP ? 8 : 1);  // outputs per item
  float acc[NO];
#pragma unroll
  for (int o = 0; o < NO; ++o) acc[o] = 0.f;
  // factor rows and M, loaded with the first chunk's reads: thread t < 256 takes As[t / 32]
  // [t % 32], and entries t and t + 512 of MsT[r][s] = M[s][r] (32 x 32 with zero padding)
  const int RR = R * R;
  const int ai = tid >> 5, ac = tid & 31;
  const bool aok = tid < kRB * 32 && ai < nr && ac < R;
  const float av0 = A[(int64_t)i0 * R + (aok ? ai * R + ac : 0)];
  const int mr0 = tid >> 5, ms0 = tid & 31, mr1 = mr0 + 16;
  const bool mok0 = mr0 < R && ms0 < R, mok1 = mr1 < R && ms0 < R;
  const float mv0 = M[mok0 ? ms0 * R + mr0 : 0];
  const float mv1 = M[mok1 ? ms0 * R + mr1 : 0];
  constexpr int kSG = 16, kSY = 8;  // staged values per thread and round
  bool first = true;
  // SPLIT: block (b, ks) takes part ks of the contracted index (a range of p, or with
  // pre < ksplit a quad-aligned range of q in slices of one p, PC == 1) and leaves its
  // partial numerator in npart[ks]; mu_fin_k adds the parts in order and updates the rows
  int pb = 0, pe = pre, qb = 0, qe = post;
  if (SPLIT) {
    const int ks = blockIdx.y;
    if (pre >= ksplit) {
      pb = (int)((int64_t)pre * ks / ksplit);
      pe = (int)((int64_t)pre * (ks + 1) / ksplit);
    } else {
      const int nq4 = (post + 3) >> 2;
      qb = 4 * (int)((int64_t)nq4 * ks / ksplit);
      qe = min(post, 4 * (int)((int64_t)nq4 * (ks + 1) / ksplit));
    }
  }
  for (int p0 = pb; p0 < pe; p0 += PC) {
    const int pn = (pe - p0) < PC ? (pe - p0) : PC;
    for (int q0 = qb; q0 < qe; q0 += QC) {
      const int qn = (qe - q0) < QC ? (qe - q0) : QC;
      const bool whole = qn == post;  // whole slices: G and Y chunk offsets are linear
      const int ng = pn * R * qn, ny = pn * nr * qn;  // both at most 2^15 (the LDS budget)
      const int nrq = nr * qn;
      const int qs = PATH == kPathQ4 && ((qn >> 2) & 1) == 0 ? qn + 4 : qn;
      float *Gs = dynr, *Ys = dynr + pn * R * qs;
      const float inv_qn = 1.0f / (float)qn, inv_nrq = 1.0f / (float)nrq;
      const float *Gc = G + (int64_t)p0 * R * post + q0;
      const float *Yc = Y + ((int64_t)p0 * Nn + i0) * post + q0;
      const int64_t ystride = (int64_t)Nn * post;  // from one slice p of Y to the next
      __syncthreads();  // the previous chunk's reads are done
      auto lds_index = [&](int e) -> int {  // row e / qn at stride qs
        if (PATH != kPathQ4) return e;
        return e + (qs - qn) * qdiv(e, inv_qn);
      };
      auto stage = [&](auto goff, auto yoff) {
        for (int gb = 0, yb = 0; gb < ng || yb < ny; gb += kSG * kRowThreads, yb += kSY * kRowThreads) {
          float vg[kSG], vy[kSY];
#pragma unroll
          for (int u = 0; u < kSG; ++u) {
            const int e = gb + tid + u * kRowThreads;
            vg[u] = Gc[goff(e < ng ? e : ng - 1)];  // past the end: the last value again
          }
#pragma unroll
          for (int u = 0; u < kSY; ++u) {
            const int e = yb + tid + u * kRowThreads;
            vy[u] = Yc[yoff(e < ny ? e : ny - 1)];
          }
#pragma unroll
          for (int u = 0; u < kSG; ++u) {
            const int e = gb + tid + u * kRowThreads;
            Gs[lds_index(e < ng ? e : ng - 1)] = vg[u];
          }
#pragma unroll
          for (int u = 0; u < kSY; ++u) {
            const int e = yb + tid + u * kRowThreads;
            Ys[lds_index(e < ny ? e : ny - 1)] = vy[u];
          }
        }
      };
      // 16-byte staging when G and Y are 16-byte aligned: the quad path (rows of qn / 4 quads,
      // at qs / 4 in LDS) and the slice path when its rows come in whole quads (nr and Nn
      // multiples of 4).  Offsets and LDS indices count quads; G and Y rows are
      // row_G = pl * R + r and row_Y = pl * nr + i of the chunk.
      const bool al = ((reinterpret_cast<uintptr_t>(G) | reinterpret_cast<uintptr_t>(Y)) & 15) == 0;
      if (al && (PATH == kPathQ4 || (PATH == kPathP && (nr & 3) == 0 && (Nn & 3) == 0))) {
        const int nq = PATH == kPathQ4 ? qn >> 2 : nr >> 2;  // quads of a row / of one p
        const int sq = qs >> 2, post4 = post >> 2;
        const float inv_nq = 1.0f / (float)nq, inv_nr = 1.0f / (float)nr;
        const int64_t ys4 = ystride >> 2;
        const int ngq = ng >> 2, nyq = ny >> 2;
        const float4 *G4 = reinterpret_cast<const float4 *>(Gc);
        const float4 *Y4 = reinterpret_cast<const float4 *>(Yc);
        float4 *Gs4 = reinterpret_cast<float4 *>(Gs), *Ys4 = reinterpret_cast<float4 *>(Ys);
        constexpr int kQG = 4, kQY = 2;
        for (int gb = 0, yb = 0; gb < ngq || yb < nyq; gb += kQG * kRowThreads, yb += kQY * kRowThreads) {
          float4 vg[kQG], vy[kQY];
          int gl[kQG], yl[kQY];
#pragma unroll
          for (int u = 0; u < kQG; ++u) {
            const int e = min(gb + tid + u * kRowThreads, ngq - 1);  // past the end: the last again
            int64_t off = e;
            int l = e;
            if (PATH == kPathQ4) {
              const int row = qdiv(e, inv_nq), c = e - __umul24(row, nq);
              off = (int64_t)row * post4 + c;
              l = __umul24(row, sq) + c;
            }
            vg[u] = G4[off];
            gl[u] = l;
          }
#pragma unroll
          for (int u = 0; u < kQY; ++u) {
            const int e = min(yb + tid + u * kRowThreads, nyq - 1);
            int64_t off;
            int l = e;
            if (PATH == kPathQ4) {
              const int row = qdiv(e, inv_nq), c = e - __umul24(row, nq);
              const int pl = qdiv(row, inv_nr), i = row - __umul24(pl, nr);
              off = (int64_t)pl * ys4 + (int64_t)i * post4 + c;
              l = __umul24(row, sq) + c;
            } else {
              const int pl = qdiv(e, inv_nq);
              off = (int64_t)pl * ys4 + (e - __umul24(pl, nq));
            }
            vy[u] = Y4[off];
            yl[u] = l;
          }
#pragma unroll
          for (int u = 0; u < kQG; ++u) Gs4[gl[u]] = vg[u];
#pragma unroll
          for (int u = 0; u < kQY; ++u) Ys4[yl[u]] = vy[u];
        }
      } else if (whole && ystride < ((int64_t)1 << 32)) {
        // the uniform choice made once, outside the loads; whole slices: e = pl * nr * qn +
        // (i * qn + qq) in Y, one 32 x 32 -> 64-bit multiply when the slice stride allows
        const unsigned ys = (unsigned)ystride;
        stage([&](int e) -> int64_t { return e; },
              [&](int e) -> int64_t {
                const int pl = qdiv(e, inv_nrq);
                return (int64_t)((uint64_t)(unsigned)pl * ys) + (e - __umul24(pl, nrq));
              });
      } else if (whole) {
        stage([&](int e) -> int64_t { return e; },
              [&](int e) -> int64_t {
                const int pl = qdiv(e, inv_nrq);
                return (int64_t)pl * ystride + (e - __umul24(pl, nrq));
              });
      } else  // one slice, e = r * qn + qq (G) or i * qn + qq (Y)
        stage([&](int e) -> int64_t {
                const int r = qdiv(e, inv_qn);
                return (int64_t)r * post + (e - __umul24(r, qn));
              },
              [&](int e) -> int64_t {
                const int i = qdiv(e, inv_qn);
                return (int64_t)i * post + (e - __umul24(i, qn));
              });
      if (first) {
        if (tid < kRB * 32) As[ai][ac] = aok ? av0 : 0.f;
        MsT[mr0][ms0] = mok0 ? mv0 : 0.f;
        MsT[mr1][ms0] = mok1 ? mv1 : 0.f;
        first = false;
      }
      __syncthreads();
      if (act) {
        if (PATH == kPathQ4) {
          // quads u = pl * (qn / 4) + q4 over [u0, u1)
          const int nq4 = qn >> 2, U = pn * nq4;
          const int u0 = qdiv(U * sp, inv_spl), u1 = qdiv(U * (sp + 1), inv_spl);
          int pl = qdiv(u0, 1.0f / (float)nq4), q4 = u0 - pl * nq4;
          const float *yp = Ys + (pl * nr + ii) * qs + 4 * q4;
          const float *gp = Gs + (pl * R + rr) * qs + 4 * q4;
          const int go = rr + 1 < R ? qs : 0;                   // the item's second column
          const int yj = nr * qs - qn, gj = R * qs - qn;        // row end -> same row, next slice
          auto step = [&](float4 &y, float4 &ga, float4 &gb) {
            y = *reinterpret_cast<const float4 *>(yp);
            ga = *reinterpret_cast<const float4 *>(gp);
            gb = *reinterpret_cast<const float4 *>(gp + go);
            yp += 4;
            gp += 4;
            const bool wrap = ++q4 == nq4;
            q4 = wrap ? 0 : q4;
            yp += wrap ? yj : 0;
            gp += wrap ? gj : 0;
          };
          auto prod = [&](const float4 &y, const float4 &ga, const float4 &gb) {
            acc[0] = fmaf(y.x, ga.x, acc[0]);
            acc[0] = fmaf(y.y, ga.y, acc[0]);
            acc[0] = fmaf(y.z, ga.z, acc[0]);
            acc[0] = fmaf(y.w, ga.w, acc[0]);
            acc[1] = fmaf(y.x, gb.x, acc[1]);
            acc[1] = fmaf(y.y, gb.y, acc[1]);
            acc[1] = fmaf(y.z, gb.z, acc[1]);
            acc[1] = fmaf(y.w, gb.w, acc[1]);
          };
          int u = u0;
          for (; u + kUn <= u1; u += kUn) {
            float4 y[kUn], ga[kUn], gb[kUn];
#pragma unroll
            for (int k = 0; k < kUn; ++k) step(y[k], ga[k], gb[k]);
#pragma unroll
            for (int k = 0; k < kUn; ++k) prod(y[k], ga[k], gb[k]);
          }
          for (; u < u1; ++u) {
            float4 y, ga, gb;
            step(y, ga, gb);
            prod(y, ga, gb);
          }
        } else if (PATH == kPathP) {
          // qn == 1: Ys[pl * nr + i], Gs[pl * R + r]
          const int u0 = qdiv(pn * sp, inv_spl), u1 = qdiv(pn * (sp + 1), inv_spl);
          const int yo = ii + 1 < nr ? 1 : 0;  // the item's second row
          const float *yp = Ys + u0 * nr + ii;
          const float *gp = Gs + u0 * R + rr;
          auto step = [&](float &y0, float &y1, float4 &g) {
            y0 = yp[0];
            y1 = yp[yo];
            g = *reinterpret_cast<const float4 *>(gp);
            yp += nr;
            gp += R;
          };
          auto prod = [&](float y0, float y1, const float4 &g) {
            acc[0] = fmaf(y0, g.x, acc[0]);
            acc[1] = fmaf(y0, g.y, acc[1]);
            acc[2] = fmaf(y0, g.z, acc[2]);
            acc[3] = fmaf(y0, g.w, acc[3]);
            acc[4] = fmaf(y1, g.x, acc[4]);
            acc[5] = fmaf(y1, g.y, acc[5]);
            acc[6] = fmaf(y1, g.z, acc[6]);
            acc[7] = fmaf(y1, g.w, acc[7]);
          };
          int u = u0;
          for (; u + kUn <= u1; u += kUn) {
            float y0[kUn], y1[kUn];
            float4 g[kUn];
#pragma unroll
            for (int k = 0; k < kUn; ++k) step(y0[k], y1[k], g[k]);
#pragma unroll
            for (int k = 0; k < kUn; ++k) prod(y0[k], y1[k], g[k]);
          }
          for (; u < u1; ++u) {
            float y0, y1;
            float4 g;
            step(y0, y1, g);
            prod(y0, y1, g);
          }
        } else {
          // c = pl * qn + qq over [u0, u1), one output
          const int Cn = pn * qn;
          const int u0 = qdiv(Cn * sp, inv_spl), u1 = qdiv(Cn * (sp + 1), inv_spl);
          int pl = qdiv(u0, inv_qn), qq = u0 - pl * qn;
          const float *yp = Ys + (pl * nr + ii) * qn + qq;
          const float *gp = Gs + (pl * R + rr) * qn + qq;
          const int yj = (nr - 1) * qn, gj = (R - 1) * qn;
          auto step = [&](float &y, float &g) {
            y = *yp++;
            g = *gp++;
            const bool wrap = ++qq == qn;
            qq = wrap ? 0 : qq;
            yp += wrap ? yj : 0;
            gp += wrap ? gj : 0;
          };
          int u = u0;
          for (; u + kUn <= u1; u += kUn) {
            float y[kUn], g[kUn];
#pragma unroll
            for (int k = 0; k < kUn; ++k) step(y[k], g[k]);
#pragma unroll
            for (int k = 0; k < kUn; ++k) acc[0] = fmaf(y[k], g[k], acc[0]);
          }
          for (; u < u1; ++u) {
            float y, g;
            step(y, g);
            acc[0] = fmaf(y, g, acc[0]);
          }
        }
      }
    }
  }
  __syncthreads();
  // partial sums red[sp][i][r], added in split order by the output's owner
  const int NRR = nr * R;
  if (act) {
    if (PATH == kPathQ4) {
      red[sp * NRR + ii * R + rr] = acc[0];
      if (rr + 1 < R) red[sp * NRR + ii * R + rr + 1] = acc[1];
    } else if (PATH == kPathP) {
#pragma unroll
      for (int k = 0; k < 4; ++k) red[sp * NRR + ii * R + rr + k] = acc[k];
      if (ii + 1 < nr) {
#pragma unroll
        for (int k = 0; k < 4; ++k) red[sp * NRR + (ii + 1) * R + rr + k] = acc[4 + k];
      }
    } else {
      red[sp * NRR + ii * R + rr] = acc[0];
    }
  }
  __syncthreads();
  const bool own = tid < NRR;  // thread tid owns output (tid / R, tid % R) from here
  const int oi = qdiv(tid, inv_R), orr = tid - oi * R;
  if (SPLIT) {
    if (own) {
      float num = 0.f;
#pragma unroll 8
      for (int k = 0; k < SPL; ++k) num += red[k * NRR + tid];
      npart[((int64_t)blockIdx.y * Nn + i0) * R + tid] = num;
    }
    return;
  }
  float nv = 0.f;
  if (own) {
    float num = 0.f;
#pragma unroll 8
    for (int k = 0; k < SPL; ++k) num += red[k * NRR + tid];
    // s = 0 .. 31 in order; the terms past R are zero times zero and leave den unchanged
    const float4 *arow = reinterpret_cast<const float4 *>(As[oi]);
    const float4 *mrow = reinterpret_cast<const float4 *>(MsT[orr]);
    float den = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float4 a = arow[q], m = mrow[q];
      den = fmaf(a.x, m.x, den);
      den = fmaf(a.y, m.y, den);
      den = fmaf(a.z, m.z, den);
      den = fmaf(a.w, m.w, den);
    }
    if (grad) {
      nv = den - num;
    } else {
      double dd = (double)den;
      if (dd < eps) {
        dd = eps;
        atomicAdd(&nclip, 1u);
      }
      nv = (float)(((double)As[oi][orr] * (double)num) / dd);
    }
  }
  __syncthreads();
  if (own) {
    if (grad) {
      grad[(int64_t)i0 * R + tid] = nv;
    } else {
      A[(int64_t)i0 * R + tid] = nv;
      As[oi][orr] = nv;
    }
  }
  __syncthreads();
  if (tid == 0 && nclip) atomicAdd(clips, (unsigned long long)nclip);
  if (grad) return;
  if (gram) {  // Gram of this block's new rows (the arithmetic of gram_parts_k)
    float *gb = gram + (int64_t)blockIdx.x * R * R;
    for (int idx = tid; idx < RR; idx += kRowThreads) {
      const int x = qdiv(idx, inv_R), y = idx - x * R;
      float s2 = 0.f;
#pragma unroll
      for (int i = 0; i < kRB; ++i) {  // rows past nr read row nr - 1 and are not added
        const int ic = i < nr ? i : nr - 1;
        const float t = fmaf(As[ic][x], As[ic][y], s2);
        s2 = i < nr ? t : s2;
      }
      gb[idx] = s2;
    }
  }
  if (gpart) {
    // last mode (post == 1): gpart[block][p][r] = sum_i Y[p][i0 + i] Anew[i][r]
    float *gp = gpart + (int64_t)blockIdx.x * pre * R;
    if (PC >= pre) {
      // one chunk: the Y rows are still in LDS, Ys[p * nr + i]; thread (g, r4) keeps
      // columns r4 .. r4 + 3 of the new rows in registers (zero past R)
      const float *Ys = dynr + pre * R;
      const int RQ4 = (R + 3) / 4;
      const float inv_rq4 = 1.0f / (float)RQ4;
      const int ng2 = qdiv(kRowThreads, inv_rq4);
      const int g = qdiv(tid, inv_rq4), r4 = 4 * (tid - g * RQ4);
      const bool vec = (R & 3) == 0;  // whole float4 rows (gpart is 16-byte aligned)
      if (g < ng2) {
        float ar[kRB][4];
#pragma unroll
        for (int i = 0; i < kRB; ++i)
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int ic = i < nr ? i : nr - 1, kc = r4 + k < R ? r4 + k : R - 1;
            const float a = As[ic][kc];
            ar[i][k] = r4 + k < R ? a : 0.f;
          }
        auto put = [&](int pp, const float (&s4)[4]) {
          float *dst = gp + (int64_t)pp * R + r4;
          if (vec) {
            *reinterpret_cast<float4 *>(dst) = make_float4(s4[0], s4[1], s4[2], s4[3]);
          } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
              if (r4 + k < R) dst[k] = s4[k];
          }
        };
        if (nr == kRB && vec) {
          // whole blocks: the 8 values of row p are two 16-byte reads (Ys is 16-byte aligned)
          for (int pp = g; pp < pre; pp += ng2) {
            const float4 *yr = reinterpret_cast<const float4 *>(Ys + pp * kRB);
            const float4 y0 = yr[0], y1 = yr[1];
            const float yv[kRB] = {y0.x, y0.y, y0.z, y0.w, y1.x, y1.y, y1.z, y1.w};
            float s4[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int i = 0; i < kRB; ++i)
#pragma unroll
              for (int k = 0; k < 4; ++k) s4[k] = fmaf(yv[i], ar[i][k], s4[k]);
            put(pp, s4);
          }
        } else {
          for (int pp = g; pp < pre; pp += ng2) {
            float s4[4] = {0.f, 0.f, 0.f, 0.f};
            const float *yr = Ys + pp * nr;
#pragma unroll
            for (int i = 0; i < kRB; ++i) {
              const float y = yr[i < nr ? i : nr - 1];  // rows past nr are not added
#pragma unroll
              for (int k = 0; k < 4; ++k) {
                const float t = fmaf(y, ar[i][k], s4[k]);
                s4[k] = i < nr ? t : s4[k];
              }
            }
            put(pp, s4);
          }
        }
      }
    } else {
      // several chunks: read the Y rows again, pieces of PC2 rows p (the block's dynamic LDS
      // holds PC * (R + kRB) floats when post == 1)
      const int PC2 = PC * (R + kRB) / kRB;
      for (int p0 = 0; p0 < pre; p0 += PC2) {
        const int pn = (pre - p0) < PC2 ? (pre - p0) : PC2;
        __syncthreads();
        for (int idx = tid; idx < pn * nr; idx += kRowThreads) {
          const int pp = idx / nr, i = idx - (idx / nr) * nr;
          dynr[idx] = Y[(int64_t)(p0 + pp) * Nn + i0 + i];
        }
        __syncthreads();
        for (int idx = tid; idx < pn * R; idx += kRowThreads) {
          const int pp = idx / R, r = idx - (idx / R) * R;
          float s2 = 0.f;
          for (int i = 0; i < nr; ++i) s2 = fmaf(dynr[pp * nr + i], As[i][r], s2);
          gp[(int64_t)(p0 + pp) * R + r] = s2;
        }
      }
    }
  }
}

// The row update after a split numerator (mu_rows_k<PATH, true>): rows [i0, i0 + kRB) of
// A_n, num = the ksplit parts added in order, den = A M (s in order, as in mu_rows_k), the
// multiplicative step with the FP64 division (or grad = den - num), the clip count and the
// Gram partial of the new rows.
constexpr int kFinThreads = kRB * 32;
__global__ __launch_bounds__(kFinThreads) void mu_fin_k(const float *__restrict__ npart, int ksplit,
                                                       float *__restrict__ A, const float *__restrict__ M,
                                                       int Nn, int R, double eps, unsigned long long *clips,
                                                       float *__restrict__ gram, float *__restrict__ grad) {
  __shared__ __attribute__((aligned(16))) float As[kRB][36];
  __shared__ __attribute__((aligned(16))) float MsT[32][36];
  __shared__ unsigned int nclip;
  const int tid = threadIdx.x;
  const int i0 = blockIdx.x * kRB;
  const int nr = (Nn - i0) < kRB ? (Nn - i0) : kRB;
  const int NRR = nr * R;
  const bool own = tid < NRR;
  const float inv_R = 1.0f / (float)R;
  const int oi = qdiv(tid, inv_R), orr = tid - oi * R;
  // the parts of the thread's output, all loads issued together
  constexpr int kFP = 16;
  float pv[kFP];
#pragma unroll
  for (int k = 0; k < kFP; ++k) {
    const int kk = k < ksplit ? k : ksplit - 1;
    pv[k] = own ? npart[((int64_t)kk * Nn + i0) * R + tid] : 0.f;
  }
  {
    const int ai = tid >> 5, ac = tid & 31;  // kFinThreads == kRB * 32
    As[ai][ac] = (ai < nr && ac < R) ? A[(int64_t)(i0 + ai) * R + ac] : 0.f;
    for (int e = tid; e < 32 * 32; e += kFinThreads) {
      const int r = e >> 5, s2 = e & 31;
      MsT[r][s2] = (r < R && s2 < R) ? M[s2 * R + r] : 0.f;
    }
  }
  if (tid == 0) nclip = 0;
  __syncthreads();
  float nv = 0.f;
  if (own) {
    float num = 0.f;
#pragma unroll
    for (int k = 0; k < kFP; ++k)
      if (k < ksplit) num += pv[k];
    for (int k = kFP; k < ksplit; ++k) num += npart[((int64_t)k * Nn + i0) * R + tid];
    const float4 *arow = reinterpret_cast<const float4 *>(As[oi]);
    const float4 *mrow = reinterpret_cast<const float4 *>(MsT[orr]);
    float den = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float4 a = arow[q], m = mrow[q];
      den = fmaf(a.x, m.x, den);
      den = fmaf(a.y, m.y, den);
      den = fmaf(a.z, m.z, den);
      den = fmaf(a.w, m.w, den);
    }
    if (grad) {
      nv = den - num;
    } else {
      double dd = (double)den;
      if (dd < eps) {
        dd = eps;
        atomicAdd(&nclip, 1u);
      }
      nv = (float)(((double)As[oi][orr] * (double)num) / dd);
    }
  }
  __syncthreads();
  if (own) {
    if (grad) {
      grad[(int64_t)i0 * R + tid] = nv;
    } else {
      A[(int64_t)i0 * R + tid] = nv;
      As[oi][orr] = nv;
    }
  }
  __syncthreads();
  if (tid == 0 && nclip) atomicAdd(clips, (unsigned long long)nclip);
  if (grad || !gram) return;
  float *gb = gram + (int64_t)blockIdx.x * R * R;  // the arithmetic of mu_rows_k's partials
  for (int idx = tid; idx < R * R; idx += kFinThreads) {
    const int x = qdiv(idx, inv_R), y = idx - x * R;
    float s2 = 0.f;
#pragma unroll
    for (int i = 0; i < kRB; ++i) {
      const int ic = i < nr ? i : nr - 1;
      const float t = fmaf(As[ic][x], As[ic][y], s2);
      s2 = i < nr ? t : s2;
    }
    gb[idx] = s2;
  }
}

nnc_status launch_mu_rows(const float *Y, const float *G, float *A, const float *M, int64_t pre,
                          int64_t Nn, int64_t post, int64_t R, double eps, unsigned long long *clips,
                          float *gram, float *gpart, float *grad, hipStream_t s, float *npart) {
  if (R > 32) return fail(NNC_EUNSUPPORTED, "mu_rows: R %lld above 32", (long long)R);
  if (pre * post > (int64_t)1 << 30 || Nn > (int64_t)1 << 30)
    return fail(NNC_EUNSUPPORTED, "mu_rows: sizes above 2^30");
  if (gpart && post != 1) return fail(NNC_EINVAL, "mu_rows: core-numerator partials need post == 1");
  // chunks: whole slices p when one fits, else quad-aligned q ranges of one slice; rows
  // in the quad path take up to 4 floats of padding in LDS
  const int path = (post % 4 == 0) ? kPathQ4 : ((post == 1 && R % 4 == 0) ? kPathP : kPathS);
  const int64_t pad = path == kPathQ4 ? 4 : 0;
  int64_t PC, QC;
  const int64_t slice = (R + kRB) * (post + pad);
  if (slice <= kRowLdsFloats) {
    PC = kRowLdsFloats / slice;
    if (PC > pre) PC = pre;
    QC = post;
  } else {
    PC = 1;
    QC = (kRowLdsFloats / (R + kRB) - pad) / 4 * 4;
  }
  const int64_t blocks = (Nn + kRB - 1) / kRB;
  // few row blocks over a long contracted index (the factors of large cores): the index is
  // split over blocks and the parts added in order by mu_fin_k
  const int64_t K = pre * post;
  int ksplit = 1;
  if (npart && !gpart && blocks < 64 && K >= 2048) {
    ksplit = (int)std::min<int64_t>(std::min<int64_t>(kMuSplitMax, 256 / blocks), K / 512);
    if (ksplit < 2) ksplit = 1;
  }
  if (ksplit > 1 && pre < ksplit) {  // q ranges of one slice at a time
    const int64_t qr = ((post + ksplit - 1) / ksplit + 3) / 4 * 4;
    PC = 1;
    if (QC > qr) QC = qr;
  } else if (ksplit > 1 && PC > (pre + ksplit - 1) / ksplit) {
    PC = (pre + ksplit - 1) / ksplit;  // no chunk longer than one part's range of p
  }
  const size_t lds = (size_t)(PC * (R + kRB) * (QC + pad)) * sizeof(float);
  if (lds > 64 * 1024) {
    static bool attr[6] = {false, false, false, false, false, false};
    const int ai = path + 3 * (ksplit > 1);
    if (!attr[ai]) {
      const void *k = nullptr;
      if (ksplit > 1)
        k = path == kPathQ4 ? reinterpret_cast<const void *>(mu_rows_k<kPathQ4, true>)
            : path == kPathP ? reinterpret_cast<const void *>(mu_rows_k<kPathP, true>)
                             : reinterpret_cast<const void *>(mu_rows_k<kPathS, true>);
      else
        k = path == kPathQ4 ? reinterpret_cast<const void *>(mu_rows_k<kPathQ4, false>)
            : path == kPathP ? reinterpret_cast<const void *>(mu_rows_k<kPathP, false>)
                             : reinterpret_cast<const void *>(mu_rows_k<kPathS, false>);
      NNC_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kRowLdsFloats * (int)sizeof(float)));
      attr[ai] = true;
    }
  }
#define NNC_MU(PV, SV)                                                                                 \
  hipLaunchKernelGGL((mu_rows_k<PV, SV>), dim3((unsigned)blocks, (unsigned)ksplit), dim3(kRowThreads), \
                     lds, s, Y, G, A, M, (int)pre, (int)Nn, (int)post, (int)R, (int)PC, (int)QC, eps,   \
                     clips, gram, gpart, grad, ksplit, npart)
  if (ksplit > 1) {
    if (path == kPathQ4) NNC_MU(kPathQ4, true);
    else if (path == kPathP) NNC_MU(kPathP, true);
    else NNC_MU(kPathS, true);
    hipLaunchKernelGGL(mu_fin_k, dim3((unsigned)blocks), dim3(kFinThreads), 0, s, npart, ksplit, A, M, (int)Nn,
                       (int)R, eps, clips, gram, grad);
  } else {
    if (path == kPathQ4) NNC_MU(kPathQ4, false);
    else if (path == kPathP) NNC_MU(kPathP, false);
    else NNC_MU(kPathS, false);
  }
#undef NNC_MU
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

// Gram partials of a factor from its rows: gram[b][x][y] = sum_{i in [8b, 8b+8)} A[i][x] A[i][y],
// the same arithmetic as the epilogue of mu_rows_k.
__global__ __launch_bounds__(256) void gram_parts_k(const float *__restrict__ A, int Nn, int R,
                                                    float *__restrict__ gram) {
  const int i0 = blockIdx.x * kRB;
  const int nr = (Nn - i0) < kRB ? (Nn - i0) : kRB;
  for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) {
    const int x = idx / R, y = idx - (idx / R) * R;
    float s2 = 0.f;
    for (int i = 0; i < nr; ++i) s2 = fmaf(A[(int64_t)(i0 + i) * R + x], A[(int64_t)(i0 + i) * R + y], s2);
    gram[(int64_t)blockIdx.x * R * R + idx] = s2;
  }
}

nnc_status launch_gram_parts(const float *A, int64_t Nn, int64_t R, float *gram, hipStream_t s) {
  hipLaunchKernelGGL(gram_parts_k, dim3((unsigned)((Nn + kRB - 1) / kRB)), dim3(256), 0, s, A, (int)Nn,
                     (int)R, gram);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

int64_t mu_rows_blocks(int64_t Nn) { return (Nn + kRB - 1) / kRB; }
int64_t mu_rows_split_floats(int64_t Nn, int64_t R) { return kMuSplitMax * Nn * R; }

// out[e] = sum_{b < nparts} part[b][e], blocks added in order (loads issued 8 at a time).
__global__ __launch_bounds__(256) void sum_parts_k(const float *__restrict__ part, int nparts,
                                                   int64_t n, float *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  float s2 = 0.f;
  for (int b0 = 0; b0 < nparts; b0 += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = (b0 + u < nparts) ? part[(int64_t)(b0 + u) * n + e] : 0.f;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (b0 + u < nparts) s2 += v[u];
  }
  out[e] = s2;
}

nnc_status launch_sum_parts(const float *part, int nparts, int64_t n, float *out, hipStream_t s) {
  hipLaunchKernelGGL(sum_parts_k, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, nparts, n, out);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

// =====================================================================================
// Core-space step, one workgroup.  The core and its temporaries live in LDS when they fit
// (lds != 0), else in global scratch; every phase ends with a barrier (and a device-scope
// fence when global scratch carries data between phases).
//   1. Gram S_k = A_k^T A_k for k in [gram_from, gram_to), the factor staged in LDS
//   2. if do_core: num_G = sum of the row-block partials, den_G = G x_0 S_0 ... x_{d-1} S_{d-1},
//      G <- G * num_G / max(den_G, eps)
//   3. M = unfold_next(G x_{k != next} S_k) unfold_next(G)^T       (R_next x R_next)
// =====================================================================================
struct CoreArgs {
  int d;
  int R[kMaxDim];
  int N[kMaxDim];
  const float *A[kMaxDim];
  float *S[kMaxDim];
  float *G;
  float *M;
  const float *gpart;
  int nparts;
  const float *gram;
  int gram_parts;
  int64_t gram_stride;
  float *t0, *t1, *numG;
  double eps;
  unsigned long long *clips;
  int gram_from, gram_to, do_core, next;
  int lds;
  int gsize;
};

constexpr int kCoreThreads = 512;
constexpr int kCoreLdsMax = 8192;  // cores up to this many entries are kept in LDS

static __device__ inline void phase_sync(bool global) {
  if (global) __threadfence();
  __syncthreads();
}

// out = in x_k S (S symmetric R_k x R_k, stored with row stride RM and zero padding),
// core-shaped.  Thread t owns column group g = t % ng (4 output columns r) for (p, q) pairs
// t / ng, t / ng + kCoreThreads / ng, ...; it keeps its RM x 4 block of S in registers, so
// a task reads only its RM inputs (rows l >= R_k read row R_k - 1 again, which the zero rows
// of S cancel).
template <int RM>
static __device__ inline void core_ttm(const CoreArgs &a, const float *in, int k, const float *S,
                                       float *out) {
  int pre = 1, post = 1;
#pragma unroll
  for (int j = 0; j < kMaxDim; ++j) {
    if (j < k) pre *= a.R[j];
    if (j > k && j < a.d) post *= a.R[j];
  }
  const int Rk = a.R[k];
  const int ng = (Rk + 3) / 4;
  const int lanes = kCoreThreads / ng;  // threads per column group
  const int g = threadIdx.x % ng, t0 = threadIdx.x / ng;
  if (t0 >= lanes) return;
  float4 sb[RM];
#pragma unroll
  for (int l = 0; l < RM; ++l) sb[l] = reinterpret_cast<const float4 *>(S + l * RM)[g];
  // row offsets, the same for every task; kept opaque (readfirstlane) so that the compiler
  // does not fold them back into one multiply per load
  int off[RM];
#pragma unroll
  for (int l = 0; l < RM; ++l) off[l] = __builtin_amdgcn_readfirstlane((l < Rk ? l : Rk - 1) * post);
  const int npq = pre * post;
  for (int pq = t0; pq < npq; pq += lanes) {
    const int p = pq / post, q = pq - (pq / post) * post;
    const float *src = in + p * Rk * post + q;
    float x[RM];
#pragma unroll
    for (int l = 0; l < RM; ++l) x[l] = src[off[l]];
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int l = 0; l < RM; ++l) {
      acc.x = fmaf(sb[l].x, x[l], acc.x);
      acc.y = fmaf(sb[l].y, x[l], acc.y);
      acc.z = fmaf(sb[l].z, x[l], acc.z);
      acc.w = fmaf(sb[l].w, x[l], acc.w);
    }
    float *dst = out + p * Rk * post + q;
    const int r0 = 4 * g;
    dst[r0 * post] = acc.x;
    if (r0 + 1 < Rk) dst[(r0 + 1) * post] = acc.y;
    if (r0 + 2 < Rk) dst[(r0 + 2) * post] = acc.z;
    if (r0 + 3 < Rk) dst[(r0 + 3) * post] = acc.w;
  }
}

// LDS: the core and its two temporaries live in LDS (G | t0 | t1 | partial-sum scratch), so
// every access is an LDS access; otherwise they are global scratch (cores above 8192
// entries) and each phase ends with a device-scope fence.
template <int RM, bool LDS>
__global__ __launch_bounds__(kCoreThreads) void core_step_k(CoreArgs a) {
  extern __shared__ __attribute__((aligned(16))) float dyn[];
  __shared__ float part[kCoreThreads];
  __shared__ __attribute__((aligned(16))) float Sp[kMaxDim][32 * RM];
  const int tid = threadIdx.x;
  const int d = a.d;
  constexpr bool glb = !LDS;
  float *G = LDS ? dyn : a.G;
  float *t0 = LDS ? dyn + a.gsize : a.t0;
  float *t1 = LDS ? dyn + 2 * a.gsize : a.t1;
  // ---- every global read of the step is issued before the first is used (each serial
  // round of global loads costs microseconds here): the core (LDS form), the Grams padded
  // to RM columns, the core numerator (core update), and the first 32 Gram partials of
  // the entries this thread sums.
  constexpr int GU = (kCoreLdsMax + kCoreThreads - 1) / kCoreThreads;  // core values per thread
  constexpr int kPB = 32;                                              // partials per batch
  const int nsp = 32 * RM;
  // (every load reads a valid address, clamped where the index runs past the data, and is
  // masked only where the value is used: a select right after a load would make the
  // compiler wait for that load at once)
  float gv[LDS ? GU : 1], nv[LDS ? GU : 1];
  if (LDS) {
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const int e = tid + u * kCoreThreads;
      gv[u] = a.G[e < a.gsize ? e : a.gsize - 1];
    }
    if (a.do_core) {
#pragma unroll
      for (int u = 0; u < GU; ++u) {
        const int e = tid + u * kCoreThreads;
        nv[u] = a.numG[e < a.gsize ? e : a.gsize - 1];
      }
    }
  }
  constexpr int SU = (32 * RM + kCoreThreads - 1) / kCoreThreads;
  float sv[SU][kMaxDim];
#pragma unroll
  for (int u = 0; u < SU; ++u) {
    const int e = tid + u * kCoreThreads;
    const int l = e / RM, r = e - (e / RM) * RM;
#pragma unroll
    for (int k = 0; k < kMaxDim; ++k) {
      const bool ok = k < d && e < nsp && l < a.R[k] && r < a.R[k];
      sv[u][k] = a.S[k < d ? k : 0][ok ? l * a.R[k] + r : 0];
    }
  }
  // Gram partials: gram[b][R][R] holds the Gram of factor rows [8b, 8b+8) (see mu_rows_k /
  // gram_parts_k); entry e is summed over b in order, by one thread (R_k^2 > kCoreThreads:
  // entries tid, tid + kCoreThreads, ...) or by nch threads over contiguous ranges of b,
  // whose sums are then added in order.  The partials and this order are the same at the
  // start of a fit and within it, so a fit resumed from its outputs continues bit for bit.
  const int gk_mode = a.gram_from;  // one Gram per step (gram_to == gram_from + 1) here
  const bool has_gram = a.gram_to > a.gram_from;
  const int Rg = has_gram ? a.R[gk_mode] : 1;
  const int RRg = Rg * Rg;
  const int nch = RRg > kCoreThreads ? 1 : kCoreThreads / RRg;
  const int ge0 = RRg > kCoreThreads ? tid : tid % RRg, gch = RRg > kCoreThreads ? 0 : tid / RRg;
  const bool gact = has_gram && gch < nch && ge0 < RRg;
  const int gb0 = gact ? (int)((int64_t)a.gram_parts * gch / nch) : 0;
  const int gb1 = gact ? (int)((int64_t)a.gram_parts * (gch + 1) / nch) : 0;
  const float *gsrc = has_gram ? a.gram : a.G;  // a valid address even without a Gram
  float pv[kPB];
#pragma unroll
  for (int u = 0; u < kPB; ++u)
    pv[u] = gsrc[(gb0 + u < gb1) ? (int64_t)(gb0 + u) * RRg + ge0 : 0];
  // ---- the values above land in LDS
  if (LDS) {
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const int e = tid + u * kCoreThreads;
      if (e < a.gsize) G[e] = gv[u];
    }
  }
#pragma unroll
  for (int u = 0; u < SU; ++u) {
    const int e = tid + u * kCoreThreads;
    const int l = e / RM, r = e - (e / RM) * RM;
#pragma unroll
    for (int k = 0; k < kMaxDim; ++k)
      if (k < d && e < nsp) Sp[k][e] = (l < a.R[k] && r < a.R[k]) ? sv[u][k] : 0.f;
  }
  __syncthreads();  // the staged (old) Grams are in place before the new one overwrites its own
  // ---- 1. Gram of the factor updated before this step (gram_from; at most one per step)
  for (int k = a.gram_from; k < a.gram_to; ++k) {
    if (k != gk_mode) break;  // launch_core_step passes one mode at a time
    auto finish = [&](int e, float v) {
      Sp[k][(e / Rg) * RM + e % Rg] = v;
      a.S[k][e] = v;
    };
    float acc = 0.f;
#pragma unroll
    for (int u = 0; u < kPB; ++u)
      if (gb0 + u < gb1) acc += pv[u];
    for (int bb = gb0 + kPB; bb < gb1; bb += kPB) {
#pragma unroll
      for (int u = 0; u < kPB; ++u) pv[u] = (bb + u < gb1) ? a.gram[(int64_t)(bb + u) * RRg + ge0] : 0.f;
#pragma unroll
      for (int u = 0; u < kPB; ++u)
        if (bb + u < gb1) acc += pv[u];
    }
    if (RRg > kCoreThreads) {
      // one thread per entry; entries beyond the first kCoreThreads are summed here
      if (gact) finish(ge0, acc);
      for (int e = tid + kCoreThreads; e < RRg; e += kCoreThreads) {
        float a2 = 0.f;
        for (int bb = 0; bb < a.gram_parts; bb += kPB) {
#pragma unroll
          for (int u = 0; u < kPB; ++u) pv[u] = (bb + u < a.gram_parts) ? a.gram[(int64_t)(bb + u) * RRg + e] : 0.f;
#pragma unroll
          for (int u = 0; u < kPB; ++u)
            if (bb + u < a.gram_parts) a2 += pv[u];
        }
        finish(e, a2);
      }
    } else {
      part[tid] = gact ? acc : 0.f;
      __syncthreads();
      if (tid < RRg) {
        float s2 = 0.f;
        for (int c = 0; c < nch; ++c) s2 += part[c * RRg + tid];
        finish(tid, s2);
      }
    }
  }
  phase_sync(glb);
  // ---- 2. core update
  if (a.do_core) {
    const float *numG = a.numG;  // summed from the row-block partials by sum_parts_k
    const float *in = G;
    for (int k = 0; k < d; ++k) {
      float *o = (k % 2) ? t1 : t0;
      core_ttm<RM>(a, in, k, Sp[k], o);
      phase_sync(glb);
      in = o;
    }
    unsigned int nclip = 0;
    auto update = [&](int e, float num) {
      double dd = (double)in[e];
      if (dd < a.eps) {
        dd = a.eps;
        ++nclip;
      }
      const float g = (float)(((double)G[e] * (double)num) / dd);
      G[e] = g;
      if (LDS) a.G[e] = g;
    };
    if (LDS) {
#pragma unroll
      for (int u = 0; u < GU; ++u) {
        const int e = tid + u * kCoreThreads;
        if (e < a.gsize) update(e, nv[u]);
      }
    } else {
      for (int e = tid; e < a.gsize; e += kCoreThreads) update(e, numG[e]);
    }
    if (nclip) atomicAdd(a.clips, (unsigned long long)nclip);
    phase_sync(glb);
  }
  // ---- 3. M for the next mode
  if (a.next >= 0) {
    const int n = a.next;
    const float *in = G;
    int cnt = 0;
    for (int k = 0; k < d; ++k) {
      if (k == n) continue;
      float *o = (cnt % 2) ? t1 : t0;
      core_ttm<RM>(a, in, k, Sp[k], o);
      phase_sync(glb);
      in = o;
      ++cnt;
    }
    const float *H = in;
    float *freebuf = (H == t0) ? t1 : t0;  // the temporary not holding H
    int pre = 1, post = 1;
    for (int j = 0; j < n; ++j) pre *= a.R[j];
    for (int j = n + 1; j < d; ++j) post *= a.R[j];
    const int Rn = a.R[n];
    // M[x][y] = sum_{c=(p,q)} H[p][x][q] G[p][y][q]: thread (4x4 block, split) sums a
    // contiguous range of c for its block; the ranges are then added in order.  The partial
    // sums go to the free temporary (gsize floats; split is lowered to fit).
    const int nb4 = (Rn + 3) / 4;
    const int blocks4 = nb4 * nb4;
    const int C = pre * post;
    int split = kCoreThreads / blocks4;
    const int cap = a.gsize / (blocks4 * 16);
    if (split > cap) split = cap > 0 ? cap : 1;
    if (split > C) split = C;
    float *pm = (a.gsize >= split * blocks4 * 16) ? freebuf : (LDS ? dyn + 3 * a.gsize : a.numG);
    const int bi = tid % blocks4, sp = tid / blocks4;
    const int x0 = 4 * (bi / nb4), y0 = 4 * (bi % nb4);
    float m[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) m[i][j] = 0.f;
    if (sp < split) {
      int xs[4], ys[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        xs[i] = (x0 + i < Rn ? x0 + i : Rn - 1) * post;
        ys[i] = (y0 + i < Rn ? y0 + i : Rn - 1) * post;
      }
      const int c0 = (int)((int64_t)C * sp / split), c1 = (int)((int64_t)C * (sp + 1) / split);
      int q = c0 - (c0 / post) * post;
      int base = (c0 / post) * Rn * post + q;  // advanced in step with (p, q)
      const int jump = (Rn - 1) * post;
      for (int c = c0; c < c1; ++c) {
        float h[4], gg[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          h[i] = H[base + xs[i]];
          gg[i] = G[base + ys[i]];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) m[i][j] = fmaf(h[i], gg[j], m[i][j]);
        ++base;
        if (++q == post) {
          q = 0;
          base += jump;
        }
      }
    }
    if (pm != freebuf) __syncthreads();  // fallback scratch: wait until every thread is done
    if (sp < split) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) pm[((sp * blocks4 + bi) * 4 + i) * 4 + j] = m[i][j];
    }
    phase_sync(glb);
    for (int e = tid; e < Rn * Rn; e += kCoreThreads) {
      const int x = e / Rn, y = e % Rn;
      const int b4 = (x / 4) * nb4 + (y / 4), j = (x % 4) * 4 + (y % 4);
      float s2 = 0.f;
      for (int c = 0; c < split; ++c) s2 += pm[(c * blocks4 + b4) * 16 + j];
      a.M[e] = s2;
    }
  }
}

nnc_status launch_slice_step(const CoreArgsHost &h, hipStream_t s);

// The core step as a chain of grid-wide launches, for cores larger than one workgroup's LDS
// (every rank <= 32): the Gram summed from its row-block partials in order, the core update
// (den_G by small contractions with the Grams, the FP64 MU step) and M_next (the core with
// every other mode multiplied by its Gram, contracted with the core over all modes but
// next).  Each sum runs in a fixed order.
static nnc_status core_step_multi(const CoreArgsHost &h, hipStream_t s) {
  const int d = h.d;
  int64_t gs = 1;
  for (int k = 0; k < d; ++k) gs *= h.R[k];
  auto pre = [&](int k) {
    int64_t v = 1;
    for (int j = 0; j < k; ++j) v *= h.R[j];
    return v;
  };
  auto post = [&](int k) {
    int64_t v = 1;
    for (int j = k + 1; j < d; ++j) v *= h.R[j];
    return v;
  };
  for (int k = h.gram_from; k < h.gram_to; ++k)
    NNC_TRY(launch_sum_parts(h.gram, h.gram_parts, h.R[k] * h.R[k], h.S[k], s));
  if (h.do_core) {
    if (h.gpart && h.nparts > 0) NNC_TRY(launch_sum_parts(h.gpart, h.nparts, gs, h.numG, s));
    const float *in = h.G;
    for (int k = 0; k < d; ++k) {  // den_G = G x_0 S_0 ... x_{d-1} S_{d-1} (S_k symmetric)
      float *o = (k % 2) ? h.t1 : h.t0;
      NNC_TRY(launch_ttm_small(in, pre(k), h.R[k], post(k), h.S[k], h.R[k], 1, h.R[k], o, s));
      in = o;
    }
    NNC_TRY(launch_mu_elem(h.G, h.numG, in, gs, h.eps, h.clips, s));
  }
  if (h.next >= 0) {
    const float *in = h.G;
    int cnt = 0;
    for (int k = 0; k < d; ++k) {
      if (k == h.next) continue;
      float *o = (cnt % 2) ? h.t1 : h.t0;
      NNC_TRY(launch_ttm_small(in, pre(k), h.R[k], post(k), h.S[k], h.R[k], 1, h.R[k], o, s));
      in = o;
      ++cnt;
    }
    NNC_TRY(launch_contract_except(in, h.G, pre(h.next), h.R[h.next], h.R[h.next], post(h.next), h.M, s));
  }
  return NNC_OK;
}

nnc_status launch_core_step(const CoreArgsHost &h, hipStream_t s) {
  // small cores: the work spread over one workgroup per slice (core_kernels.hip), the core
  // numerator summed from h.gpart there too
  {
    const nnc_status st = launch_slice_step(h, s);
    if (st != NNC_EUNSUPPORTED) return st;
  }
  {
    int64_t gs = 1;
    int maxr = 1;
    for (int k = 0; k < h.d; ++k) {
      gs *= h.R[k];
      maxr = std::max(maxr, (int)h.R[k]);
    }
    // cores beyond one workgroup's LDS: grid-wide launches
    if (gs > kCoreLdsMax && maxr <= 32 && h.gram_to - h.gram_from <= 1 && h.t0 && h.t1) return core_step_multi(h, s);
  }
  if (h.do_core && h.gpart && h.nparts > 0) {
    int64_t gs = 1;
    for (int k = 0; k < h.d; ++k) gs *= h.R[k];
    NNC_TRY(launch_sum_parts(h.gpart, h.nparts, gs, h.numG, s));
  }
  CoreArgs a;
  memset(&a, 0, sizeof a);
  a.d = h.d;
  int64_t gsize = 1, ssum = 0;
  for (int k = 0; k < kMaxDim; ++k) {
    a.R[k] = k < h.d ? (int)h.R[k] : 1;
    a.N[k] = k < h.d ? (int)h.N[k] : 1;
    a.A[k] = k < h.d ? h.A[k] : nullptr;
    a.S[k] = k < h.d ? h.S[k] : nullptr;
  }
  for (int k = 0; k < h.d; ++k) {
    if (h.R[k] > 32) return fail(NNC_EUNSUPPORTED, "core_step: rank above 32");
    gsize *= h.R[k];
    ssum += h.R[k] * h.R[k];
  }
  if (gsize > (int64_t)1 << 28) return fail(NNC_EUNSUPPORTED, "core_step: core too large");
  a.gsize = (int)gsize;
  a.G = h.G;
  a.M = h.M;
  a.gpart = h.gpart;
  a.nparts = h.nparts;
  a.gram = h.gram;
  a.gram_parts = h.gram_parts;
  a.gram_stride = h.gram_stride;
  a.t0 = h.t0;
  a.t1 = h.t1;
  a.numG = h.numG;
  a.eps = h.eps;
  a.clips = h.clips;
  a.gram_from = h.gram_from;
  a.gram_to = h.gram_to;
  a.do_core = h.do_core;
  a.next = h.next;
  int maxr = 1;
  for (int k = 0; k < h.d; ++k) maxr = std::max(maxr, (int)h.R[k]);
  size_t lds = 0;
  if (gsize <= kCoreLdsMax) {
    a.lds = 1;
    lds = (size_t)(3 * gsize + 4 * kCoreThreads) * sizeof(float);
  }
#define NNC_CORE_LAUNCH2(RM, LDSV)                                                              \
  do {                                                                                          \
    static bool attr = false;                                                                   \
    if (!attr) {                                                                                \
      NNC_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(core_step_k<RM, LDSV>),        \
                                  hipFuncAttributeMaxDynamicSharedMemorySize,                   \
                                  (int)((3 * kCoreLdsMax + 4 * kCoreThreads) * sizeof(float)))); \
      attr = true;                                                                              \
    }                                                                                           \
    hipLaunchKernelGGL((core_step_k<RM, LDSV>), dim3(1), dim3(kCoreThreads), lds, s, a);        \
  } while (0)
#define NNC_CORE_LAUNCH(RM)            \
  do {                                 \
    if (a.lds)                         \
      NNC_CORE_LAUNCH2(RM, true);      \
    else                               \
      NNC_CORE_LAUNCH2(RM, false);     \
  } while (0)
  if (maxr <= 8)
    NNC_CORE_LAUNCH(8);
  else if (maxr <= 16)
    NNC_CORE_LAUNCH(16);
  else if (maxr <= 24)
    NNC_CORE_LAUNCH(24);
  else
    NNC_CORE_LAUNCH(32);
#undef NNC_CORE_LAUNCH
#undef NNC_CORE_LAUNCH2
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

}  // namespace nnc
