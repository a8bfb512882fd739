// The two X-streaming passes of a three-way sweep with the next small contraction done in
// the same launch, so neither pass-1 partial P = X x_2 A_2^T nor a separate contraction
// launch is needed (modes 0, 1, 2; X is N0 x N1 x N2, row-major):
//
//   pass1y_k : Y0[i0][r1][r2] = sum_i1 A1[i1][r1] sum_i2 X[i0][i1][i2] A2[i2][r2]
//              (the mode-0 numerator chain).  The last-mode contraction of a 16-row tile
//              lands in MFMA accumulators whose layout is already the B operand of a
//              v_mfma_f32_16x16x4_f32 over the tile's rows, so the second contraction runs
//              on the FP32 matrix cores straight from registers, with A1 entries read from
//              L2.  A block owns whole i0 slabs; its waves split a slab's tiles and add
//              their partial sums in wave order through LDS (fixed order, deterministic).
//   pass2y_k : T[r0][i1][i2] = sum_i0 A0[i0][r0] X[i0][i1][i2] (written, it feeds mode 2 and
//              the core) and Y1[r0][i1][r2] = sum_i2 T[r0][i1][i2] A2[i2][r2] (the mode-1
//              numerator chain).  The accumulators of a T tile are the A operand of the
//              FP32 MFMA over the tile's columns; the waves holding the tiles of one i1 row
//              add their partial sums in wave order through LDS.
//
// Each pass also runs a side job in the first blocks to finish their share of the stream:
// one row each of the next mode's R x R matrix M_n = unfold_n(G x_{k!=n} S_k) unfold_n(G)^T
// (and, for pass 2, the new Gram S_0 summed from the row-block partials of the mode-0
// update), so that the update of mode n needs no launch of its own for it.
//
// X is bfloat16 (v_mfma_f32_16x16x32_bf16 with FP32 accumulation, the factor applied as a
// bf16 hi + lo pair); FP32 X takes the general schedule, whose FP32 passes measured faster
// than these contractions added to them.  The contracted factor of the stream (<= 32
// columns, zero-padded to 16-column tiles) lives in LDS.  X is read with ordinary loads:
// at 512^3 they measured about 4 us per pass faster here than non-temporal ones (the
// plain pass kernels measured the other way round and keep non-temporal loads).
#include <map>
#include <mutex>

#include "nnc_internal.h"

namespace nnc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef float fl2 __attribute__((ext_vector_type(2)));

// two floats to a pair of bfloat16 (round to nearest even; v_cvt_pk_bf16_f32), the first
// in the low half
static __device__ inline uint32_t y_pk_bf16(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((fl2){a, b}, bf2));
}

static __device__ inline uint16_t y_f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
static __device__ inline float y_bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
static __device__ inline f4 y_mfma_bf16(u4 a, u4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b),
                                                c, 0, 0, 0);
}
static __device__ inline f4 y_mfma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int kYThreads = 512;
constexpr int kYWaves = kYThreads / 64;
constexpr int kYS = 33;                   // row stride of a wave's 32 x 32 partial sum in LDS
constexpr int kYPartBytes = 32 * kYS * 4;  // bytes of one such partial

// ------------------------------------------------------------------------------ side job
// Row a of M_n for a three-way core G (R0 x R1 x R2): with p < q the two other
// modes and G_a the R_p x R_q slice of G at i_n = a,
//   H_a = S_p G_a S_q,   M_n[a][b] = sum_{u,v} H_a[u][v] G_b[u][v]
// (the Grams are symmetric, so this is G x_p S_p x_q S_q restricted to the slice).  With
// SUMMED, the Gram of mode gmode is first summed from its row-block partials and the job of
// row 0 stores it.  issue() starts every global read the job needs, as wide coalesced loads;
// finish() consumes them:
//   - G goes to LDS in the mode-n unfolding Gn[b][u * R_q + v];
//   - the partials: entry groups of 4 (or single entries), each group's partials split into
//     nch contiguous chunks added in order, then the chunks added in order;
//   - G_a S_q and S_p (G_a S_q) on the FP32 matrix cores, operands zero-padded to 32 x 32
//     in LDS, one 16 x 16 output tile per wave (waves 0..3);
//   - the dot products: 16 lanes per b, lane l taking rows u = l and l + 16 (v in order),
//     then a fixed butterfly.
// LDS: side_lds_floats(R0 R1 R2) floats.
constexpr int kSidePB = 16;  // partial groups in flight per thread
constexpr int kSideG4 = 8;   // float4 of G per thread (cores up to 16384 entries)

__host__ __device__ constexpr int side_lds_floats(int gsize) { return 4 * 32 * kYS + 4 * kYThreads + gsize; }

template <bool SUMMED>
struct SideJob {
  float4 pv[SUMMED ? kSidePB : 1];
  float4 gq[kSideG4];
  float sv[2][2];
  int p, q, Rp, Rq, Rn, RPQ, gsize, RR, Rg, W, ngrp, nch, ch, grp, b0, b1, row;
  bool vec, pact;

  __device__ void issue(const Side3 &a, int ia) {
    const int tid = threadIdx.x;
    row = ia;
    const int n = a.n;
    p = n == 0 ? 1 : 0;
    q = n == 2 ? 1 : 2;
    Rp = a.R[p];
    Rq = a.R[q];
    Rn = a.R[n];
    RPQ = Rp * Rq;
    gsize = Rn * RPQ;
    Rg = SUMMED ? a.R[a.gmode] : 1;
    RR = Rg * Rg;
    vec = (RR & 3) == 0;
    W = vec ? 4 : 1;
    ngrp = RR / W;
    nch = SUMMED ? (ngrp >= kYThreads ? 1 : kYThreads / ngrp) : 1;
    const int P = SUMMED ? a.gram_parts : 0;
    ch = tid / ngrp;
    grp = tid - ch * ngrp;
    pact = SUMMED && ch < nch;
    b0 = pact ? (P * ch) / nch : 0;  // P * nch < 2^31
    b1 = pact ? (P * (ch + 1)) / nch : 0;
    if (SUMMED) {
#pragma unroll
      for (int u = 0; u < kSidePB; ++u) {
        const int bb = b0 + u < b1 ? b0 + u : (b1 > 0 ? b1 - 1 : 0);
        const float *src = a.gram_part + (int64_t)bb * RR + grp * W;
        pv[u] = vec ? *reinterpret_cast<const float4 *>(src) : make_float4(src[0], 0.f, 0.f, 0.f);
      }
    }
    // G as float4 (the last one may run past gsize: it is read from the start instead)
    const int g4 = (gsize + 3) >> 2;
#pragma unroll
    for (int u = 0; u < kSideG4; ++u) {
      const int e4 = tid + u * kYThreads;
      gq[u] = *reinterpret_cast<const float4 *>(a.G + (e4 < g4 && 4 * e4 + 4 <= gsize ? 4 * e4 : 0));
    }
#pragma unroll
    for (int which = 0; which < 2; ++which) {
      const int k = which ? q : p;
      const int Rk = a.R[k];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int e = tid + u * kYThreads;
        sv[which][u] = a.S[k][e < Rk * Rk ? e : 0];
      }
    }
  }

  // offset of core entry (i0, i1, i2) in the mode-n unfolding Gn[b][u * R_q + v]
  __device__ int gn_index(int n, int i0, int i1, int i2) const {
    const int b = n == 0 ? i0 : (n == 1 ? i1 : i2);
    const int u = n == 0 ? i1 : i0;
    const int v = n == 2 ? i1 : i2;
    return b * RPQ + u * Rq + v;
  }

  // Ends with every wave past a barrier.
  __device__ void finish(const Side3 &a, float *lds) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, li = lane & 15, lg = lane >> 4;
    float *Sp = lds, *Sq = Sp + 32 * kYS, *Ga = Sq + 32 * kYS, *T1 = Ga + 32 * kYS;
    float *red = T1 + 32 * kYS;  // chunk sums of the partials: up to kYThreads float4
    float *Gn = red + 4 * kYThreads;
    for (int e = tid; e < 4 * 32 * kYS; e += kYThreads) lds[e] = 0.f;  // zero padding
    // G into its mode-n unfolding: entry (i0, i1, i2) -> (b, u, v) = (i_n, i_p, i_q)
    const int R1 = a.R[1], R2 = a.R[2];
    const int g4 = (gsize + 3) >> 2;
    const float inv12 = 1.0f / (float)(R1 * R2), inv2 = 1.0f / (float)R2;
#pragma unroll
    for (int u = 0; u < kSideG4; ++u) {
      const int e4 = tid + u * kYThreads;
      if (e4 < g4) {
        const float gvv[4] = {gq[u].x, gq[u].y, gq[u].z, gq[u].w};
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const int e = 4 * e4 + w;
          if (e < gsize) {
            const int i0 = qdiv(e, inv12), r = e - i0 * R1 * R2;
            const int i1 = qdiv(r, inv2), i2 = r - i1 * R2;
            Gn[gn_index(a.n, i0, i1, i2)] = gvv[w];
          }
        }
      }
    }
    if (4 * g4 > gsize) {  // the tail past the last whole float4
      for (int e = 4 * (gsize >> 2) + tid; e < gsize; e += kYThreads) {
        const int i0 = qdiv(e, inv12), r = e - i0 * R1 * R2;
        const int i1 = qdiv(r, inv2), i2 = r - i1 * R2;
        Gn[gn_index(a.n, i0, i1, i2)] = a.G[e];
      }
    }
    __syncthreads();
    if (SUMMED && pact) {
      float4 s4 = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int u = 0; u < kSidePB; ++u)
        if (b0 + u < b1) {
          s4.x += pv[u].x;
          s4.y += pv[u].y;
          s4.z += pv[u].z;
          s4.w += pv[u].w;
        }
      for (int bb = b0 + kSidePB; bb < b1; ++bb) {  // chunks longer than kSidePB
        const float *src = a.gram_part + (int64_t)bb * RR + grp * W;
        const float4 v = vec ? *reinterpret_cast<const float4 *>(src) : make_float4(src[0], 0.f, 0.f, 0.f);
        s4.x += v.x;
        s4.y += v.y;
        s4.z += v.z;
        s4.w += v.w;
      }
      reinterpret_cast<float4 *>(red)[ch * ngrp + grp] = s4;
    }
#pragma unroll
    for (int which = 0; which < 2; ++which) {
      const int k = which ? q : p;
      if (SUMMED && k == a.gmode) continue;
      const int Rk = a.R[k];
      float *dst = which ? Sq : Sp;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int e = tid + u * kYThreads;
        if (e < Rk * Rk) dst[(e / Rk) * kYS + e % Rk] = sv[which][u];
      }
    }
    const int ia = row;
    for (int e = tid; e < RPQ; e += kYThreads) Ga[(e / Rq) * kYS + e % Rq] = Gn[ia * RPQ + e];
    __syncthreads();
    if (SUMMED) {  // chunks in order, into the LDS Gram of mode gmode
      float *dst = a.gmode == p ? Sp : Sq;
      for (int g = tid; g < ngrp; g += kYThreads) {
        float4 t4 = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int c = 0; c < nch; ++c) {
          const float4 v = reinterpret_cast<const float4 *>(red)[c * ngrp + g];
          t4.x += v.x;
          t4.y += v.y;
          t4.z += v.z;
          t4.w += v.w;
        }
        const float tv[4] = {t4.x, t4.y, t4.z, t4.w};
        for (int w = 0; w < W; ++w) {
          const int e = g * W + w;
          dst[(e / Rg) * kYS + e % Rg] = tv[w];
          if (row == 0) a.S_store[e] = tv[w];
        }
      }
      __syncthreads();
    }
    // C = L R on 32 x 32 zero-padded LDS operands; wave w < 4 forms output tile (w >> 1, w & 1).
    // flat: C is written as an R_p x R_q matrix without padding (C[u * R_q + v]).
    auto mm32 = [&](const float *L, const float *Rm, float *C, bool flat) {
      if (wave < 4) {
        const int mt = wave >> 1, nt = wave & 1;
        f4 c4 = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 8; ++ks)
          c4 = y_mfma_f32(L[(16 * mt + li) * kYS + 4 * ks + lg], Rm[(4 * ks + lg) * kYS + 16 * nt + li], c4);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int u = 16 * mt + 4 * lg + v, w = 16 * nt + li;
          if (!flat)
            C[u * kYS + w] = c4[v];
          else if (u < Rp && w < Rq)
            C[u * Rq + w] = c4[v];
        }
      }
      __syncthreads();
    };
    mm32(Ga, Sq, T1, false);  // T1 = G_a S_q
    mm32(Sp, T1, Ga, true);   // H = S_p T1, flat into Ga
    // M_n[a][b] = <H, G_b>: lane l16 of b's group adds c = l16, l16 + 16, ... (both flat)
    const int bq = tid >> 4, l16 = tid & 15;
    const int nk = (RPQ - l16 + 15) >> 4;
    const float *gb = Gn + (bq < Rn ? bq : 0) * RPQ + l16;
    const float *hb = Ga + l16;
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < 64; ++k)
      if (k < nk) acc = fmaf(hb[16 * k], gb[16 * k], acc);
    if (bq >= Rn) acc = 0.f;
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
    if (bq < Rn && l16 == 0) a.M[ia * Rn + bq] = acc;
    __syncthreads();
  }
};

// The side job runs after the block's share of the stream, in the first side.nrows blocks to
// finish it (a ticket counter): the blocks end their shares a few microseconds apart, and the
// side rows fill that spread instead of delaying the shares of fixed blocks.  Which block
// forms a row depends on timing, the row does not.  The block that takes the last ticket
// sets the counter back to zero.  Every wave calls it; the stream's LDS is free.
template <bool SUMMED>
static __device__ void side_after_stream(const Side3 &side, unsigned char *lds_b, int fbytes) {
  unsigned int *tk = reinterpret_cast<unsigned int *>(lds_b);
  if (threadIdx.x == 0) {
    const unsigned int t = atomicAdd(side.ticket, 1u);
    if (t == gridDim.x - 1) atomicExch(side.ticket, 0u);
    *tk = t;
  }
  __syncthreads();
  const int t = (int)*tk;
  if (t >= side.nrows) return;
  SideJob<SUMMED> sj;
  sj.issue(side, t);
  sj.finish(side, reinterpret_cast<float *>(lds_b + fbytes));
}

// ------------------------------------------------------------------------------ pass 1
// Rows m = i0 * N1 + i1 of X (K = N2 contiguous bf16 values each).  A tile is 16 rows (so
// N1 % 16 == 0 and a tile never straddles two slabs) and is read in pieces of 16 rows x CPR
// 16-byte chunks with row-contiguous loads, staged through the wave's LDS region and read
// back in the MFMA layout (the scheme of the row-contiguous last-mode pass).  Block b owns
// slabs i0 = b, b + grid, ...; wave w takes tiles w, w + 8, ... of each slab.  The pieces
// of a wave form one sequence across its slabs, with one piece in flight while the
// previous one is multiplied; A1 entries of a tile are loaded when the tile's first piece
// is, one tile ahead of their use (double buffer a1n -> a1c).
template <int RT, int CPR>
__global__ __launch_bounds__(kYThreads) __attribute__((amdgpu_waves_per_eu(CPR <= 16 ? 4 : 1))) void pass1y_k(const uint16_t *__restrict__ X, int N0, int N1, int K,
                                                      const float *__restrict__ F, int R2,
                                                      const float *__restrict__ A1, int R1,
                                                      float *__restrict__ Y0, Side3 side) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_b[];
  constexpr int KC = CPR * 8;  // k-values per piece (8 per 16-byte chunk)
  constexpr int LPI = CPR / 4;
  constexpr int RPI = 64 / CPR;
  constexpr int SS = CPR * 16 + 16;
  constexpr int RP = 16 * RT;
  constexpr int kFB = 32;
  constexpr int WSB = 16 * SS > kYPartBytes ? 16 * SS : kYPartBytes;
  const int Kp = (K + KC - 1) / KC * KC;
  const int KS = Kp + 8;
  // factor rows in LDS: the R2 columns of A2 and one zero row that the MFMA tiles' rows past
  // R2 read (RP rows when R2 fills the tiles)
  const int FR = RP < R2 + 1 ? RP : R2 + 1;
  uint16_t *hi = reinterpret_cast<uint16_t *>(lds_b);
  uint16_t *lo = hi + FR * KS;
  const int fbytes = 2 * FR * KS * 2;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lg = lane >> 4;
  unsigned char *stg = lds_b + fbytes + wave * WSB;
  const int kpt = Kp / KC;
  const int Ts = N1 >> 4;
  const int tw = wave < Ts ? (Ts - wave + 7) >> 3 : 0;
  const int nsl = (int)blockIdx.x < N0 ? (N0 - 1 - (int)blockIdx.x) / (int)gridDim.x + 1 : 0;
  const int pps = tw * kpt;
  const int np = nsl * pps;
  const int crow = lane / CPR, cch = lane % CPR;
  // first row of piece i's tile (pieces past the end repeat the last one; a wave without
  // pieces reads row 0)
  auto tile_row0 = [&](int i) -> int64_t {
    if (np == 0) return 0;
    const int ii = i < np ? i : np - 1;
    const int j = ii / pps, r = ii - j * pps, k = r / kpt;
    return ((int64_t)blockIdx.x + (int64_t)j * gridDim.x) * N1 + (int64_t)(wave + 8 * k) * 16;
  };
  auto piece_h = [&](int i) { return np == 0 ? 0 : (i < np ? i : np - 1) % kpt; };
  auto load_piece = [&](u4 (&b)[LPI], int i) {
    const int64_t row0 = tile_row0(i);
    const int k = piece_h(i) * KC + cch * 8;
    const int kc = k < K ? k : 0;
#pragma unroll
    for (int j = 0; j < LPI; ++j) {
      const int64_t row = row0 + j * RPI + crow;
      b[j] = *reinterpret_cast<const u4 *>(X + row * (int64_t)K + kc);
    }
  };
  auto store_piece = [&](const u4 (&b)[LPI]) {
#pragma unroll
    for (int j = 0; j < LPI; ++j) *reinterpret_cast<u4 *>(stg + (j * RPI + crow) * SS + cch * 16) = b[j];
  };
  // A1 rows of piece i's tile: a[mt][jj] = A1[i1 + 4 lg + jj][16 mt + li] (column clamped;
  // columns past R1 are zeroed where used)
  const int c1 = li < R1 ? li : R1 - 1, c2 = 16 + li < R1 ? 16 + li : R1 - 1;
  auto load_a1 = [&](float (&a)[2][4], int i) {
    const int i1 = (int)(tile_row0(i) % N1) + 4 * lg;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      a[0][jj] = A1[(int64_t)(i1 + jj) * R1 + c1];
      a[1][jj] = A1[(int64_t)(i1 + jj) * R1 + c2];
    }
  };
  f4 acc[RT];
  f4 yacc[2][RT];
  float a1n[2][4], a1c[2][4];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < RT; ++nt) yacc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
  auto compute_piece = [&](int i) {
    const int h = i % kpt;
    if (h == 0) {
#pragma unroll
      for (int nt = 0; nt < RT; ++nt) acc[nt] = f4{0.f, 0.f, 0.f, 0.f};
    }
    const unsigned char *srow = stg + li * SS + lg * 16;
#pragma unroll
    for (int st = 0; st < CPR / 4; ++st) {
      const u4 av = *reinterpret_cast<const u4 *>(srow + st * 64);
      const int kk = h * KC + st * 32;
#pragma unroll
      for (int nt = 0; nt < RT; ++nt) {
        const int off = min(nt * 16 + li, FR - 1) * KS + kk + 8 * lg;
        acc[nt] = y_mfma_bf16(av, *reinterpret_cast<const u4 *>(hi + off), acc[nt]);
        acc[nt] = y_mfma_bf16(av, *reinterpret_cast<const u4 *>(lo + off), acc[nt]);
      }
    }
    if (h == kpt - 1) {
      // the tile's P rows (lane: rows 4 lg + jj, column 16 nt + li) are the B operand of the
      // FP32 MFMA whose K slot lg stands for row 4 lg + jj; A = A1^T
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const float x0 = li < R1 ? a1c[0][jj] : 0.f;
        const float x1 = 16 + li < R1 ? a1c[1][jj] : 0.f;
#pragma unroll
        for (int nt = 0; nt < RT; ++nt) {
          yacc[0][nt] = y_mfma_f32(x0, acc[nt][jj], yacc[0][nt]);
          yacc[1][nt] = y_mfma_f32(x1, acc[nt][jj], yacc[1][nt]);
        }
      }
    }
  };
  // the waves' partial sums of slab j, added in wave order
  auto slab_end = [&](int j) {
    float *yw = reinterpret_cast<float *>(stg);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < RT; ++nt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) yw[(16 * mt + 4 * lg + v) * kYS + 16 * nt + li] = yacc[mt][nt][v];
        yacc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
      }
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x + (int64_t)j * gridDim.x;
    const int RR = R1 * R2;
    for (int e = threadIdx.x; e < RR; e += kYThreads) {
      const int r1 = e / R2, r2 = e - (e / R2) * R2;
      float sum = 0.f;
#pragma unroll
      for (int w = 0; w < kYWaves; ++w)
        sum += reinterpret_cast<const float *>(lds_b + fbytes + w * WSB)[r1 * kYS + r2];
      Y0[s * RR + e] = sum;
    }
    __syncthreads();
  };

  // ---- prologue: a first batch of factor loads, the first piece of X and its A1 rows, then
  // the factor's conversion into LDS
  constexpr int KSTR = kYThreads / RP;
  const int fr = threadIdx.x % RP, fk = threadIdx.x / RP;
  const int frc = fr < R2 ? fr : R2 - 1;
  auto fac_load = [&](int k) { return F[(int64_t)(k < K ? k : K - 1) * R2 + frc]; };
  auto fac_store = [&](int k, float x) {
    const float a = (k < K && fr < R2) ? x : 0.f;
    const int kk = k < Kp ? k : Kp;
    const uint16_t h = y_f2bf(a);
    if (fr < FR) {
      hi[fr * KS + kk] = h;
      lo[fr * KS + kk] = y_f2bf(a - y_bf2f(h));
    }
  };
  float fv[kFB];
#pragma unroll
  for (int u = 0; u < kFB; ++u) fv[u] = fac_load(fk + u * KSTR);
  __builtin_amdgcn_sched_barrier(0);
  u4 bb[LPI];
  load_a1(a1n, 0);
  load_piece(bb, 0);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int u = 0; u < kFB; ++u) fac_store(fk + u * KSTR, fv[u]);
  for (int k0 = kFB * KSTR; k0 < Kp; k0 += kFB * KSTR) {
#pragma unroll
    for (int u = 0; u < kFB; ++u) fv[u] = fac_load(k0 + fk + u * KSTR);
#pragma unroll
    for (int u = 0; u < kFB; ++u) fac_store(k0 + fk + u * KSTR, fv[u]);
  }
  __syncthreads();
  int i = 0;
  for (int j = 0; j < nsl; ++j) {
    for (int r = 0; r < pps; ++r, ++i) {
      store_piece(bb);
      const int il = i + 1;
      if (il % kpt == 0) {
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) a1c[mt][jj] = a1n[mt][jj];
        load_a1(a1n, il);
      }
      load_piece(bb, il);
      __builtin_amdgcn_sched_barrier(0);
      compute_piece(i);
    }
    slab_end(j);
  }
  __syncthreads();
  side_after_stream<false>(side, lds_b, 16);  // the stream's LDS, factor included, is free
}

// ------------------------------------------------------------------------------ pass 2
// X (bf16) as [N][Q] with N = N0 contracted and Q = N1 * N2; tiles of 128 consecutive q
// (N2 % 128 == 0, so a tile lies in one i1 row).  The tile schedule and operand forms are
// those of the earlier-mode pass: a wave walks n in steps of 32 rows with one step of loads
// in flight.  The Tg = N2 / 128 tiles of one i1 row form a group (Tg divides 8); a unit of 8
// consecutive tiles (8 / Tg groups) goes to one block, wave w taking tile w, and at the end
// of a unit the waves of each group add their partial sums in wave order.
template <int RT>
__global__ __launch_bounds__(kYThreads) void pass2y_k(const uint16_t *__restrict__ X, int N, int N1, int N2,
                                                      const float *__restrict__ F, int R,
                                                      const float *__restrict__ A2, int R2,
                                                      float *__restrict__ out, float *__restrict__ Y1,
                                                      Side3 side) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_b[];
  constexpr int RP = 16 * RT;
  constexpr int TQ = 128;
  const int64_t Q = (int64_t)N1 * N2;
  const int Np = (N + 31) & ~31;
  const int NS = Np + 8;
  const int fbytes = 2 * RP * NS * 2;
  // the wave's LDS region: the T tile's staging, the tile's A2 rows, the unit's partial sums
  const int WSB = 4 * max(max(R, R2) * TQ, kYPartBytes / 4);
  uint16_t *hi = reinterpret_cast<uint16_t *>(lds_b);
  uint16_t *lo = hi + RP * NS;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lg = lane >> 4;
  const int nsteps = Np >> 5;
  float *stg = reinterpret_cast<float *>(lds_b + fbytes + wave * WSB);
  const int Tg = N2 / TQ;
  const int ng = 8 / Tg;  // groups per unit
  const int64_t nunits = (int64_t)N1 / ng;
  const int64_t nub = (int64_t)blockIdx.x < nunits ? (nunits - 1 - blockIdx.x) / gridDim.x + 1 : 0;
  auto tile_of = [&](int64_t j) -> int64_t { return ((int64_t)blockIdx.x + j * gridDim.x) * 8 + wave; };
  u4 v[8];
  const uint16_t *xp = X;
  int nlim = 0;
  auto tile_base = [&](int64_t t) {
    xp = X + t * TQ + 8 * li;
    nlim = N - 1;
  };
  auto load = [&](int s) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int n = min(32 * s + 8 * lg + j, nlim);
      v[j] = *reinterpret_cast<const u4 *>(xp + (int64_t)n * Q);
    }
  };
  if (nub > 0) tile_base(tile_of(0));
  load(0);
  __builtin_amdgcn_sched_barrier(0);  // the X loads go out before the factor is staged
  {
    const int total = RP * Np;
    constexpr int kB = 8;
    for (int e0 = 0; e0 < total; e0 += kB * kYThreads) {
      float fv[kB];
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const int e = e0 + threadIdx.x + u * kYThreads;
        const int n = e / RP, r = e - (e / RP) * RP;
        const bool ok = e < total && n < N && r < R;
        fv[u] = F[(ok ? n : 0) * R + (ok ? r : 0)];
      }
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const int e = e0 + threadIdx.x + u * kYThreads;
        const int n = e / RP, r = e - (e / RP) * RP;
        const bool ok = e < total && n < N && r < R;
        const float a = ok ? fv[u] : 0.f;
        if (e < total) {
          const uint16_t h = y_f2bf(a);
          hi[r * NS + n] = h;
          lo[r * NS + n] = y_f2bf(a - y_bf2f(h));
        }
      }
    }
  }
  __syncthreads();
  const int cc0 = li < R2 ? li : 0, cc1 = 16 + li < R2 ? 16 + li : 0;
  const float m0 = li < R2 ? 1.f : 0.f, m1 = 16 + li < R2 ? 1.f : 0.f;
  for (int64_t j = 0; j < nub; ++j) {
    const int64_t t = tile_of(j);
    const int64_t q0 = t * TQ;
    f4 acc[8][RT];
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
      for (int nt = 0; nt < RT; ++nt) acc[c][nt] = f4{0.f, 0.f, 0.f, 0.f};
    // the tile's A2 rows [i20, i20 + 128) (contiguous, 128 R2 floats) go to the wave's LDS
    // region in chunks of 512 floats, chunk c loaded in step c and stored in step c + 1
    const int64_t a2base = (q0 % N2) * R2;
    const int nfa = TQ * R2, nca = (nfa + 511) >> 9;
    f4 av[2];
    auto a2_load = [&](int c) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int e = 512 * c + 8 * lane + 4 * h;
        av[h] = *reinterpret_cast<const f4 *>(A2 + a2base + (e + 4 <= nfa ? e : nfa - 4));
      }
    };
    auto a2_store = [&](int c) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int e = 512 * c + 8 * lane + 4 * h;
        if (e + 4 <= nfa) *reinterpret_cast<f4 *>(stg + e) = av[h];
      }
    };
    for (int s = 0; s < nsteps; ++s) {
      if (s >= 1 && s - 1 < nca) a2_store(s - 1);
      u4 bh[RT], bl[RT];
#pragma unroll
      for (int nt = 0; nt < RT; ++nt) {
        const int off = (nt * 16 + li) * NS + s * 32 + 8 * lg;
        bh[nt] = *reinterpret_cast<const u4 *>(hi + off);
        bl[nt] = *reinterpret_cast<const u4 *>(lo + off);
      }
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        u4 op;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const uint32_t a = v[2 * w][c >> 1], b = v[2 * w + 1][c >> 1];
          op[w] = (c & 1) ? ((a >> 16) | (b & 0xffff0000u)) : ((a & 0xffffu) | (b << 16));
        }
#pragma unroll
        for (int nt = 0; nt < RT; ++nt) {
          acc[c][nt] = y_mfma_bf16(op, bh[nt], acc[c][nt]);
          acc[c][nt] = y_mfma_bf16(op, bl[nt], acc[c][nt]);
        }
      }
      if (s < nca) a2_load(s);
      load(s + 1);
      __builtin_amdgcn_sched_barrier(0);  // the refill stays ahead of the next step
    }
    // chunks the steps did not cover (short contracted modes)
    if (nsteps - 1 < nca) a2_store(nsteps - 1);
    for (int c = nsteps; c < nca; ++c) {
      a2_load(c);
      a2_store(c);
    }
    __builtin_amdgcn_wave_barrier();  // the wave reads back only what it wrote
    // the next tile's first step goes out before this tile's products and output
    if (j + 1 < nub)
      tile_base(tile_of(j + 1));
    else
      nlim = 0;
    load(0);
    __builtin_amdgcn_sched_barrier(0);
    // Y partial on bf16 MFMAs with hi + lo splits of both operands (hi*hi + hi*lo + lo*hi):
    // A = the T accumulators (K slot lg stands for the tile's columns 32 lg + 8 jj + c),
    // B = the staged A2 rows
    f4 yacc[RT][2];
#pragma unroll
    for (int nt = 0; nt < RT; ++nt) yacc[nt][0] = yacc[nt][1] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      u4 ah[RT], al[RT];
#pragma unroll
      for (int nt = 0; nt < RT; ++nt) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const float x0 = acc[2 * w][nt][jj], x1 = acc[2 * w + 1][nt][jj];
          const uint32_t h2 = y_pk_bf16(x0, x1);
          ah[nt][w] = h2;
          al[nt][w] = y_pk_bf16(x0 - y_bf2f((uint16_t)(h2 & 0xffffu)), x1 - y_bf2f((uint16_t)(h2 >> 16)));
        }
      }
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        const int col = mt ? cc1 : cc0;
        const float msk = mt ? m1 : m0;
        u4 bh2, bl2;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const float b0 = msk * stg[(32 * lg + 8 * jj + 2 * w) * R2 + col];
          const float b1 = msk * stg[(32 * lg + 8 * jj + 2 * w + 1) * R2 + col];
          const uint32_t h2 = y_pk_bf16(b0, b1);
          bh2[w] = h2;
          bl2[w] = y_pk_bf16(b0 - y_bf2f((uint16_t)(h2 & 0xffffu)), b1 - y_bf2f((uint16_t)(h2 >> 16)));
        }
#pragma unroll
        for (int nt = 0; nt < RT; ++nt) {
          yacc[nt][mt] = y_mfma_bf16(ah[nt], bh2, yacc[nt][mt]);
          yacc[nt][mt] = y_mfma_bf16(ah[nt], bl2, yacc[nt][mt]);
          yacc[nt][mt] = y_mfma_bf16(al[nt], bh2, yacc[nt][mt]);
        }
      }
    }
    __builtin_amdgcn_wave_barrier();  // the A2 rows are read before the T tile overwrites them
    // T tile: through the wave's LDS region, whole rows per store instruction (ordinary
    // stores: the launch after this one reads T back)
#pragma unroll
    for (int nt = 0; nt < RT; ++nt) {
      const int r = nt * 16 + li;
      if (r < R) {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int qq = 32 * lg + 8 * jj;
          *reinterpret_cast<f4 *>(stg + r * 128 + qq) =
              f4{acc[0][nt][jj], acc[1][nt][jj], acc[2][nt][jj], acc[3][nt][jj]};
          *reinterpret_cast<f4 *>(stg + r * 128 + qq + 4) =
              f4{acc[4][nt][jj], acc[5][nt][jj], acc[6][nt][jj], acc[7][nt][jj]};
        }
      }
    }
    __builtin_amdgcn_wave_barrier();  // the wave reads back only what it wrote
    for (int rr = 0; rr < R; rr += 2) {
      const int r = rr + (lane >> 5);
      const int qq = (lane & 31) * 4;
      if (r < R)
        *reinterpret_cast<f4 *>(out + (int64_t)r * Q + q0 + qq) = *reinterpret_cast<const f4 *>(stg + r * 128 + qq);
    }
    __builtin_amdgcn_wave_barrier();
    // unit end: partial sums of each group (waves g Tg .. g Tg + Tg - 1, in order) into
    // Y1[r0][i1][r2]
#pragma unroll
    for (int nt = 0; nt < RT; ++nt)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) stg[(16 * nt + 4 * lg + vv) * kYS + 16 * mt + li] = yacc[nt][mt][vv];
    __syncthreads();
    const int64_t u = (int64_t)blockIdx.x + j * gridDim.x;
    const int RR = R * R2;
    for (int e = threadIdx.x; e < ng * RR; e += kYThreads) {
      const int g = e / RR, rem = e - g * RR;
      const int r0 = rem / R2, r2 = rem - (rem / R2) * R2;
      float sum = 0.f;
      for (int w = g * Tg; w < (g + 1) * Tg; ++w)
        sum += reinterpret_cast<const float *>(lds_b + fbytes + w * WSB)[r0 * kYS + r2];
      const int64_t i1 = u * ng + g;
      Y1[((int64_t)r0 * N1 + i1) * R2 + r2] = sum;
    }
    __syncthreads();
  }
  __syncthreads();
  side_after_stream<true>(side, lds_b, fbytes);
}

// ------------------------------------------------------------------------------ launchers
static nnc_status allow_y_lds(const void *kern, size_t bytes) {
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

constexpr size_t kYCuLds = 160 * 1024;

static int pass1y_cpr(int64_t K) { return K >= 256 ? 32 : (K >= 128 ? 16 : 8); }

static size_t pass1y_lds(int RT, int CPR, int64_t K, int64_t R2, int64_t gsize) {
  const int64_t KC = CPR * 8;
  const int64_t Kp = (K + KC - 1) / KC * KC;
  const int64_t FR = std::min<int64_t>(16 * RT, R2 + 1);
  const int64_t fbytes = 2 * FR * (Kp + 8) * 2;
  const int64_t wsb = std::max<int64_t>(16 * (CPR * 16 + 16), kYPartBytes);
  // the side job runs after the stream, over the stream's LDS (from byte 16)
  return (size_t)std::max<int64_t>(fbytes + kYWaves * wsb, 16 + 4 * (int64_t)side_lds_floats((int)gsize));
}

// Pass 1's piece width and blocks per CU: pieces of 16 chunks (127 VGPRs) and two blocks per
// CU when two blocks' LDS fits a CU, else pieces by K and one block per CU.
static void pass1y_config(int RT, int64_t K, int64_t R2, int64_t gsize, int *cpr, int *per_cu) {
  if (K >= 128 && 2 * pass1y_lds(RT, 16, K, R2, gsize) <= kYCuLds) {
    *cpr = 16;
    *per_cu = 2;
  } else {
    *cpr = pass1y_cpr(K);
    *per_cu = 1;
  }
}

static size_t pass2y_lds(int RT, int64_t N, int64_t R, int64_t R2, int64_t gsize) {
  const int64_t Np = (N + 31) / 32 * 32;
  const int64_t fbytes = 2 * 16 * RT * (Np + 8) * 2;
  const int64_t wsb = 4 * std::max<int64_t>(std::max(R, R2) * 128, kYPartBytes / 4);
  return (size_t)(fbytes + std::max<int64_t>(kYWaves * wsb, 4 * (int64_t)side_lds_floats((int)gsize)));
}

bool pass1y_ok(nnc_dtype dt, int64_t N0, int64_t N1, int64_t N2, int64_t R0, int64_t R1, int64_t R2) {
  if (dt != NNC_BF16) return false;
  if (R0 < 1 || R0 > 32 || R1 < 1 || R1 > 32 || R2 < 1 || R2 > 32) return false;
  if (R0 * R1 * R2 > kSideG4 * kYThreads * 4) return false;
  if (N1 % 16 || N2 % 8 || N2 < 64 || N2 > (1 << 20)) return false;
  if (N0 * N1 >= ((int64_t)1 << 31) || N0 * R1 * R2 >= ((int64_t)1 << 31)) return false;
  int cpr, per_cu;
  pass1y_config(R2 <= 16 ? 1 : 2, N2, R2, R0 * R1 * R2, &cpr, &per_cu);
  return pass1y_lds(R2 <= 16 ? 1 : 2, cpr, N2, R2, R0 * R1 * R2) <= kYCuLds;
}

bool pass2y_ok(nnc_dtype dt, int64_t N0, int64_t N1, int64_t N2, int64_t R0, int64_t R1, int64_t R2) {
  if (dt != NNC_BF16) return false;
  if (R0 < 1 || R0 > 32 || R1 < 1 || R1 > 32 || R2 < 1 || R2 > 32) return false;
  if (R0 * R1 * R2 > kSideG4 * kYThreads * 4) return false;
  if (N2 % 128 || N0 > (1 << 20) || N0 * R0 >= ((int64_t)1 << 31)) return false;
  const int64_t Tg = N2 / 128;
  if (Tg > 8 || 8 % Tg || N1 % (8 / Tg)) return false;
  if (N1 * N2 >= ((int64_t)1 << 40)) return false;
  return pass2y_lds(R0 <= 16 ? 1 : 2, N0, R0, R2, R0 * R1 * R2) <= kYCuLds;
}

nnc_status launch_pass1y(const void *X, nnc_dtype dt, int64_t N0, int64_t N1, int64_t N2, const float *A2,
                         int64_t R2, const float *A1, int64_t R1, float *Y0, const Side3 &side, hipStream_t s) {
  if (!pass1y_ok(dt, N0, N1, N2, side.R[0], R1, R2) || side.R[1] != R1 || side.R[2] != R2 ||
      (reinterpret_cast<uintptr_t>(X) & 15u) || (side.nrows > 0 && (reinterpret_cast<uintptr_t>(side.G) & 15u)))
    return fail(NNC_EUNSUPPORTED, "pass1y: unsupported shape");
  if (side.nrows > 0 && side.gram_part) return fail(NNC_EINVAL, "pass1y: its side job sums no partials");
  if (side.nrows > 0 && !side.ticket) return fail(NNC_EINVAL, "pass1y: the side job needs its ticket counter");
  const int RT = R2 <= 16 ? 1 : 2;
  int CPR, per_cu;
  pass1y_config(RT, N2, R2, (int64_t)side.R[0] * R1 * R2, &CPR, &per_cu);
  const size_t lds = pass1y_lds(RT, CPR, N2, R2, (int64_t)side.R[0] * R1 * R2);
  const int grid = (int)std::max<int64_t>(std::min<int64_t>(N0, (int64_t)per_cu * device_cu_count()), side.nrows);
  const uint16_t *Xb = (const uint16_t *)X;
#define NNC_P1(RTV, CPRV)                                                                         \
  do {                                                                                            \
    NNC_TRY(allow_y_lds(reinterpret_cast<const void *>(pass1y_k<RTV, CPRV>), lds));               \
    hipLaunchKernelGGL((pass1y_k<RTV, CPRV>), dim3(grid), dim3(kYThreads), lds, s, Xb, (int)N0,   \
                       (int)N1, (int)N2, A2, (int)R2, A1, (int)R1, Y0, side);                    \
  } while (0)
#define NNC_P1C(RTV)        \
  do {                      \
    if (CPR == 32)          \
      NNC_P1(RTV, 32);      \
    else if (CPR == 16)     \
      NNC_P1(RTV, 16);      \
    else                    \
      NNC_P1(RTV, 8);       \
  } while (0)
  if (RT == 1)
    NNC_P1C(1);
  else
    NNC_P1C(2);
#undef NNC_P1C
#undef NNC_P1
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

nnc_status launch_pass2y(const void *X, nnc_dtype dt, int64_t N0, int64_t N1, int64_t N2, const float *A0,
                         int64_t R0, const float *A2, int64_t R2, float *T, float *Y1, const Side3 &side,
                         hipStream_t s) {
  if (!pass2y_ok(dt, N0, N1, N2, R0, side.R[1], R2) || side.R[0] != R0 || side.R[2] != R2 ||
      (reinterpret_cast<uintptr_t>(X) & 15u) || (reinterpret_cast<uintptr_t>(T) & 15u) ||
      (reinterpret_cast<uintptr_t>(A2) & 15u) || (side.nrows > 0 && (reinterpret_cast<uintptr_t>(side.G) & 15u)))
    return fail(NNC_EUNSUPPORTED, "pass2y: unsupported shape");
  if (side.nrows > 0 && !side.gram_part) return fail(NNC_EINVAL, "pass2y: its side job sums partials");
  if (side.nrows > 0 && !side.ticket) return fail(NNC_EINVAL, "pass2y: the side job needs its ticket counter");
  const int RT = R0 <= 16 ? 1 : 2;
  const size_t lds = pass2y_lds(RT, N0, R0, R2, (int64_t)R0 * side.R[1] * R2);
  const int64_t units = N1 / (8 / (N2 / 128));
  const int grid = (int)std::max<int64_t>(std::min<int64_t>(units, device_cu_count()), side.nrows);
  const uint16_t *Xb = (const uint16_t *)X;
#define NNC_P2(RTV)                                                                               \
  do {                                                                                            \
    NNC_TRY(allow_y_lds(reinterpret_cast<const void *>(pass2y_k<RTV>), lds));                     \
    hipLaunchKernelGGL((pass2y_k<RTV>), dim3(grid), dim3(kYThreads), lds, s, Xb, (int)N0, (int)N1, \
                       (int)N2, A0, (int)R0, A2, (int)R2, T, Y1, side);                           \
  } while (0)
  if (RT == 1)
    NNC_P2(1);
  else
    NNC_P2(2);
#undef NNC_P2
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

}  // namespace nnc
