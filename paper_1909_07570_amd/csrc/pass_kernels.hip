// The X-streaming contractions of a sweep (the two passes over X), software-pipelined:
// every wave keeps the loads of its next work unit in flight while the MFMAs consume the
// current one.
//
//   ttm_last_lds_k     : out[m][r] = sum_k X[m][k] F(k, r)   (contraction index contiguous)
//   ttm_last_pipe_k    : the same, for rows too short for ttm_last_lds_k's pieces
//   ttm_mid_lds_k      : out[p][r][q] = sum_n F(n, r) X[p][n][q]  (contraction index strided, bf16)
//   ttm_mid_lds_f32_k  : the same for FP32 X
// X is FP32 (v_mfma_f32_16x16x4_f32) or bfloat16 (v_mfma_f32_16x16x32_bf16, FP32
// accumulation, factor applied as bf16 hi + lo parts).  The factor (R <= 32 columns,
// zero-padded to 16-column tiles) lives in LDS.
#include <map>
#include <mutex>

#include "nnc_internal.h"

namespace nnc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

static __device__ inline uint16_t p_f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
static __device__ inline float p_bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
static __device__ inline f4 p_mfma_bf16(u4 a, u4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b),
                                                c, 0, 0, 0);
}
static __device__ inline f4 p_mfma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int kPassThreads = 256;
constexpr int kUnitChunks = 16;  // 16-byte loads per lane per work unit

// =====================================================================================
// Last-mode contraction.  A work unit is 16 rows x KU k-values: lane (li = lane%16,
// lg = lane/16) loads, for each of 16 chunks c, the 16 bytes X[row li][kb*KU + c*KPC + EPC*lg ..]
// (EPC elements; KPC = 4*EPC k-values per chunk across the four lane groups).
//   bf16: the 8 elements are the lane's MFMA A operand (k-slots 8 lg .. 8 lg + 7), paired
//         with 8 consecutive k of the factor's transposed bf16 rows in LDS.
//   f32 : element e of the chunk feeds the MFMA whose k-slot lg stands for k = .. + 4 lg + e.
// Output tile: lane holds rows 4 lg + j, column li of each 16-column tile.
// =====================================================================================
template <bool BF, int RT>
__global__ __launch_bounds__(kPassThreads) void ttm_last_pipe_k(const void *__restrict__ Xv, int64_t M,
                                                                int K, const float *__restrict__ F,
                                                                int64_t ldl, int64_t ldr, int R,
                                                                float *__restrict__ out) {
  extern __shared__ __attribute__((aligned(16))) uint16_t lds_u16[];
  constexpr int EPC = BF ? 8 : 4;
  constexpr int KPC = 4 * EPC;
  constexpr int KU = kUnitChunks * KPC;
  constexpr int RP = 16 * RT;
  const int Kp = (K + KPC - 1) / KPC * KPC;
  // ---- factor staging
  const int KS = Kp + 8;    // bf16: [RP][KS] hi then lo
  const int RS = RP + 4;    // f32: [Kp][RS]
  uint16_t *hi = lds_u16;
  uint16_t *lo = lds_u16 + RP * KS;
  float *fl = reinterpret_cast<float *>(lds_u16);
  if (BF) {
    for (int e = threadIdx.x; e < RP * Kp; e += blockDim.x) {
      const int r = e / Kp, k = e - r * Kp;
      const float a = (k < K && r < R) ? F[k * ldl + r * ldr] : 0.f;
      const uint16_t h = p_f2bf(a);
      hi[r * KS + k] = h;
      lo[r * KS + k] = p_f2bf(a - p_bf2f(h));
    }
  } else {
    for (int e = threadIdx.x; e < Kp * RP; e += blockDim.x) {
      const int k = e / RP, r = e - k * RP;
      fl[k * RS + r] = (k < K && r < R) ? F[k * ldl + r * ldr] : 0.f;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int nw = blockDim.x >> 6;
  const int64_t ntile = (M + 15) >> 4;
  const int upt = (Kp + KU - 1) / KU;  // units per tile
  const int64_t tstride = (int64_t)gridDim.x * nw;

  auto load_unit = [&](u4 (&buf)[kUnitChunks], int64_t t, int kb) {
    const int64_t row = t * 16 + li;
    const bool rv = row < M;
    const char *xr = reinterpret_cast<const char *>(Xv) + (rv ? row : 0) * (int64_t)K * (BF ? 2 : 4);
#pragma unroll
    for (int c = 0; c < kUnitChunks; ++c) {
      const int k = kb * KU + c * KPC + EPC * lg;
      buf[c] = (rv && k < K) ? *reinterpret_cast<const u4 *>(xr + (int64_t)k * (BF ? 2 : 4))
                             : u4{0u, 0u, 0u, 0u};
    }
  };
  f4 acc[RT];
  auto compute_unit = [&](const u4 (&buf)[kUnitChunks], int64_t t, int kb) {
    if (kb == 0) {
#pragma unroll
      for (int nt = 0; nt < RT; ++nt) acc[nt] = f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int c = 0; c < kUnitChunks; ++c) {
      const int kc = kb * KU + c * KPC;
      if (kc >= Kp) break;  // uniform
      if (BF) {
        const int kk = kc + 8 * lg;
#pragma unroll
        for (int nt = 0; nt < RT; ++nt) {
          const int off = (nt * 16 + li) * KS + kk;
          acc[nt] = p_mfma_bf16(buf[c], *reinterpret_cast<const u4 *>(hi + off), acc[nt]);
          acc[nt] = p_mfma_bf16(buf[c], *reinterpret_cast<const u4 *>(lo + off), acc[nt]);
        }
      } else {
        const int kk = kc + 4 * lg;
        const f4 xv = __builtin_bit_cast(f4, buf[c]);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float *brow = fl + (kk + e) * RS + li;
#pragma unroll
          for (int nt = 0; nt < RT; ++nt) acc[nt] = p_mfma_f32(xv[e], brow[nt * 16], acc[nt]);
        }
      }
    }
    if (kb == upt - 1) {
#pragma unroll
      for (int nt = 0; nt < RT; ++nt) {
        const int r = nt * 16 + li;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t m = t * 16 + 4 * lg + j;
          if (m < M && r < R) out[m * R + r] = acc[nt][j];
        }
      }
    }
  };
  auto advance = [&](int64_t &t, int &kb) {
    if (++kb == upt) {
      kb = 0;
      t += tstride;
    }
  };

  u4 b0[kUnitChunks], b1[kUnitChunks];
  int64_t t = (int64_t)blockIdx.x * nw + wave;
  int kb = 0;
  if (t < ntile) load_unit(b0, t, kb);
  while (t < ntile) {
    int64_t tn = t;
    int kbn = kb;
    advance(tn, kbn);
    if (tn < ntile) load_unit(b1, tn, kbn);
    compute_unit(b0, t, kb);
    t = tn;
    kb = kbn;
    if (t >= ntile) break;
    tn = t;
    kbn = kb;
    advance(tn, kbn);
    if (tn < ntile) load_unit(b0, tn, kbn);
    compute_unit(b1, t, kb);
    t = tn;
    kb = kbn;
  }
}

// =====================================================================================
// Earlier-mode contraction, bf16 X: out[p][r][q] = sum_n F(n, r) X[p][n][q].
// A wave owns a Q-tile (p, q0 .. q0 + 128) and walks n in steps of 32 rows.  Lane (li, lg)
// loads the 16 bytes X[p][n][q0 + 8 li ..] of rows n = 32 s + 8 lg + j (j < 8) and
// transposes that 8 x 8 block in registers into eight A operands (operand c: the 8 n values
// of q = q0 + 8 i + c, i = li), so MFMA c's output row i stands for q0 + 8 i + c.  Each step
// refills its buffer for the step kMidDepth ahead right after its MFMAs, and every refill
// is issued on every path (rows past N and steps past the tile read the tile's last row,
// which is cached), so the waits are exact.  One step in flight per wave measured fastest
// (51.5 us against 53.6 with two and 55 with three at 512^3): with the HBM saturated, more
// outstanding loads only add queueing and concurrent DRAM row streams.  Every block issues
// its first tile's loads before it builds the factor's bf16 hi / lo rows in LDS, and a wave
// issues its next tile's loads before it writes the current tile's output, which goes
// through the wave's LDS region so that each store instruction covers two whole rows,
// written non-temporally (the output is read back only by the next kernel).
// =====================================================================================
constexpr int kMidWaves = 8;
constexpr int kMidDepth = 1;
constexpr int kMidDepthF32 = 1;  // steps in flight per wave, FP32 X (one measured fastest, as for bf16)

template <int RT, bool HS>
__global__ __launch_bounds__(64 * kMidWaves) __attribute__((amdgpu_waves_per_eu(RT == 1 ? 4 : 1))) void ttm_mid_lds_k(const uint16_t *__restrict__ X,
                                                               int64_t P, int N, int64_t Q,
                                                               const float *__restrict__ F,
                                                               int64_t ldl, int64_t ldr, int R,
                                                               float *__restrict__ out, int64_t ldp,
                                                               int acc_out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_b[];
  constexpr int RP = 16 * RT;
  const int Np = (N + 31) & ~31;
  const int NS = Np + 8;
  uint16_t *hi = reinterpret_cast<uint16_t *>(lds_b);
  uint16_t *lo = hi + RP * NS;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lg = lane >> 4;
  const int64_t qt = (Q + 127) >> 7;
  const int64_t ntile = P * qt;
  const int nsteps = Np >> 5;
  float *stg = reinterpret_cast<float *>(lds_b + 2 * RP * NS * 2) + wave * (R * (HS ? 64 : 128));
  u4 v[kMidDepth][8];
  const uint16_t *xp = X;  // lane's column of the current tile
  int nlim = 0;            // last row a load may touch (0: one line, for loads past the work)
  auto tile_base = [&](int64_t t) {
    const int64_t p = t / qt;
    const int64_t q0 = (t - p * qt) * 128;
    const int64_t qa = q0 + 8 * li;
    xp = X + p * ldp + (qa < Q ? qa : Q - 8);
    nlim = N - 1;
  };
  auto load = [&](u4 (&vv)[8], int s) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int n = min(32 * s + 8 * lg + j, nlim);
      vv[j] = __builtin_nontemporal_load(reinterpret_cast<const u4 *>(xp + (int64_t)n * Q));
    }
  };
  int64_t t = (int64_t)blockIdx.x * kMidWaves + wave;
  const int64_t tstride = (int64_t)gridDim.x * kMidWaves;
  if (t < ntile) tile_base(t);
#pragma unroll
  for (int b = 0; b < kMidDepth; ++b) load(v[b], b);
  __builtin_amdgcn_sched_barrier(0);  // the X loads go out before the factor is staged
  {
    const int total = RP * Np;
    constexpr int kB = 8;
    for (int e0 = 0; e0 < total; e0 += kB * 64 * kMidWaves) {
      float fv[kB];
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const int e = e0 + threadIdx.x + u * 64 * kMidWaves;
        const int n = e / RP, r = e - (e / RP) * RP;
        const bool ok = e < total && n < N && r < R;
        fv[u] = F[(ok ? n : 0) * (int)ldl + (ok ? r : 0) * (int)ldr];  // the factor has < 2^31 entries
      }
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const int e = e0 + threadIdx.x + u * 64 * kMidWaves;
        const int n = e / RP, r = e - (e / RP) * RP;
        const bool ok = e < total && n < N && r < R;
        const float a = ok ? fv[u] : 0.f;  // masked where the value is awaited
        const uint16_t h = p_f2bf(a);
        if (e < total) {
          hi[r * NS + n] = h;
          lo[r * NS + n] = p_f2bf(a - p_bf2f(h));
        }
      }
    }
  }
  __syncthreads();
  for (; t < ntile; t += tstride) {
    const int64_t p = t / qt;
    const int64_t q0 = (t - p * qt) * 128;
    f4 acc[8][RT];
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
      for (int nt = 0; nt < RT; ++nt) acc[c][nt] = f4{0.f, 0.f, 0.f, 0.f};
    auto step = [&](u4 (&vv)[8], int s) {
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
          const uint32_t a = vv[2 * w][c >> 1], b = vv[2 * w + 1][c >> 1];
          op[w] = (c & 1) ? ((a >> 16) | (b & 0xffff0000u)) : ((a & 0xffffu) | (b << 16));
        }
#pragma unroll
        for (int nt = 0; nt < RT; ++nt) {
          acc[c][nt] = p_mfma_bf16(op, bh[nt], acc[c][nt]);
          acc[c][nt] = p_mfma_bf16(op, bl[nt], acc[c][nt]);
        }
      }
      load(vv, s + kMidDepth);
      __builtin_amdgcn_sched_barrier(0);  // the refill stays ahead of the next step
    };
    int s = 0;
    for (; s + kMidDepth <= nsteps; s += kMidDepth) {
#pragma unroll
      for (int b = 0; b < kMidDepth; ++b) step(v[b], s + b);
    }
#pragma unroll
    for (int b = 0; b < kMidDepth - 1; ++b)
      if (s + b < nsteps) step(v[b], s + b);
    // the next tile's first steps (or, after the last tile, one cached line) go out
    // before this tile's output is written
    const int64_t tn = t + tstride;
    if (tn < ntile)
      tile_base(tn);
    else
      nlim = 0;
#pragma unroll
    for (int b = 0; b < kMidDepth; ++b) load(v[b], b);
    __builtin_amdgcn_sched_barrier(0);
    if (!HS) {
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
        if (r < R && q0 + qq < Q) {
          f4 *o = reinterpret_cast<f4 *>(out + (p * R + r) * Q + q0 + qq);
          f4 val = *reinterpret_cast<const f4 *>(stg + r * 128 + qq);
          if (acc_out) {
            val += *o;  // a later chunk of the contracted index: added in chunk order
            *o = val;
          } else {
            __builtin_nontemporal_store(val, o);
          }
        }
      }
      __builtin_amdgcn_wave_barrier();
    } else {
      // half staging (large R): columns 64 h .. 64 h + 63 of the tile in turn; lanes with
      // lg >> 1 == h hold them (column 32 (lg & 1) + 8 jj + c of the half)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if ((lg >> 1) == h) {
#pragma unroll
          for (int nt = 0; nt < RT; ++nt) {
            const int r = nt * 16 + li;
            if (r < R) {
#pragma unroll
              for (int jj = 0; jj < 4; ++jj) {
                const int qq = 32 * (lg & 1) + 8 * jj;
                *reinterpret_cast<f4 *>(stg + r * 64 + qq) =
                    f4{acc[0][nt][jj], acc[1][nt][jj], acc[2][nt][jj], acc[3][nt][jj]};
                *reinterpret_cast<f4 *>(stg + r * 64 + qq + 4) =
                    f4{acc[4][nt][jj], acc[5][nt][jj], acc[6][nt][jj], acc[7][nt][jj]};
              }
            }
          }
        }
        __builtin_amdgcn_wave_barrier();  // the wave reads back only what it wrote
        for (int rr = 0; rr < R; rr += 4) {
          const int r = rr + (lane >> 4);
          const int qq = (lane & 15) * 4;
          const int64_t qc = q0 + 64 * h + qq;
          if (r < R && qc < Q) {
            f4 *o = reinterpret_cast<f4 *>(out + (p * R + r) * Q + qc);
            f4 val = *reinterpret_cast<const f4 *>(stg + r * 64 + qq);
            if (acc_out) {
              val += *o;
              *o = val;
            } else {
              __builtin_nontemporal_store(val, o);
            }
          }
        }
        __builtin_amdgcn_wave_barrier();  // the half is read before the next one overwrites it
      }
    }
  }
}

// =====================================================================================
// Earlier-mode contraction, FP32 X (v_mfma_f32_16x16x4_f32), same schedule as ttm_mid_lds_k.
// A wave owns a Q-tile of 64 columns.  Lane (li, lg) loads the 16 bytes X[p][n][q0 + 4 li ..]
// of rows n = 32 s + 8 lg + j (j < 8); for each j, component c of that float4 is the A
// operand of MFMA (j, c): its K index lg stands for row 32 s + 8 lg + j and its output row i
// for column q0 + 4 i + c.  The factor (FP32, [n][RS] in LDS) is the B operand.  Lane
// (li, lg) ends up holding, for output column r = 16 nt + li and i = 0..3, the four
// adjacent columns q0 + 16 lg + 4 i + (0..3) of each accumulator set c.
// =====================================================================================
template <int RT, int DEPTH>
__global__ __launch_bounds__(64 * kMidWaves) __attribute__((amdgpu_waves_per_eu(4))) void ttm_mid_lds_f32_k(const float *__restrict__ X,
                                                                   int64_t P, int N, int64_t Q,
                                                                   const float *__restrict__ F,
                                                                   int64_t ldl, int64_t ldr, int R,
                                                                   float *__restrict__ out, int64_t ldp,
                                                                   int acc_out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_b[];
  constexpr int RP = 16 * RT;
  constexpr int RS = RP + 2;  // factor row stride: the four row groups of a read land on
                              // different banks
  const int Np = (N + 31) & ~31;
  float *fl = reinterpret_cast<float *>(lds_b);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lg = lane >> 4;
  const int64_t qt = (Q + 63) >> 6;
  const int64_t ntile = P * qt;
  const int nsteps = Np >> 5;
  float *stg = fl + Np * RS + wave * (R * 64);
  u4 v[DEPTH][8];
  const float *xp = X;
  int nlim = 0;
  auto tile_base = [&](int64_t t) {
    const int64_t p = t / qt;
    const int64_t q0 = (t - p * qt) * 64;
    const int64_t qa = q0 + 4 * li;
    xp = X + p * ldp + (qa < Q ? qa : Q - 4);
    nlim = N - 1;
  };
  auto load = [&](u4 (&vv)[8], int s) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int n = min(32 * s + 8 * lg + j, nlim);
      vv[j] = __builtin_nontemporal_load(reinterpret_cast<const u4 *>(xp + (int64_t)n * Q));
    }
  };
  int64_t t = (int64_t)blockIdx.x * kMidWaves + wave;
  const int64_t tstride = (int64_t)gridDim.x * kMidWaves;
  if (t < ntile) tile_base(t);
#pragma unroll
  for (int b = 0; b < DEPTH; ++b) load(v[b], b);
  __builtin_amdgcn_sched_barrier(0);  // the X loads go out before the factor is staged
  {
    const int total = Np * RP;
    constexpr int kB = 8;
    for (int e0 = 0; e0 < total; e0 += kB * 64 * kMidWaves) {
      float fv[kB];
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const int e = e0 + threadIdx.x + u * 64 * kMidWaves;
        const int n = e / RP, r = e - (e / RP) * RP;
        const bool ok = e < total && n < N && r < R;
        fv[u] = F[(ok ? n : 0) * (int)ldl + (ok ? r : 0) * (int)ldr];
      }
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const int e = e0 + threadIdx.x + u * 64 * kMidWaves;
        const int n = e / RP, r = e - (e / RP) * RP;
        const bool ok = e < total && n < N && r < R;
        if (e < total) fl[n * RS + r] = ok ? fv[u] : 0.f;  // masked where the value is awaited
      }
    }
  }
  __syncthreads();
  for (; t < ntile; t += tstride) {
    const int64_t p = t / qt;
    const int64_t q0 = (t - p * qt) * 64;
    f4 acc[4][RT];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int nt = 0; nt < RT; ++nt) acc[c][nt] = f4{0.f, 0.f, 0.f, 0.f};
    auto step = [&](u4 (&vv)[8], int s) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const f4 xv = __builtin_bit_cast(f4, vv[j]);
        const float *brow = fl + (32 * s + 8 * lg + j) * RS + li;
#pragma unroll
        for (int nt = 0; nt < RT; ++nt) {
          const float b = brow[nt * 16];
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[c][nt] = p_mfma_f32(xv[c], b, acc[c][nt]);
        }
      }
      load(vv, s + DEPTH);
      __builtin_amdgcn_sched_barrier(0);  // the refill stays ahead of the next step
    };
    int s = 0;
    for (; s + DEPTH <= nsteps; s += DEPTH) {
#pragma unroll
      for (int b = 0; b < DEPTH; ++b) step(v[b], s + b);
    }
#pragma unroll
    for (int b = 0; b < DEPTH - 1; ++b)
      if (s + b < nsteps) step(v[b], s + b);
    const int64_t tn = t + tstride;
    if (tn < ntile)
      tile_base(tn);
    else
      nlim = 0;
#pragma unroll
    for (int b = 0; b < DEPTH; ++b) load(v[b], b);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int nt = 0; nt < RT; ++nt) {
      const int r = nt * 16 + li;
      if (r < R) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          *reinterpret_cast<f4 *>(stg + r * 64 + 16 * lg + 4 * i) =
              f4{acc[0][nt][i], acc[1][nt][i], acc[2][nt][i], acc[3][nt][i]};
      }
    }
    __builtin_amdgcn_wave_barrier();  // the wave reads back only what it wrote
    for (int rr = 0; rr < R; rr += 4) {  // four rows of 64 columns per instruction
      const int r = rr + (lane >> 4);
      const int qq = (lane & 15) * 4;
      if (r < R && q0 + qq < Q) {
        f4 *o = reinterpret_cast<f4 *>(out + (p * R + r) * Q + q0 + qq);
        f4 val = *reinterpret_cast<const f4 *>(stg + r * 64 + qq);
        if (acc_out) {
          val += *o;  // a later chunk of the contracted index: added in chunk order
          *o = val;
        } else {
          __builtin_nontemporal_store(val, o);
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// =====================================================================================
// Last-mode contraction with row-contiguous loads.  Fed straight from memory, the MFMA
// operand layout makes every load instruction touch 16 rows (64 bytes of each), which
// splits each 128-byte line over two requests and keeps the stream well short of HBM speed.
// Here each load instruction covers whole row segments instead: a piece is 16 rows x CPR
// 16-byte chunks, and lane l of load j reads chunk l % CPR of row j * (64 / CPR) + l / CPR,
// so one instruction reads 64 / CPR segments of CPR * 16 contiguous bytes, non-temporally.
// The wave writes the piece to its own padded LDS region and reads it back in the MFMA
// layout (lane (li, lg) takes row li, chunk 4 s + lg at k-step s).  NB register buffers
// keep NB pieces in flight while one is consumed from LDS; every load is issued on every
// path, so the wait before each store leaves the two younger pieces outstanding.
//   bf16: chunk = 8 k, k-step = 32 k; A = the chunk, B = the factor's bf16 hi and lo rows.
//   f32 : chunk = 4 k, k-step = 16 k; element e of the chunk feeds MFMA e, whose k-slot lg
//         stands for k = 16 s + 4 lg + e; B = the matching 4 floats of the factor.
// The factor is stored transposed, [16 RT][Kp + pad], so both operand reads are 16-byte
// LDS loads free of bank conflicts.  One 512-thread block per CU.
// =====================================================================================
constexpr int kLdsThreads = 512;
constexpr int kLdsWaves = kLdsThreads / 64;

template <bool BF, int RT, int CPR, int NB>
__global__ __launch_bounds__(kLdsThreads) __attribute__((amdgpu_waves_per_eu(CPR <= 16 ? 4 : 1))) void ttm_last_lds_k(const void *__restrict__ Xv, int64_t M,
                                                              int K, const float *__restrict__ F,
                                                              int64_t ldl, int64_t ldr, int R,
                                                              float *__restrict__ out, int64_t ldx,
                                                              int acc_out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_b[];
  constexpr int EPC = BF ? 8 : 4;    // elements per 16-byte chunk
  constexpr int ESZ = BF ? 2 : 4;    // bytes per element
  constexpr int KC = CPR * EPC;      // k-values per piece
  constexpr int LPI = CPR / 4;       // loads per lane per piece
  constexpr int RPI = 64 / CPR;      // rows per load instruction
  constexpr int SS = CPR * 16 + 16;  // staging row stride in bytes (16 bytes of padding)
  constexpr int KSTEP = BF ? 32 : 16;
  constexpr int RP = 16 * RT;
  constexpr int kFB = 32;            // factor loads in flight per thread while staging
  const int Kp = (K + KC - 1) / KC * KC;
  const int KS = Kp + (BF ? 8 : 4);  // factor row stride (elements)
  // factor rows in LDS: the R columns of the factor and one zero row that the MFMA tiles'
  // rows past R read (RP rows when R fills the tiles)
  const int FR = RP < R + 1 ? RP : R + 1;
  uint16_t *hi = reinterpret_cast<uint16_t *>(lds_b);
  uint16_t *lo = hi + FR * KS;
  float *fl = reinterpret_cast<float *>(lds_b);
  const int fbytes = BF ? 2 * FR * KS * 2 : FR * KS * 4;  // a multiple of 16
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int li = lane & 15, lg = lane >> 4;
  unsigned char *stg = lds_b + fbytes + wave * 16 * SS;
  const int64_t ntile = (M + 15) >> 4;
  const int kpt = Kp / KC;  // pieces per tile
  const int64_t gw = (int64_t)blockIdx.x * kLdsWaves + wave;
  const int64_t tstride = (int64_t)gridDim.x * kLdsWaves;

  const int crow = lane / CPR, cch = lane % CPR;
  // Lanes outside X load from inside it instead: rows past the end read the last row
  // (their output rows are never stored) and chunks past K read the row's first chunk (the
  // factor is zero there, so they add 0 for finite X; a row holding Inf or NaN has a
  // non-finite result either way).  So every lane issues every load and the loaded values
  // go to LDS untouched, which keeps the waits exact.
  auto load_piece = [&](u4 (&b)[LPI], int64_t t, int h) {
    const int k = h * KC + cch * EPC;
    const int kc = k < K ? k : 0;
#pragma unroll
    for (int j = 0; j < LPI; ++j) {
      int64_t row = t * 16 + j * RPI + crow;
      row = row < M ? row : M - 1;
      b[j] = __builtin_nontemporal_load(reinterpret_cast<const u4 *>(
          reinterpret_cast<const char *>(Xv) + (row * ldx + kc) * ESZ));
    }
  };
  auto store_piece = [&](const u4 (&b)[LPI]) {
#pragma unroll
    for (int j = 0; j < LPI; ++j)
      *reinterpret_cast<u4 *>(stg + (j * RPI + crow) * SS + cch * 16) = b[j];
  };
  f4 acc[RT];
  auto compute_piece = [&](int64_t t, int h) {
    if (h == 0) {
#pragma unroll
      for (int nt = 0; nt < RT; ++nt) acc[nt] = f4{0.f, 0.f, 0.f, 0.f};
    }
    const unsigned char *srow = stg + li * SS + lg * 16;
#pragma unroll
    for (int st = 0; st < CPR / 4; ++st) {
      const u4 a = *reinterpret_cast<const u4 *>(srow + st * 64);
      const int kk = h * KC + st * KSTEP;
      if (BF) {
#pragma unroll
        for (int nt = 0; nt < RT; ++nt) {
          const int off = min(nt * 16 + li, FR - 1) * KS + kk + 8 * lg;
          acc[nt] = p_mfma_bf16(a, *reinterpret_cast<const u4 *>(hi + off), acc[nt]);
          acc[nt] = p_mfma_bf16(a, *reinterpret_cast<const u4 *>(lo + off), acc[nt]);
        }
      } else {
        const f4 xv = __builtin_bit_cast(f4, a);
#pragma unroll
        for (int nt = 0; nt < RT; ++nt) {
          const f4 bv = *reinterpret_cast<const f4 *>(fl + min(nt * 16 + li, FR - 1) * KS + kk + 4 * lg);
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[nt] = p_mfma_f32(xv[e], bv[e], acc[nt]);
        }
      }
    }
    if (h == kpt - 1) {
      // The tile's output rows t*16 .. t*16+15 are one contiguous block of out: the wave
      // puts its accumulators into its staging region (free once the reads above are done;
      // LDS operations of a wave complete in order) and writes the block in 16-byte pieces,
      // non-temporally (only the next kernel reads it).
      float *ot = reinterpret_cast<float *>(stg);
#pragma unroll
      for (int nt = 0; nt < RT; ++nt) {
        const int r = nt * 16 + li;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (r < R) ot[(4 * lg + j) * R + r] = acc[nt][j];
      }
      const int64_t rows = (M - t * 16) < 16 ? (M - t * 16) : 16;
      const int nfl = (int)rows * R;
      float *dst = out + t * 16 * (int64_t)R;
#pragma unroll
      for (int e0 = 0; e0 < 16 * RP; e0 += 256) {
        const int e = e0 + 4 * lane;
        if (e + 4 <= nfl) {
          f4 val = *reinterpret_cast<const f4 *>(ot + e);
          if (acc_out) {  // a later chunk of the contracted index: added in chunk order
            val += *reinterpret_cast<const f4 *>(dst + e);
            *reinterpret_cast<f4 *>(dst + e) = val;
          } else {
            __builtin_nontemporal_store(val, reinterpret_cast<f4 *>(dst + e));
          }
        } else if (e < nfl) {
          for (int q = e; q < nfl; ++q) dst[q] = acc_out ? dst[q] + ot[q] : ot[q];
        }
      }
    }
  };
  auto adv = [&](int64_t &t, int &h) {
    if (++h == kpt) {
      h = 0;
      t += tstride;
    }
  };
  // piece i lives in buffer i % NB: it is stored to LDS once it has arrived, the buffer is
  // refilled at once with piece i + NB, and the MFMAs then consume piece i from LDS, so
  // NB pieces are in flight during every compute step
  u4 bb[NB][LPI];
  int64_t lt = gw, ct = gw;  // load and compute cursors (tile, piece)
  int lh = 0, ch = 0;
  // Prologue, in this order: the first batch of factor loads, the first NB pieces of X,
  // then the factor's conversion into LDS.  The conversion waits only for the factor loads
  // (the older ones), so the X requests stay in flight through it and the barrier.  The
  // scheduling barriers keep this order, which the waits count on.  A wave without tiles
  // loads clamped rows and leaves after the barrier.
  // thread -> column r = tid % RP of the factor and rows k = tid / RP + u * KSTR
  constexpr int KSTR = kLdsThreads / RP;
  const int fr = threadIdx.x % RP, fk = threadIdx.x / RP;
  const int frc = fr < R ? fr : R - 1;
  auto fac_load = [&](int k) { return F[(int64_t)(k < K ? k : K - 1) * ldl + (int64_t)frc * ldr]; };
  // Rows k >= Kp go to the padding column Kp, which no MFMA reads, and columns past the
  // zero row write their zeros into it: the store is then unconditional, so every factor
  // load is consumed on every path.
  const int frs = fr < FR ? fr : FR - 1;
  auto fac_store = [&](int k, float x) {
    const float a = (k < K && fr < R) ? x : 0.f;
    const int kk = k < Kp ? k : Kp;
    if (BF) {
      const uint16_t h = p_f2bf(a);
      hi[frs * KS + kk] = h;
      lo[frs * KS + kk] = p_f2bf(a - p_bf2f(h));
    } else {
      fl[frs * KS + kk] = a;
    }
  };
  float fv[kFB];
#pragma unroll
  for (int u = 0; u < kFB; ++u) fv[u] = fac_load(fk + u * KSTR);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    load_piece(bb[j], lt, lh);
    adv(lt, lh);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int u = 0; u < kFB; ++u) fac_store(fk + u * KSTR, fv[u]);
  // longer factors: further batches (these waits also cover the X requests above)
  for (int k0 = kFB * KSTR; k0 < Kp; k0 += kFB * KSTR) {
#pragma unroll
    for (int u = 0; u < kFB; ++u) fv[u] = fac_load(k0 + fk + u * KSTR);
#pragma unroll
    for (int u = 0; u < kFB; ++u) fac_store(k0 + fk + u * KSTR, fv[u]);
  }
  __syncthreads();
  if (gw >= ntile) return;  // no barrier follows
  const int64_t np = ((ntile - 1 - gw) / tstride + 1) * kpt;  // pieces of this wave
  auto step = [&](u4 (&b)[LPI]) {
    store_piece(b);
    load_piece(b, lt, lh);
    adv(lt, lh);
    __builtin_amdgcn_sched_barrier(0);
    compute_piece(ct, ch);
    adv(ct, ch);
  };
  // whole rounds of NB steps (a single back edge, so the waits stay exact), then the
  // remaining pieces; the loads issued for pieces past the end read the last row of X
  // again and are never used
  int64_t i = 0;
  for (; i + NB <= np; i += NB) {
#pragma unroll
    for (int j = 0; j < NB; ++j) step(bb[j]);
  }
#pragma unroll
  for (int j = 0; j < NB - 1; ++j)
    if (i + j < np) step(bb[j]);
}

// ------------------------------------------------------------------ launchers
static nnc_status allow_lds_bytes(const void *kern, size_t bytes) {
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

constexpr size_t kPassLdsMax = 96 * 1024;
constexpr int kPassBlocks = 512;  // persistent: two blocks per CU

size_t pass_last_lds(bool bf, int RT, int64_t K) {
  if (bf) {
    const int64_t Kp = (K + 31) / 32 * 32;
    return (size_t)(2 * 16 * RT * (Kp + 8) * 2);
  }
  const int64_t Kp = (K + 15) / 16 * 16;
  return (size_t)(Kp * (16 * RT + 4) * 4);
}

// Earlier-mode kernels: the factor (bf16 hi / lo rows, or FP32 rows) plus each wave's
// output staging.
size_t pass_mid_lds(bool bf, int RT, int64_t N, int64_t R, bool hs) {
  const int64_t Np = (N + 31) / 32 * 32;
  if (bf) return (size_t)(2 * 16 * RT * (Np + 8) * 2 + (int64_t)kMidWaves * R * (hs ? 64 : 128) * 4);
  return (size_t)(Np * (16 * RT + 2) * 4 + (int64_t)kMidWaves * R * 64 * 4);
}

// Row-contiguous last-mode kernel: chunks per piece row (CPR) is the largest of 32, 16, 8
// whose piece width does not exceed K; the whole LDS (factor + staging) must fit a CU.
constexpr size_t kCuLdsBytes = 160 * 1024;

int device_cu_count() {
  static int n = 0;
  if (!n) {
    int dev = 0, c = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && c > 0)
      n = c;
    else
      n = 256;
  }
  return n;
}

size_t last_lds_bytes(bool bf, int RT, int CPR, int64_t K, int64_t R) {
  const int64_t EPC = bf ? 8 : 4, KC = CPR * EPC;
  const int64_t Kp = (K + KC - 1) / KC * KC;
  const int64_t KS = Kp + (bf ? 8 : 4);
  const int64_t FR = std::min<int64_t>(16 * RT, R + 1);
  const int64_t fbytes = bf ? 2 * FR * KS * 2 : FR * KS * 4;
  return (size_t)(fbytes + (int64_t)kLdsWaves * 16 * (CPR * 16 + 16));
}

static nnc_status launch_last_lds(const void *X, bool bf, int64_t M, int64_t K, const float *F,
                                  int64_t ldl, int64_t ldr, int64_t R, float *out, hipStream_t s,
                                  const char **kernel_name, int reserve, int64_t ldx, int acc_out) {
  const int EPC = bf ? 8 : 4;
  if (K % EPC || K > (1 << 20) || K < 8 * EPC) return NNC_EUNSUPPORTED;
  const int RT = R <= 16 ? 1 : 2;
  // pieces of 16 chunks and two blocks per CU when two blocks' LDS fits a CU (every variant
  // of 16 chunks stays within 128 VGPRs, four waves per SIMD), else the widest pieces that fit
  int CPR = K >= 32 * EPC ? 32 : (K >= 16 * EPC ? 16 : 8), per_cu = 1;
  if (K >= 16 * EPC && 2 * last_lds_bytes(bf, RT, 16, K, R) <= kCuLdsBytes) {
    CPR = 16;
    per_cu = 2;
  }
  const size_t lds = last_lds_bytes(bf, RT, CPR, K, R);
  if (lds > kCuLdsBytes) return NNC_EUNSUPPORTED;
  const int64_t tiles = (M + 15) / 16;
  const int grid = (int)std::max<int64_t>(
      1, std::min<int64_t>((tiles + kLdsWaves - 1) / kLdsWaves,
                           (int64_t)per_cu * (device_cu_count() - std::max(reserve, 0))));
  // one piece in flight per wave (measured fastest at 512^3 with random data, 51.5-52 us
  // against 53.5-54 with two and 54-55 with three for bf16 X: with the HBM saturated, more
  // outstanding loads only queue)
#define NNC_LL(BFV, RTV, CPRV)                                                                    \
  do {                                                                                            \
    constexpr int NBV = 1;                                                                        \
    NNC_TRY(allow_lds_bytes(reinterpret_cast<const void *>(ttm_last_lds_k<BFV, RTV, CPRV, NBV>), lds)); \
    hipLaunchKernelGGL((ttm_last_lds_k<BFV, RTV, CPRV, NBV>), dim3(grid), dim3(kLdsThreads), lds, s, X, \
                       M, (int)K, F, ldl, ldr, (int)R, out, ldx, acc_out);                        \
  } while (0)
#define NNC_LL_CPR(BFV, RTV)           \
  do {                                 \
    if (CPR == 32)                     \
      NNC_LL(BFV, RTV, 32);            \
    else if (CPR == 16)                \
      NNC_LL(BFV, RTV, 16);            \
    else                               \
      NNC_LL(BFV, RTV, 8);             \
  } while (0)
  if (bf && RT == 1)
    NNC_LL_CPR(true, 1);
  else if (bf)
    NNC_LL_CPR(true, 2);
  else if (RT == 1)
    NNC_LL_CPR(false, 1);
  else
    NNC_LL_CPR(false, 2);
#undef NNC_LL_CPR
#undef NNC_LL
  if (kernel_name) *kernel_name = bf ? "ttm_last_lds_bf16" : "ttm_last_lds_f32";
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

// Returns NNC_EUNSUPPORTED (without recording an error) when the shape does not suit the
// pipelined kernels, so the caller can fall back.  A contracted index too long for the
// factor to fit in LDS is split into chunks, each a launch on its slab of X (with X's own
// strides) whose output is added to the previous chunks' in chunk order.
nnc_status launch_pass(const void *X, nnc_dtype xdt, int64_t P, int64_t N, int64_t Q, const float *F,
                       int64_t ldl, int64_t ldr, int64_t R, float *out, hipStream_t s,
                       const char **kernel_name, int reserve_cus) {
  if (R > 32 || R < 1) return NNC_EUNSUPPORTED;
  if ((reinterpret_cast<uintptr_t>(X) & 15u) || (reinterpret_cast<uintptr_t>(out) & 15u))
    return NNC_EUNSUPPORTED;
  const bool bf = xdt == NNC_BF16;
  const int esz = bf ? 2 : 4;
  const int RT = R <= 16 ? 1 : 2;
  const int waves = kPassThreads / 64;
  if (Q == 1) {
    if (N > (1 << 20)) return NNC_EUNSUPPORTED;
    nnc_status st = launch_last_lds(X, bf, P, N, F, ldl, ldr, R, out, s, kernel_name, reserve_cus, N, 0);
    if (st != NNC_EUNSUPPORTED) return st;
    const int EPC = bf ? 8 : 4, KC = 32 * EPC;
    if (N % EPC == 0 && N >= 8 * EPC && last_lds_bytes(bf, RT, 32, KC, R) <= kCuLdsBytes) {
      // chunks of Kc (a multiple of the 32-chunk piece width, so every slab starts 16-byte
      // aligned), the last one long enough for the kernel's pieces
      int64_t Kmax = KC;
      while (last_lds_bytes(bf, RT, 32, Kmax + KC, R) <= kCuLdsBytes) Kmax += KC;
      int64_t Kc = Kmax, nch = 1;
      for (; Kc >= KC; Kc -= KC) {
        nch = (N + Kc - 1) / Kc;
        if (N - (nch - 1) * Kc >= 8 * EPC) break;
      }
      if (Kc >= KC) {
        for (int64_t c = 0; c < nch; ++c) {
          const int64_t k0 = c * Kc, kc = std::min(Kc, N - k0);
          NNC_TRY(launch_last_lds(static_cast<const char *>(X) + k0 * esz, bf, P, kc, F + k0 * ldl, ldl, ldr, R,
                                  out, s, nullptr, reserve_cus, N, c > 0));
        }
        if (kernel_name) *kernel_name = bf ? "ttm_last_lds_bf16 (chunked)" : "ttm_last_lds_f32 (chunked)";
        return NNC_OK;
      }
    }
    if (N % (bf ? 8 : 4)) return NNC_EUNSUPPORTED;
    const size_t lds = pass_last_lds(bf, RT, N);
    if (lds > kPassLdsMax) return NNC_EUNSUPPORTED;
    const int64_t tiles = (P + 15) / 16;
    const int grid = (int)std::min<int64_t>(std::max<int64_t>((tiles + waves - 1) / waves, 1), kPassBlocks);
#define NNC_LAST(BFV, RTV)                                                                        \
  do {                                                                                            \
    NNC_TRY(allow_lds_bytes(reinterpret_cast<const void *>(ttm_last_pipe_k<BFV, RTV>), lds));     \
    hipLaunchKernelGGL((ttm_last_pipe_k<BFV, RTV>), dim3(grid), dim3(kPassThreads), lds, s, X, P, \
                       (int)N, F, ldl, ldr, (int)R, out);                                         \
  } while (0)
    if (bf && RT == 1) NNC_LAST(true, 1);
    else if (bf) NNC_LAST(true, 2);
    else if (RT == 1) NNC_LAST(false, 1);
    else NNC_LAST(false, 2);
#undef NNC_LAST
    if (kernel_name) *kernel_name = bf ? "ttm_last_pipe_bf16" : "ttm_last_pipe_f32";
  } else {
    // earlier mode: ttm_mid_lds_k (bf16 X) / ttm_mid_lds_f32_k (FP32 X)
    if (Q % (bf ? 8 : 4)) return NNC_EUNSUPPORTED;
    if (N > (1 << 20) || N * ldl + R * ldr >= ((int64_t)1 << 31)) return NNC_EUNSUPPORTED;  // 32-bit factor indexing
    // bf16 output staging by halves of the tile when the whole tile's does not fit beside the
    // factor (R above 20 at N = 512); rows of the factor per launch: all of them, or chunks of
    // a multiple of 32
    const bool hs = bf && pass_mid_lds(bf, RT, N, R, false) > kCuLdsBytes;
    int64_t Nc = N;
    if (pass_mid_lds(bf, RT, N, R, hs) > kCuLdsBytes) {
      int64_t Nmax = 0;
      while (pass_mid_lds(bf, RT, Nmax + 32, R, hs) <= kCuLdsBytes) Nmax += 32;
      if (Nmax == 0) return NNC_EUNSUPPORTED;
      const int64_t nch = (N + Nmax - 1) / Nmax;
      Nc = ((N + nch - 1) / nch + 31) / 32 * 32;
    }
    const size_t lds = pass_mid_lds(bf, RT, Nc, R, hs);
    const int64_t tiles = P * ((Q + (bf ? 127 : 63)) / (bf ? 128 : 64));
    // two blocks per CU when their LDS fits and the variant stays within 128 VGPRs (four
    // waves per SIMD: the FP32 kernels and the bf16 ones of one rank tile)
    const int per_cu = ((!bf || RT == 1) && 2 * lds <= kCuLdsBytes) ? 2 : 1;
    int grid = (int)std::min<int64_t>((tiles + kMidWaves - 1) / kMidWaves, (int64_t)per_cu * device_cu_count());
    if (grid < 1) grid = 1;
    for (int64_t n0 = 0; n0 < N; n0 += Nc) {
      const int64_t nc = std::min(Nc, N - n0);
      const void *Xc = static_cast<const char *>(X) + n0 * Q * esz;
      const float *Fc = F + n0 * ldl;
      const int acc = n0 > 0;
#define NNC_MID(KERN)                                                                                \
  do {                                                                                               \
    NNC_TRY(allow_lds_bytes(reinterpret_cast<const void *>(KERN), lds));                             \
    hipLaunchKernelGGL(KERN, dim3(grid), dim3(64 * kMidWaves), lds, s, XARG, P, (int)nc, Q, Fc, ldl, \
                       ldr, (int)R, out, N * Q, acc);                                                \
  } while (0)
      if (bf) {
#define XARG (const uint16_t *)Xc
        if (RT == 1 && !hs) NNC_MID((ttm_mid_lds_k<1, false>));
        else if (RT == 1) NNC_MID((ttm_mid_lds_k<1, true>));
        else if (!hs) NNC_MID((ttm_mid_lds_k<2, false>));
        else NNC_MID((ttm_mid_lds_k<2, true>));
#undef XARG
      } else {
#define XARG (const float *)Xc
        if (RT == 1) NNC_MID((ttm_mid_lds_f32_k<1, kMidDepthF32>));
        else NNC_MID((ttm_mid_lds_f32_k<2, kMidDepthF32>));
#undef XARG
      }
#undef NNC_MID
    }
    if (kernel_name)
      *kernel_name = Nc < N ? (bf ? "ttm_mid_bf16 (chunked)" : "ttm_mid_f32 (chunked)") : (bf ? "ttm_mid_bf16" : "ttm_mid_f32");
  }
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

}  // namespace nnc
