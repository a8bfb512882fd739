// Nonnegative CP of a small tensor (the Tucker core) by multiplicative updates, entirely
// inside one workgroup: the CP factors, their Grams and the update temporaries live in LDS,
// and so does the tensor when it fits.  One workgroup per fit, so a launch can run many
// independent fits (random restarts, uneven ranks) at once, and every sweep of every fit
// happens inside that single launch.
//
// Sweep (factors 1..d in order):  M_n = MTTKRP(T, {B_k}_{k!=n}),  H_n = Hadamard_{k!=n} B_k^T B_k,
//   B_n <- B_n * M_n / max(B_n H_n, eps),  then B_n^T B_n is refreshed.
// With ALS set (the real-valued CP fit of the core, Section 2.2) the update is the least-squares
// step B_n <- M_n H_n^{-1} instead, H_n inverted in FP64 by Gauss-Jordan elimination.
// MTTKRP M_n[i, rho] = sum over entries with i_n = i of T[idx] prod_{k!=n} B_k[i_k, rho] is
// evaluated in two stages: first the last mode L != n is contracted for every rho at once,
//   Z[o][rho] = sum_l T[.., l (mode L), ..] B_L[l, rho]        (o = the other indices of T),
// then Z is summed over the remaining modes != n with their factor entries.  Partial sums
// are added in a fixed order, so results are reproducible.
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "nnc_internal.h"

namespace nnc {

struct CpPtrs {
  float *p[kMaxDim];
};

struct CpArgs {
  int d;
  int dims[kMaxDim];
  int size;
  int maxdim;
  int t_lds;  // 1: T staged in LDS
  int z_lds;  // 1: Z in LDS, else in global scratch
  int zmax;   // rows of Z (max over modes of size / dims[L])
};

static __device__ inline float mu_cp(float x, float num, float den, double eps, unsigned int *nclip) {
  double dd = (double)den;
  if (dd < eps) {
    dd = eps;
    atomicAdd(nclip, 1u);
  }
  return (float)(((double)x * (double)num) / dd);
}

// LDS floats of one fit of rank r with `threads` threads:
//   [T if t_lds] B_k (dims[k] x r) | Gram_k (r x r) | H (r x r)
//   | part (max(threads, maxdim * r)) | new factor values (maxdim x RM)
//   | red (2 * threads doubles) | [2 r x r doubles if ALS]
//   | [Z (zmax x r) if z_lds]
static int64_t cp_lds_floats(const CpArgs &a, int r, int threads, bool t_lds, bool z_lds, bool als) {
  int64_t s = t_lds ? a.size : 0;
  s = (s + 3) & ~(int64_t)3;  // factor rows are read as float4
  const int RM = r <= 8 ? 8 : (r <= 16 ? 16 : 32);  // factor rows and Z rows are padded to RM
  for (int k = 0; k < a.d; ++k) s += (int64_t)a.dims[k] * RM;
  s += (int64_t)(a.d + 1) * r * r;
  s += std::max<int64_t>(threads, (int64_t)a.maxdim * r);
  s = (s + 3) & ~(int64_t)3;
  s += (int64_t)a.maxdim * RM;  // new values of the last updated factor
  s += (s & 1);               // keep the doubles 8-byte aligned
  s += 4 * (int64_t)threads;  // 2 * threads doubles
  if (als) s += 4 * (int64_t)r * r;  // two r x r double buffers for the inverse of H
  s = (s + 3) & ~(int64_t)3;  // Z rows are written as float4
  if (z_lds) s += (int64_t)a.zmax * RM;
  return s;
}

// Every per-mode array below is indexed only by loop counters of fully unrolled loops over
// kMaxDim, so it lives in registers (no scratch memory); factor blocks are addressed by
// offsets kept in LDS.
template <int RM, bool ALS, int DC>
__global__ __launch_bounds__(1024) void nncp_k(const float *__restrict__ Tg, CpArgs a, int rank0,
                                               CpPtrs ptr0, const int *__restrict__ ranks,
                                               float *const *__restrict__ fptrs, int iters,
                                               double eps, double *__restrict__ resid,
                                               unsigned long long *clips, float *__restrict__ zg) {
  extern __shared__ __attribute__((aligned(16))) float sm[];
  __shared__ unsigned int nclip;
  __shared__ int boff[kMaxDim + 1];
  const int b = blockIdx.x;
  const int r = ranks ? ranks[b] : rank0;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int d = DC > 0 ? DC : a.d;  // DC > 0: the order fixed at compile time
  float *p = sm;
  const float *T = Tg;
  if (a.t_lds) {
    for (int e = tid; e < a.size; e += nt) p[e] = Tg[e];
    T = p;
    p += a.size;
  }
  p += (4 - ((p - sm) & 3)) & 3;
  float *sB = p;  // B_k at sB + boff[k], rows padded to RM columns (zeros past r)
  int nb = 0;
#pragma unroll
  for (int k = 0; k < kMaxDim; ++k)
    if (k < d) nb += a.dims[k] * RM;
  p += nb;
  float *sW = p;  // Gram_k at sW + k*r*r
  p += d * r * r;
  float *H = p;
  p += r * r;
  float *part = p;
  p += (nt > a.maxdim * r ? nt : a.maxdim * r);
  p += (4 - ((p - sm) & 3)) & 3;  // fnew rows are read as float4
  float *fnew = p;  // the new values of the factor just updated (rows padded to RM, zeros past r)
  p += a.maxdim * RM;
  p += ((p - sm) & 1);
  double *red = reinterpret_cast<double *>(p);
  p += 4 * nt;
  double *Hd = reinterpret_cast<double *>(p);  // ALS: two r x r buffers
  if (ALS) p += 4 * r * r;
  p += (4 - ((p - sm) & 3)) & 3;
  float *Z = a.z_lds ? p : zg + (int64_t)b * a.zmax * RM;
  for (int e = tid; e < a.maxdim * RM; e += nt) fnew[e] = 0.f;
  if (tid == 0) {
    nclip = 0;
    int o = 0;
    for (int k = 0; k < d; ++k) {
      boff[k] = o;
      o += a.dims[k] * RM;
    }
    boff[d] = o;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kMaxDim; ++k) {
    if (k >= d) break;
    const float *src = ranks ? fptrs[(int64_t)b * d + k] : ptr0.p[k];
    for (int e = tid; e < a.dims[k] * RM; e += nt) {
      const int i = e / RM, c = e - (e / RM) * RM;
      sB[boff[k] + e] = c < r ? src[i * r + c] : 0.f;
    }
  }
  __syncthreads();
  for (int k = 0; k < d; ++k) {
    const float *Bk = sB + boff[k];
    for (int e = tid; e < r * r; e += nt) {
      const int x = e / r, y = e - (e / r) * r;
      float acc = 0.f;
      for (int i = 0; i < a.dims[k]; ++i) acc = fmaf(Bk[i * RM + x], Bk[i * RM + y], acc);
      sW[k * r * r + e] = acc;
    }
  }
  __syncthreads();

  // Multiplicative updates leave the new values of B_n in fnew; the phase that starts the next
  // mode copies them into place and forms their Gram (`pending`, mode `np`), so a mode takes
  // three barriers.  A stage-1 contraction over that same factor reads fnew directly.
  bool pending = false;
  int np = 0;
  const float inv_r = 1.0f / (float)r;
  for (int it = 0; it < iters; ++it) {
    for (int n = 0; n < d; ++n) {
      const int L = (n == d - 1) ? d - 2 : d - 1;
      const int mL = a.dims[L];
      int postL = 1;
      for (int k = L + 1; k < d; ++k) postL *= a.dims[k];
      const int zrows = a.size / mL;
      const float *BL = (pending && L == np) ? fnew : sB + boff[L];
      // ---- stage 1: Z[o][rho] = sum_l T[(pre*mL + l)*postL + q] B_L[l][rho], o = pre*postL + q;
      // one thread per (row, quad of columns), quads past the rank left out.  H_n (Hadamard
      // product of the other Grams, final since the last update) in the same phase.
      const int nq = (r + 3) >> 2;
      // index divisions through float reciprocals (qdiv; nncp_check_shape keeps every
      // index here below 2^22)
      const float inv_nq = 1.0f / (float)nq, inv_postL = 1.0f / (float)postL;
      // modes 1 .. d-2 contract the same mode L = d-1 as mode 0, whose factor has not changed
      // since mode 0's stage 1 in this sweep: Z is already there
      const bool z_current = n >= 1 && n <= d - 2;
      for (int w = z_current ? nq * zrows : tid; w < nq * zrows; w += nt) {
        const int o = qdiv(w, inv_nq), c4 = (w - o * nq) * 4;
        const int pre = qdiv(o, inv_postL), q = o - pre * postL;
        const float *t = T + pre * mL * postL + q;
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 4
        for (int l = 0; l < mL; ++l) {
          const float x = t[l * postL];
          const float4 bv = *reinterpret_cast<const float4 *>(BL + l * RM + c4);
          acc.x = fmaf(x, bv.x, acc.x);
          acc.y = fmaf(x, bv.y, acc.y);
          acc.z = fmaf(x, bv.z, acc.z);
          acc.w = fmaf(x, bv.w, acc.w);
        }
        *reinterpret_cast<float4 *>(Z + o * RM + c4) = acc;
      }
      if (pending) {
        float *Bp = sB + boff[np];
        const int Ip = a.dims[np];
        for (int e = tid; e < Ip * RM; e += nt) Bp[e] = fnew[e];
        for (int e = tid; e < r * r; e += nt) {
          const int x = qdiv(e, inv_r), y = e - x * r;
          float acc = 0.f;
#pragma unroll 4
          for (int i = 0; i < Ip; ++i) acc = fmaf(fnew[i * RM + x], fnew[i * RM + y], acc);
          sW[np * r * r + e] = acc;
        }
        pending = false;
      }
      if (!a.z_lds) __threadfence_block();
      __syncthreads();
      // H_n: Hadamard product of the other Grams (all final since the phase above)
      for (int e = tid; e < r * r; e += nt) {
        float h = 1.f;
        for (int k = 0; k < d; ++k)
          if (k != n) h *= sW[k * r * r + e];
        H[e] = h;
      }
      // ---- stage 2: M[i][rho] = sum over Z rows with i_n = i of Z[o][rho] prod_{k!=n,L} B_k[i_k][rho]
      // Z's modes are T's modes without L (row-major).  With one mode j besides n and L
      // (d = 3), Z is 2-D and the sum runs over j's index directly (split s taking the
      // indices j = s (mod S)); otherwise an odometer walks the modes other than n over
      // contiguous ranges.  Pairs (i, rho) take S threads each, whose partial sums are added
      // in split order by the update below.
      const int In = a.dims[n];
      const int npairs = In * r;
      const int other = zrows / In;
      const int S = npairs >= nt ? 1 : nt / npairs;
      const float inv_npairs = 1.0f / (float)npairs;
      if (d <= 3) {
        // position of n among Z's modes and the other mode (if any)
        int jo = -1;
        for (int k = 0; k < d; ++k)
          if (k != n && k != L) jo = k;
        const bool n_first = jo < 0 || n < jo;  // Z = [n][jo] or [jo][n]
        const int Bo = jo >= 0 ? boff[jo] : 0;
        const int zstep = (n_first ? 1 : In) * S;
        for (int w = tid; w < npairs * S; w += nt) {
          const int s = qdiv(w, inv_npairs), pr = w - s * npairs;
          const int i = qdiv(pr, inv_r), rho = pr - i * r;
          int zoff = n_first ? i * other + s : s * In + i;
          float acc = 0.f;
          if (jo >= 0) {
            const float *bo = sB + Bo + rho;
            for (int j = s; j < other; j += S, zoff += zstep) acc += Z[zoff * RM + rho] * bo[j * RM];
          } else {
            for (int j = s; j < other; j += S, zoff += zstep) acc += Z[zoff * RM + rho];
          }
          part[w] = acc;
        }
      } else {
        int zdims[kMaxDim], zstride[kMaxDim], zb[kMaxDim], idx[kMaxDim];
        int nz = 0, npos = 0;
#pragma unroll
        for (int j = 0; j < kMaxDim; ++j) {
          zdims[j] = 1;
          zstride[j] = 0;
          zb[j] = 0;
          idx[j] = 0;
        }
#pragma unroll
        for (int k = 0; k < kMaxDim; ++k) {
          if (k < d && k != L) {
            if (k == n) npos = nz;
#pragma unroll
            for (int j = 0; j < kMaxDim; ++j)
              if (j == nz) {
                zdims[j] = a.dims[k];
                zb[j] = boff[k];
              }
            ++nz;
          }
        }
        {
          int st = 1;
#pragma unroll
          for (int j = kMaxDim - 1; j >= 0; --j)
            if (j < nz) {
              zstride[j] = st;
              st *= zdims[j];
            }
        }
        int nstride = 0;
#pragma unroll
        for (int j = 0; j < kMaxDim; ++j)
          if (j == npos) nstride = zstride[j];
        for (int w = tid; w < npairs * S; w += nt) {
          const int s = qdiv(w, inv_npairs), pr = w - s * npairs;
          const int i = qdiv(pr, inv_r), rho = pr - i * r;
          const int o0 = (int)((int64_t)other * s / S), o1 = (int)((int64_t)other * (s + 1) / S);
          int rem = o0, zoff = i * nstride;
#pragma unroll
          for (int j = kMaxDim - 1; j >= 0; --j) {
            if (j < nz && j != npos) {
              idx[j] = rem % zdims[j];
              rem /= zdims[j];
              zoff += idx[j] * zstride[j];
            }
          }
          float acc = 0.f;
          for (int o = o0; o < o1; ++o) {
            float prod = Z[zoff * RM + rho];
#pragma unroll
            for (int j = 0; j < kMaxDim; ++j)
              if (j < nz && j != npos) prod *= sB[zb[j] + idx[j] * RM + rho];
            acc += prod;
            bool carry = true;  // odometer over the modes != n of Z, last fastest
#pragma unroll
            for (int j = kMaxDim - 1; j >= 0; --j) {
              if (carry && j < nz && j != npos) {
                zoff += zstride[j];
                if (++idx[j] == zdims[j]) {
                  zoff -= zdims[j] * zstride[j];
                  idx[j] = 0;
                } else {
                  carry = false;
                }
              }
            }
          }
          part[w] = acc;
        }
      }
      __syncthreads();
      float *Bn = sB + boff[n];
      if (ALS) {
        // ---- B_n <- M H^{-1}: the S partial sums of each pair (split order) into part[e]
        // (a thread reads only its own pair's partials, and part[e] is one of them)
        for (int e = tid; e < npairs; e += nt) {
          float m = 0.f;
#pragma unroll 4
          for (int s = 0; s < S; ++s) m += part[s * npairs + e];
          part[e] = m;
        }
        for (int e = tid; e < r * r; e += nt) Hd[e] = (double)H[e];
        __syncthreads();
        const double *Hinv = gj_inverse(Hd, Hd + r * r, r, &nclip);
        for (int e = tid; e < npairs; e += nt) {
          const int i = qdiv(e, inv_r), c = e - i * r;
          double v = 0.0;
          for (int s2 = 0; s2 < r; ++s2) v += (double)part[i * r + s2] * Hinv[s2 * r + c];
          Bn[i * RM + c] = (float)v;
        }
        __syncthreads();
        for (int e = tid; e < r * r; e += nt) {
          const int x = qdiv(e, inv_r), y = e - x * r;
          float acc = 0.f;
#pragma unroll 4
          for (int i = 0; i < In; ++i) acc = fmaf(Bn[i * RM + x], Bn[i * RM + y], acc);
          sW[n * r * r + e] = acc;
        }
        __syncthreads();
        continue;
      }
      // ---- B_n <- B_n * M / max(B_n H, eps): new values go to fnew (moved into place, and
      // their Gram formed, by the first phase of the next mode or after the last sweep)
      for (int e = tid; e < npairs; e += nt) {
        const int i = qdiv(e, inv_r), c = e - i * r;
        float m = 0.f;  // the S partial sums of pair e, in split order
#pragma unroll 4
        for (int s = 0; s < S; ++s) m += part[s * npairs + e];
        float den = 0.f;
#pragma unroll 4
        for (int s2 = 0; s2 < r; ++s2) den = fmaf(Bn[i * RM + s2], H[s2 * r + c], den);
        fnew[i * RM + c] = mu_cp(Bn[i * RM + c], m, den, eps, &nclip);
      }
      pending = true;
      np = n;
      __syncthreads();
    }
  }
  if (pending) {
    float *Bp = sB + boff[np];
    for (int e = tid; e < a.dims[np] * RM; e += nt) Bp[e] = fnew[e];
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kMaxDim; ++k) {
    if (k >= d) break;
    float *dst = ranks ? fptrs[(int64_t)b * d + k] : ptr0.p[k];
    for (int e = tid; e < a.dims[k] * r; e += nt) dst[e] = sB[boff[k] + (e / r) * RM + e % r];
  }
  if (tid == 0 && nclip) atomicAdd(clips, (unsigned long long)nclip);

  if (resid) {  // ||T - cp(B)|| / ||T||, double accumulation, fixed tree
    double sr = 0.0, sx = 0.0;
    for (int e = tid; e < a.size; e += nt) {
      int ix[kMaxDim];
      int rem = e;
#pragma unroll
      for (int k = kMaxDim - 1; k >= 0; --k) {
        ix[k] = 0;
        if (k < d) {
          ix[k] = rem % a.dims[k];
          rem /= a.dims[k];
        }
      }
      float xh = 0.f;
      for (int rho = 0; rho < r; ++rho) {
        float pp = 1.f;
#pragma unroll
        for (int k = 0; k < kMaxDim; ++k)
          if (k < d) pp *= sB[boff[k] + ix[k] * RM + rho];
        xh += pp;
      }
      const double x = T[e];
      const double df = x - (double)xh;
      sr += df * df;
      sx += x * x;
    }
    red[tid] = sr;
    red[nt + tid] = sx;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
      if (tid < w && tid + w < nt) {
        red[tid] += red[tid + w];
        red[nt + tid] += red[nt + tid + w];
      }
      __syncthreads();
    }
    if (tid == 0) resid[b] = red[nt] > 0.0 ? sqrt(red[0] / red[nt]) : 0.0;
  }
}

static CpArgs make_args(const CpProblem &pb) {
  CpArgs a;
  memset(&a, 0, sizeof a);
  a.d = pb.d;
  a.size = (int)pb.size;
  a.maxdim = 0;
  for (int k = 0; k < pb.d; ++k) {
    a.dims[k] = (int)pb.dims[k];
    if (a.dims[k] > a.maxdim) a.maxdim = a.dims[k];
  }
  const int mlast = a.dims[pb.d - 1], mprev = a.dims[pb.d - 2];
  a.zmax = a.size / (mlast < mprev ? mlast : mprev);
  return a;
}

// Dynamic LDS a single fit may use (one workgroup per CU; gfx950 has 160 KiB per CU).
constexpr int64_t kCpLdsBudget = 150 * 1024;

struct CpLayout {
  CpArgs a;
  int64_t lds_bytes;
};

// Keep T in LDS when possible (it is read every stage), then Z.
static CpLayout cp_layout(const CpProblem &pb, int max_rank, int threads, bool als, bool t_global = false) {
  CpLayout L;
  L.a = make_args(pb);
  const bool opts[4][2] = {{true, true}, {true, false}, {false, true}, {false, false}};
  for (const auto &o : opts) {
    if (t_global && o[0]) continue;  // the tensor read from global memory (L2) on request
    const int64_t bytes = cp_lds_floats(L.a, max_rank, threads, o[0], o[1], als) * 4;
    if (bytes <= kCpLdsBudget || (!o[0] && !o[1])) {
      L.a.t_lds = o[0];
      L.a.z_lds = o[1];
      L.lds_bytes = bytes;
      return L;
    }
  }
  return L;
}

int64_t nncp_lds_bytes(const CpProblem &pb, int max_rank, int threads, bool als, bool t_global) {
  return cp_layout(pb, max_rank, threads, als, t_global).lds_bytes;
}

int64_t nncp_zscratch_floats(const CpProblem &pb, int max_rank) {
  const CpArgs a = make_args(pb);
  const int RM = max_rank <= 8 ? 8 : (max_rank <= 16 ? 16 : 32);
  return (int64_t)a.zmax * RM;
}

int nncp_default_threads(const CpProblem &pb, int max_rank) {
  const int64_t work = pb.size * (int64_t)max_rank;
  if (work >= (1 << 16)) return 1024;
  if (work >= (1 << 13)) return 512;
  return 256;
}

// Raise a kernel's dynamic-LDS limit to `bytes` (once per larger size).
static nnc_status allow_lds(const void *kern, int64_t bytes) {
  static std::mutex mu;
  static std::map<const void *, int64_t> done;
  if (bytes <= 64 * 1024) return NNC_OK;
  std::lock_guard<std::mutex> lk(mu);
  auto it = done.find(kern);
  if (it != done.end() && it->second >= bytes) return NNC_OK;
  NNC_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  done[kern] = bytes;
  return NNC_OK;
}

// The kernel splits its loop indices with qdiv, exact below 2^22: stage 1 runs
// ceil(r/4) * size / dims[L] items (L = the contracted mode of that update), stage 2 and the
// update run dims[n] * r pairs (times a split factor only while that stays below the thread
// count).  Shapes whose index ranges reach 2^22 are refused here, before any HIP call.
nnc_status nncp_check_shape(const CpProblem &pb, int max_rank, int threads, bool als) {
  if (pb.d < 2 || pb.size < 1) return fail(NNC_EINVAL, "nnCP needs a tensor of 2 or more modes");
  if (pb.size > (1 << 26)) return fail(NNC_EUNSUPPORTED, "nnCP tensor too large for one workgroup");
  if (max_rank < 1) return fail(NNC_EINVAL, "nnCP rank %d < 1", max_rank);
  if (max_rank > 32) return fail(NNC_EUNSUPPORTED, "nnCP rank above 32");
  constexpr int64_t kIdxLimit = (int64_t)1 << 22;
  const int64_t nq = (max_rank + 3) / 4;
  for (int n = 0; n < pb.d; ++n) {
    const int L = (n == pb.d - 1) ? pb.d - 2 : pb.d - 1;
    const int64_t zrows = pb.size / pb.dims[L];
    if (nq * zrows >= kIdxLimit)
      return fail(NNC_EUNSUPPORTED,
                  "nnCP tensor of %lld entries at rank %d: %lld contraction items reach the 2^22 index limit",
                  (long long)pb.size, max_rank, (long long)(nq * zrows));
    if (pb.dims[n] * max_rank >= kIdxLimit)
      return fail(NNC_EUNSUPPORTED, "nnCP mode %d of length %lld at rank %d reaches the 2^22 index limit", n,
                  (long long)pb.dims[n], max_rank);
  }
  if (threads <= 0) threads = nncp_default_threads(pb, max_rank);
  if (threads > 1024 || threads % 64)
    return fail(NNC_EINVAL, "threads_per_fit must be a multiple of 64 <= 1024");
  const CpLayout L = cp_layout(pb, max_rank, threads, als);
  if (L.lds_bytes > kCpLdsBudget)
    return fail(NNC_EUNSUPPORTED, "nnCP working set %lld bytes exceeds the LDS budget",
                (long long)L.lds_bytes);
  return NNC_OK;
}

nnc_status launch_nncp(const float *T, const CpProblem &pb, int nbatch, const int *d_ranks,
                       int max_rank, float *const *d_factor_ptrs, float *const *single_ptrs,
                       int iters, double eps, double *d_resid, unsigned long long *clips,
                       float *zscratch, int threads, hipStream_t s, bool als, bool t_global) {
  NNC_TRY(nncp_check_shape(pb, max_rank, threads, als));
  if (threads <= 0) threads = nncp_default_threads(pb, max_rank);
  const CpLayout L = cp_layout(pb, max_rank, threads, als, t_global);
  if (L.lds_bytes > kCpLdsBudget)
    return fail(NNC_EUNSUPPORTED, "nnCP working set %lld bytes exceeds the LDS budget", (long long)L.lds_bytes);
  if (!L.a.z_lds && !zscratch) return fail(NNC_EWORKSPACE, "nnCP needs Z scratch in the workspace");
  CpPtrs p0;
  for (int k = 0; k < kMaxDim; ++k) p0.p[k] = (single_ptrs && k < pb.d) ? single_ptrs[k] : nullptr;
  const size_t lds = (size_t)L.lds_bytes;
  // Orders 2 to 5 have kernels of their own: with the order a constant, the loops over modes
  // unroll and their index bookkeeping folds away (300 sweeps of a 20^3 core at rank 10:
  // 4.3 -> 3.3 ms).
#define NNC_CP_LAUNCH3(RM, ALSV, DCV)                                                                  \
  do {                                                                                                 \
    NNC_TRY(allow_lds(reinterpret_cast<const void *>(nncp_k<RM, ALSV, DCV>), L.lds_bytes));            \
    hipLaunchKernelGGL((nncp_k<RM, ALSV, DCV>), dim3(nbatch), dim3(threads), lds, s, T, L.a, max_rank, \
                       p0, d_ranks, d_factor_ptrs, iters, eps, d_resid, clips, zscratch);              \
  } while (0)
#define NNC_CP_LAUNCH(RM, ALSV)                  \
  do {                                           \
    switch (pb.d) {                              \
      case 2: NNC_CP_LAUNCH3(RM, ALSV, 2); break; \
      case 3: NNC_CP_LAUNCH3(RM, ALSV, 3); break; \
      case 4: NNC_CP_LAUNCH3(RM, ALSV, 4); break; \
      case 5: NNC_CP_LAUNCH3(RM, ALSV, 5); break; \
      default: NNC_CP_LAUNCH3(RM, ALSV, 0);      \
    }                                            \
  } while (0)
  if (als) {
    if (max_rank <= 8)
      NNC_CP_LAUNCH(8, true);
    else if (max_rank <= 16)
      NNC_CP_LAUNCH(16, true);
    else
      NNC_CP_LAUNCH(32, true);
  } else {
    if (max_rank <= 8)
      NNC_CP_LAUNCH(8, false);
    else if (max_rank <= 16)
      NNC_CP_LAUNCH(16, false);
    else
      NNC_CP_LAUNCH(32, false);
  }
#undef NNC_CP_LAUNCH
#undef NNC_CP_LAUNCH3
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

}  // namespace nnc
