// Nonnegative CP of a small tensor (the Tucker core) by multiplicative updates, entirely
// inside one workgroup: the CP factors, their Grams and the update temporaries live in LDS;
// the tensor is read through the cache.  One workgroup per fit, so a launch can run many
// independent fits (random restarts, uneven ranks) at once, and every sweep of every fit
// happens inside that single launch.
//
// Sweep (factors 1..d in order):  M_n = MTTKRP(T, {B_k}_{k!=n}),  H_n = Hadamard_{k!=n} B_k^T B_k,
//   B_n <- B_n * M_n / max(B_n H_n, eps),  then B_n^T B_n is refreshed.
// MTTKRP by its definition: M_n[i, rho] = sum over entries with i_n = i of
// T[idx] * prod_{k!=n} B_k[i_k, rho].  Each (i, rho) pair is split over several threads that
// sum fixed index ranges; the partial sums are then added in a fixed order.
#include "nnc_internal.h"

namespace nnc {

struct CpPtrs {
  float *p[kMaxDim];
};

struct CpArgs {
  int d;
  int64_t dims[kMaxDim];
  int64_t size;
  int maxdim;
};

static __device__ inline float mu_cp(float x, float num, float den, double eps,
                                     unsigned long long *clips) {
  double dd = (double)den;
  if (dd < eps) {
    dd = eps;
    atomicAdd(clips, 1ull);
  }
  return (float)(((double)x * (double)num) / dd);
}

// LDS layout (floats): B_k (dims[k] x r) for every k | Gram_k (r x r) for every k | H (r x r)
//                      | M (maxdim x r) | part (blockDim)
__host__ __device__ inline int64_t cp_lds_floats(const CpArgs &a, int r, int threads) {
  int64_t s = 0;
  for (int k = 0; k < a.d; ++k) s += a.dims[k] * r;
  s += (int64_t)a.d * r * r + (int64_t)r * r + (int64_t)a.maxdim * r + threads;
  return s;
}

// A single fit passes its rank and factor pointers by value (ranks == nullptr); a batch
// passes device tables.
__global__ void nncp_k(const float *__restrict__ T, CpArgs a, int rank0, CpPtrs ptr0,
                       const int *__restrict__ ranks, float *const *__restrict__ fptrs, int iters,
                       double eps, double *__restrict__ resid, unsigned long long *clips) {
  extern __shared__ float sm[];
  const int b = blockIdx.x;
  const int r = ranks ? ranks[b] : rank0;
  float *const *Bg = ranks ? fptrs + (int64_t)b * a.d : ptr0.p;
  const int tid = threadIdx.x, nt = blockDim.x;
  float *Bs[kMaxDim];
  float *Wg[kMaxDim];
  float *p = sm;
  for (int k = 0; k < a.d; ++k) {
    Bs[k] = p;
    p += a.dims[k] * r;
  }
  for (int k = 0; k < a.d; ++k) {
    Wg[k] = p;
    p += r * r;
  }
  float *H = p;
  p += r * r;
  float *Mm = p;
  p += a.maxdim * r;
  float *part = p;

  for (int k = 0; k < a.d; ++k)
    for (int64_t e = tid; e < a.dims[k] * r; e += nt) Bs[k][e] = Bg[k][e];
  __syncthreads();
  for (int k = 0; k < a.d; ++k)
    for (int e = tid; e < r * r; e += nt) {
      const int x = e / r, y = e - (e / r) * r;
      float acc = 0.f;
      for (int64_t i = 0; i < a.dims[k]; ++i) acc = fmaf(Bs[k][i * r + x], Bs[k][i * r + y], acc);
      Wg[k][e] = acc;
    }
  __syncthreads();

  for (int it = 0; it < iters; ++it) {
    for (int n = 0; n < a.d; ++n) {
      const int64_t In = a.dims[n];
      const int64_t npairs = In * r;
      int64_t post = 1;
      for (int k = n + 1; k < a.d; ++k) post *= a.dims[k];
      const int64_t other = a.size / In;
      const int S = npairs >= nt ? 1 : (int)(nt / npairs);
      // ---- MTTKRP, split into S fixed index ranges per (i, rho)
      for (int64_t w = tid; w < npairs * S; w += nt) {
        const int64_t pr = w % npairs;
        const int s = (int)(w / npairs);
        const int64_t i = pr / r;
        const int rho = (int)(pr - i * r);
        const int64_t o0 = other * s / S, o1 = other * (s + 1) / S;
        // decode o0 into the other indices (odometer, modes != n, last fastest)
        int64_t idx[kMaxDim];
        int64_t rem = o0;
        for (int k = a.d - 1; k >= 0; --k) {
          if (k == n) {
            idx[k] = i;
            continue;
          }
          idx[k] = rem % a.dims[k];
          rem /= a.dims[k];
        }
        float acc = 0.f;
        for (int64_t o = o0; o < o1; ++o) {
          const int64_t pre = o / post, q = o - (o / post) * post;
          float prod = T[(pre * In + i) * post + q];
          for (int k = 0; k < a.d; ++k)
            if (k != n) prod *= Bs[k][idx[k] * r + rho];
          acc += prod;
          for (int k = a.d - 1; k >= 0; --k) {  // advance the odometer
            if (k == n) continue;
            if (++idx[k] < a.dims[k]) break;
            idx[k] = 0;
          }
        }
        if (S == 1)
          Mm[pr] = acc;
        else
          part[w] = acc;
      }
      __syncthreads();
      if (S > 1) {
        for (int64_t pr = tid; pr < npairs; pr += nt) {
          float acc = 0.f;
          for (int s = 0; s < S; ++s) acc += part[s * npairs + pr];
          Mm[pr] = acc;
        }
      }
      // ---- H = Hadamard product of the other Grams
      for (int e = tid; e < r * r; e += nt) {
        float h = 1.f;
        for (int k = 0; k < a.d; ++k)
          if (k != n) h *= Wg[k][e];
        H[e] = h;
      }
      __syncthreads();
      // ---- B_n <- B_n * M / max(B_n H, eps)   (read phase, barrier, write phase)
      float nv[4];
      int cnt = 0;
      for (int64_t e = tid; e < npairs; e += nt) {
        const int64_t i = e / r;
        const int c = (int)(e - i * r);
        float den = 0.f;
        for (int s = 0; s < r; ++s) den = fmaf(Bs[n][i * r + s], H[s * r + c], den);
        const float v = mu_cp(Bs[n][e], Mm[e], den, eps, clips);
        if (cnt < 4) nv[cnt] = v;
        else part[e] = v;
        ++cnt;
      }
      __syncthreads();
      cnt = 0;
      for (int64_t e = tid; e < npairs; e += nt) {
        Bs[n][e] = cnt < 4 ? nv[cnt] : part[e];
        ++cnt;
      }
      __syncthreads();
      // ---- Gram of the new B_n
      for (int e = tid; e < r * r; e += nt) {
        const int x = e / r, y = e - (e / r) * r;
        float acc = 0.f;
        for (int64_t i = 0; i < In; ++i) acc = fmaf(Bs[n][i * r + x], Bs[n][i * r + y], acc);
        Wg[n][e] = acc;
      }
      __syncthreads();
    }
  }
  for (int k = 0; k < a.d; ++k)
    for (int64_t e = tid; e < a.dims[k] * r; e += nt) Bg[k][e] = Bs[k][e];

  // relative residual ||T - cp(B)|| / ||T||, double accumulation, fixed tree
  if (resid) {
    double sr = 0.0, sx = 0.0;
    for (int64_t e = tid; e < a.size; e += nt) {
      int64_t rem = e;
      int64_t idx[kMaxDim];
      for (int k = a.d - 1; k >= 0; --k) {
        idx[k] = rem % a.dims[k];
        rem /= a.dims[k];
      }
      float xh = 0.f;
      for (int rho = 0; rho < r; ++rho) {
        float pp = 1.f;
        for (int k = 0; k < a.d; ++k) pp *= Bs[k][idx[k] * r + rho];
        xh += pp;
      }
      const double x = T[e];
      const double df = x - (double)xh;
      sr += df * df;
      sx += x * x;
    }
    __shared__ double red[1024];
    red[tid] = sr;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
      if (tid < w && tid + w < nt) red[tid] += red[tid + w];
      __syncthreads();
    }
    const double tr = red[0];
    __syncthreads();
    red[tid] = sx;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
      if (tid < w && tid + w < nt) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) resid[b] = red[0] > 0.0 ? sqrt(tr / red[0]) : 0.0;
  }
}

int nncp_default_threads(const CpProblem &pb, int max_rank) {
  int64_t maxpairs = 0;
  for (int k = 0; k < pb.d; ++k) maxpairs = pb.dims[k] * max_rank > maxpairs ? pb.dims[k] * max_rank : maxpairs;
  // enough threads to give every (i, rho) pair a few slices of the index range
  if (pb.size * max_rank >= 1 << 16) return 1024;
  if (maxpairs * 4 >= 512) return 512;
  return 256;
}

static CpArgs make_args(const CpProblem &pb) {
  CpArgs a;
  a.d = pb.d;
  a.size = pb.size;
  a.maxdim = 0;
  for (int k = 0; k < pb.d; ++k) {
    a.dims[k] = pb.dims[k];
    if (pb.dims[k] > a.maxdim) a.maxdim = (int)pb.dims[k];
  }
  return a;
}

// LDS of one fit: the layout above, with `part` holding max(threads, maxdim * r) floats
// (MTTKRP partial sums need at most `threads`; the update may park up to maxdim * r values).
int64_t nncp_lds_bytes(const CpProblem &pb, int max_rank, int threads) {
  const CpArgs a = make_args(pb);
  int64_t part = threads;
  if ((int64_t)a.maxdim * max_rank > part) part = (int64_t)a.maxdim * max_rank;
  return (cp_lds_floats(a, max_rank, 0) + part) * (int64_t)sizeof(float);
}

// Dynamic LDS per fit the nnCP kernel may request (the static reduction array adds 8 KiB).
constexpr int64_t kCpLdsBudget = 56 * 1024;

nnc_status launch_nncp(const float *T, const CpProblem &pb, int nbatch, const int *d_ranks,
                       int max_rank, float *const *d_factor_ptrs, float *const *single_ptrs,
                       int iters, double eps, double *d_resid, unsigned long long *clips,
                       int threads, hipStream_t s) {
  const CpArgs a = make_args(pb);
  if (threads <= 0) threads = nncp_default_threads(pb, max_rank);
  if (threads > 1024 || threads % 64)
    return fail(NNC_EINVAL, "threads_per_fit must be a multiple of 64 <= 1024");
  const int64_t lds = nncp_lds_bytes(pb, max_rank, threads);
  if (lds > kCpLdsBudget)
    return fail(NNC_EUNSUPPORTED, "nnCP working set %lld bytes exceeds the LDS budget",
                (long long)lds);
  CpPtrs p0;
  for (int k = 0; k < kMaxDim; ++k) p0.p[k] = (single_ptrs && k < pb.d) ? single_ptrs[k] : nullptr;
  hipLaunchKernelGGL(nncp_k, dim3(nbatch), dim3(threads), (size_t)lds, s, T, a, max_rank, p0, d_ranks,
                     d_factor_ptrs, iters, eps, d_resid, clips);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

}  // namespace nnc
