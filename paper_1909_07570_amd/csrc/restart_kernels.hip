// Many complete nnCANDELINC fits of one small 3-way tensor from different random starts,
// one workgroup (one wave) per start with everything in LDS: the study of Section 4.2, which
// runs Algorithms 1 and 2 a thousand times on the 4x4x4 example with known nnCPD at several
// assumed multiranks and compares the distributions of relative error and mean congruence.
//
//   Algorithm 1: nnTucker (multirank m) by the blockwise multiplicative rule, nnCP of the
//                core (rank r), lift C_n = A_n B_n.
//   Algorithm 2: nnCP of X (rank r), NMF of each CP factor A_n ~ W_n H_n (m_n columns),
//                lift C_n = W_n H_n.
// Each fit runs a fixed number of sweeps.  Then ||X - cp(C)|| / ||X|| (FP64 sums) and, when
// the true factors are given, the mean congruence of the r rank-one terms of cp(C) with the
// true ones under the component matching that maximises it (Section 4.1 scoring).
//
// Every dimension, multirank and rank is <= kTinyDim.  An NMF is the CP of the (N, r, 1)
// tensor A with factors W, H^T and a fixed all-ones third factor (two-way Lee-Seung rule).
#include <string.h>

#include "nnc_internal.h"

namespace nnc {

constexpr int kTinyDim = 8;
constexpr int kTinyThreads = 64;
constexpr int kTinyCube = kTinyDim * kTinyDim * kTinyDim;
constexpr int kTinySq = kTinyDim * kTinyDim;

struct TinyArgs {
  const float *X;
  int N[3], M[3], r, alg, nres;
  int outer, inner;       // sweeps of the first (nnTucker / nnCP of X) and second fit
  const float *inits;     // per start, see tiny_init_floats()
  int64_t init_stride;    // floats per start
  const float *truth[3];  // N_n x r true factors, or null (no congruence)
  double eps;
  double *rel, *cong;     // [nres]
  float *fout;            // lifted factors of every start (nullable): [nres][N0 + N1 + N2][r]
  unsigned long long *clips;
};

struct TinyLds {
  float X[kTinyCube], G[kTinyCube], T0[kTinyCube], T1[kTinyCube], T2[kTinyCube];
  float A[3][kTinySq], B[3][kTinySq], E[3][kTinySq], S[3][kTinySq], C[3][kTinySq];
  float ones[kTinySq];  // Gram of the all-ones third factor of an NMF
  float num[kTinySq], Mm[kTinySq], cg[kTinySq];
  double red[2][kTinyThreads];
};

struct TinyCtx {
  int lane;
  double eps;
  unsigned int clips;
};

static __device__ inline void tsync() { __syncthreads(); }

static __device__ inline float tiny_mu(TinyCtx &c, float x, float num, float den) {
  double dd = (double)den;
  if (dd < c.eps) {
    dd = c.eps;
    ++c.clips;
  }
  return (float)(((double)x * (double)num) / dd);
}

static __device__ inline int lin3(const int *d, int i0, int i1, int i2) { return (i0 * d[1] + i1) * d[2] + i2; }

// out = in with mode n contracted against F (L x C, row-major):
//   out[.., c, ..] = sum_l in[.., l, ..] F[l][c]     (in: sizes d, out: sizes d with d[n] = C)
static __device__ void tiny_ttm(const TinyCtx &c, const float *in, const int *d, int n, const float *F, int C,
                                float *out) {
  int od[3] = {d[0], d[1], d[2]};
  od[n] = C;
  const int total = od[0] * od[1] * od[2];
  for (int o = c.lane; o < total; o += kTinyThreads) {
    int idx[3] = {o / (od[1] * od[2]), (o / od[2]) % od[1], o % od[2]};
    const int cc = idx[n];
    float s = 0.f;
    for (int l = 0; l < d[n]; ++l) {
      idx[n] = l;
      s = fmaf(in[lin3(d, idx[0], idx[1], idx[2])], F[l * C + cc], s);
    }
    out[o] = s;
  }
  tsync();
}

// out[i][a] = sum over the other two modes of U[.., i, ..] V[.., a, ..]; U has sizes ud and
// V the same sizes except Nv in mode n; out is ud[n] x Nv.
static __device__ void tiny_contract_except(const TinyCtx &c, const float *U, const int *ud, const float *V,
                                            int Nv, int n, float *out) {
  int vd[3] = {ud[0], ud[1], ud[2]};
  vd[n] = Nv;
  const int p = n == 0 ? 1 : 0, q = n == 2 ? 1 : 2;
  for (int o = c.lane; o < ud[n] * Nv; o += kTinyThreads) {
    const int i = o / Nv, a = o % Nv;
    float s = 0.f;
    for (int x = 0; x < ud[p]; ++x)
      for (int y = 0; y < ud[q]; ++y) {
        int ju[3], jv[3];
        ju[n] = i;
        jv[n] = a;
        ju[p] = jv[p] = x;
        ju[q] = jv[q] = y;
        s = fmaf(U[lin3(ud, ju[0], ju[1], ju[2])], V[lin3(vd, jv[0], jv[1], jv[2])], s);
      }
    out[o] = s;
  }
  tsync();
}

static __device__ void tiny_gram(const TinyCtx &c, const float *A, int N, int R, float *S) {
  for (int o = c.lane; o < R * R; o += kTinyThreads) {
    const int a = o / R, b = o % R;
    float s = 0.f;
    for (int i = 0; i < N; ++i) s = fmaf(A[i * R + a], A[i * R + b], s);
    S[o] = s;
  }
  tsync();
}

// A (N x R) <- A * num / max(A Mm, eps), Mm R x R.
static __device__ void tiny_update(TinyCtx &c, float *A, const float *num, const float *Mm, int N, int R) {
  constexpr int kU = kTinySq / kTinyThreads;
  float nv[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int o = c.lane + u * kTinyThreads;
    nv[u] = 0.f;
    if (o < N * R) {
      const int i = o / R, b = o % R;
      float dn = 0.f;
      for (int a = 0; a < R; ++a) dn = fmaf(A[i * R + a], Mm[a * R + b], dn);
      nv[u] = tiny_mu(c, A[o], num[o], dn);
    }
  }
  tsync();
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int o = c.lane + u * kTinyThreads;
    if (o < N * R) A[o] = nv[u];
  }
  tsync();
}

// One sweep of the blockwise nnTucker rule: factors 0, 1, 2, then the core.
static __device__ void tiny_tucker_sweep(TinyCtx &c, TinyLds &L, const int *N, const int *M) {
  for (int n = 0; n < 3; ++n) {
    const int k1 = n == 0 ? 1 : 0, k2 = n == 2 ? 1 : 2;
    int d[3] = {N[0], N[1], N[2]};
    tiny_ttm(c, L.X, d, k1, L.A[k1], M[k1], L.T0);  // X x_{k != n} A_k^T
    d[k1] = M[k1];
    tiny_ttm(c, L.T0, d, k2, L.A[k2], M[k2], L.T1);
    d[k2] = M[k2];
    tiny_contract_except(c, L.T1, d, L.G, M[n], n, L.num);  // num_n: N_n x M_n
    const int g[3] = {M[0], M[1], M[2]};
    tiny_ttm(c, L.G, g, k1, L.S[k1], M[k1], L.T0);  // G x_{k != n} S_k
    tiny_ttm(c, L.T0, g, k2, L.S[k2], M[k2], L.T1);
    tiny_contract_except(c, L.T1, g, L.G, M[n], n, L.Mm);  // M_n x M_n
    tiny_update(c, L.A[n], L.num, L.Mm, N[n], M[n]);
    tiny_gram(c, L.A[n], N[n], M[n], L.S[n]);
  }
  int d[3] = {N[0], N[1], N[2]};
  tiny_ttm(c, L.X, d, 0, L.A[0], M[0], L.T0);  // X x_0 A_0^T x_1 A_1^T x_2 A_2^T
  d[0] = M[0];
  tiny_ttm(c, L.T0, d, 1, L.A[1], M[1], L.T1);
  d[1] = M[1];
  tiny_ttm(c, L.T1, d, 2, L.A[2], M[2], L.T2);  // numerator in T2
  const int g[3] = {M[0], M[1], M[2]};
  tiny_ttm(c, L.G, g, 0, L.S[0], M[0], L.T0);  // G x_0 S_0 x_1 S_1 x_2 S_2
  tiny_ttm(c, L.T0, g, 1, L.S[1], M[1], L.T1);
  tiny_ttm(c, L.T1, g, 2, L.S[2], M[2], L.T0);  // denominator in T0
  const int gs = M[0] * M[1] * M[2];
  for (int o = c.lane; o < gs; o += kTinyThreads) L.G[o] = tiny_mu(c, L.G[o], L.T2[o], L.T0[o]);
  tsync();
}

// One sweep of the CP rule on the 3-way tensor T (sizes d) with factors F[n] (d[n] x r) and
// Grams S[n]; modes with upd[n] == 0 keep their factor.
static __device__ void tiny_cp_sweep(TinyCtx &c, TinyLds &L, const float *T, const int *d, float *const *F,
                                     float *const *S, const int *upd, int r) {
  for (int n = 0; n < 3; ++n) {
    if (!upd[n]) continue;
    const int p = n == 0 ? 1 : 0, q = n == 2 ? 1 : 2;
    for (int o = c.lane; o < d[n] * r; o += kTinyThreads) {  // MTTKRP
      const int i = o / r, rho = o % r;
      float s = 0.f;
      for (int x = 0; x < d[p]; ++x)
        for (int y = 0; y < d[q]; ++y) {
          int j[3];
          j[n] = i;
          j[p] = x;
          j[q] = y;
          s = fmaf(T[lin3(d, j[0], j[1], j[2])], F[p][x * r + rho] * F[q][y * r + rho], s);
        }
      L.num[o] = s;
    }
    for (int o = c.lane; o < r * r; o += kTinyThreads) L.Mm[o] = S[p][o] * S[q][o];  // H_n
    tsync();
    tiny_update(c, F[n], L.num, L.Mm, d[n], r);
    tiny_gram(c, F[n], d[n], r, S[n]);
  }
}

// C = P Q (P: N x K, Q: K x r, or Q^T given as r x K when qt).
static __device__ void tiny_lift(const TinyCtx &c, const float *P, const float *Q, int N, int K, int r, int qt,
                                 float *C) {
  for (int o = c.lane; o < N * r; o += kTinyThreads) {
    const int i = o / r, rho = o % r;
    float s = 0.f;
    for (int k = 0; k < K; ++k) s = fmaf(P[i * K + k], qt ? Q[rho * K + k] : Q[k * r + rho], s);
    C[o] = s;
  }
  tsync();
}

__global__ __launch_bounds__(kTinyThreads) void tiny_candelinc_k(TinyArgs a) {
  __shared__ TinyLds L;
  const int start = blockIdx.x;
  TinyCtx c{(int)threadIdx.x, a.eps, 0u};
  const int *N = a.N, *M = a.M;
  const int r = a.r;
  const int xs = N[0] * N[1] * N[2];
  for (int o = c.lane; o < xs; o += kTinyThreads) L.X[o] = a.X[o];
  for (int o = c.lane; o < kTinySq; o += kTinyThreads) L.ones[o] = 1.f;
  const float *in = a.inits + (int64_t)start * a.init_stride;
  // initial values, laid out as documented for tiny_init_floats()
  if (a.alg == 1) {
    for (int n = 0; n < 3; ++n) {
      for (int o = c.lane; o < N[n] * M[n]; o += kTinyThreads) L.A[n][o] = in[o];
      in += N[n] * M[n];
    }
    for (int o = c.lane; o < M[0] * M[1] * M[2]; o += kTinyThreads) L.G[o] = in[o];
    in += M[0] * M[1] * M[2];
    for (int n = 0; n < 3; ++n) {
      for (int o = c.lane; o < M[n] * r; o += kTinyThreads) L.B[n][o] = in[o];
      in += M[n] * r;
    }
  } else {
    for (int n = 0; n < 3; ++n) {
      for (int o = c.lane; o < N[n] * r; o += kTinyThreads) L.A[n][o] = in[o];
      in += N[n] * r;
    }
    for (int n = 0; n < 3; ++n) {
      for (int o = c.lane; o < N[n] * M[n]; o += kTinyThreads) L.B[n][o] = in[o];
      in += N[n] * M[n];
    }
    for (int n = 0; n < 3; ++n) {  // H_n (M_n x r) stored transposed as the CP factor H^T
      for (int o = c.lane; o < M[n] * r; o += kTinyThreads) L.E[n][(o % r) * M[n] + o / r] = in[o];
      in += M[n] * r;
    }
  }
  tsync();
  if (a.alg == 1) {
    for (int n = 0; n < 3; ++n) tiny_gram(c, L.A[n], N[n], M[n], L.S[n]);
    for (int t = 0; t < a.outer; ++t) tiny_tucker_sweep(c, L, N, M);
    // nnCP of the core
    float *F[3] = {L.B[0], L.B[1], L.B[2]};
    float *S[3] = {L.S[0], L.S[1], L.S[2]};
    const int upd[3] = {1, 1, 1};
    for (int n = 0; n < 3; ++n) tiny_gram(c, L.B[n], M[n], r, L.S[n]);
    for (int t = 0; t < a.inner; ++t) tiny_cp_sweep(c, L, L.G, M, F, S, upd, r);
    for (int n = 0; n < 3; ++n) tiny_lift(c, L.A[n], L.B[n], N[n], M[n], r, 0, L.C[n]);
  } else {
    float *F[3] = {L.A[0], L.A[1], L.A[2]};
    float *S[3] = {L.S[0], L.S[1], L.S[2]};
    const int upd[3] = {1, 1, 1};
    for (int n = 0; n < 3; ++n) tiny_gram(c, L.A[n], N[n], r, L.S[n]);
    for (int t = 0; t < a.outer; ++t) tiny_cp_sweep(c, L, L.X, N, F, S, upd, r);
    for (int n = 0; n < 3; ++n) {  // NMF A_n ~ W_n H_n: CP of (N_n, r, 1) with W, H^T, ones
      const int dn[3] = {N[n], r, 1};
      float *Fn[3] = {L.B[n], L.E[n], L.ones};
      float *Sn[3] = {L.S[0], L.S[1], L.S[2]};
      const int un[3] = {1, 1, 0};
      for (int o = c.lane; o < M[n] * M[n]; o += kTinyThreads) L.S[2][o] = 1.f;  // Gram of ones
      tsync();
      tiny_gram(c, L.B[n], N[n], M[n], L.S[0]);
      tiny_gram(c, L.E[n], r, M[n], L.S[1]);
      for (int t = 0; t < a.inner; ++t) tiny_cp_sweep(c, L, L.A[n], dn, Fn, Sn, un, M[n]);
      tiny_lift(c, L.B[n], L.E[n], N[n], M[n], r, 1, L.C[n]);
    }
  }
  // relative error of cp(C), FP64 sums
  double se = 0.0, sx = 0.0;
  for (int o = c.lane; o < xs; o += kTinyThreads) {
    const int i = o / (N[1] * N[2]), j = (o / N[2]) % N[1], k = o % N[2];
    float xh = 0.f;
    for (int rho = 0; rho < r; ++rho) xh = fmaf(L.C[0][i * r + rho] * L.C[1][j * r + rho], L.C[2][k * r + rho], xh);
    const double dl = (double)L.X[o] - (double)xh;
    se += dl * dl;
    sx += (double)L.X[o] * (double)L.X[o];
  }
  L.red[0][c.lane] = se;
  L.red[1][c.lane] = sx;
  // congruence of component rho with true component sigma: product over modes of cosines
  if (a.truth[0]) {
    for (int o = c.lane; o < r * r; o += kTinyThreads) {
      const int rho = o / r, sg = o % r;
      double prod = 1.0;
      for (int n = 0; n < 3; ++n) {
        double dot = 0.0, n1 = 0.0, n2 = 0.0;
        for (int i = 0; i < N[n]; ++i) {
          const double u = L.C[n][i * r + rho], v = a.truth[n][i * r + sg];
          dot += u * v;
          n1 += u * u;
          n2 += v * v;
        }
        prod *= (n1 > 0 && n2 > 0) ? dot / sqrt(n1 * n2) : 0.0;
      }
      L.cg[o] = (float)prod;
    }
  }
  tsync();
  if (c.lane == 0) {
    double e = 0.0, x = 0.0;
    for (int l = 0; l < kTinyThreads; ++l) {
      e += L.red[0][l];
      x += L.red[1][l];
    }
    a.rel[start] = x > 0 ? sqrt(e / x) : 0.0;
  }
  tsync();  // the residual sums are read before red[] is reused
  if (a.truth[0]) {  // best matching: every permutation of r components, lanes in turn
    int nperm = 1;
    for (int k = 2; k <= r; ++k) nperm *= k;
    double best = -1e300;
    for (int pidx = c.lane; pidx < nperm; pidx += kTinyThreads) {
      int avail[kTinyDim];
      for (int k = 0; k < r; ++k) avail[k] = k;
      int code = pidx, left = r;
      double s = 0.0;
      for (int rho = 0; rho < r; ++rho) {  // factorial-base digits pick the unused targets
        int f = 1;
        for (int k = 2; k < left; ++k) f *= k;
        const int dgt = code / f;
        code -= dgt * f;
        s += L.cg[rho * r + avail[dgt]];
        for (int k = dgt; k < left - 1; ++k) avail[k] = avail[k + 1];
        --left;
      }
      best = fmax(best, s / r);
    }
    L.red[0][c.lane] = best;
    tsync();
    if (c.lane == 0) {
      double b = -1e300;
      for (int l = 0; l < kTinyThreads; ++l) b = fmax(b, L.red[0][l]);
      a.cong[start] = b;
    }
  }
  if (a.fout) {
    float *out = a.fout + (int64_t)start * (N[0] + N[1] + N[2]) * r;
    for (int n = 0; n < 3; ++n) {
      for (int o = c.lane; o < N[n] * r; o += kTinyThreads) out[o] = L.C[n][o];
      out += N[n] * r;
    }
  }
  if (c.clips && a.clips) atomicAdd(a.clips, (unsigned long long)c.clips);
}

int64_t tiny_init_floats(int alg, const int *N, const int *M, int r) {
  int64_t s = 0;
  if (alg == 1) {
    for (int n = 0; n < 3; ++n) s += (int64_t)N[n] * M[n] + (int64_t)M[n] * r;
    s += (int64_t)M[0] * M[1] * M[2];
  } else {
    for (int n = 0; n < 3; ++n) s += (int64_t)N[n] * r + (int64_t)N[n] * M[n] + (int64_t)M[n] * r;
  }
  return s;
}

nnc_status launch_tiny_candelinc(const float *X, const int *N, const int *M, int r, int alg, int nres,
                                 int outer, int inner, const float *inits, const float *const *truth,
                                 double eps, double *rel, double *cong, float *fout,
                                 unsigned long long *clips, hipStream_t s) {
  TinyArgs a;
  memset(&a, 0, sizeof a);
  a.X = X;
  for (int n = 0; n < 3; ++n) {
    a.N[n] = N[n];
    a.M[n] = M[n];
    a.truth[n] = truth ? truth[n] : nullptr;
  }
  a.r = r;
  a.alg = alg;
  a.nres = nres;
  a.outer = outer;
  a.inner = inner;
  a.inits = inits;
  a.init_stride = tiny_init_floats(alg, N, M, r);
  a.eps = eps;
  a.rel = rel;
  a.cong = cong;
  a.fout = fout;
  a.clips = clips;
  hipLaunchKernelGGL(tiny_candelinc_k, dim3(nres), dim3(kTinyThreads), 0, s, a);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

}  // namespace nnc

namespace nnc {

// Mean congruence of two rank-r CP models with factors P[n], Q[n] (dims[n] x r): the
// congruence of components rho and sigma is the product over modes of the cosines of their
// factor columns (FP64), and the score is the largest mean over the matchings of components
// (every permutation).  One workgroup; a zero column has cosine 0.
struct CongArgs {
  int d, r;
  int64_t dims[kMaxDim];
  const float *P[kMaxDim], *Q[kMaxDim];
  double *out;
};

__global__ __launch_bounds__(256) void congruence_k(CongArgs a) {
  __shared__ double cg[kTinyDim * kTinyDim];
  __shared__ double best[256];
  const int tid = threadIdx.x, r = a.r;
  if (tid < r * r) {
    const int rho = tid / r, sg = tid % r;
    double prod = 1.0;
    for (int n = 0; n < a.d; ++n) {
      double dot = 0.0, n1 = 0.0, n2 = 0.0;
      for (int64_t i = 0; i < a.dims[n]; ++i) {
        const double u = a.P[n][i * r + rho], v = a.Q[n][i * r + sg];
        dot += u * v;
        n1 += u * u;
        n2 += v * v;
      }
      prod *= (n1 > 0 && n2 > 0) ? dot / sqrt(n1 * n2) : 0.0;
    }
    cg[tid] = prod;
  }
  __syncthreads();
  int nperm = 1;
  for (int k = 2; k <= r; ++k) nperm *= k;
  double b = -1e300;
  for (int pidx = tid; pidx < nperm; pidx += 256) {
    int avail[kTinyDim];
    for (int k = 0; k < r; ++k) avail[k] = k;
    int code = pidx, left = r;
    double s = 0.0;
    for (int rho = 0; rho < r; ++rho) {  // factorial-base digits pick the unused targets
      int f = 1;
      for (int k = 2; k < left; ++k) f *= k;
      const int dgt = code / f;
      code -= dgt * f;
      s += cg[rho * r + avail[dgt]];
      for (int k = dgt; k < left - 1; ++k) avail[k] = avail[k + 1];
      --left;
    }
    b = fmax(b, s / r);
  }
  best[tid] = b;
  __syncthreads();
  if (tid == 0) {
    double m = -1e300;
    for (int t = 0; t < 256; ++t) m = fmax(m, best[t]);
    *a.out = m;
  }
}

nnc_status launch_congruence(int d, const int64_t *dims, int r, const float *const *P, const float *const *Q,
                             double *out, hipStream_t s) {
  CongArgs a;
  memset(&a, 0, sizeof a);
  a.d = d;
  a.r = r;
  for (int n = 0; n < d; ++n) {
    a.dims[n] = dims[n];
    a.P[n] = P[n];
    a.Q[n] = Q[n];
  }
  a.out = out;
  hipLaunchKernelGGL(congruence_k, dim3(1), dim3(256), 0, s, a);
  NNC_HIP(hipGetLastError());
  return NNC_OK;
}

}  // namespace nnc
