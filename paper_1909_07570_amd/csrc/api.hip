// C ABI of the library: argument validation (before any HIP call), workspace planning,
// the sweep schedule of the nonnegative Tucker multiplicative updates, the nnCP / lift /
// residual / adjoint entry points.
//
// Sweep schedule (d modes, factors 0..d-1 updated in order, then the core):
//   pass 1: P = X x_{d-1} A_{d-1}^T                     (streams X; contraction index contiguous)
//   for n < d-1:  Y_n = P x_{k<n} A_k^T(new) x_{n<k<d-1} A_k^T(old); update A_n
//           (A_{d-1} has not changed yet, so P serves every one of these modes; the prefix
//            P x_0 A_0^T ... x_{n-1} A_{n-1}^T is kept and extended mode by mode)
//   pass 2: T = X x_0 A_0^T(new)                          (streams X; contraction index strided)
//           Y_{d-1} = T x_1 A_1^T ... x_{d-2} A_{d-2}^T;  update A_{d-1}
//   core:   num_G = Y_{d-1} x_{d-1} A_{d-1}^T(new),  den_G = G x_k A_k^T A_k;  update G
// By the commutativity of mode products (Appendix A) every Y_n equals X x_{k!=n} A_k^T with
// the Gauss-Seidel factors, so two passes over X per sweep suffice for any d.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "nnc_internal.h"

namespace nnc {

static thread_local std::string g_err = "no error";
static int g_timing = 0;

nnc_status fail(nnc_status st, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

static int64_t prod(const int64_t *a, int lo, int hi) {
  int64_t p = 1;
  for (int k = lo; k < hi; ++k) p *= a[k];
  return p;
}

static nnc_status check_dims(int ndim, const int64_t *dims, const char *what) {
  if (ndim < 2 || ndim > kMaxDim) return fail(NNC_EINVAL, "ndim %d outside [2, %d]", ndim, kMaxDim);
  if (!dims) return fail(NNC_EINVAL, "%s is NULL", what);
  double p = 1.0;
  for (int k = 0; k < ndim; ++k) {
    if (dims[k] < 1) return fail(NNC_EINVAL, "%s[%d] = %lld < 1", what, k, (long long)dims[k]);
    p *= (double)dims[k];
  }
  if (p > 4.0e18) return fail(NNC_EINVAL, "%s: element count overflows", what);
  return NNC_OK;
}

static nnc_status check_ptrs(const void *const *ptrs, int n, const char *what) {
  if (!ptrs) return fail(NNC_EINVAL, "%s is NULL", what);
  for (int k = 0; k < n; ++k)
    if (!ptrs[k]) return fail(NNC_EINVAL, "%s[%d] is NULL", what, k);
  return NNC_OK;
}

// ------------------------------------------------------------------ static scratch
// Scratch of the entry point that allocates nothing (nncp_fit_noalloc).  In host code the
// name `scratch` is only a stand-in for the symbol: its device address is looked up once
// per device, with that device current, and only that address is passed to kernels.  Every
// call on one device shares that device's copy, so calls that overlap on a device race.
constexpr size_t kStaticScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static char *g_scratch_ptr[kMaxDevices];

static nnc_status static_scratch(char **out) {
  int dev = -1;
  NNC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(NNC_EUNSUPPORTED, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(NNC_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = (char *)p;
  }
  *out = g_scratch_ptr[dev];
  return NNC_OK;
}

// ------------------------------------------------------------------ workspace layout
struct Layout {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  }
};

struct TuckerPlan {
  int d = 0;
  int64_t N[kMaxDim], R[kMaxDim];
  int64_t size = 0, gsize = 0;
  int64_t nP = 0, nT = 0, nU = 0, nC = 0, nY = 0, nNum = 0, nS = 0, nM = 0, nGp = 0, nGr = 0, nNp = 0;
  bool fast = false;  // every multirank <= 32: fused small-step kernels
  size_t oP, oT, oU0, oU1, oC0, oC1, oY, oNum, oDen, oS, oM, oG0, oG1, oG2, oG3, oGp, oGr, oNp, oClip,
      oFlag, oTicket, oRed, oPart, oLsT, oLsL, oLsS, total;
};

static void grow(int64_t &v, int64_t x) {
  if (x > v) v = x;
}

// Sizes of every intermediate of the schedule above (and of the residual's expansion
// G x_0 A_0 ... x_{d-2} A_{d-2}), so that the same code paths fit in the buffers.
static TuckerPlan plan_tucker(int d, const int64_t *dims, const int64_t *rk) {
  TuckerPlan p;
  p.d = d;
  for (int k = 0; k < d; ++k) {
    p.N[k] = dims[k];
    p.R[k] = rk[k];
  }
  p.size = prod(p.N, 0, d);
  p.gsize = prod(p.R, 0, d);
  p.nP = p.size / p.N[d - 1] * p.R[d - 1];
  p.nT = p.size / p.N[0] * p.R[0];
  int64_t cur[kMaxDim];
  for (int n = 0; n < d - 1; ++n) {
    // U_n = P x_{k<n} A_k^T : dims R_0..R_{n-1}, N_n..N_{d-2}, R_{d-1}
    for (int k = 0; k < d; ++k) cur[k] = (k < n || k == d - 1) ? p.R[k] : p.N[k];
    if (n >= 1) grow(p.nU, prod(cur, 0, d));
    for (int k = n + 1; k < d - 1; ++k) {
      cur[k] = p.R[k];
      if (k < d - 2) grow(p.nC, prod(cur, 0, d));
    }
  }
  for (int k = 0; k < d; ++k) cur[k] = (k == 0) ? p.R[0] : p.N[k];
  for (int k = 1; k < d - 1; ++k) {
    cur[k] = p.R[k];
    if (k < d - 2) grow(p.nC, prod(cur, 0, d));
  }
  for (int k = 0; k < d; ++k) cur[k] = p.R[k];
  for (int k = 0; k < d - 1; ++k) {
    cur[k] = p.N[k];
    if (k < d - 2) grow(p.nC, prod(cur, 0, d));
  }
  for (int n = 0; n < d; ++n) {
    grow(p.nY, p.gsize / p.R[n] * p.N[n]);
    grow(p.nNum, p.N[n] * p.R[n]);
    grow(p.nNp, mu_rows_split_floats(p.N[n], p.R[n]));
    grow(p.nM, p.R[n] * p.R[n]);
    p.nS += p.R[n] * p.R[n];
  }
  p.fast = true;
  for (int n = 0; n < d; ++n)
    if (p.R[n] > 32) p.fast = false;
  p.nGp = mu_rows_blocks(p.N[d - 1]) * p.gsize;
  for (int n = 0; n < d; ++n) grow(p.nGr, mu_rows_blocks(p.N[n]) * p.R[n] * p.R[n]);
  p.nGr *= d;  // the prologue keeps the partials of every factor
  Layout L;
  p.oP = L.take(sizeof(float) * p.nP);
  p.oT = L.take(sizeof(float) * p.nT);
  p.oU0 = L.take(sizeof(float) * p.nU);
  p.oU1 = L.take(sizeof(float) * p.nU);
  p.oC0 = L.take(sizeof(float) * p.nC);
  p.oC1 = L.take(sizeof(float) * p.nC);
  p.oY = L.take(sizeof(float) * p.nY);
  p.oNum = L.take(sizeof(float) * p.nNum);
  p.oDen = L.take(sizeof(float) * p.nNum);
  p.oS = L.take(sizeof(float) * p.nS);
  p.oM = L.take(sizeof(float) * p.nM);
  p.oG0 = L.take(sizeof(float) * p.gsize);
  p.oG1 = L.take(sizeof(float) * p.gsize);
  p.oG2 = L.take(sizeof(float) * p.gsize);
  p.oG3 = L.take(sizeof(float) * p.gsize);
  p.oGp = L.take(sizeof(float) * p.nGp);
  p.oGr = L.take(sizeof(float) * p.nGr);
  p.oNp = L.take(sizeof(float) * p.nNp);
  p.oClip = L.take(sizeof(unsigned long long));
  p.oFlag = L.take(sizeof(unsigned int));
  p.oTicket = L.take(sizeof(unsigned int));
  p.oRed = L.take(2 * sizeof(double));
  p.oPart = L.take(2 * sizeof(double) * resid_stream_max_blocks());
  p.oLsT = L.take(sizeof(double) * 32 * 32);         // the real-valued fit's R x R transform,
  p.oLsL = L.take(sizeof(float) * 32 * 32);          // its Cholesky factor
  p.oLsS = L.take(sizeof(float) * kMaxDim * 32 * 32);  // and the inverse Grams
  p.total = L.off;
  return p;
}

struct TuckerBufs {
  char *base;
  const TuckerPlan *p;
  float *f(size_t off) const { return reinterpret_cast<float *>(base + off); }
  float *P() const { return f(p->oP); }
  float *T() const { return f(p->oT); }
  float *U(int i) const { return f(i ? p->oU1 : p->oU0); }
  float *C(int i) const { return f(i ? p->oC1 : p->oC0); }
  float *Y() const { return f(p->oY); }
  float *num() const { return f(p->oNum); }
  float *npart() const { return f(p->oNp); }
  float *den() const { return f(p->oDen); }
  float *S(int k) const {
    size_t o = p->oS;
    for (int j = 0; j < k; ++j) o += sizeof(float) * p->R[j] * p->R[j];
    return f(o);
  }
  float *M() const { return f(p->oM); }
  float *G(int i) const {
    const size_t o[4] = {p->oG0, p->oG1, p->oG2, p->oG3};
    return f(o[i]);
  }
  float *gpart() const { return f(p->oGp); }
  float *gram() const { return f(p->oGr); }
  unsigned long long *clips() const { return reinterpret_cast<unsigned long long *>(base + p->oClip); }
  unsigned int *flag() const { return reinterpret_cast<unsigned int *>(base + p->oFlag); }
  unsigned int *ticket() const { return reinterpret_cast<unsigned int *>(base + p->oTicket); }
  double *red() const { return reinterpret_cast<double *>(base + p->oRed); }
  double *part() const { return reinterpret_cast<double *>(base + p->oPart); }
  double *lsT() const { return reinterpret_cast<double *>(base + p->oLsT); }
  float *lsL() const { return f(p->oLsL); }
  float *lsSinv(int k) const { return f(p->oLsS + sizeof(float) * 32 * 32 * k); }
};

// ------------------------------------------------------------------ TTM helpers
// out = in x_k A^T where `in` has dims cur (float) and A is cur[k] x R (row-major).
static nnc_status ttm_mode(const void *in, nnc_dtype dt, int d, const int64_t *cur, int k,
                           const float *A, int64_t R, float *out, hipStream_t s,
                           bool mfma = true) {
  return launch_ttm(in, dt, prod(cur, 0, k), cur[k], prod(cur, k + 1, d), A, R, 1, R, out, s, mfma);
}

// out = in x_k A where A is N x cur[k] stored as a factor (N rows of cur[k]): the expansion
// of mode k from a rank index back to a data index.
static nnc_status expand_mode(const float *in, int d, const int64_t *cur, int k, const float *A,
                              int64_t N, float *out, hipStream_t s) {
  return launch_ttm(in, NNC_F32, prod(cur, 0, k), cur[k], prod(cur, k + 1, d), A, 1, cur[k], N, out,
                    s, false);
}

// Chain of contractions of the modes in `modes` (in order) of `src` (dims cur, updated in
// place), factors A[k] (cur[k] x R[k]).  Intermediates ping-pong in C0/C1, the result goes
// to `dst`.  With no modes, returns src.
static nnc_status chain(const float *src, int d, int64_t *cur, const int *modes, int nm,
                        float *const *A, const int64_t *R, float *c0, float *c1, float *dst,
                        const float **result, hipStream_t s) {
  const float *in = src;
  for (int i = 0; i < nm; ++i) {
    const int k = modes[i];
    float *out = (i == nm - 1) ? dst : ((i % 2) ? c1 : c0);
    NNC_TRY(ttm_mode(in, NNC_F32, d, cur, k, A[k], R[k], out, s));
    cur[k] = R[k];
    in = out;
  }
  *result = in;
  return NNC_OK;
}

// H = G x_{k != skip} S_k (core space), skip = -1: every mode.  Ping-pongs in G buffers 0/1,
// result pointer returned.
static nnc_status core_chain(const TuckerBufs &b, const float *G, int skip, float *dst,
                             const float **result, hipStream_t s) {
  const TuckerPlan &p = *b.p;
  int64_t cur[kMaxDim];
  for (int k = 0; k < p.d; ++k) cur[k] = p.R[k];
  const float *in = G;
  int cnt = 0, total = 0;
  for (int k = 0; k < p.d; ++k)
    if (k != skip) ++total;
  for (int k = 0; k < p.d; ++k) {
    if (k == skip) continue;
    float *out = (cnt == total - 1 && dst) ? dst : b.G(cnt % 2);
    if (p.fast)
      NNC_TRY(launch_ttm_small(in, prod(cur, 0, k), cur[k], prod(cur, k + 1, p.d), b.S(k), p.R[k], 1, p.R[k],
                               out, s));
    else
      NNC_TRY(ttm_mode(in, NNC_F32, p.d, cur, k, b.S(k), p.R[k], out, s, false));
    in = out;
    ++cnt;
  }
  *result = in;
  return NNC_OK;
}

// num_n, M_n and, when `grad` is null, the MU update of A_n and its new Gram; when `grad`
// is given, grad = A_n M_n - num_n instead (no update).
static nnc_status factor_block(const TuckerBufs &b, int n, const float *Y, const float *G,
                               float *A, double eps, float *grad, hipStream_t s) {
  const TuckerPlan &p = *b.p;
  const int64_t pre = prod(p.R, 0, n), post = prod(p.R, n + 1, p.d);
  if (!p.fast || !grad) NNC_TRY(launch_contract_except(Y, G, pre, p.N[n], p.R[n], post, b.num(), s));
  if (p.fast) {  // M_n by the core step of the fused sweep (every Gram is current)
    CoreArgsHost h;
    memset(&h, 0, sizeof h);
    h.d = p.d;
    for (int k = 0; k < p.d; ++k) {
      h.R[k] = p.R[k];
      h.N[k] = p.N[k];
      h.S[k] = b.S(k);
    }
    h.G = const_cast<float *>(G);
    h.M = b.M();
    h.t0 = b.G(0);
    h.t1 = b.G(1);
    h.numG = b.G(2);
    h.next = n;
    NNC_TRY(launch_core_step(h, s));
  } else {
    const float *H = nullptr;
    NNC_TRY(core_chain(b, G, n, nullptr, &H, s));
    NNC_TRY(launch_contract_except(H, G, pre, p.R[n], p.R[n], post, b.M(), s));
  }
  if (grad && p.fast)  // grad = A_n M_n - num_n by the row kernel (num formed there)
    return launch_mu_rows(Y, G, A, b.M(), pre, p.N[n], post, p.R[n], 0.0, b.clips(), nullptr, nullptr, grad, s,
                          b.npart());
  if (grad) {
    NNC_TRY(launch_matmul_small(A, b.M(), p.N[n], p.R[n], p.R[n], b.den(), s));
    NNC_TRY(launch_sub(b.den(), b.num(), grad, p.N[n] * p.R[n], s));
    return NNC_OK;
  }
  NNC_TRY(launch_mu_factor(A, b.num(), b.M(), p.N[n], p.R[n], eps, b.clips(), s));
  NNC_TRY(launch_gram(A, p.N[n], p.R[n], b.S(n), s));
  return NNC_OK;
}

// ------------------------------------------------------------------ pass timing
struct PassTimer {
  std::vector<hipEvent_t> ev;
  std::vector<int> kind;  // 0: the sweep's first X pass, 1: its second
  size_t used = 0;
  nnc_status start(hipStream_t s, int k) {
    if (used + 2 > ev.size()) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t e;
        NNC_HIP(hipEventCreate(&e));
        ev.push_back(e);
      }
    }
    NNC_HIP(hipEventRecord(ev[used], s));
    kind.push_back(k);
    return NNC_OK;
  }
  nnc_status stop(hipStream_t s) {
    NNC_HIP(hipEventRecord(ev[used + 1], s));
    used += 2;
    return NNC_OK;
  }
  // total and per-kind milliseconds and launch counts
  nnc_status total_ms(double *ms, double per_ms[2], long long per_n[2]) {
    double t = 0;
    per_ms[0] = per_ms[1] = 0.0;
    per_n[0] = per_n[1] = 0;
    for (size_t i = 0; i + 1 < used; i += 2) {
      NNC_HIP(hipEventSynchronize(ev[i + 1]));
      float x = 0.f;
      NNC_HIP(hipEventElapsedTime(&x, ev[i], ev[i + 1]));
      t += x;
      per_ms[kind[i / 2]] += x;
      per_n[kind[i / 2]] += 1;
    }
    *ms = t;
    return NNC_OK;
  }
  ~PassTimer() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

// Per-pass timing of this thread's last timed fit (nnc_last_pass_times).
static thread_local double g_pass_ms[2] = {0.0, 0.0};
static thread_local long long g_pass_n[2] = {0, 0};

// ------------------------------------------------------------------ fused sweep (R <= 32)
static CoreArgsHost core_args(const TuckerBufs &b, float *G, float *const *A, double eps) {
  const TuckerPlan &p = *b.p;
  CoreArgsHost h;
  memset(&h, 0, sizeof h);
  h.d = p.d;
  for (int k = 0; k < p.d; ++k) {
    h.R[k] = p.R[k];
    h.N[k] = p.N[k];
    h.A[k] = A[k];
    h.S[k] = b.S(k);
  }
  h.G = G;
  h.M = b.M();
  h.t0 = b.G(0);
  h.t1 = b.G(1);
  h.numG = b.G(2);
  h.gpart = b.gpart();
  h.eps = eps;
  h.clips = b.clips();
  h.next = -1;
  return h;
}

// Every Gram and the R x R matrix of mode 0: the state a fused sweep starts from.
static nnc_status fused_prologue(const TuckerBufs &b, float *G, float *const *A, double eps,
                                 hipStream_t s) {
  const TuckerPlan &p = *b.p;
  int64_t stride = 0;
  for (int k = 0; k < p.d; ++k) stride = std::max(stride, mu_rows_blocks(p.N[k]) * p.R[k] * p.R[k]);
  // one core step per factor: the partials of factors with different sizes differ in count
  for (int k = 0; k < p.d; ++k) {
    NNC_TRY(launch_gram_parts(A[k], p.N[k], p.R[k], b.gram(), s));
    CoreArgsHost h = core_args(b, G, A, eps);
    h.gram_from = k;
    h.gram_to = k + 1;
    h.gram = b.gram();
    h.gram_parts = (int)mu_rows_blocks(p.N[k]);
    h.gram_stride = stride;
    h.next = -1;
    NNC_TRY(launch_core_step(h, s));
  }
  return NNC_OK;
}

static nnc_status ttm_f32(const float *in, int d, const int64_t *cur, int k, const float *A,
                          int64_t R, float *out, hipStream_t s) {
  return launch_ttm_small(in, prod(cur, 0, k), cur[k], prod(cur, k + 1, d), A, R, 1, R, out, s);
}

// Contract modes `modes` of `src` (dims cur, updated) with ttm_small; result pointer out.
static nnc_status chain_small(const float *src, int d, int64_t *cur, const int *modes, int nm,
                              float *const *A, const int64_t *R, float *c0, float *c1, float *dst,
                              const float **result, hipStream_t s) {
  const float *in = src;
  for (int i = 0; i < nm; ++i) {
    const int k = modes[i];
    float *out = (i == nm - 1) ? dst : ((i % 2) ? c1 : c0);
    NNC_TRY(ttm_f32(in, d, cur, k, A[k], R[k], out, s));
    cur[k] = R[k];
    in = out;
  }
  *result = in;
  return NNC_OK;
}

// The core step that closes a sweep: core numerator from the last mode's row-block
// partials, Gram of the last factor and the core update.  (M_0 of the next sweep is formed
// at that sweep's start, beside its first small contraction.)
static nnc_status core_tail(const TuckerBufs &b, float *G, float *const *A, double eps, hipStream_t s,
                            bool from_parts = true) {
  const TuckerPlan &p = *b.p;
  const int d = p.d;
  CoreArgsHost h = core_args(b, G, A, eps);  // core numerator summed from b.gpart() there,
  h.gram_from = d - 1;                       // or already in b.G(2) (from_parts false)
  h.gram_to = d;
  h.gram = b.gram();
  h.gram_parts = (int)mu_rows_blocks(p.N[d - 1]);
  h.do_core = 1;
  h.nparts = from_parts ? (int)mu_rows_blocks(p.N[d - 1]) : 0;
  if (!from_parts) h.gpart = nullptr;
  h.next = -1;
  return launch_core_step(h, s);
}

// Sweeps captured in one graph when no objective is recorded in between.
constexpr int kSweepsPerGraph = 16;

// Sweeps per graph for a run of n: a divisor of n between kSweepsPerGraph / 2 and
// kSweepsPerGraph when there is one, so the run needs one capture instead of two (capture and
// instantiation cost more than the extra graph launches), else kSweepsPerGraph (n at most).
static int sweeps_per_graph(int n) {
  for (int d = kSweepsPerGraph; d >= kSweepsPerGraph / 2; --d)
    if (n >= d && n % d == 0) return d;
  return std::min(n, kSweepsPerGraph);
}

// Chain of small contractions (chain_small) whose first launch also carries the core step
// `h` (independent of the chain); without contractions the core step runs alone.
static nnc_status chain_with_core(const TuckerBufs &b, const float *src, int d, int64_t *cur,
                                  const int *modes, int nm, float *const *A, const int64_t *R,
                                  const CoreArgsHost &h, const float **result, hipStream_t s) {
  if (nm == 0) {
    NNC_TRY(launch_core_step(h, s));
    *result = src;
    return NNC_OK;
  }
  const int k = modes[0];
  float *out = (nm == 1) ? b.Y() : b.C(0);
  NNC_TRY(launch_small_with_core(src, prod(cur, 0, k), cur[k], prod(cur, k + 1, d), A[k], R[k], 1,
                                 R[k], out, h, s));
  cur[k] = R[k];
  // the rest of the chain continues from `out` (ping-pong buffers shifted by one)
  return chain_small(out, d, cur, modes + 1, nm - 1, A, R, b.C(1), b.C(0), b.Y(), result, s);
}

// One sweep of the fused schedule (every multirank <= 32).  Two X passes: pass 1
// (P = X x_{d-1} A_{d-1}^T) feeds modes 0 .. d-2, pass 2 (T = X x_0 A_0^T, with the new
// A_0) feeds mode d-1 and the core.  Each core step that only forms a Gram and the next
// mode's R x R matrix shares a launch with a small contraction it does not depend on:
//   M_0 (from G and every Gram)           with the first contraction of P,
//   Gram of A_n, M_{n+1}  (n < d-2)       with U_{n+1} = U_n x_n A_n^T,
//   Gram of A_{d-2}, M_{d-1}              with the first contraction of T.
static nnc_status fused_sweep(const TuckerBufs &b, const void *X, nnc_dtype dt, float *G,
                              float *const *A, double eps, hipStream_t s, PassTimer *tm) {
  const TuckerPlan &p = *b.p;
  const int d = p.d;
  if (tm) NNC_TRY(tm->start(s, 0));
  NNC_TRY(launch_ttm(X, dt, p.size / p.N[d - 1], p.N[d - 1], 1, A[d - 1], p.R[d - 1], 1, p.R[d - 1],
                     b.P(), s, true));
  if (tm) NNC_TRY(tm->stop(s));
  const float *U = b.P();
  CoreArgsHost pending = core_args(b, G, A, eps);  // M_0: no new Gram
  pending.gram_from = pending.gram_to = 0;
  pending.next = 0;
  for (int n = 0; n < d - 1; ++n) {
    int64_t cur[kMaxDim];
    for (int k = 0; k < d; ++k) cur[k] = (k < n || k == d - 1) ? p.R[k] : p.N[k];
    int modes[kMaxDim], nm = 0;
    for (int k = n + 1; k < d - 1; ++k) modes[nm++] = k;
    int64_t ycur[kMaxDim];
    memcpy(ycur, cur, sizeof ycur);
    const float *Y = nullptr;
    if (n == 0)
      NNC_TRY(chain_with_core(b, U, d, ycur, modes, nm, A, p.R, pending, &Y, s));
    else
      NNC_TRY(chain_small(U, d, ycur, modes, nm, A, p.R, b.C(0), b.C(1), b.Y(), &Y, s));
    NNC_TRY(launch_mu_rows(Y, G, A[n], b.M(), prod(p.R, 0, n), p.N[n], prod(p.R, n + 1, d), p.R[n],
                           eps, b.clips(), b.gram(), nullptr, nullptr, s, b.npart()));
    // core step n: Gram of the new A_n and M_{n+1}
    CoreArgsHost h = core_args(b, G, A, eps);
    h.gram_from = n;
    h.gram_to = n + 1;
    h.gram = b.gram();
    h.gram_parts = (int)mu_rows_blocks(p.N[n]);
    h.next = n + 1;
    if (n < d - 2) {
      float *Un = b.U(n % 2);
      NNC_TRY(launch_small_with_core(U, prod(cur, 0, n), cur[n], prod(cur, n + 1, d), A[n], p.R[n],
                                     1, p.R[n], Un, h, s));
      U = Un;
    } else {
      pending = h;  // M_{d-1} is not needed before the last mode
    }
  }
  if (tm) NNC_TRY(tm->start(s, 1));
  NNC_TRY(launch_ttm(X, dt, 1, p.N[0], p.size / p.N[0], A[0], p.R[0], 1, p.R[0], b.T(), s, true));
  if (tm) NNC_TRY(tm->stop(s));
  int64_t cur[kMaxDim];
  for (int k = 0; k < d; ++k) cur[k] = (k == 0) ? p.R[0] : p.N[k];
  int modes[kMaxDim], nm = 0;
  for (int k = 1; k < d - 1; ++k) modes[nm++] = k;
  const float *Y = nullptr;
  NNC_TRY(chain_with_core(b, b.T(), d, cur, modes, nm, A, p.R, pending, &Y, s));
  // the core numerator X x_k A_k^T: from the last mode's row-block partials, or, for cores
  // beyond the slice kernels (where per-block partials of the whole core cost more than the
  // contraction itself), by one small contraction with the new A_{d-1}
  const bool big_core = p.gsize > 16384;
  NNC_TRY(launch_mu_rows(Y, G, A[d - 1], b.M(), prod(p.R, 0, d - 1), p.N[d - 1], 1, p.R[d - 1], eps,
                         b.clips(), b.gram(), big_core ? nullptr : b.gpart(), nullptr, s, b.npart()));
  if (big_core) NNC_TRY(ttm_f32(Y, d, cur, d - 1, A[d - 1], p.R[d - 1], b.G(2), s));
  return core_tail(b, G, A, eps, s, !big_core);
}

// ------------------------------------------------------------------ fused three-way sweep
// d = 3 with both X passes carrying the next small contraction (fused3_kernels.hip):
//   pass 1:  Y0 = X x_2 A2^T x_1 A1^T         (side blocks: M_0)          -> rows of A0
//   pass 2:  T = X x_0 A0^T, Y1 = T x_2 A2^T  (side blocks: S_0, M_1)     -> rows of A1
//   Y2 = T x_1 A1^T beside the Gram of A1, M_2 and U = G x_0 S_0 x_1 S_1   -> rows of A2
//   core update in one launch: den_G = U x_2 S_2 (its numerator from the last rows' partials).
// P = X x_2 A2^T is never stored; seven launches per sweep.  NNC_NO_FUSED3 in the
// environment selects the general fused schedule instead (for comparisons).
static bool fused3_ok(const TuckerPlan &p, nnc_dtype dt, const void *X, const float *G, float *const *A) {
  // FP32 X: the general schedule measured faster (the FP32 passes are already near their
  // matrix-core bound, so the in-pass contractions lengthen them more than they save)
  if (p.d != 3 || !p.fast || dt != NNC_BF16 || getenv("NNC_NO_FUSED3")) return false;
  for (const void *ptr : {X, (const void *)A[0], (const void *)A[1], (const void *)A[2]})
    if (reinterpret_cast<uintptr_t>(ptr) & 15u) return false;
  if (reinterpret_cast<uintptr_t>(G) & 15u) return false;
  return pass1y_ok(dt, p.N[0], p.N[1], p.N[2], p.R[0], p.R[1], p.R[2]) &&
         pass2y_ok(dt, p.N[0], p.N[1], p.N[2], p.R[0], p.R[1], p.R[2]);
}

static Side3 side3(const TuckerBufs &b, const float *G, int n) {
  const TuckerPlan &p = *b.p;
  Side3 sd;
  memset(&sd, 0, sizeof sd);
  sd.nrows = (int)p.R[n];
  sd.n = n;
  for (int k = 0; k < 3; ++k) {
    sd.R[k] = (int)p.R[k];
    sd.S[k] = b.S(k);
  }
  sd.G = G;
  sd.M = b.M();
  sd.gmode = -1;
  sd.ticket = b.ticket();
  return sd;
}

static nnc_status fused3_sweep(const TuckerBufs &b, const void *X, nnc_dtype dt, float *G,
                               float *const *A, double eps, hipStream_t s, PassTimer *tm) {
  const TuckerPlan &p = *b.p;
  if (tm) NNC_TRY(tm->start(s, 0));
  NNC_TRY(launch_pass1y(X, dt, p.N[0], p.N[1], p.N[2], A[2], p.R[2], A[1], p.R[1], b.Y(), side3(b, G, 0), s));
  if (tm) NNC_TRY(tm->stop(s));
  NNC_TRY(launch_mu_rows(b.Y(), G, A[0], b.M(), 1, p.N[0], p.R[1] * p.R[2], p.R[0], eps, b.clips(), b.gram(),
                         nullptr, nullptr, s));
  Side3 s1 = side3(b, G, 1);
  s1.gram_part = b.gram();
  s1.gmode = 0;
  s1.gram_parts = (int)mu_rows_blocks(p.N[0]);
  s1.S_store = b.S(0);
  if (tm) NNC_TRY(tm->start(s, 1));
  NNC_TRY(launch_pass2y(X, dt, p.N[0], p.N[1], p.N[2], A[0], p.R[0], A[2], p.R[2], b.T(), b.Y(), s1, s));
  if (tm) NNC_TRY(tm->stop(s));
  NNC_TRY(launch_mu_rows(b.Y(), G, A[1], b.M(), p.R[0], p.N[1], p.R[2], p.R[1], eps, b.clips(), b.gram(),
                         nullptr, nullptr, s));
  CoreArgsHost h = core_args(b, G, A, eps);  // Gram of A1 and M_2 beside Y2 = T x_1 A1^T
  h.gram_from = 1;
  h.gram_to = 2;
  h.gram = b.gram();
  h.gram_parts = (int)mu_rows_blocks(p.N[1]);
  h.next = 2;
  h.u_out = b.G(0);  // U = G x_0 S_0 x_1 S_1 for the core update
  NNC_TRY(launch_small_with_core(b.T(), p.R[0], p.N[1], p.N[2], A[1], p.R[1], 1, p.R[1], b.Y(), h, s));
  NNC_TRY(launch_mu_rows(b.Y(), G, A[2], b.M(), p.R[0] * p.R[1], p.N[2], 1, p.R[2], eps, b.clips(), b.gram(),
                         b.gpart(), nullptr, s));
  CoreArgsHost c = core_args(b, G, A, eps);  // numerator, Gram of A2, den = U x_2 S_2, update
  c.gram_from = 2;
  c.gram_to = 3;
  c.gram = b.gram();
  c.gram_parts = (int)mu_rows_blocks(p.N[2]);
  c.do_core = 1;
  c.nparts = (int)mu_rows_blocks(p.N[2]);
  c.next = -1;
  return launch_core_last(c, s);
}

// ------------------------------------------------------------------ one sweep
static nnc_status tucker_sweep(const TuckerBufs &b, const void *X, nnc_dtype dt, float *G,
                               float *const *A, double eps, hipStream_t s, PassTimer *tm) {
  const TuckerPlan &p = *b.p;
  const int d = p.d;
  // pass 1
  if (tm) NNC_TRY(tm->start(s, 0));
  NNC_TRY(launch_ttm(X, dt, p.size / p.N[d - 1], p.N[d - 1], 1, A[d - 1], p.R[d - 1], 1, p.R[d - 1],
                     b.P(), s, true));
  if (tm) NNC_TRY(tm->stop(s));
  const float *U = b.P();
  CoreArgsHost deferred;
  bool have_deferred = false;
  for (int n = 0; n < d - 1; ++n) {
    int64_t cur[kMaxDim];
    for (int k = 0; k < d; ++k) cur[k] = (k < n || k == d - 1) ? p.R[k] : p.N[k];
    int modes[kMaxDim], nm = 0;
    for (int k = n + 1; k < d - 1; ++k) modes[nm++] = k;
    const float *Y = nullptr;
    int64_t ycur[kMaxDim];
    memcpy(ycur, cur, sizeof ycur);
    NNC_TRY(chain(U, d, ycur, modes, nm, A, p.R, b.C(0), b.C(1), b.Y(), &Y, s));
    NNC_TRY(factor_block(b, n, Y, G, A[n], eps, nullptr, s));
    if (n < d - 2) {
      float *Un = b.U(n % 2);
      NNC_TRY(ttm_mode(U, NNC_F32, d, cur, n, A[n], p.R[n], Un, s));
      U = Un;
    }
  }
  // pass 2
  if (tm) NNC_TRY(tm->start(s, 1));
  NNC_TRY(launch_ttm(X, dt, 1, p.N[0], p.size / p.N[0], A[0], p.R[0], 1, p.R[0], b.T(), s, true));
  if (tm) NNC_TRY(tm->stop(s));
  {
    int64_t cur[kMaxDim];
    for (int k = 0; k < d; ++k) cur[k] = (k == 0) ? p.R[0] : p.N[k];
    int modes[kMaxDim], nm = 0;
    for (int k = 1; k < d - 1; ++k) modes[nm++] = k;
    const float *Y = nullptr;
    NNC_TRY(chain(b.T(), d, cur, modes, nm, A, p.R, b.C(0), b.C(1), b.Y(), &Y, s));
    NNC_TRY(factor_block(b, d - 1, Y, G, A[d - 1], eps, nullptr, s));
    // core: num_G = Y x_{d-1} A_{d-1}^T (cur[d-1] is N_{d-1} here)
    NNC_TRY(ttm_mode(Y, NNC_F32, d, cur, d - 1, A[d - 1], p.R[d - 1], b.G(2), s, false));
  }
  const float *den = nullptr;
  NNC_TRY(core_chain(b, G, -1, b.G(3), &den, s));
  NNC_TRY(launch_mu_elem(G, b.G(2), den, p.gsize, eps, b.clips(), s));
  return NNC_OK;
}

// One sweep by the schedule that fits the shape.
static nnc_status any_sweep(const TuckerBufs &b, const void *X, nnc_dtype dt, float *G, float *const *A,
                            double eps, hipStream_t s, PassTimer *tm) {
  if (fused3_ok(*b.p, dt, X, G, A)) return fused3_sweep(b, X, dt, G, A, eps, s, tm);
  if (b.p->fast) return fused_sweep(b, X, dt, G, A, eps, s, tm);
  return tucker_sweep(b, X, dt, G, A, eps, s, tm);
}

// ------------------------------------------------------------------ real Tucker sweep
// One sweep of the real-valued Tucker fit (alternating least squares with orthonormalized
// factors, Section 2.2): the X passes and small contractions of the general sweep above, with
// the least-squares updates of ls_kernels.hip in place of the multiplicative ones.
// G <- G x_n L^T for the Cholesky factor L of the last factor step: the small contraction
// with "factor" L (out[.., i, ..] = sum_l L[l][i] G[.., l, ..]) into G(3), copied back.
static nnc_status ls_core_rotate(const TuckerBufs &b, int n, float *G, hipStream_t s) {
  const TuckerPlan &p = *b.p;
  NNC_TRY(launch_ttm_small(G, prod(p.R, 0, n), p.R[n], prod(p.R, n + 1, p.d), b.lsL(), p.R[n], 1, p.R[n],
                           b.G(3), s));
  NNC_HIP(hipMemcpyAsync(G, b.G(3), sizeof(float) * p.gsize, hipMemcpyDeviceToDevice, s));
  return NNC_OK;
}

// Orthonormalization of a given factor (Q of its positive-diagonal QR replaces it, R goes
// into the core): the factor is copied to num first, since the row kernel writes A apart
// from its input.
static nnc_status ls_orthonormalize(const TuckerBufs &b, int n, float *G, float *A, hipStream_t s) {
  const TuckerPlan &p = *b.p;
  NNC_HIP(hipMemcpyAsync(b.num(), A, sizeof(float) * p.N[n] * p.R[n], hipMemcpyDeviceToDevice, s));
  NNC_TRY(launch_ls_factor(b.num(), nullptr, p.N[n], p.R[n], A, b.lsT(), b.lsL(), b.S(n), b.clips(), s));
  return ls_core_rotate(b, n, G, s);
}

static nnc_status ls_factor(const TuckerBufs &b, int n, const float *Y, float *G, float *const *A,
                            hipStream_t s) {
  const TuckerPlan &p = *b.p;
  const int64_t pre = prod(p.R, 0, n), post = prod(p.R, n + 1, p.d);
  NNC_TRY(launch_contract_except(Y, G, pre, p.N[n], p.R[n], post, b.num(), s));  // num_n
  CoreArgsHost h = core_args(b, G, A, 0.0);  // K_n (the M_n of the multiplicative sweep)
  h.gram_from = h.gram_to = 0;
  h.next = n;
  NNC_TRY(launch_core_step(h, s));
  NNC_TRY(launch_ls_factor(b.num(), b.M(), p.N[n], p.R[n], A[n], b.lsT(), b.lsL(), b.S(n), b.clips(), s));
  return ls_core_rotate(b, n, G, s);
}

// Every multirank <= 32 here, so the small contractions are those of the fused sweep.
static nnc_status ls_sweep(const TuckerBufs &b, const void *X, nnc_dtype dt, float *G, float *const *A,
                           hipStream_t s, PassTimer *tm) {
  const TuckerPlan &p = *b.p;
  const int d = p.d;
  if (tm) NNC_TRY(tm->start(s, 0));
  NNC_TRY(launch_ttm(X, dt, p.size / p.N[d - 1], p.N[d - 1], 1, A[d - 1], p.R[d - 1], 1, p.R[d - 1],
                     b.P(), s, true));
  if (tm) NNC_TRY(tm->stop(s));
  const float *U = b.P();
  for (int n = 0; n < d - 1; ++n) {
    int64_t cur[kMaxDim];
    for (int k = 0; k < d; ++k) cur[k] = (k < n || k == d - 1) ? p.R[k] : p.N[k];
    int modes[kMaxDim], nm = 0;
    for (int k = n + 1; k < d - 1; ++k) modes[nm++] = k;
    const float *Y = nullptr;
    int64_t ycur[kMaxDim];
    memcpy(ycur, cur, sizeof ycur);
    NNC_TRY(chain_small(U, d, ycur, modes, nm, A, p.R, b.C(0), b.C(1), b.Y(), &Y, s));
    NNC_TRY(ls_factor(b, n, Y, G, A, s));
    if (n < d - 2) {
      float *Un = b.U(n % 2);
      NNC_TRY(ttm_f32(U, d, cur, n, A[n], p.R[n], Un, s));
      U = Un;
    }
  }
  if (tm) NNC_TRY(tm->start(s, 1));
  NNC_TRY(launch_ttm(X, dt, 1, p.N[0], p.size / p.N[0], A[0], p.R[0], 1, p.R[0], b.T(), s, true));
  if (tm) NNC_TRY(tm->stop(s));
  int64_t cur[kMaxDim];
  for (int k = 0; k < d; ++k) cur[k] = (k == 0) ? p.R[0] : p.N[k];
  int modes[kMaxDim], nm = 0;
  for (int k = 1; k < d - 1; ++k) modes[nm++] = k;
  const float *Y = nullptr;
  NNC_TRY(chain_small(b.T(), d, cur, modes, nm, A, p.R, b.C(0), b.C(1), b.Y(), &Y, s));
  NNC_TRY(ls_factor(b, d - 1, Y, G, A, s));
  // core: numerator X x_k A_k^T (every factor new), then G = numerator x_k S_k^{-1}
  NNC_TRY(ttm_f32(Y, d, cur, d - 1, A[d - 1], p.R[d - 1], b.G(2), s));
  float *S[kMaxDim], *Sinv[kMaxDim];
  for (int k = 0; k < d; ++k) {
    S[k] = b.S(k);
    Sinv[k] = b.lsSinv(k);
  }
  NNC_TRY(launch_ls_inverses(d, p.R, S, Sinv, b.clips(), s));
  int64_t gc[kMaxDim];
  for (int k = 0; k < d; ++k) gc[k] = p.R[k];
  const float *src = b.G(2);
  for (int k = 0; k < d; ++k) {  // S_k^{-1} is symmetric: the contraction with it as "factor"
    float *dst = (k == d - 1) ? G : b.G(k % 2);
    NNC_TRY(ttm_f32(src, d, gc, k, Sinv[k], p.R[k], dst, s));
    src = dst;
  }
  return NNC_OK;
}

// ||X - G x {A}||^2 and ||X||^2 into b.red() (device), Tucker model.
static nnc_status tucker_resid(const TuckerBufs &b, const void *X, nnc_dtype dt, const float *G,
                               const float *const *A, hipStream_t s) {
  const TuckerPlan &p = *b.p;
  const int d = p.d;
  int64_t cur[kMaxDim];
  for (int k = 0; k < d; ++k) cur[k] = p.R[k];
  const float *in = G;
  for (int k = 0; k < d - 1; ++k) {
    float *out = (k == d - 2) ? b.P() : b.C(k % 2);
    NNC_TRY(expand_mode(in, d, cur, k, A[k], p.N[k], out, s));
    cur[k] = p.N[k];
    in = out;
  }
  int nb = 0;
  NNC_TRY(launch_resid_stream(X, dt, p.size / p.N[d - 1], p.N[d - 1], in, A[d - 1], p.R[d - 1],
                              b.part(), &nb, s));
  NNC_TRY(launch_reduce_pairs(b.part(), nb, b.red(), s));
  return NNC_OK;
}

static nnc_status read_red(const TuckerBufs &b, double out[2], hipStream_t s) {
  NNC_HIP(hipMemcpyAsync(out, b.red(), 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  NNC_HIP(hipStreamSynchronize(s));
  return NNC_OK;
}

static double rel_of(const double red[2]) { return red[1] > 0 ? sqrt(red[0] / red[1]) : 0.0; }

// A library-owned stream for graph capture when the caller passes the default stream
// (which cannot be captured).  Default priority.
static hipStream_t capture_stream() {
  static std::mutex mu;
  static hipStream_t st = nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (!st) {
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
  }
  return st;
}

// Executable sweep graphs of the fits, kept across calls of one host thread: a later fit
// whose key matches (every pointer, size and setting its launches take, and the schedule
// switches read from the environment) replays them instead of capturing and instantiating
// again.  The graphs capture pointers, not data, so new values in the same buffers are read
// by the replay.  Each fit synchronises before it returns, so no cached graph is in flight
// when another call evicts it.
struct SweepGraphKey {
  const void *X, *ws, *core, *A[kMaxDim];
  int64_t N[kMaxDim], R[kMaxDim];
  double eps;
  hipStream_t stream;
  int dt, d, count, device, ls, no_fused3, no_big_slices, pad;  // pad: no trailing padding bytes
};
static_assert(sizeof(SweepGraphKey) % 8 == 0 && offsetof(SweepGraphKey, pad) + sizeof(int) == sizeof(SweepGraphKey),
              "the key is compared bytewise and must have no padding");
struct SweepGraphKeyLess {
  bool operator()(const SweepGraphKey &a, const SweepGraphKey &b) const { return memcmp(&a, &b, sizeof a) < 0; }
};
constexpr size_t kSweepGraphCacheMax = 16;  // executable graphs per host thread
static std::map<SweepGraphKey, hipGraphExec_t, SweepGraphKeyLess> &sweep_graph_cache() {
  // never destroyed: graphs are not torn down after the runtime at process exit
  static thread_local auto *c = new std::map<SweepGraphKey, hipGraphExec_t, SweepGraphKeyLess>();
  return *c;
}

// Run `n` sweeps, each enqueued by `sweep(stream)`, captured sweeps_per_graph(n) at a time into
// HIP graphs when `graphs` is set (a library stream stands in for the default stream, which
// cannot be captured).  Returns after the sweeps are enqueued on `s` (synchronised once).
static nnc_status run_sweeps(hipStream_t s, bool graphs, int n,
                             const std::function<nnc_status(hipStream_t)> &sweep) {
  if (n <= 0) return NNC_OK;
  if (!graphs) {
    for (int t = 0; t < n; ++t) NNC_TRY(sweep(s));
    return NNC_OK;
  }
  hipStream_t cs = s;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  if (!s) {
    cs = capture_stream();
    if (!cs) return fail(NNC_EHIP, "could not create a capture stream");
    NNC_HIP(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming));
    NNC_HIP(hipEventCreateWithFlags(&ev_out, hipEventDisableTiming));
    NNC_HIP(hipEventRecord(ev_in, s));
    NNC_HIP(hipStreamWaitEvent(cs, ev_in, 0));
  }
  auto capture = [&](hipGraphExec_t *ge, int count) -> nnc_status {
    hipGraph_t g = nullptr;
    NNC_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    nnc_status st = NNC_OK;
    for (int c = 0; c < count && st == NNC_OK; ++c) st = sweep(cs);
    const hipError_t ec = hipStreamEndCapture(cs, &g);
    if (st != NNC_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (ec != hipSuccess) return fail(NNC_EHIP, "graph capture failed: %s", hipGetErrorString(ec));
    const hipError_t ei = hipGraphInstantiate(ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(NNC_EHIP, "graph instantiation failed: %s", hipGetErrorString(ei));
    return NNC_OK;
  };
  const int per = sweeps_per_graph(n);
  hipGraphExec_t gb = nullptr, gr = nullptr;
  nnc_status st = capture(&gb, per);
  if (st == NNC_OK && n % per) st = capture(&gr, n % per);
  for (int t = 0; st == NNC_OK && t + per <= n; t += per)
    if (hipGraphLaunch(gb, cs) != hipSuccess) st = fail(NNC_EHIP, "graph launch failed");
  if (st == NNC_OK && gr && hipGraphLaunch(gr, cs) != hipSuccess) st = fail(NNC_EHIP, "graph launch failed");
  // an executable graph is destroyed only after its queued launches have finished
  if (hipStreamSynchronize(cs) != hipSuccess && st == NNC_OK)
    st = fail(NNC_EHIP, "stream synchronization after the sweeps failed");
  for (hipGraphExec_t e : {gb, gr})
    if (e) (void)hipGraphExecDestroy(e);
  NNC_TRY(st);
  if (!s) {
    NNC_HIP(hipEventRecord(ev_out, cs));
    NNC_HIP(hipStreamWaitEvent(s, ev_out, 0));
    NNC_HIP(hipEventDestroy(ev_in));
    NNC_HIP(hipEventDestroy(ev_out));
  }
  return NNC_OK;
}

// ------------------------------------------------------------------ nnCP of the data tensor
// (the nnCPD step of Algorithm 2).  Two X passes per sweep, as in the Tucker sweep:
// Z = X x_{d-1} B_{d-1}^T serves modes 0 .. d-2 (B_{d-1} is unchanged until the last mode),
// T = X x_0 B_0^T (new B_0) serves mode d-1.  Each mode: rank-wise contraction of Z or T with
// the other current factors (MTTKRP), multiplicative update, new Gram.
struct CpxPlan {
  int d = 0, r = 0;
  int64_t N[kMaxDim];
  int64_t size = 0;
  size_t oZ, oT, oM, oPart, oWA, oWC, oS, oClip, oFlag, oRed, oRpart, total;
};

static CpxPlan plan_cpx(int d, const int64_t *dims, int r) {
  CpxPlan p;
  p.d = d;
  p.r = r;
  p.size = prod(dims, 0, d);
  int64_t maxN = 1, part = 0, wa = 0, wc = 0;
  for (int k = 0; k < d; ++k) {
    p.N[k] = dims[k];
    maxN = std::max(maxN, dims[k]);
  }
  for (int n = 0; n < d - 1; ++n) {  // modes served by Z
    const int64_t A = prod(dims, 0, n), C = prod(dims, n + 1, d - 1);
    part = std::max(part, diag_part_floats(A, dims[n], C, r));
    if (n >= 2) wa = std::max(wa, A * r);
    if (d - 1 - (n + 1) >= 2) wc = std::max(wc, C * r);
  }
  {  // the last mode, served by T
    const int64_t A = prod(dims, 1, d - 1);
    part = std::max(part, diag_part_floats(A, dims[d - 1], 1, r));
    if (d - 2 >= 2) wa = std::max(wa, A * r);
  }
  Layout L;
  p.oZ = L.take(sizeof(float) * (size_t)(p.size / dims[d - 1] * r));  // also the residual's rows
  p.oT = L.take(sizeof(float) * (size_t)(p.size / dims[0] * r));
  p.oM = L.take(sizeof(float) * (size_t)(maxN * r));
  p.oPart = L.take(sizeof(float) * (size_t)part);
  p.oWA = L.take(sizeof(float) * (size_t)wa);
  p.oWC = L.take(sizeof(float) * (size_t)wc);
  p.oS = L.take(sizeof(float) * (size_t)(d * r * r));
  p.oClip = L.take(sizeof(unsigned long long));
  p.oFlag = L.take(sizeof(unsigned int));
  p.oRed = L.take(2 * sizeof(double));
  p.oRpart = L.take(2 * sizeof(double) * resid_stream_max_blocks());
  p.total = L.off;
  return p;
}

// Khatri-Rao rows of the factors of modes [lo, hi) (row-major over those modes): none -> NULL,
// one -> the factor itself, more -> built into buf.
static nnc_status kr_weights(float *const *B, const int64_t *N, int lo, int hi, int r, float *buf,
                             const float **w, int64_t *rows, hipStream_t s) {
  *rows = prod(N, lo, hi);
  if (hi <= lo) {
    *w = nullptr;
    return NNC_OK;
  }
  if (hi - lo == 1) {
    *w = B[lo];
    return NNC_OK;
  }
  int64_t dims[kMaxDim];
  const float *C[kMaxDim];
  for (int k = lo; k < hi; ++k) {
    dims[k - lo] = N[k];
    C[k - lo] = B[k];
  }
  dims[hi - lo] = 1;  // the rows exclude the last listed mode of launch_kr_rows
  C[hi - lo] = B[lo];
  NNC_TRY(launch_kr_rows(hi - lo + 1, dims, r, C, buf, s));
  *w = buf;
  return NNC_OK;
}

static nnc_status cpx_sweep(const CpxPlan &p, char *base, const void *X, nnc_dtype dt, float *const *B,
                            double eps, hipStream_t s) {
  const int d = p.d, r = p.r;
  float *Z = (float *)(base + p.oZ), *T = (float *)(base + p.oT), *M = (float *)(base + p.oM);
  float *part = (float *)(base + p.oPart), *WA = (float *)(base + p.oWA), *WC = (float *)(base + p.oWC);
  float *S = (float *)(base + p.oS);
  unsigned long long *clips = (unsigned long long *)(base + p.oClip);
  NNC_TRY(launch_ttm(X, dt, p.size / p.N[d - 1], p.N[d - 1], 1, B[d - 1], r, 1, r, Z, s, true));
  for (int n = 0; n < d - 1; ++n) {
    const float *wa, *wc;
    int64_t A, C;
    NNC_TRY(kr_weights(B, p.N, 0, n, r, WA, &wa, &A, s));
    NNC_TRY(kr_weights(B, p.N, n + 1, d - 1, r, WC, &wc, &C, s));
    NNC_TRY(launch_diag(Z, 0, A, p.N[n], C, wa, wc, r, M, part, s));
    NNC_TRY(launch_cp_mu(B[n], M, S, d, n, p.N[n], r, eps, clips, s));
    NNC_TRY(launch_gram_block(B[n], p.N[n], r, S + (size_t)n * r * r, s));
  }
  NNC_TRY(launch_ttm(X, dt, 1, p.N[0], p.size / p.N[0], B[0], r, 1, r, T, s, true));
  const float *wa;
  int64_t A;
  NNC_TRY(kr_weights(B, p.N, 1, d - 1, r, WA, &wa, &A, s));
  NNC_TRY(launch_diag(T, 1, A, p.N[d - 1], 1, wa, nullptr, r, M, part, s));
  NNC_TRY(launch_cp_mu(B[d - 1], M, S, d, d - 1, p.N[d - 1], r, eps, clips, s));
  NNC_TRY(launch_gram_block(B[d - 1], p.N[d - 1], r, S + (size_t)(d - 1) * r * r, s));
  return NNC_OK;
}

// ||X - cp(B)||^2 and ||X||^2 into the plan's red buffer.
static nnc_status cpx_resid(const CpxPlan &p, char *base, const void *X, nnc_dtype dt,
                            float *const *B, hipStream_t s) {
  float *W = (float *)(base + p.oZ);
  NNC_TRY(launch_kr_rows(p.d, p.N, p.r, (const float *const *)B, W, s));
  int nb = 0;
  NNC_TRY(launch_resid_stream(X, dt, p.size / p.N[p.d - 1], p.N[p.d - 1], W, B[p.d - 1], p.r,
                              (double *)(base + p.oRpart), &nb, s));
  return launch_reduce_pairs((double *)(base + p.oRpart), nb, (double *)(base + p.oRed), s);
}

}  // namespace nnc

using namespace nnc;

extern "C" {

const char *nnc_last_error(void) { return g_err.c_str(); }

void nnc_set_timing(int on) { g_timing = on ? 1 : 0; }

void nnc_last_pass_times(double *ms, long long *launches) {
  for (int k = 0; k < 2; ++k) {
    if (ms) ms[k] = g_pass_ms[k];
    if (launches) launches[k] = g_pass_n[k];
  }
}

int nnc_device_ok(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  return strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
}

static thread_local const char *g_last_ttm_kernel = "";

nnc_status nnc_ttm(const void *X, nnc_dtype xdt, int ndim, const int64_t *dims, int n,
                   const float *A, int64_t R, float *out, void *stream) {
  NNC_TRY(check_dims(ndim, dims, "dims"));
  if (!X || !A || !out) return fail(NNC_EINVAL, "X, A and out must be non-NULL");
  if (xdt != NNC_F32 && xdt != NNC_BF16) return fail(NNC_EINVAL, "unknown dtype %d", (int)xdt);
  if (n < 0 || n >= ndim) return fail(NNC_EINVAL, "mode %d outside [0, %d)", n, ndim);
  if (R < 1) return fail(NNC_EINVAL, "R = %lld < 1", (long long)R);
  g_last_ttm_kernel = "";
  return launch_ttm(X, xdt, prod(dims, 0, n), dims[n], prod(dims, n + 1, ndim), A, R, 1, R, out,
                    (hipStream_t)stream, true, &g_last_ttm_kernel);
}

const char *nnc_last_ttm_kernel(void) { return g_last_ttm_kernel; }

nnc_status nnc_convert_f32_bf16(const float *in, uint16_t *out, int64_t count, void *stream) {
  if (!in || !out) return fail(NNC_EINVAL, "in and out must be non-NULL");
  if (count < 0) return fail(NNC_EINVAL, "count < 0");
  if (count == 0) return NNC_OK;
  return launch_convert_bf16(in, out, count, (hipStream_t)stream);
}

nnc_status nnc_fill_uniform(uint64_t seed, uint64_t stream_id, float *ptr, int64_t n, void *stream) {
  if (n < 0) return fail(NNC_EINVAL, "n = %lld < 0", (long long)n);
  if (n == 0) return NNC_OK;
  if (!ptr) return fail(NNC_EINVAL, "ptr is NULL");
  return launch_fill_uniform(uniform_stream_key(seed, stream_id), 0, n, ptr, nullptr, (hipStream_t)stream);
}

nnc_status nnc_fill_uniform_f64(uint64_t seed, uint64_t stream_id, int64_t offset, double *ptr, int64_t n,
                                void *stream) {
  if (n < 0 || offset < 0) return fail(NNC_EINVAL, "n = %lld and offset = %lld must be >= 0", (long long)n,
                                       (long long)offset);
  if (n == 0) return NNC_OK;
  if (!ptr) return fail(NNC_EINVAL, "ptr is NULL");
  return launch_fill_uniform(uniform_stream_key(seed, stream_id), offset, n, nullptr, ptr, (hipStream_t)stream);
}

size_t nntucker_workspace_bytes(int ndim, const int64_t *dims, const int64_t *multirank) {
  if (check_dims(ndim, dims, "dims") != NNC_OK) return 0;
  if (check_dims(ndim, multirank, "multirank") != NNC_OK) return 0;
  return plan_tucker(ndim, dims, multirank).total;
}

// The driver shared by the nonnegative fit (multiplicative updates) and the real-valued fit
// (least squares, `ls`): argument checks, sweeps (optionally in graphs), objective history
// and the final report.
static nnc_status tucker_fit_impl(bool ls, const void *X, nnc_dtype xdt, int ndim, const int64_t *dims,
                                  const int64_t *multirank, int iters, float *core, float *const *factors,
                                  const nnc_options *opt, nnc_report *rep, void *stream) {
  const auto t0 = std::chrono::steady_clock::now();
  NNC_TRY(check_dims(ndim, dims, "dims"));
  NNC_TRY(check_dims(ndim, multirank, "multirank"));
  if (!X) return fail(NNC_EINVAL, "X is NULL");
  if (!core) return fail(NNC_EINVAL, "core is NULL");
  NNC_TRY(check_ptrs((const void *const *)factors, ndim, "factors"));
  if (xdt != NNC_F32 && xdt != NNC_BF16) return fail(NNC_EINVAL, "unknown dtype %d", (int)xdt);
  if (iters < 0) return fail(NNC_EINVAL, "iters = %d < 0", iters);
  const int64_t max_rank = ls ? 32 : 256;
  for (int k = 0; k < ndim; ++k)
    if (multirank[k] > max_rank)
      return fail(NNC_EUNSUPPORTED, "multirank[%d] = %lld above %lld", k, (long long)multirank[k],
                  (long long)max_rank);
  nnc_options o;
  memset(&o, 0, sizeof o);
  if (opt) o = *opt;
  if (o.eps < 0) return fail(NNC_EINVAL, "eps < 0");
  const double eps = o.eps > 0 ? o.eps : 1e-12;
  if (o.fp32_final_sweeps < 0) return fail(NNC_EINVAL, "fp32_final_sweeps < 0");
  if (o.fp32_final_sweeps > 0 && xdt != NNC_BF16)
    return fail(NNC_EINVAL, "fp32_final_sweeps needs X in NNC_BF16");
  if (o.fp32_final_sweeps > 0 && !o.x_fp32)
    return fail(NNC_EINVAL, "fp32_final_sweeps > 0 needs x_fp32");
  if (o.objective_every < 0) return fail(NNC_EINVAL, "objective_every < 0");
  if (o.objective_every > 0 && (!rep || !rep->objective_history))
    return fail(NNC_EINVAL, "objective_every > 0 needs rep->objective_history");
  const TuckerPlan p = plan_tucker(ndim, dims, multirank);
  if (!o.workspace) return fail(NNC_EWORKSPACE, "workspace is NULL (need %zu bytes)", p.total);
  if (o.workspace_bytes < p.total)
    return fail(NNC_EWORKSPACE, "workspace has %zu bytes, need %zu", o.workspace_bytes, p.total);

  hipStream_t s = (hipStream_t)stream;
  TuckerBufs b{(char *)o.workspace, &p};
  NNC_HIP(hipMemsetAsync(b.clips(), 0, sizeof(unsigned long long), s));
  NNC_HIP(hipMemsetAsync(b.flag(), 0, sizeof(unsigned int), s));
  NNC_HIP(hipMemsetAsync(b.ticket(), 0, sizeof(unsigned int), s));
  if (ls)  // orthonormal initial factors (A_n = Q R, G <- G x_n R: the same initial model)
    for (int k = 0; k < ndim; ++k)
      NNC_TRY(ls_orthonormalize(b, k, core, factors[k], s));
  else if (p.fast)
    NNC_TRY(fused_prologue(b, core, factors, eps, s));
  else
    for (int k = 0; k < ndim; ++k) NNC_TRY(launch_gram(factors[k], p.N[k], p.R[k], b.S(k), s));
  auto sweep = [&](const void *Xs, nnc_dtype dts, hipStream_t st, PassTimer *t) -> nnc_status {
    return ls ? ls_sweep(b, Xs, dts, core, factors, st, t) : any_sweep(b, Xs, dts, core, factors, eps, st, t);
  };

  PassTimer timer;
  PassTimer *tm = g_timing ? &timer : nullptr;
  const bool graphs = o.use_graph && !g_timing;
  const int split = (xdt == NNC_BF16 && o.fp32_final_sweeps > 0)
                        ? (iters > o.fp32_final_sweeps ? iters - o.fp32_final_sweeps : 0)
                        : iters;
  const float *xres = o.x_fp32 ? o.x_fp32 : (const float *)X;
  const nnc_dtype dres = o.x_fp32 ? NNC_F32 : xdt;
  int hist = 0;

  // run sweeps [t0, t1) on (Xs, dts)
  auto run_range = [&](int ta, int tb, const void *Xs, nnc_dtype dts) -> nnc_status {
    if (ta >= tb) return NNC_OK;
    const bool every = o.objective_every > 0;
    if (!graphs) {
      for (int t = ta; t < tb; ++t) {
        NNC_TRY(sweep(Xs, dts, s, tm));
        if (every && (t + 1) % o.objective_every == 0) {
          NNC_TRY(tucker_resid(b, xres, dres, core, factors, s));
          double red[2];
          NNC_TRY(read_red(b, red, s));
          rep->objective_history[hist++] = rel_of(red);
        }
      }
      return NNC_OK;
    }
    hipStream_t cs = s;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    if (!s) {
      cs = capture_stream();
      if (!cs) return fail(NNC_EHIP, "could not create a capture stream");
      NNC_HIP(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming));
      NNC_HIP(hipEventCreateWithFlags(&ev_out, hipEventDisableTiming));
      NNC_HIP(hipEventRecord(ev_in, s));
      NNC_HIP(hipStreamWaitEvent(cs, ev_in, 0));
    }
    // capture `count` sweeps into an executable graph
    auto capture = [&](hipGraphExec_t *ge, int count) -> nnc_status {
      hipGraph_t g = nullptr;
      NNC_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      nnc_status st = NNC_OK;
      for (int c = 0; c < count && st == NNC_OK; ++c)
        st = sweep(Xs, dts, cs, nullptr);
      hipError_t ec = hipStreamEndCapture(cs, &g);
      if (st != NNC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (ec != hipSuccess) return fail(NNC_EHIP, "graph capture failed: %s", hipGetErrorString(ec));
      const hipError_t ei = hipGraphInstantiate(ge, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) return fail(NNC_EHIP, "graph instantiation failed: %s", hipGetErrorString(ei));
      return NNC_OK;
    };
    if (!every && tb - ta > 1) {
      // several sweeps per graph: the turnaround between two graph launches (several
      // microseconds) is paid once per sweeps_per_graph(n) sweeps.  The executable graphs
      // are cached (see sweep_graph_cache) and destroyed only after their launches have
      // finished: their resources must not be released (and reused by the next
      // instantiation) while queued launches read them.
      const int n = tb - ta;
      const int per = sweeps_per_graph(n);
      // the cache key of `count` sweeps on (Xs, dts)
      auto key_of = [&](int count, SweepGraphKey *k) -> nnc_status {
        memset(k, 0, sizeof *k);
        k->X = Xs;
        k->ws = o.workspace;
        k->core = core;
        for (int j = 0; j < ndim; ++j) {
          k->A[j] = factors[j];
          k->N[j] = p.N[j];
          k->R[j] = p.R[j];
        }
        k->eps = eps;
        k->stream = cs;
        k->dt = (int)dts;
        k->d = ndim;
        k->count = count;
        NNC_HIP(hipGetDevice(&k->device));
        k->ls = ls ? 1 : 0;
        k->no_fused3 = getenv("NNC_NO_FUSED3") ? 1 : 0;
        k->no_big_slices = getenv("NNC_NO_BIG_SLICES") ? 1 : 0;
        return NNC_OK;
      };
      const int rem = n % per;
      SweepGraphKey kb, kr;
      NNC_TRY(key_of(per, &kb));
      NNC_TRY(key_of(rem, &kr));
      auto &c = sweep_graph_cache();
      auto ib = c.find(kb);
      auto ir = rem ? c.find(kr) : c.end();
      const size_t misses = (ib == c.end() ? 1 : 0) + (rem && ir == c.end() ? 1 : 0);
      if (misses && c.size() + misses > kSweepGraphCacheMax) {
        // make room, keeping the graphs this range replays (every fit has synchronized its
        // launches before returning, so none of the others is in flight)
        for (auto it = c.begin(); it != c.end();) {
          if (it == ib || it == ir) {
            ++it;
            continue;
          }
          (void)hipGraphExecDestroy(it->second);
          it = c.erase(it);
        }
      }
      hipGraphExec_t gb = nullptr, gr = nullptr;
      nnc_status st = NNC_OK;
      if (ib != c.end()) {
        gb = ib->second;
      } else if ((st = capture(&gb, per)) == NNC_OK) {
        c.emplace(kb, gb);
      }
      if (st == NNC_OK && rem) {
        if (ir != c.end()) {
          gr = ir->second;
        } else if ((st = capture(&gr, rem)) == NNC_OK) {
          c.emplace(kr, gr);
        }
      }
      for (int t = 0; st == NNC_OK && t + per <= n; t += per)
        if (hipGraphLaunch(gb, cs) != hipSuccess) st = fail(NNC_EHIP, "graph launch failed");
      if (st == NNC_OK && gr && hipGraphLaunch(gr, cs) != hipSuccess) st = fail(NNC_EHIP, "graph launch failed");
      if (hipStreamSynchronize(cs) != hipSuccess && st == NNC_OK)
        st = fail(NNC_EHIP, "stream synchronization after the sweeps failed");
      if (st != NNC_OK) {  // a failed range leaves no graph in the cache
        for (const SweepGraphKey *kk : {&kb, &kr}) {
          const auto it = c.find(*kk);
          if (it != c.end()) {
            (void)hipGraphExecDestroy(it->second);
            c.erase(it);
          }
        }
        return st;
      }  // else the graphs stay in the cache
    } else {
      hipGraphExec_t ge = nullptr;
      NNC_TRY(capture(&ge, 1));
      for (int t = ta; t < tb; ++t) {
        NNC_HIP(hipGraphLaunch(ge, cs));
        if (every && (t + 1) % o.objective_every == 0) {
          NNC_TRY(tucker_resid(b, xres, dres, core, factors, cs));
          double red[2];
          NNC_TRY(read_red(b, red, cs));
          rep->objective_history[hist++] = rel_of(red);
        }
      }
      NNC_HIP(hipStreamSynchronize(cs));  // see above: no destruction while launches are queued
      NNC_HIP(hipGraphExecDestroy(ge));
    }
    if (!s) {
      NNC_HIP(hipEventRecord(ev_out, cs));
      NNC_HIP(hipStreamWaitEvent(s, ev_out, 0));
      NNC_HIP(hipEventDestroy(ev_in));
      NNC_HIP(hipEventDestroy(ev_out));
    }
    return NNC_OK;
  };
  NNC_TRY(run_range(0, split, X, xdt));
  NNC_TRY(run_range(split, iters, o.x_fp32, NNC_F32));

  if (rep) {
    NNC_TRY(tucker_resid(b, xres, dres, core, factors, s));
    NNC_TRY(launch_check_finite(core, p.gsize, b.flag(), s));
    for (int k = 0; k < ndim; ++k) NNC_TRY(launch_check_finite(factors[k], p.N[k] * p.R[k], b.flag(), s));
    double red[2];
    unsigned long long clips = 0;
    unsigned int flag = 0;
    NNC_HIP(hipMemcpyAsync(red, b.red(), sizeof red, hipMemcpyDeviceToHost, s));
    NNC_HIP(hipMemcpyAsync(&clips, b.clips(), sizeof clips, hipMemcpyDeviceToHost, s));
    NNC_HIP(hipMemcpyAsync(&flag, b.flag(), sizeof flag, hipMemcpyDeviceToHost, s));
    NNC_HIP(hipStreamSynchronize(s));
    rep->sweeps_done = iters;
    rep->rel_residual = rel_of(red);
    rep->eps_clips = ls ? 0 : (long long)clips;
    rep->history_len = hist;
    rep->ttm_pass_ms = 0;
    rep->ttm_pass_launches = (long long)(timer.used / 2);
    if (tm) {
      NNC_TRY(timer.total_ms(&rep->ttm_pass_ms, g_pass_ms, g_pass_n));
    }
    rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (ls && clips)
      return fail(NNC_ENUMERIC, "%llu least-squares systems were not positive definite (rank-deficient "
                  "core or factor: lower the multirank)", clips);
    if (flag || !std::isfinite(rep->rel_residual))
      return fail(NNC_ENUMERIC, "non-finite values in the fitted model (NaN or Inf in X?)");
  }
  return NNC_OK;
}

nnc_status nntucker_fit(const void *X, nnc_dtype xdt, int ndim, const int64_t *dims,
                        const int64_t *multirank, int iters, float *core, float *const *factors,
                        const nnc_options *opt, nnc_report *rep, void *stream) {
  return tucker_fit_impl(false, X, xdt, ndim, dims, multirank, iters, core, factors, opt, rep, stream);
}

size_t tucker_ls_workspace_bytes(int ndim, const int64_t *dims, const int64_t *multirank) {
  return nntucker_workspace_bytes(ndim, dims, multirank);
}

nnc_status tucker_ls_fit(const void *X, nnc_dtype xdt, int ndim, const int64_t *dims,
                         const int64_t *multirank, int iters, float *core, float *const *factors,
                         const nnc_options *opt, nnc_report *rep, void *stream) {
  return tucker_fit_impl(true, X, xdt, ndim, dims, multirank, iters, core, factors, opt, rep, stream);
}

size_t reconstruct_workspace_bytes(int ndim, const int64_t *dims, const int64_t *model_dims,
                                   int is_cp) {
  if (check_dims(ndim, dims, "dims") != NNC_OK || !model_dims) return 0;
  if (is_cp) {
    if (model_dims[0] < 1) return 0;
    Layout L;
    L.take(sizeof(float) * (size_t)(prod(dims, 0, ndim - 1) * model_dims[0]));
    L.take(2 * sizeof(double));
    L.take(2 * sizeof(double) * resid_stream_max_blocks());
    return L.off;
  }
  if (check_dims(ndim, model_dims, "model_dims") != NNC_OK) return 0;
  return plan_tucker(ndim, dims, model_dims).total;
}

static nnc_status resid_impl(const void *X, nnc_dtype xdt, int ndim, const int64_t *dims,
                             const float *core, const int64_t *model_dims,
                             const float *const *factors, double red[2], void *workspace,
                             size_t workspace_bytes, void *stream) {
  NNC_TRY(check_dims(ndim, dims, "dims"));
  if (!X || !model_dims) return fail(NNC_EINVAL, "X and model_dims must be non-NULL");
  if (xdt != NNC_F32 && xdt != NNC_BF16) return fail(NNC_EINVAL, "unknown dtype %d", (int)xdt);
  NNC_TRY(check_ptrs((const void *const *)factors, ndim, "factors"));
  const bool cp = core == nullptr;
  if (cp && model_dims[0] < 1) return fail(NNC_EINVAL, "rank %lld < 1", (long long)model_dims[0]);
  if (!cp) NNC_TRY(check_dims(ndim, model_dims, "model_dims"));
  const size_t need = reconstruct_workspace_bytes(ndim, dims, model_dims, cp ? 1 : 0);
  if (!workspace || workspace_bytes < need)
    return fail(NNC_EWORKSPACE, "workspace has %zu bytes, need %zu", workspace ? workspace_bytes : 0, need);
  hipStream_t s = (hipStream_t)stream;
  if (cp) {
    const int64_t r = model_dims[0];
    Layout L;
    const size_t oW = L.take(sizeof(float) * (size_t)(prod(dims, 0, ndim - 1) * r));
    const size_t oRed = L.take(2 * sizeof(double));
    const size_t oPart = L.take(2 * sizeof(double) * resid_stream_max_blocks());
    char *base = (char *)workspace;
    float *W = (float *)(base + oW);
    NNC_TRY(launch_kr_rows(ndim, dims, r, factors, W, s));
    int nb = 0;
    NNC_TRY(launch_resid_stream(X, xdt, prod(dims, 0, ndim - 1), dims[ndim - 1], W, factors[ndim - 1],
                                r, (double *)(base + oPart), &nb, s));
    NNC_TRY(launch_reduce_pairs((double *)(base + oPart), nb, (double *)(base + oRed), s));
    NNC_HIP(hipMemcpyAsync(red, base + oRed, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    NNC_HIP(hipStreamSynchronize(s));
  } else {
    const TuckerPlan p = plan_tucker(ndim, dims, model_dims);
    TuckerBufs b{(char *)workspace, &p};
    NNC_TRY(tucker_resid(b, X, xdt, core, factors, s));
    NNC_TRY(read_red(b, red, s));
  }
  if (!std::isfinite(red[0]) || !std::isfinite(red[1]))
    return fail(NNC_ENUMERIC, "non-finite residual (NaN or Inf in X or the model)");
  return NNC_OK;
}

nnc_status reconstruct_residual(const void *X, nnc_dtype xdt, int ndim, const int64_t *dims,
                                const float *core, const int64_t *model_dims,
                                const float *const *factors, double *rel_residual,
                                void *workspace, size_t workspace_bytes, void *stream) {
  if (!rel_residual) return fail(NNC_EINVAL, "rel_residual is NULL");
  double red[2];
  NNC_TRY(resid_impl(X, xdt, ndim, dims, core, model_dims, factors, red, workspace, workspace_bytes,
                     stream));
  *rel_residual = rel_of(red);
  return NNC_OK;
}

nnc_status reconstruct_sq_sums(const void *X, nnc_dtype xdt, int ndim, const int64_t *dims,
                               const float *core, const int64_t *model_dims,
                               const float *const *factors, double *sq_error, double *sq_norm,
                               void *workspace, size_t workspace_bytes, void *stream) {
  if (!sq_error || !sq_norm) return fail(NNC_EINVAL, "sq_error and sq_norm must be non-NULL");
  double red[2];
  NNC_TRY(resid_impl(X, xdt, ndim, dims, core, model_dims, factors, red, workspace, workspace_bytes,
                     stream));
  *sq_error = red[0];
  *sq_norm = red[1];
  return NNC_OK;
}

nnc_status nntucker_grad(const void *X, nnc_dtype xdt, int ndim, const int64_t *dims,
                         const int64_t *multirank, const float *core, const float *const *factors,
                         float *grad_core, float *const *grad_factors, double *loss,
                         void *workspace, size_t workspace_bytes, void *stream) {
  NNC_TRY(check_dims(ndim, dims, "dims"));
  NNC_TRY(check_dims(ndim, multirank, "multirank"));
  if (!X || !core || !grad_core) return fail(NNC_EINVAL, "X, core and grad_core must be non-NULL");
  if (xdt != NNC_F32 && xdt != NNC_BF16) return fail(NNC_EINVAL, "unknown dtype %d", (int)xdt);
  NNC_TRY(check_ptrs((const void *const *)factors, ndim, "factors"));
  NNC_TRY(check_ptrs((const void *const *)grad_factors, ndim, "grad_factors"));
  for (int k = 0; k < ndim; ++k)
    if (multirank[k] > 256)
      return fail(NNC_EUNSUPPORTED, "multirank[%d] = %lld above 256", k, (long long)multirank[k]);
  const TuckerPlan p = plan_tucker(ndim, dims, multirank);
  if (!workspace || workspace_bytes < p.total)
    return fail(NNC_EWORKSPACE, "workspace has %zu bytes, need %zu", workspace ? workspace_bytes : 0, p.total);
  hipStream_t s = (hipStream_t)stream;
  TuckerBufs b{(char *)workspace, &p};
  const int d = ndim;
  float *const *A = const_cast<float *const *>(factors);
  if (p.fast) {
    float *Sk[kMaxDim];
    for (int k = 0; k < d; ++k) Sk[k] = b.S(k);
    NNC_TRY(launch_gram_set(d, A, p.N, p.R, Sk, s));
  } else {
    for (int k = 0; k < d; ++k) NNC_TRY(launch_gram(A[k], p.N[k], p.R[k], b.S(k), s));
  }
  // factors 0..d-2 from P = X x_{d-1} A_{d-1}^T (all factors held fixed)
  NNC_TRY(launch_ttm(X, xdt, p.size / p.N[d - 1], p.N[d - 1], 1, A[d - 1], p.R[d - 1], 1, p.R[d - 1],
                     b.P(), s, true));
  for (int n = 0; n < d - 1; ++n) {
    int64_t cur[kMaxDim];
    for (int k = 0; k < d; ++k) cur[k] = (k == d - 1) ? p.R[k] : p.N[k];
    int modes[kMaxDim], nm = 0;
    for (int k = 0; k < d - 1; ++k)
      if (k != n) modes[nm++] = k;
    const float *Y = nullptr;
    if (p.fast)
      NNC_TRY(chain_small(b.P(), d, cur, modes, nm, A, p.R, b.C(0), b.C(1), b.Y(), &Y, s));
    else
      NNC_TRY(chain(b.P(), d, cur, modes, nm, A, p.R, b.C(0), b.C(1), b.Y(), &Y, s));
    NNC_TRY(factor_block(b, n, Y, core, A[n], 0.0, grad_factors[n], s));
  }
  // factor d-1 and the core from T = X x_0 A_0^T
  NNC_TRY(launch_ttm(X, xdt, 1, p.N[0], p.size / p.N[0], A[0], p.R[0], 1, p.R[0], b.T(), s, true));
  int64_t cur[kMaxDim];
  for (int k = 0; k < d; ++k) cur[k] = (k == 0) ? p.R[0] : p.N[k];
  int modes[kMaxDim], nm = 0;
  for (int k = 1; k < d - 1; ++k) modes[nm++] = k;
  const float *Y = nullptr;
  if (p.fast)
    NNC_TRY(chain_small(b.T(), d, cur, modes, nm, A, p.R, b.C(0), b.C(1), b.Y(), &Y, s));
  else
    NNC_TRY(chain(b.T(), d, cur, modes, nm, A, p.R, b.C(0), b.C(1), b.Y(), &Y, s));
  NNC_TRY(factor_block(b, d - 1, Y, core, A[d - 1], 0.0, grad_factors[d - 1], s));
  if (p.fast)
    NNC_TRY(ttm_f32(Y, d, cur, d - 1, A[d - 1], p.R[d - 1], b.G(2), s));
  else
    NNC_TRY(ttm_mode(Y, NNC_F32, d, cur, d - 1, A[d - 1], p.R[d - 1], b.G(2), s, false));
  nnc_status cst = NNC_EUNSUPPORTED;
  if (p.fast) {  // den_G - num_G slice by slice
    CoreArgsHost h = core_args(b, const_cast<float *>(core), A, 0.0);
    cst = launch_core_grad(h, grad_core, s);
    if (cst != NNC_EUNSUPPORTED) NNC_TRY(cst);
  }
  if (cst == NNC_EUNSUPPORTED) {
    const float *den = nullptr;
    NNC_TRY(core_chain(b, core, -1, b.G(3), &den, s));
    NNC_TRY(launch_sub(den, b.G(2), grad_core, p.gsize, s));
  }
  if (loss) {
    NNC_TRY(tucker_resid(b, X, xdt, core, factors, s));
    double red[2];
    NNC_TRY(read_red(b, red, s));
    *loss = 0.5 * red[0];
    if (!std::isfinite(*loss)) return fail(NNC_ENUMERIC, "non-finite loss");
  }
  return NNC_OK;
}

// ------------------------------------------------------------------ nnCP of the core
static nnc_status check_cp(const float *core, int ndim, const int64_t *core_dims, int rank,
                           int iters) {
  NNC_TRY(check_dims(ndim, core_dims, "core_dims"));
  if (!core) return fail(NNC_EINVAL, "core is NULL");
  if (rank < 1) return fail(NNC_EINVAL, "rank %d < 1", rank);
  if (iters < 0) return fail(NNC_EINVAL, "iters = %d < 0", iters);
  return NNC_OK;
}

static CpProblem cp_problem(int ndim, const int64_t *core_dims) {
  CpProblem pb;
  pb.d = ndim;
  pb.size = 1;
  for (int k = 0; k < ndim; ++k) {
    pb.dims[k] = core_dims[k];
    pb.size *= core_dims[k];
  }
  return pb;
}

// Workspace of nnCP fits: rank table, factor-pointer table, residuals, clip counter, the
// contraction scratch (used when it does not fit in LDS) and, for the batched entry point,
// the tuner's scratch factors and their pointer table.
struct CpWs {
  size_t oRank, oPtr, oRes, oClip, oZ, oTune, oTunePtr, oTuneRank, total;
};

static CpWs cp_ws(const CpProblem &pb, int nbatch, const int *ranks, bool tune) {
  int maxr = 1;
  int64_t facs = 0;
  for (int j = 0; j < nbatch; ++j) {
    maxr = std::max(maxr, ranks[j]);
    for (int k = 0; k < pb.d; ++k) facs += pb.dims[k] * ranks[j];
  }
  Layout L;
  CpWs w;
  w.oRank = L.take(sizeof(int) * nbatch);
  w.oPtr = L.take(sizeof(float *) * (size_t)nbatch * pb.d);
  w.oRes = L.take(sizeof(double) * nbatch);
  w.oClip = L.take(sizeof(unsigned long long));
  w.oZ = L.take(sizeof(float) * (size_t)(nbatch * nncp_zscratch_floats(pb, maxr)));
  w.oTune = L.take(tune ? sizeof(float) * (size_t)facs : 0);
  w.oTunePtr = L.take(tune ? sizeof(float *) * (size_t)nbatch * pb.d : 0);
  w.oTuneRank = L.take(tune ? sizeof(int) * (size_t)nbatch : 0);
  w.total = L.off;
  return w;
}

size_t nncp_workspace_bytes(int ndim, const int64_t *core_dims, int rank) {
  if (check_cp((const float *)1, ndim, core_dims, rank, 0) != NNC_OK) return 0;
  const CpProblem pb = cp_problem(ndim, core_dims);
  return cp_ws(pb, 1, &rank, false).total;
}

size_t nncp_batched_workspace_bytes(int ndim, const int64_t *core_dims, int nbatch, const int *ranks) {
  if (nbatch < 1 || !ranks) return 0;
  if (check_dims(ndim, core_dims, "core_dims") != NNC_OK) return 0;
  for (int j = 0; j < nbatch; ++j)
    if (ranks[j] < 1) return 0;
  return cp_ws(cp_problem(ndim, core_dims), nbatch, ranks, true).total;
}

static nnc_status check_nncp_args(const float *core, int ndim, const int64_t *core_dims, int rank, int iters,
                                  float *const *cp_factors, double eps) {
  NNC_TRY(check_cp(core, ndim, core_dims, rank, iters));
  NNC_TRY(check_ptrs((const void *const *)cp_factors, ndim, "cp_factors"));
  if (eps < 0) return fail(NNC_EINVAL, "eps < 0");
  if (rank > 32) return fail(NNC_EUNSUPPORTED, "rank %d above 32", rank);
  return nncp_check_shape(cp_problem(ndim, core_dims), rank, 0);
}

// One CP fit of the core with its scratch (layout cp_ws) at `base`: multiplicative updates,
// or least-squares ones (`als`); fills `rep` (and syncs) if given.
static nnc_status nncp_fit_at(const float *core, int ndim, const int64_t *core_dims, int rank, int iters,
                              float *const *cp_factors, double eps, nnc_report *rep, char *base,
                              hipStream_t s, bool als = false) {
  const auto t0 = std::chrono::steady_clock::now();
  const CpProblem pb = cp_problem(ndim, core_dims);
  const CpWs w = cp_ws(pb, 1, &rank, false);
  unsigned long long *clips = (unsigned long long *)(base + w.oClip);
  NNC_TRY(launch_fill_u64(clips, 1, 0ull, s));
  NNC_TRY(launch_nncp(core, pb, 1, nullptr, rank, nullptr, cp_factors, iters, eps > 0 ? eps : 1e-12,
                      rep ? (double *)(base + w.oRes) : nullptr, clips, (float *)(base + w.oZ), 0, s,
                      als));
  if (rep) {
    double res = 0.0;
    unsigned long long nclip = 0;
    NNC_HIP(hipMemcpyAsync(&res, base + w.oRes, sizeof(double), hipMemcpyDeviceToHost, s));
    NNC_HIP(hipMemcpyAsync(&nclip, clips, sizeof nclip, hipMemcpyDeviceToHost, s));
    NNC_HIP(hipStreamSynchronize(s));
    rep->sweeps_done = iters;
    rep->rel_residual = res;
    rep->eps_clips = als ? 0 : (long long)nclip;
    rep->history_len = 0;
    rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    rep->ttm_pass_ms = 0.0;
    rep->ttm_pass_launches = 0;
    if (als && nclip)
      return fail(NNC_ENUMERIC, "%llu least-squares systems of the CP fit were not positive definite", nclip);
    if (!std::isfinite(res)) return fail(NNC_ENUMERIC, "non-finite CP residual");
  }
  return NNC_OK;
}

nnc_status nncp_fit(const float *core, int ndim, const int64_t *core_dims, int rank, int iters,
                    float *const *cp_factors, const nnc_options *opt, nnc_report *rep, void *stream) {
  const double eps = opt ? opt->eps : 0.0;
  NNC_TRY(check_nncp_args(core, ndim, core_dims, rank, iters, cp_factors, eps));
  const CpWs w = cp_ws(cp_problem(ndim, core_dims), 1, &rank, false);
  if (!opt || !opt->workspace || opt->workspace_bytes < w.total)
    return fail(NNC_EWORKSPACE, "workspace has %zu bytes, need %zu",
                (opt && opt->workspace) ? opt->workspace_bytes : 0, w.total);
  return nncp_fit_at(core, ndim, core_dims, rank, iters, cp_factors, eps, rep, (char *)opt->workspace,
                     (hipStream_t)stream);
}

size_t cp_ls_workspace_bytes(int ndim, const int64_t *core_dims, int rank) {
  return nncp_workspace_bytes(ndim, core_dims, rank);
}

nnc_status cp_ls_fit(const float *core, int ndim, const int64_t *core_dims, int rank, int iters,
                     float *const *cp_factors, const nnc_options *opt, nnc_report *rep, void *stream) {
  NNC_TRY(check_cp(core, ndim, core_dims, rank, iters));
  NNC_TRY(check_ptrs((const void *const *)cp_factors, ndim, "cp_factors"));
  if (rank > 32) return fail(NNC_EUNSUPPORTED, "rank %d above 32", rank);
  NNC_TRY(nncp_check_shape(cp_problem(ndim, core_dims), rank, 0, true));
  const CpWs w = cp_ws(cp_problem(ndim, core_dims), 1, &rank, false);
  if (!opt || !opt->workspace || opt->workspace_bytes < w.total)
    return fail(NNC_EWORKSPACE, "workspace has %zu bytes, need %zu",
                (opt && opt->workspace) ? opt->workspace_bytes : 0, w.total);
  return nncp_fit_at(core, ndim, core_dims, rank, iters, cp_factors, 0.0, rep, (char *)opt->workspace,
                     (hipStream_t)stream, true);
}

size_t nncp_noalloc_max_scratch_bytes(void) { return kStaticScratchBytes; }

nnc_status nncp_fit_noalloc(const float *core, int ndim, const int64_t *core_dims, int rank, int iters,
                            float *const *cp_factors, const nnc_options *opt, nnc_report *rep, void *stream) {
  const double eps = opt ? opt->eps : 0.0;
  NNC_TRY(check_nncp_args(core, ndim, core_dims, rank, iters, cp_factors, eps));
  const CpWs w = cp_ws(cp_problem(ndim, core_dims), 1, &rank, false);
  if (w.total > kStaticScratchBytes)
    return fail(NNC_EUNSUPPORTED, "this nnCP needs %zu bytes of scratch, above the %zu-byte static maximum "
                "of nncp_fit_noalloc (use nncp_fit with a workspace)", w.total, kStaticScratchBytes);
  char *base = nullptr;
  NNC_TRY(static_scratch(&base));
  return nncp_fit_at(core, ndim, core_dims, rank, iters, cp_factors, eps, rep, base, (hipStream_t)stream);
}

size_t nncpx_workspace_bytes(int ndim, const int64_t *dims, int rank) {
  if (check_dims(ndim, dims, "dims") != NNC_OK || rank < 1 || rank > 32) return 0;
  return plan_cpx(ndim, dims, rank).total;
}

nnc_status nncpx_fit(const void *X, nnc_dtype xdt, int ndim, const int64_t *dims, int rank, int iters,
                     float *const *factors, const nnc_options *opt, nnc_report *rep, void *stream) {
  const auto t0 = std::chrono::steady_clock::now();
  NNC_TRY(check_dims(ndim, dims, "dims"));
  if (!X) return fail(NNC_EINVAL, "X is NULL");
  NNC_TRY(check_ptrs((const void *const *)factors, ndim, "factors"));
  if (xdt != NNC_F32 && xdt != NNC_BF16) return fail(NNC_EINVAL, "unknown dtype %d", (int)xdt);
  if (rank < 1) return fail(NNC_EINVAL, "rank %d < 1", rank);
  if (rank > 32) return fail(NNC_EUNSUPPORTED, "rank %d above 32", rank);
  if (iters < 0) return fail(NNC_EINVAL, "iters = %d < 0", iters);
  nnc_options o;
  memset(&o, 0, sizeof o);
  if (opt) o = *opt;
  if (o.eps < 0) return fail(NNC_EINVAL, "eps < 0");
  const double eps = o.eps > 0 ? o.eps : 1e-12;
  if (o.fp32_final_sweeps < 0) return fail(NNC_EINVAL, "fp32_final_sweeps < 0");
  if (o.fp32_final_sweeps > 0 && xdt != NNC_BF16)
    return fail(NNC_EINVAL, "fp32_final_sweeps needs X in NNC_BF16");
  if (o.fp32_final_sweeps > 0 && !o.x_fp32) return fail(NNC_EINVAL, "fp32_final_sweeps > 0 needs x_fp32");
  if (o.objective_every < 0) return fail(NNC_EINVAL, "objective_every < 0");
  if (o.objective_every > 0 && (!rep || !rep->objective_history))
    return fail(NNC_EINVAL, "objective_every > 0 needs rep->objective_history");
  const CpxPlan p = plan_cpx(ndim, dims, rank);
  if (!o.workspace) return fail(NNC_EWORKSPACE, "workspace is NULL (need %zu bytes)", p.total);
  if (o.workspace_bytes < p.total)
    return fail(NNC_EWORKSPACE, "workspace has %zu bytes, need %zu", o.workspace_bytes, p.total);

  hipStream_t s = (hipStream_t)stream;
  char *base = (char *)o.workspace;
  NNC_TRY(launch_fill_u64((unsigned long long *)(base + p.oClip), 1, 0ull, s));
  NNC_HIP(hipMemsetAsync(base + p.oFlag, 0, sizeof(unsigned int), s));
  for (int k = 0; k < ndim; ++k)
    NNC_TRY(launch_gram_block(factors[k], dims[k], rank, (float *)(base + p.oS) + (size_t)k * rank * rank, s));
  const int split = (xdt == NNC_BF16 && o.fp32_final_sweeps > 0)
                        ? (iters > o.fp32_final_sweeps ? iters - o.fp32_final_sweeps : 0)
                        : iters;
  const void *xres = o.x_fp32 ? (const void *)o.x_fp32 : X;
  const nnc_dtype dres = o.x_fp32 ? NNC_F32 : xdt;
  const bool graphs = o.use_graph && !g_timing && o.objective_every == 0;
  int hist = 0;
  auto run = [&](int ta, int tb, const void *Xs, nnc_dtype dts) -> nnc_status {
    if (o.objective_every == 0)
      return run_sweeps(s, graphs, tb - ta,
                        [&](hipStream_t cs) { return cpx_sweep(p, base, Xs, dts, factors, eps, cs); });
    for (int t = ta; t < tb; ++t) {
      NNC_TRY(cpx_sweep(p, base, Xs, dts, factors, eps, s));
      if ((t + 1) % o.objective_every == 0) {
        NNC_TRY(cpx_resid(p, base, xres, dres, factors, s));
        double red[2];
        NNC_HIP(hipMemcpyAsync(red, base + p.oRed, sizeof red, hipMemcpyDeviceToHost, s));
        NNC_HIP(hipStreamSynchronize(s));
        rep->objective_history[hist++] = rel_of(red);
      }
    }
    return NNC_OK;
  };
  NNC_TRY(run(0, split, X, xdt));
  NNC_TRY(run(split, iters, o.x_fp32, NNC_F32));
  if (rep) {
    NNC_TRY(cpx_resid(p, base, xres, dres, factors, s));
    for (int k = 0; k < ndim; ++k)
      NNC_TRY(launch_check_finite(factors[k], dims[k] * rank, (unsigned int *)(base + p.oFlag), s));
    double red[2];
    unsigned long long clips = 0;
    unsigned int flag = 0;
    NNC_HIP(hipMemcpyAsync(red, base + p.oRed, sizeof red, hipMemcpyDeviceToHost, s));
    NNC_HIP(hipMemcpyAsync(&clips, base + p.oClip, sizeof clips, hipMemcpyDeviceToHost, s));
    NNC_HIP(hipMemcpyAsync(&flag, base + p.oFlag, sizeof flag, hipMemcpyDeviceToHost, s));
    NNC_HIP(hipStreamSynchronize(s));
    rep->sweeps_done = iters;
    rep->rel_residual = rel_of(red);
    rep->eps_clips = (long long)clips;
    rep->history_len = hist;
    rep->ttm_pass_ms = 0;
    rep->ttm_pass_launches = 0;
    rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (flag || !std::isfinite(rep->rel_residual))
      return fail(NNC_ENUMERIC, "non-finite values in the fitted model (NaN or Inf in X?)");
  }
  return NNC_OK;
}

size_t nmf_workspace_bytes(int64_t rows, int64_t cols, int rank) {
  if (rows < 1 || cols < 1 || rank < 1 || rank > 32) return 0;
  const int64_t dims[2] = {rows, cols};
  const CpProblem pb = cp_problem(2, dims);
  Layout L;
  L.take(cp_ws(pb, 1, &rank, false).total);
  L.take(sizeof(float) * (size_t)(cols * rank));
  L.take(sizeof(unsigned long long));
  L.take(2 * sizeof(double));
  return L.off;
}

// One NMF on the one-workgroup kernel when it fits (clip counter and FP64 sums at the end of
// the workspace), else as the two-way nnCP.
static nnc_status nmf_one(const float *A, int64_t rows, int64_t cols, int rank, int iters, float *W,
                          float *H, double eps, double *rel_residual, char *base, hipStream_t s) {
  const int64_t dims[2] = {rows, cols};
  const CpProblem pb = cp_problem(2, dims);
  const CpWs w = cp_ws(pb, 1, &rank, false);
  Layout L;
  L.take(w.total);
  float *Ht = (float *)(base + L.take(sizeof(float) * (size_t)(cols * rank)));
  unsigned long long *clips = (unsigned long long *)(base + L.take(sizeof(unsigned long long)));
  double *red = (double *)(base + L.take(2 * sizeof(double)));
  if (rows < (1 << 30) && nmf_block_fits((int)rows, (int)cols, rank)) {
    const int r32 = (int)rows, m32 = rank;
    NNC_TRY(launch_fill_u64(clips, 1, 0ull, s));
    NNC_TRY(launch_nmf_block(1, &A, &r32, (int)cols, &m32, iters, &W, &H, eps, clips,
                             rel_residual ? red : nullptr, s));
    if (rel_residual) {
      double h[2];
      NNC_HIP(hipMemcpyAsync(h, red, sizeof h, hipMemcpyDeviceToHost, s));
      NNC_HIP(hipStreamSynchronize(s));
      *rel_residual = rel_of(h);
    }
    return NNC_OK;
  }
  // A ~ W H is the two-way nonnegative CP with factors W (rows x rank) and H^T (cols x rank)
  NNC_TRY(nncp_check_shape(pb, rank, 0));
  NNC_TRY(launch_transpose(H, rank, cols, Ht, s));
  float *fac[2] = {W, Ht};
  NNC_TRY(launch_fill_u64((unsigned long long *)(base + w.oClip), 1, 0ull, s));
  NNC_TRY(launch_nncp(A, pb, 1, nullptr, rank, nullptr, fac, iters, eps,
                      rel_residual ? (double *)(base + w.oRes) : nullptr,
                      (unsigned long long *)(base + w.oClip), (float *)(base + w.oZ), 0, s));
  NNC_TRY(launch_transpose(Ht, cols, rank, H, s));
  if (rel_residual) {
    NNC_HIP(hipMemcpyAsync(rel_residual, base + w.oRes, sizeof(double), hipMemcpyDeviceToHost, s));
    NNC_HIP(hipStreamSynchronize(s));
  }
  return NNC_OK;
}

nnc_status nmf_fit(const float *A, int64_t rows, int64_t cols, int rank, int iters, float *W, float *H,
                   double eps, double *rel_residual, void *workspace, size_t workspace_bytes,
                   void *stream) {
  if (!A || !W || !H) return fail(NNC_EINVAL, "A, W and H must be non-NULL");
  if (rows < 1 || cols < 1) return fail(NNC_EINVAL, "matrix %lld x %lld is empty", (long long)rows, (long long)cols);
  if (rank < 1) return fail(NNC_EINVAL, "rank %d < 1", rank);
  if (rank > 32) return fail(NNC_EUNSUPPORTED, "rank %d above 32", rank);
  if (iters < 0) return fail(NNC_EINVAL, "iters = %d < 0", iters);
  if (eps < 0) return fail(NNC_EINVAL, "eps < 0");
  const size_t need = nmf_workspace_bytes(rows, cols, rank);
  if (!workspace || workspace_bytes < need)
    return fail(NNC_EWORKSPACE, "workspace has %zu bytes, need %zu", workspace ? workspace_bytes : 0, need);
  NNC_TRY(nmf_one(A, rows, cols, rank, iters, W, H, eps > 0 ? eps : 1e-12, rel_residual,
                  (char *)workspace, (hipStream_t)stream));
  if (rel_residual && !std::isfinite(*rel_residual)) return fail(NNC_ENUMERIC, "non-finite NMF residual");
  return NNC_OK;
}

size_t nmf_batched_workspace_bytes(int nbatch, const int64_t *rows, int64_t cols, const int *ranks) {
  if (nbatch < 1 || !rows || !ranks) return 0;
  size_t one = 0;
  for (int j = 0; j < nbatch; ++j) {
    const size_t b = nmf_workspace_bytes(rows[j], cols, ranks[j]);
    if (b == 0) return 0;
    one = std::max(one, b);
  }
  Layout L;
  L.take(one);
  L.take(sizeof(unsigned long long));
  L.take(2 * sizeof(double) * (size_t)nbatch);
  return L.off;
}

nnc_status nmf_fit_batched(int nbatch, const float *const *A, const int64_t *rows, int64_t cols,
                           const int *ranks, int iters, float *const *W, float *const *H, double eps,
                           double *rel_residuals, void *workspace, size_t workspace_bytes, void *stream) {
  if (nbatch < 1 || !rows || !ranks) return fail(NNC_EINVAL, "nbatch %d < 1 or NULL rows / ranks", nbatch);
  NNC_TRY(check_ptrs((const void *const *)A, nbatch, "A"));
  NNC_TRY(check_ptrs((const void *const *)W, nbatch, "W"));
  NNC_TRY(check_ptrs((const void *const *)H, nbatch, "H"));
  if (cols < 1) return fail(NNC_EINVAL, "cols %lld < 1", (long long)cols);
  for (int j = 0; j < nbatch; ++j) {
    if (rows[j] < 1) return fail(NNC_EINVAL, "rows[%d] = %lld < 1", j, (long long)rows[j]);
    if (ranks[j] < 1) return fail(NNC_EINVAL, "ranks[%d] = %d < 1", j, ranks[j]);
    if (ranks[j] > 32) return fail(NNC_EUNSUPPORTED, "ranks[%d] = %d above 32", j, ranks[j]);
  }
  if (iters < 0) return fail(NNC_EINVAL, "iters = %d < 0", iters);
  if (eps < 0) return fail(NNC_EINVAL, "eps < 0");
  const size_t need = nmf_batched_workspace_bytes(nbatch, rows, cols, ranks);
  if (!workspace || workspace_bytes < need)
    return fail(NNC_EWORKSPACE, "workspace has %zu bytes, need %zu", workspace ? workspace_bytes : 0, need);
  hipStream_t s = (hipStream_t)stream;
  const double e = eps > 0 ? eps : 1e-12;
  char *base = (char *)workspace;
  Layout L;
  size_t one = 0;
  for (int j = 0; j < nbatch; ++j) one = std::max(one, nmf_workspace_bytes(rows[j], cols, ranks[j]));
  L.take(one);
  unsigned long long *clips = (unsigned long long *)(base + L.take(sizeof(unsigned long long)));
  double *red = (double *)(base + L.take(2 * sizeof(double) * (size_t)nbatch));
  NNC_TRY(launch_fill_u64(clips, 1, 0ull, s));
  // the problems the one-workgroup kernel takes run side by side, kNmfMax per launch
  std::vector<int> fast, slow;
  for (int j = 0; j < nbatch; ++j)
    (rows[j] < (1 << 30) && nmf_block_fits((int)rows[j], (int)cols, ranks[j]) ? fast : slow).push_back(j);
  for (size_t i0 = 0; i0 < fast.size(); i0 += 8) {
    const int n = (int)std::min<size_t>(8, fast.size() - i0);
    const float *a[8];
    float *w[8], *h[8];
    int rr[8], mm[8];
    for (int k = 0; k < n; ++k) {
      const int j = fast[i0 + k];
      a[k] = A[j];
      w[k] = W[j];
      h[k] = H[j];
      rr[k] = (int)rows[j];
      mm[k] = ranks[j];
    }
    NNC_TRY(launch_nmf_block(n, a, rr, (int)cols, mm, iters, w, h, e, clips,
                             rel_residuals ? red + 2 * i0 : nullptr, s));  // by position in `fast`
  }
  std::vector<double> res(nbatch, 0.0);
  for (int j : slow)
    NNC_TRY(nmf_one(A[j], rows[j], cols, ranks[j], iters, W[j], H[j], e,
                    rel_residuals ? &res[j] : nullptr, base, s));
  if (rel_residuals) {
    std::vector<double> h(2 * (size_t)nbatch);
    NNC_HIP(hipMemcpyAsync(h.data(), red, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
    NNC_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i < fast.size(); ++i) res[fast[i]] = rel_of(&h[2 * i]);
    for (int j = 0; j < nbatch; ++j) {
      rel_residuals[j] = res[j];
      if (!std::isfinite(res[j])) return fail(NNC_ENUMERIC, "non-finite NMF residual (problem %d)", j);
    }
  }
  return NNC_OK;
}

int64_t nncandelinc_restart_init_floats(int algorithm, const int64_t *dims, const int64_t *multirank, int rank) {
  if (!dims || !multirank || (algorithm != 1 && algorithm != 2) || rank < 1) return 0;
  int N[3], M[3];
  for (int n = 0; n < 3; ++n) {
    if (dims[n] < 1 || multirank[n] < 1) return 0;
    N[n] = (int)dims[n];
    M[n] = (int)multirank[n];
  }
  return tiny_init_floats(algorithm, N, M, rank);
}

nnc_status nncandelinc_restarts(const float *X, const int64_t *dims, int algorithm, const int64_t *multirank,
                                int rank, int nrestarts, int outer_iters, int inner_iters, const float *inits,
                                const float *const *true_factors, double eps, double *rel_errors,
                                double *congruences, float *lifted, unsigned long long *clips, void *stream) {
  NNC_TRY(check_dims(3, dims, "dims"));
  NNC_TRY(check_dims(3, multirank, "multirank"));
  if (algorithm != 1 && algorithm != 2) return fail(NNC_EINVAL, "algorithm %d is neither 1 nor 2", algorithm);
  if (rank < 1) return fail(NNC_EINVAL, "rank %d < 1", rank);
  if (nrestarts < 0 || outer_iters < 0 || inner_iters < 0)
    return fail(NNC_EINVAL, "negative restart or sweep count");
  if (eps < 0) return fail(NNC_EINVAL, "eps < 0");
  int N[3], M[3];
  for (int n = 0; n < 3; ++n) {
    if (dims[n] > 8 || multirank[n] > 8)
      return fail(NNC_EUNSUPPORTED, "dims and multirank above 8 (mode %d)", n);
    N[n] = (int)dims[n];
    M[n] = (int)multirank[n];
  }
  if (rank > 8) return fail(NNC_EUNSUPPORTED, "rank %d above 8", rank);
  if (nrestarts == 0) return NNC_OK;  // nothing to read or write
  if (!X || !inits || !rel_errors) return fail(NNC_EINVAL, "X, inits and rel_errors must be non-NULL");
  if (true_factors) {
    NNC_TRY(check_ptrs((const void *const *)true_factors, 3, "true_factors"));
    if (!congruences) return fail(NNC_EINVAL, "true_factors given without congruences");
  }
  return launch_tiny_candelinc(X, N, M, rank, algorithm, nrestarts, outer_iters, inner_iters, inits,
                               true_factors, eps > 0 ? eps : 1e-12, rel_errors, true_factors ? congruences : nullptr,
                               lifted, clips, (hipStream_t)stream);
}

nnc_status nnc_mean_congruence(int ndim, const int64_t *dims, int rank, const float *const *P,
                               const float *const *Q, double *congruence, void *stream) {
  NNC_TRY(check_dims(ndim, dims, "dims"));
  if (rank < 1) return fail(NNC_EINVAL, "rank %d < 1", rank);
  if (rank > 8) return fail(NNC_EUNSUPPORTED, "rank %d above 8", rank);
  if (!congruence) return fail(NNC_EINVAL, "congruence is NULL");
  NNC_TRY(check_ptrs((const void *const *)P, ndim, "P"));
  NNC_TRY(check_ptrs((const void *const *)Q, ndim, "Q"));
  return launch_congruence(ndim, dims, rank, P, Q, congruence, (hipStream_t)stream);
}

// ---- tuner for the batched launch: threads per fit, timed on scratch factors, cached per
// (core shape, rank multiset) for the life of the process.
// ------------------------------------------------------------------ batched nnCP tuner
// A launch configuration of the batched nnCP: threads per fit, the tensor read from global
// memory instead of LDS, and the fits ordered by descending rank (longest first, which
// shortens the tail when there are more fits than compute units).  The tuner times every
// candidate on scratch factors for a few sweeps and keeps the fastest; choices persist in a
// JSON-lines file keyed by (device, core shape, rank multiset): $NNC_TUNE_CACHE, else
// $XDG_CACHE_HOME/nncandelinc/tune.json, else ~/.cache/nncandelinc/tune.json ("off"
// disables the file; the in-process cache remains).
struct TuneChoice {
  int threads = 0;
  int t_global = 0;
  int lpt = 0;
  double ms = 0.0;
};

static std::mutex g_tune_mu;
static std::map<std::string, TuneChoice> g_tune_cache;
static std::string g_tune_file_read = "\x01";  // the cache file last read (none yet)
static thread_local std::string g_last_tune = "{}";

static std::string tune_file() {
  const char *e = getenv("NNC_TUNE_CACHE");
  if (e && *e) return strcmp(e, "off") == 0 ? std::string() : std::string(e);
  const char *x = getenv("XDG_CACHE_HOME");
  if (x && *x) return std::string(x) + "/nncandelinc/tune.json";
  const char *h = getenv("HOME");
  if (h && *h) return std::string(h) + "/.cache/nncandelinc/tune.json";
  return std::string();
}

static std::string device_tag() {
  int dev = 0;
  hipDeviceProp_t pr;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&pr, dev) != hipSuccess) return "unknown";
  std::string arch(pr.gcnArchName);
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch.resize(colon);
  return arch + "/" + std::to_string(pr.multiProcessorCount) + "cu";
}

static std::string tune_key(const CpProblem &pb, int nbatch, const int *ranks) {
  std::string k = device_tag() + "|";
  for (int i = 0; i < pb.d; ++i) k += (i ? "x" : "") + std::to_string(pb.dims[i]);
  k += "|";
  std::vector<int> rs(ranks, ranks + nbatch);
  std::sort(rs.begin(), rs.end());
  for (size_t i = 0; i < rs.size(); ++i) k += (i ? "," : "") + std::to_string(rs[i]);
  return k;
}

// One JSON object per line: {"key": "...", "threads": T, "t_global": 0, "lpt": 0, "ms": x}
static bool json_int(const std::string &line, const char *name, int *v) {
  const std::string pat = std::string("\"") + name + "\":";
  const size_t p = line.find(pat);
  if (p == std::string::npos) return false;
  *v = atoi(line.c_str() + p + pat.size());
  return true;
}

// Reads the cache file when its path differs from the one read last (entries already in the
// process are kept; the file's win for equal keys).
static void tune_file_load() {
  const std::string path = tune_file();
  if (path == g_tune_file_read) return;
  g_tune_file_read = path;
  if (path.empty()) return;
  FILE *f = fopen(path.c_str(), "r");
  if (!f) return;
  char buf[4096];
  while (fgets(buf, sizeof buf, f)) {
    const std::string line(buf);
    const size_t k0 = line.find("\"key\": \"");
    if (k0 == std::string::npos) continue;
    const size_t ks = k0 + 8, ke = line.find('"', ks);
    if (ke == std::string::npos) continue;
    TuneChoice c;
    if (!json_int(line, "threads", &c.threads) || !json_int(line, "t_global", &c.t_global) ||
        !json_int(line, "lpt", &c.lpt))
      continue;
    if (c.threads < 64 || c.threads > 1024 || c.threads % 64) continue;
    g_tune_cache[line.substr(ks, ke - ks)] = c;
  }
  fclose(f);
}

static void tune_file_store() {
  const std::string path = tune_file();
  if (path.empty()) return;
  for (size_t p = path.find('/', 1); p != std::string::npos; p = path.find('/', p + 1))
    (void)mkdir(path.substr(0, p).c_str(), 0755);
  const std::string tmp = path + ".tmp" + std::to_string((long long)getpid());
  FILE *f = fopen(tmp.c_str(), "w");
  if (!f) return;
  for (const auto &kv : g_tune_cache)
    fprintf(f, "{\"key\": \"%s\", \"threads\": %d, \"t_global\": %d, \"lpt\": %d, \"ms\": %.4f}\n",
            kv.first.c_str(), kv.second.threads, kv.second.t_global, kv.second.lpt, kv.second.ms);
  const bool ok = fclose(f) == 0;
  if (ok)
    (void)rename(tmp.c_str(), path.c_str());
  else
    (void)remove(tmp.c_str());
}

static void note_tune(const TuneChoice &c, const char *source) {
  char buf[160];
  snprintf(buf, sizeof buf, "{\"threads\": %d, \"t_global\": %d, \"lpt\": %d, \"ms\": %.4f, \"source\": \"%s\"}",
           c.threads, c.t_global, c.lpt, c.ms, source);
  g_last_tune = buf;
}

// The order of the fits under a choice: as given, or by descending rank (stable).
static std::vector<int> fit_order(int nbatch, const int *ranks, bool lpt) {
  std::vector<int> o(nbatch);
  for (int j = 0; j < nbatch; ++j) o[j] = j;
  if (lpt) std::stable_sort(o.begin(), o.end(), [&](int a, int b) { return ranks[a] > ranks[b]; });
  return o;
}

static nnc_status tune_batched(const float *core, const CpProblem &pb, int nbatch, const int *ranks,
                               int maxr, const CpWs &w, char *base, int iters, hipStream_t s,
                               TuneChoice *best) {
  const std::string key = tune_key(pb, nbatch, ranks);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_file_load();
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      *best = it->second;
      note_tune(*best, "cache");
      return NNC_OK;
    }
  }
  hipEvent_t e0, e1;
  NNC_HIP(hipEventCreate(&e0));
  NNC_HIP(hipEventCreate(&e1));
  const int titers = std::max(1, std::min(iters, 10));
  TuneChoice b;
  b.ms = 1e30;
  const bool lpt_matters = nbatch > device_cu_count();
  nnc_status st = NNC_OK;
  for (int lpt = 0; lpt <= (lpt_matters ? 1 : 0) && st == NNC_OK; ++lpt) {
    // scratch factors (constant 0.5) and the rank / pointer tables in this order
    const std::vector<int> ord = fit_order(nbatch, ranks, lpt != 0);
    std::vector<int> rk(nbatch);
    std::vector<float *> ptrs((size_t)nbatch * pb.d);
    float *fbase = (float *)(base + w.oTune);
    int64_t off = 0;
    for (int i = 0; i < nbatch; ++i) {
      rk[i] = ranks[ord[i]];
      for (int k = 0; k < pb.d; ++k) {
        ptrs[(size_t)i * pb.d + k] = fbase + off;
        off += pb.dims[k] * rk[i];
      }
    }
    NNC_HIP(hipMemcpy(base + w.oTunePtr, ptrs.data(), sizeof(float *) * ptrs.size(), hipMemcpyHostToDevice));
    NNC_HIP(hipMemcpy(base + w.oTuneRank, rk.data(), sizeof(int) * nbatch, hipMemcpyHostToDevice));
    for (int tg = 0; tg <= 1 && st == NNC_OK; ++tg) {
      // reading the tensor from global memory is a distinct layout only when it fits in LDS
      if (tg && nncp_lds_bytes(pb, maxr, 256, false, true) == nncp_lds_bytes(pb, maxr, 256, false, false)) continue;
      for (int t : {256, 512, 1024}) {
        if (nncp_lds_bytes(pb, maxr, t, false, tg != 0) > 150 * 1024) continue;
        st = launch_fill_f32(fbase, off, 0.5f, s);
        if (st != NNC_OK) break;
        NNC_HIP(hipEventRecord(e0, s));
        st = launch_nncp(core, pb, nbatch, (const int *)(base + w.oTuneRank), maxr,
                         (float *const *)(base + w.oTunePtr), nullptr, titers, 1e-12, nullptr,
                         (unsigned long long *)(base + w.oClip), (float *)(base + w.oZ), t, s, false, tg != 0);
        if (st != NNC_OK) break;
        NNC_HIP(hipEventRecord(e1, s));
        NNC_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        NNC_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < b.ms) {
          b.ms = ms;
          b.threads = t;
          b.t_global = tg;
          b.lpt = lpt;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  NNC_TRY(st);
  if (b.threads == 0) {
    b.threads = nncp_default_threads(pb, maxr);
    b.ms = 0.0;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = b;
  tune_file_store();
  *best = b;
  note_tune(b, "measured");
  return NNC_OK;
}

nnc_status nncp_fit_batched(const float *core, int ndim, const int64_t *core_dims, int nbatch,
                            const int *ranks, int iters, float *const *cp_factors, double eps,
                            double *rel_residuals, int threads_per_fit, void *workspace,
                            size_t workspace_bytes, void *stream) {
  NNC_TRY(check_cp(core, ndim, core_dims, 1, iters));
  if (nbatch < 1) return fail(NNC_EINVAL, "nbatch %d < 1", nbatch);
  if (!ranks || !rel_residuals) return fail(NNC_EINVAL, "ranks and rel_residuals must be non-NULL");
  NNC_TRY(check_ptrs((const void *const *)cp_factors, nbatch * ndim, "cp_factors"));
  if (eps < 0) return fail(NNC_EINVAL, "eps < 0");
  int maxr = 0;
  for (int j = 0; j < nbatch; ++j) {
    if (ranks[j] < 1) return fail(NNC_EINVAL, "ranks[%d] = %d < 1", j, ranks[j]);
    if (ranks[j] > 32) return fail(NNC_EUNSUPPORTED, "ranks[%d] = %d above 32", j, ranks[j]);
    if (ranks[j] > maxr) maxr = ranks[j];
  }
  if (threads_per_fit != 0 && (threads_per_fit < 64 || threads_per_fit > 1024 || threads_per_fit % 64))
    return fail(NNC_EINVAL, "threads_per_fit must be 0 or a multiple of 64 in [64, 1024]");
  const CpProblem pb = cp_problem(ndim, core_dims);
  NNC_TRY(nncp_check_shape(pb, maxr, threads_per_fit));
  const CpWs w = cp_ws(pb, nbatch, ranks, true);
  if (!workspace || workspace_bytes < w.total)
    return fail(NNC_EWORKSPACE, "workspace has %zu bytes, need %zu", workspace ? workspace_bytes : 0,
                w.total);
  hipStream_t s = (hipStream_t)stream;
  char *base = (char *)workspace;
  NNC_HIP(hipStreamSynchronize(s));
  TuneChoice tc;
  tc.threads = threads_per_fit;
  if (tc.threads == 0)
    NNC_TRY(tune_batched(core, pb, nbatch, ranks, maxr, w, base, iters, s, &tc));
  else
    note_tune(tc, "caller");
  // The tables are copied synchronously (the host arrays need only live for the call), in
  // the chosen order of the fits.
  const std::vector<int> ord = fit_order(nbatch, ranks, tc.lpt != 0);
  std::vector<int> rk(nbatch);
  std::vector<float *> fp((size_t)nbatch * ndim);
  for (int i = 0; i < nbatch; ++i) {
    rk[i] = ranks[ord[i]];
    for (int k = 0; k < ndim; ++k) fp[(size_t)i * ndim + k] = cp_factors[(size_t)ord[i] * ndim + k];
  }
  NNC_HIP(hipMemcpy(base + w.oRank, rk.data(), sizeof(int) * nbatch, hipMemcpyHostToDevice));
  NNC_HIP(hipMemcpy(base + w.oPtr, fp.data(), sizeof(float *) * (size_t)nbatch * ndim, hipMemcpyHostToDevice));
  const int threads = tc.threads;
  // One graph: clear the clip counter, then the single persistent launch of every fit.
  hipStream_t cs = s;
  if (!s) {
    cs = capture_stream();
    if (!cs) return fail(NNC_EHIP, "could not create a capture stream");
    NNC_HIP(hipStreamSynchronize(nullptr));
  }
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  NNC_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  nnc_status st = launch_fill_u64((unsigned long long *)(base + w.oClip), 1, 0ull, cs);
  if (st == NNC_OK)
    st = launch_nncp(core, pb, nbatch, (const int *)(base + w.oRank), maxr, (float *const *)(base + w.oPtr),
                     nullptr, iters, eps > 0 ? eps : 1e-12, (double *)(base + w.oRes),
                     (unsigned long long *)(base + w.oClip), (float *)(base + w.oZ), threads, cs, false,
                     tc.t_global != 0);
  hipError_t ec = hipStreamEndCapture(cs, &g);
  if (st != NNC_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (ec != hipSuccess) return fail(NNC_EHIP, "graph capture failed: %s", hipGetErrorString(ec));
  NNC_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
  NNC_HIP(hipGraphLaunch(ge, cs));
  std::vector<double> res(nbatch);
  NNC_HIP(hipMemcpyAsync(res.data(), base + w.oRes, sizeof(double) * nbatch, hipMemcpyDeviceToHost, cs));
  NNC_HIP(hipStreamSynchronize(cs));
  NNC_HIP(hipGraphExecDestroy(ge));
  NNC_HIP(hipGraphDestroy(g));
  for (int i = 0; i < nbatch; ++i) rel_residuals[ord[i]] = res[i];
  for (int j = 0; j < nbatch; ++j)
    if (!std::isfinite(rel_residuals[j])) return fail(NNC_ENUMERIC, "non-finite residual of fit %d", j);
  return NNC_OK;
}

const char *nnc_last_tune(void) { return g_last_tune.c_str(); }

nnc_status nncandelinc_lift(int ndim, const int64_t *dims, const int64_t *multirank, int rank,
                            const float *const *tucker_factors, const float *const *cp_factors,
                            float *const *out_factors, void *stream) {
  NNC_TRY(check_dims(ndim, dims, "dims"));
  NNC_TRY(check_dims(ndim, multirank, "multirank"));
  if (rank < 1) return fail(NNC_EINVAL, "rank %d < 1", rank);
  NNC_TRY(check_ptrs((const void *const *)tucker_factors, ndim, "tucker_factors"));
  NNC_TRY(check_ptrs((const void *const *)cp_factors, ndim, "cp_factors"));
  NNC_TRY(check_ptrs((const void *const *)out_factors, ndim, "out_factors"));
  hipStream_t s = (hipStream_t)stream;
  for (int k = 0; k < ndim; ++k)
    NNC_TRY(launch_lift(tucker_factors[k], cp_factors[k], dims[k], multirank[k], rank, out_factors[k], s));
  return NNC_OK;
}

}  // extern "C"
