/*
 * nncandelinc.h -- C ABI of the MI355X (gfx950) library for nonnegative CANDELINC
 * (Alexandrov, DeSantis, Manzini, Skau, "Nonnegative Canonical Tensor Decomposition with
 * Linear Constraints: nnCANDELINC", arXiv 1909.07570), which solves the constrained
 * least-squares problem of Section 4 (eq. nnCANDELINC) in two ways:
 *   Algorithm 1: a nonnegative Tucker compression X ~ G x_1 F1 x_2 F2 ... x_d Fd
 *                (nntucker_fit), a nonnegative CP of the core G ~ I x_1 B1 ... x_d Bd
 *                (nncp_fit), and the lift C_n = F_n B_n (nncandelinc_lift);
 *   Algorithm 2: a nonnegative CP of X itself (nncpx_fit), then an NMF of each CP factor,
 *                A_n ~ F_n B_n (nmf_fit, nmf_fit_batched), and the same lift.
 * Scoring (Section 4.1): reconstruct_residual and nnc_mean_congruence.  The random-restart
 * study of Section 4.2 runs as one launch (nncandelinc_restarts).
 * Real-valued CANDELINC (Section 2.2, the same problem without the nonnegativity
 * constraints): a Tucker fit by alternating least squares (tucker_ls_fit), a CP fit of its
 * core by alternating least squares (cp_ls_fit), and the same lift.
 *
 * Conventions shared by every entry point
 *   - Tensors are dense and row-major (last index fastest): element (i_1, ..., i_d) of a
 *     tensor with dims N_1..N_d lives at offset ((i_1 N_2 + i_2) N_3 + ...) + i_d.
 *     Factor matrices are row-major: F_n is dims[n] x R_n, B_n is R_n x r, C_n is dims[n] x r.
 *     In the text below F_n is written A_n.
 *   - Pointers are DEVICE pointers unless marked "host".  The caller owns every buffer.
 *     The library never allocates device memory.  Entry points that need scratch space take
 *     a caller-provided device workspace whose minimum size a *_workspace_bytes query
 *     returns; workspace contents need not be initialised and are clobbered.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Work is
 *     enqueued on it in order.  An entry point returns without synchronising unless it
 *     must hand a value back to host memory (marked "syncs").
 *   - Every argument is validated before any HIP call, so invalid calls fail the same way
 *     with or without a GPU.  Status codes are returned; nothing is thrown across the ABI.
 *     nnc_last_error() describes the most recent non-OK status of the calling thread.
 *   - ndim is 2..8.  Multiranks may exceed the dimensions they compress (Section 4.2 fits
 *     multirank [5,5,5] to a 4x4x4 tensor).
 *   - Multiplicative updates (MU): the paper delegates the solvers to library routines run
 *     for a fixed iteration count with random initialisation and no early stop (Section 4.1).
 *     This library applies Lee-Seung Frobenius multiplicative updates block by block:
 *       factor n (n = 1..d in order, Gauss-Seidel):
 *         A_n <- A_n * num_n / max(den_n, eps)
 *         num_n = unfold_n(X x_{k!=n} A_k^T) unfold_n(G)^T
 *         den_n = A_n unfold_n(G x_{k!=n} A_k^T A_k) unfold_n(G)^T
 *       core:  G <- G * (X x_1 A_1^T ... x_d A_d^T) / max(G x_1 A_1^T A_1 ... x_d A_d^T A_d, eps)
 *       nnCP of the core, factor n:  B_n <- B_n * M_n / max(B_n H_n, eps),
 *         M_n = MTTKRP of the core with the other factors, H_n = Hadamard product of their Grams.
 *     (x * num) / max(den, eps) is evaluated in double precision and rounded to float.
 *     Initial values are inputs (the caller draws them), and the results are written back
 *     in place into the same buffers, so a fit can be resumed by calling again.
 */
#ifndef NNCANDELINC_H
#define NNCANDELINC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NNC_OK = 0,
  NNC_EINVAL = -1,       /* invalid argument (null pointer, bad size, bad enum)            */
  NNC_EUNSUPPORTED = -2, /* valid request the library does not implement                   */
  NNC_EWORKSPACE = -3,   /* workspace missing or smaller than the query says               */
  NNC_EHIP = -4,         /* a HIP runtime call failed (message in nnc_last_error)          */
  NNC_ENUMERIC = -5      /* non-finite value in the result (e.g. NaN or Inf in X)          */
} nnc_status;

typedef enum { NNC_F32 = 0, NNC_BF16 = 1 } nnc_dtype;

/* Options of nntucker_fit.  Zero-initialised options are valid defaults (eps 1e-12). */
typedef struct {
  int fp32_final_sweeps;   /* with X in NNC_BF16: the last k sweeps read x_fp32 and run the
                              X-streaming contractions in FP32 (refinement)                   */
  const float *x_fp32;     /* optional FP32 copy of X (device).  Required when
                              fp32_final_sweeps > 0.  When given, residuals are measured
                              against it                                                        */
  double eps;              /* MU denominator floor; 0 selects 1e-12                            */
  int objective_every;     /* 0: residual only at the end (if a report is requested);
                              k > 0: also after every k-th sweep into report history          */
  int use_graph;           /* 1: capture one sweep in a HIP graph and replay it              */
  void *workspace;         /* device scratch of at least nntucker_workspace_bytes()          */
  size_t workspace_bytes;
} nnc_options;

/* Report of a fit (host struct).  Passing a report makes the call synchronise. */
typedef struct {
  int sweeps_done;
  double rel_residual;        /* ||X - G x {A}||_F / ||X||_F after the last sweep            */
  long long eps_clips;        /* number of MU entries whose denominator was below eps        */
  double *objective_history;  /* host, optional: relative residual after every
                                 objective_every-th sweep (length >= iters / objective_every) */
  int history_len;            /* entries written                                             */
  double seconds;             /* wall time of the call                                       */
  double ttm_pass_ms;         /* summed GPU time of the two X-streaming TTM passes (when
                                 timing is requested through nnc_set_timing)                  */
  long long ttm_pass_launches;
} nnc_report;

/* Thread-local description of the last non-OK status (never NULL). */
const char *nnc_last_error(void);

/* 1 if the library was built for and can see a gfx950 device, else 0 (no error raised). */
int nnc_device_ok(void);

/* Turn per-launch timing of the X-streaming TTM passes on (1) or off (0).  When on, the
 * library records HIP events around each pass launch on the caller's stream and nntucker_fit
 * reports their summed duration. */
void nnc_set_timing(int on);

/* The per-pass split of the last timed fit on the calling thread (a fit run while timing
 * was on and with rep != NULL): ms[0] / launches[0] for the first X pass of each sweep
 * (X x_d A_d^T; in the fused three-way BF16 schedule the pass that also forms Y_0 and M_0),
 * ms[1] / launches[1] for the second (X x_1 A_1^T; fused: also Y_1, S_1 and M_1).  Host
 * arrays of 2, either may be NULL. */
void nnc_last_pass_times(double *ms, long long *launches);

/*
 * n-mode product with a transposed factor, out = X x_n A^T (Appendix A, definition of
 * n-mode multiplication, with the matrix A^T):
 *   out[i_1..r..i_d] = sum_l X[i_1..l..i_d] * A[l, r],   l < dims[n], r < R.
 * X: dims (xdt = NNC_F32 or NNC_BF16).  A: dims[n] x R float.  out: float, the shape of X
 * with dims[n] replaced by R.  n is 0-based.  Runs the same MFMA pass kernels as the fit
 * when their shape conditions hold, else a general kernel.
 */
nnc_status nnc_ttm(const void *X, nnc_dtype xdt, int ndim, const int64_t *dims, int n,
                   const float *A, int64_t R, float *out, void *stream);

/* The kernel the calling thread's last nnc_ttm launched: "ttm_last_lds_bf16",
 * "ttm_mid_f32", ... for the matrix-core X-streaming kernels ("(chunked)" when the contracted
 * index was split into several launches), "ttm_generic" for the general kernel.  A static
 * string, never NULL. */
const char *nnc_last_ttm_kernel(void);

/* Round FP32 to bfloat16 (round to nearest, ties to even; NaN stays NaN).  out holds
 * count uint16 bit patterns. */
nnc_status nnc_convert_f32_bf16(const float *in, uint16_t *out, int64_t count, void *stream);

/*
 * Seeded uniform draws for initial values and synthetic inputs.  The paper starts every
 * solver from a random initialisation (Section 4.1) and draws the random factor matrices of
 * its generated tensors (Section 4.3); this library takes initial values as inputs, and these
 * helpers draw them on the device from a counter-based SplitMix64 stream (Steele, Lea &
 * Flood, OOPSLA 2014):
 *   key      = mix64(mix64(seed + G) ^ (stream_id * 0xD1B54A32D192ED03)),  G = 0x9E3779B97F4A7C15,
 *   draw(i)  = mix64(key + (i + 1) * G)   (arithmetic mod 2^64; mix64 = SplitMix64's finaliser),
 *   value(i) = (draw(i) >> 11) * 2^-53, a double in [0, 1).
 * Element i depends only on (seed, stream_id, i), so the values are the same whatever the
 * launch shape, and a slice can be drawn on its own.
 *   nnc_fill_uniform:      ptr[i] = value(i) rounded to float (nearest, ties to even),
 *                          i < n.  ptr: device, n floats.
 *   nnc_fill_uniform_f64:  ptr[i] = value(offset + i) as a double, i < n.  ptr: device.
 * n = 0 does nothing; n < 0, offset < 0 or a NULL ptr (with n > 0) -> NNC_EINVAL.
 * Asynchronous on `stream`.
 */
nnc_status nnc_fill_uniform(uint64_t seed, uint64_t stream_id, float *ptr, int64_t n, void *stream);
nnc_status nnc_fill_uniform_f64(uint64_t seed, uint64_t stream_id, int64_t offset, double *ptr, int64_t n,
                                void *stream);

/*
 * Nonnegative Tucker decomposition by multiplicative updates (the nnTD step of
 * Algorithm 1), exactly `iters` sweeps, no early stop (Section 4.1).  The arithmetic of the
 * two X-streaming contractions of every sweep follows xdt: NNC_F32 runs FP32 MFMA;
 * NNC_BF16 runs bf16 MFMA with FP32 accumulation (the factor is applied as a hi + lo pair
 * of bf16 values, so the rounding of X to bf16 is the only reduction of precision).
 * Everything else (partial contractions, Grams, updates) is FP32 with FP64 divisions.
 *   X          dims[0..ndim-1], dtype xdt.
 *   multirank  host, R_n = multirank[n] >= 1.
 *   core       in: initial G (prod R_n floats, entries >= 0); out: fitted G.
 *   factors    host array of ndim device pointers; factor n is dims[n] x R_n;
 *              in: initial A_n >= 0; out: fitted A_n.
 *   opt        nullable (defaults); workspace is required.
 *   rep        nullable; non-NULL makes the call synchronise and fill it.
 * iters = 0 leaves the inputs unchanged (and reports their residual).
 */
size_t nntucker_workspace_bytes(int ndim, const int64_t *dims, const int64_t *multirank);
nnc_status nntucker_fit(const void *X, nnc_dtype xdt, int ndim, const int64_t *dims,
                        const int64_t *multirank, int iters, float *core, float *const *factors,
                        const nnc_options *opt, nnc_report *rep, void *stream);

/*
 * Nonnegative CP of a (small) tensor, here the Tucker core (the nnCPD step of Algorithm 1),
 * exactly `iters` MU sweeps in one persistent launch.  rank <= 32.
 *   core        core_dims[0..ndim-1] floats.
 *   cp_factors  host array of ndim device pointers; factor n is core_dims[n] x rank;
 *               in: initial B_n >= 0; out: fitted B_n.
 *   opt         eps and the workspace (at least nncp_workspace_bytes()) are used; the other
 *               fields are ignored.  NULL or a short workspace -> NNC_EWORKSPACE.
 *   rep         nullable; non-NULL syncs and reports sweeps_done, eps_clips, seconds and
 *               rel_residual = ||core - cp(B)||_F / ||core||_F.
 */
size_t nncp_workspace_bytes(int ndim, const int64_t *core_dims, int rank);
nnc_status nncp_fit(const float *core, int ndim, const int64_t *core_dims, int rank, int iters,
                    float *const *cp_factors, const nnc_options *opt, nnc_report *rep, void *stream);

/*
 * nncp_fit for callers that cannot allocate device memory or pass a workspace: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * kernels and results as nncp_fit, except that opt is nullable and only its eps is read
 * (the workspace fields are ignored).  Its scratch is a static device array of
 * nncp_noalloc_max_scratch_bytes() bytes (8 MiB) that each device holds from library load
 * to process exit; a fit whose nncp_workspace_bytes() exceeds it is refused with
 * NNC_EUNSUPPORTED before any HIP call.  The call itself allocates nothing.  Every call on a
 * device shares that device's array, so calls that overlap on one device (from several host
 * threads, or on several streams without ordering) race; calls in one stream order are safe.
 */
size_t nncp_noalloc_max_scratch_bytes(void);
nnc_status nncp_fit_noalloc(const float *core, int ndim, const int64_t *core_dims, int rank, int iters,
                            float *const *cp_factors, const nnc_options *opt, nnc_report *rep, void *stream);

/*
 * Real-valued Tucker fit (the Tucker step of CANDELINC, Section 2.2; the paper leaves the
 * algorithm to standard tools).  Exactly `iters` sweeps of alternating least squares in the
 * nonnegative fit's order, each block replaced by the exact minimizer of
 * 0.5 ||X - G x {A}||_F^2 over that block:
 *   factor n:  A* = num_n K_n^{-1},  num_n as in nntucker_fit,
 *              K_n = unfold_n(G x_{k!=n} A_k^T A_k) unfold_n(G)^T;
 *              then the thin QR A* = Q R (R upper triangular, positive diagonal, by Cholesky
 *              of A*^T A* in FP64): A_n <- Q and G <- G x_n R, which leaves the model as is;
 *   core:      G <- (X x_1 A_1^T ... x_d A_d^T) x_1 (A_1^T A_1)^{-1} ... x_d (A_d^T A_d)^{-1}.
 * Before the first sweep each initial factor is orthonormalized the same way (the initial
 * model is unchanged), so the systems are well conditioned from the first step on.
 * On return every factor has orthonormal columns (to FP32 rounding), so the CP error of the
 * core equals the error of the lifted CP against the Tucker model.  The R x R systems are
 * solved in FP64 (Gauss-Jordan inverses, no pivoting).
 * Arguments as nntucker_fit, except: every multirank[n] <= 32 (else NNC_EUNSUPPORTED);
 * entries may have any sign; eps is ignored and eps_clips reports 0.  With rep non-NULL a
 * system that was not positive definite (a rank-deficient core unfolding or factor, e.g. a
 * multirank above the data's multilinear rank with no noise) returns NNC_ENUMERIC, and the
 * outputs are then unspecified.  Workspace: tucker_ls_workspace_bytes() (the same size as
 * nntucker_workspace_bytes()).
 */
size_t tucker_ls_workspace_bytes(int ndim, const int64_t *dims, const int64_t *multirank);
nnc_status tucker_ls_fit(const void *X, nnc_dtype xdt, int ndim, const int64_t *dims,
                         const int64_t *multirank, int iters, float *core, float *const *factors,
                         const nnc_options *opt, nnc_report *rep, void *stream);

/*
 * Real-valued CP of a (small) tensor, here the Tucker core (the CPD step of CANDELINC,
 * Section 2.2): exactly `iters` sweeps of alternating least squares in one persistent launch,
 * factor n (n = 1..d in order):  B_n <- M_n H_n^{-1}  (M_n, H_n as in nncp_fit; H_n inverted
 * in FP64 by Gauss-Jordan elimination).  rank <= 32.  Arguments and report as nncp_fit
 * (workspace at least cp_ls_workspace_bytes(), the same size as nncp_workspace_bytes());
 * eps is ignored.  With rep non-NULL an H_n that was not positive definite returns
 * NNC_ENUMERIC.
 */
size_t cp_ls_workspace_bytes(int ndim, const int64_t *core_dims, int rank);
nnc_status cp_ls_fit(const float *core, int ndim, const int64_t *core_dims, int rank, int iters,
                     float *const *cp_factors, const nnc_options *opt, nnc_report *rep, void *stream);

/*
 * Many independent nnCP fits of one core (random restarts, possibly different ranks) in a
 * single persistent launch: restart j has rank ranks[j] (host array) and factors
 * cp_factors[j*ndim + n] (core_dims[n] x ranks[j]).  rel_residuals: host, nbatch entries
 * (syncs).  Every rank must be <= 32.  threads_per_fit: 0 lets the library's tuner choose.
 */
size_t nncp_batched_workspace_bytes(int ndim, const int64_t *core_dims, int nbatch, const int *ranks);
nnc_status nncp_fit_batched(const float *core, int ndim, const int64_t *core_dims, int nbatch,
                            const int *ranks, int iters, float *const *cp_factors, double eps,
                            double *rel_residuals, int threads_per_fit, void *workspace,
                            size_t workspace_bytes, void *stream);

/* The launch configuration the calling thread's last nncp_fit_batched used, as a JSON
 * object: {"threads": T, "t_global": 0|1, "lpt": 0|1, "ms": x, "source": "measured" | "cache"
 * | "caller"} -- threads per fit, the tensor read from global memory instead of LDS, the
 * fits ordered by descending rank, the tuner's timing of a few sweeps, and where the choice
 * came from.  The tuner (threads_per_fit = 0) times each candidate once per (device, core
 * shape, rank multiset) and keeps the choice in a JSON-lines file: $NNC_TUNE_CACHE, else
 * $XDG_CACHE_HOME/nncandelinc/tune.json, else ~/.cache/nncandelinc/tune.json; "off" keeps
 * it in the process only.  A static thread-local string, never NULL. */
const char *nnc_last_tune(void);

/*
 * Nonnegative CP of the data tensor itself (the nnCPD step of Algorithm 2, which runs it on
 * X and then factors each CP factor by NMF), exactly `iters` sweeps of the multiplicative
 * update B_n <- B_n * M_n / max(B_n H_n, eps) (the nnCP rule above, applied to X, factors
 * in order 0..d-1 within a sweep).  Two X-streaming contractions per sweep, run by the
 * same kernels and with the same arithmetic as nntucker_fit (xdt = NNC_F32: FP32 MFMA;
 * NNC_BF16: bf16 MFMA with FP32 accumulation): Z = X x_d B_d^T serves modes 1..d-1 and
 * T = X x_1 B_1^T (after B_1's update) serves mode d; the MTTKRPs are rank-wise
 * contractions of Z or T with the other factors.  rank <= 32.
 *   factors  host array of ndim device pointers; factor n is dims[n] x rank;
 *            in: initial B_n >= 0; out: fitted B_n.
 *   opt      nullable (defaults); workspace (nncpx_workspace_bytes()) is required.
 *            fp32_final_sweeps / x_fp32 / objective_every / use_graph as for nntucker_fit.
 *   rep      nullable; non-NULL syncs and reports ||X - cp(B)||_F / ||X||_F.
 */
size_t nncpx_workspace_bytes(int ndim, const int64_t *dims, int rank);
nnc_status nncpx_fit(const void *X, nnc_dtype xdt, int ndim, const int64_t *dims, int rank, int iters,
                     float *const *factors, const nnc_options *opt, nnc_report *rep, void *stream);

/*
 * Nonnegative matrix factorization A ~ W H (the NMF step of Algorithm 2, applied to each CP
 * factor A^(i) with m_i latent columns: A^(i) ~ F^(i) B^(i)), exactly `iters` Lee-Seung
 * multiplicative sweeps, W first, then H:
 *   W <- W * (A H^T) / max(W H H^T, eps),   H <- H * (W^T A) / max(W^T W H, eps),
 * which is the two-way case of the nnCP rule (factors W and H^T).  One workgroup computes
 * it with A, W and H in LDS when they fit (rows * rank <= 32768, cols <= 32, about 159 KiB),
 * else the nnCP kernel runs it as a two-way nnCP.
 *   A  rows x cols (float, entries >= 0).   W  rows x rank, in: initial; out: fitted.
 *   H  rank x cols, in: initial; out: fitted.   rank <= 32.
 *   rel_residual  host, nullable: ||A - W H||_F / ||A||_F; non-NULL syncs.
 *   workspace     at least nmf_workspace_bytes().
 */
size_t nmf_workspace_bytes(int64_t rows, int64_t cols, int rank);
nnc_status nmf_fit(const float *A, int64_t rows, int64_t cols, int rank, int iters, float *W, float *H,
                   double eps, double *rel_residual, void *workspace, size_t workspace_bytes,
                   void *stream);

/*
 * Several independent NMFs with a common column count in one call (Algorithm 2 factors
 * every CP factor A^(i), i = 1..d, each with its own m_i): problem j factors A[j]
 * (rows[j] x cols) with rank ranks[j] into W[j] (rows[j] x ranks[j]) and H[j]
 * (ranks[j] x cols), in place.  Problems small enough for one workgroup's LDS run side by
 * side in one launch; the others run one after another as in nmf_fit.  A, W, H: host arrays
 * of nbatch device pointers; rows, ranks: host arrays.  rel_residuals: host, nullable,
 * nbatch entries (syncs).  workspace: nmf_batched_workspace_bytes().
 */
size_t nmf_batched_workspace_bytes(int nbatch, const int64_t *rows, int64_t cols, const int *ranks);
nnc_status nmf_fit_batched(int nbatch, const float *const *A, const int64_t *rows, int64_t cols,
                           const int *ranks, int iters, float *const *W, float *const *H, double eps,
                           double *rel_residuals, void *workspace, size_t workspace_bytes, void *stream);

/*
 * The random-restart study of Section 4.2: `nrestarts` complete nnCANDELINC fits of one small
 * 3-way tensor in a single launch, one workgroup per start, every fit in on-chip memory.
 *   algorithm 1: nnTucker (multirank) for outer_iters sweeps, nnCP of the core (rank) for
 *                inner_iters sweeps, lift C_n = A_n B_n.
 *   algorithm 2: nnCP of X (rank) for outer_iters sweeps, NMF of each CP factor with
 *                multirank[n] columns for inner_iters sweeps, lift C_n = W_n H_n.
 * The multiplicative rules are those of nntucker_fit, nncp_fit and nmf_fit.  dims, multirank
 * and rank are at most 8 (the study's tensor is 4 x 4 x 4).
 *   X            device, dims[0] x dims[1] x dims[2] floats.
 *   inits        device, nrestarts x nncandelinc_restart_init_floats() floats; per start:
 *                algorithm 1: A_0, A_1, A_2 (dims[n] x multirank[n]), G (prod multirank),
 *                             B_0, B_1, B_2 (multirank[n] x rank);
 *                algorithm 2: B_0, B_1, B_2 (dims[n] x rank, CP of X), W_0, W_1, W_2
 *                             (dims[n] x multirank[n]), H_0, H_1, H_2 (multirank[n] x rank).
 *   true_factors host array of 3 device pointers (dims[n] x rank), nullable: the known CP
 *                factors; congruences[j] is then the mean congruence of start j's rank-one
 *                terms with them under the best matching (Section 4.1 scoring).
 *   rel_errors   device, nrestarts doubles: ||X - cp(C)||_F / ||X||_F of every start.
 *   lifted       device, nullable: nrestarts x (dims[0] + dims[1] + dims[2]) x rank floats.
 *   clips        device, nullable: clipped denominators are added to *clips.
 * nrestarts = 0 validates the sizes and returns NNC_OK without reading any buffer.
 */
int64_t nncandelinc_restart_init_floats(int algorithm, const int64_t *dims, const int64_t *multirank, int rank);
nnc_status nncandelinc_restarts(const float *X, const int64_t *dims, int algorithm, const int64_t *multirank,
                                int rank, int nrestarts, int outer_iters, int inner_iters, const float *inits,
                                const float *const *true_factors, double eps, double *rel_errors,
                                double *congruences, float *lifted, unsigned long long *clips, void *stream);

/*
 * Mean congruence of two CP models of rank <= 8 (Section 4.1 scoring): the congruence of two
 * rank-one terms is the product over modes of the cosines of their factor columns, and the
 * score is the mean over components under the matching that maximises it (every permutation
 * is tried).  P, Q: host arrays of ndim device pointers, factor n dims[n] x rank.  congruence:
 * device, one double (no synchronisation).  A zero column has cosine 0.
 */
nnc_status nnc_mean_congruence(int ndim, const int64_t *dims, int rank, const float *const *P,
                               const float *const *Q, double *congruence, void *stream);

/*
 * Lift: C_n = A_n B_n for every mode (substituting the core's CP into the Tucker model,
 * Section 2.1 lemma proof and Section 2.2).  tucker_factors[n]: dims[n] x multirank[n];
 * cp_factors[n]: multirank[n] x rank; out_factors[n]: dims[n] x rank.  Host arrays of
 * device pointers.
 */
nnc_status nncandelinc_lift(int ndim, const int64_t *dims, const int64_t *multirank, int rank,
                            const float *const *tucker_factors, const float *const *cp_factors,
                            float *const *out_factors, void *stream);

/*
 * Relative reconstruction error ||X - Xhat||_F / ||X||_F (Section 4.1 scoring), with
 * squared differences accumulated in double precision.  Syncs.
 *   core != NULL: Tucker model Xhat = core x_1 A_1 ... x_d A_d, model_dims = multirank.
 *   core == NULL: CP model Xhat = sum_rho outer(A_1[:,rho], ..., A_d[:,rho]);
 *                 model_dims[0] = rank (other entries ignored).
 * factors: host array of ndim device pointers, factor n is dims[n] x model_dims[n] (Tucker)
 * or dims[n] x rank (CP).
 */
size_t reconstruct_workspace_bytes(int ndim, const int64_t *dims, const int64_t *model_dims,
                                   int is_cp);
nnc_status reconstruct_residual(const void *X, nnc_dtype xdt, int ndim, const int64_t *dims,
                                const float *core, const int64_t *model_dims,
                                const float *const *factors, double *rel_residual,
                                void *workspace, size_t workspace_bytes, void *stream);

/* The two sums behind reconstruct_residual: sq_error = ||X - Xhat||_F^2 and
 * sq_norm = ||X||_F^2 (host doubles; syncs).  Same arguments and workspace otherwise. */
nnc_status reconstruct_sq_sums(const void *X, nnc_dtype xdt, int ndim, const int64_t *dims,
                               const float *core, const int64_t *model_dims,
                               const float *const *factors, double *sq_error, double *sq_norm,
                               void *workspace, size_t workspace_bytes, void *stream);

/*
 * Adjoint of L = 0.5 ||X - G x {A}||_F^2 at one point (every block held fixed):
 *   dL/dA_n = den_n - num_n,   dL/dG = den_G - num_G,
 * the same numerators and denominators the multiplicative updates use, recomputed from X
 * (two X passes; nothing is kept from a forward call).  grad_core: prod R floats;
 * grad_factors: host array of device pointers (dims[n] x R_n).  loss: host, nullable
 * (non-NULL adds one more X pass and syncs).  Workspace: nntucker_workspace_bytes().
 */
nnc_status nntucker_grad(const void *X, nnc_dtype xdt, int ndim, const int64_t *dims,
                         const int64_t *multirank, const float *core, const float *const *factors,
                         float *grad_core, float *const *grad_factors, double *loss,
                         void *workspace, size_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* NNCANDELINC_H */
