/*
 * libtvs -- TV-Stokes denoising by dual (Chambolle-type) iterations inside an
 * overlapping Schwarz decomposition, on one AMD Instinct MI355X (gfx950).
 *
 * The method is that of Langer, Runft, Rahman, Tai and Wu, "Functional
 * Analysis and Parallel Domain Decomposition for the TV-Stokes Model"
 * (arXiv 2602.17494):
 *   Step 1 (tangent field smoothing, TFS): the dual problem eq. tfsdualdis,
 *     min_{|p_k| <= 1} || P_K vecdiv p - delta^{-1} P_K tau_0 ||^2 on the
 *     extended grid Omega-tilde, solved by Algorithm 1 (alg:chambTfs), and
 *     tau = P_K tau_0 - delta P_K vecdiv p (Corollary Cor:tfsdual with
 *     eq. tfs_dualPK);
 *   Step 2 (image reconstruction, IRV2 of Section 3.3): the dual problem
 *     eq. ir2dualdis, min_{|p| <= 1} || div p - alpha (d0 - g) ||^2 on Omega
 *     with (D^-_x, D^-_y) g = (R_Omega tau)^perp, solved by Chambolle's
 *     iteration, and d = d0 - div p / alpha;  IRV1 (eq. ir1dualdis with
 *     eq. eq:defXi2:discrete and eq. eq:tau_hat) is available as a variant;
 *   both inside the parallel overlapping Schwarz iteration of Algorithm 2
 *     (alg:disalgsubsp) with the subdomain loops of Algorithm 3
 *     (alg:tfsparinner, Step 2) and Algorithm 5 (alg:tfsparinnertfsloc,
 *     Step 1, with the projection of locally supported data restricted to
 *     the subdomain, eqs. locglobprojpart1 and locglobprojpart3).
 *
 * Grids, layout and ownership
 *   The image grid Omega has N2 rows (y) and N1 columns (x), 2 <= N2, N1 <=
 *   5119 and (N2+1)(N1+1) <= 2^28: the inverse Laplacian of Omega-tilde runs
 *   as FFTs of smooth lengths >= 2(N+1) - 1 held in one workgroup's LDS
 *   (at most 10240 points per axis); larger shapes give TVS_EINVAL.
 *   The Step-1 grid Omega-tilde has (N2+1) x (N1+1) points and holds Omega as
 *   its first N2 rows and N1 columns (Section 4.1).  Arrays are row-major:
 *     image  d0, d      : N2 * N1 values
 *     field  tau        : 2 planes of (N2+1) * (N1+1) values, plane 0 = tau_1
 *                         (x-component), plane 1 = tau_2 (y-component)
 *   All array pointers are DEVICE pointers owned by the caller, of the element
 *   type given by `dtype` (float or double).  The library owns only its
 *   context, the per-problem plans and work buffers it caches inside the
 *   context, all released by tvs_ctx_destroy.
 *
 * Streams
 *   `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Work is enqueued on it in order.  When `stats` is non-NULL the call
 *   waits for the stream before returning (it reads FP64 reductions back);
 *   otherwise outputs are valid once the stream has been synchronised.  Calls
 *   sharing one context must not overlap (the context's work buffers are
 *   reused); use one context per concurrent caller.
 *
 * Errors
 *   Every call returns TVS_OK (0) or a negative code; tvs_last_error()
 *   returns a thread-local message for the last failure.  No C++ exception
 *   crosses this interface.
 */
#ifndef TVS_H_
#define TVS_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  TVS_OK = 0,
  TVS_EINVAL = -1,    /* shape, parameter or layout out of range */
  TVS_ENOMEM = -2,    /* device allocation failed */
  TVS_EHIP = -3,       /* a HIP runtime call or kernel launch failed */
  TVS_ENONFINITE = -4, /* an FP64 reduction found NaN or Inf */
  TVS_EBUSY = -5       /* a job's result was asked for before it finished */
};

typedef enum { TVS_F32 = 0, TVS_F64 = 1 } tvs_dtype;

/* Step-2 reconstruction variant (Section 5.1). */
typedef enum { TVS_IRV2 = 0, TVS_IRV1 = 1 } tvs_variant;

/* Model and iteration parameters.
 *   delta  > 0      TFS weight (eq. eq:cTFS)
 *   alpha  > 0      Step-2 weight (eq. modifiedStep2; IRV1: alpha = 1/mu)
 *   t in (0, 1/8]   dual step size (Algorithm 1 and the convergence theorem after it)
 *   h      > 0      mesh size (the paper's experiments use h = 1)
 *   eps    > 0      IRV1 smoothing of |tau^perp| (eq. eq:defXi2); unused by IRV2
 *   variant         TVS_IRV2 or TVS_IRV1 */
typedef struct {
  double delta, alpha, t, h, eps;
  int variant;
} tvs_params;

/* Subdomain layout (Section 6.1).  M2 x M1 subdomains (1 <= M <= 32 per
 * axis); s_y, s_x = width of the stripe two neighbours share, centred on the
 * core cut floor(k n / M) of the Omega-tilde axis (n = N+1); every core must
 * be at least max(s, 2) points wide, and s >= 1 where M > 1.  The weights
 * theta_m are linear ramps across the shared stripes.  alpha_hat <= 0 selects
 * the colouring rule after Algorithm 2 (1, 1/2 or 1/4); otherwise it must lie
 * in (0, 1].  M2 = M1 = 1 is the plain single-domain solve (theta = 1). */
typedef struct {
  int M2, M1, s_y, s_x;
  double alpha_hat;
} tvs_layout;

/* Iteration counts: `sweeps` outer iterations of Algorithm 2 (>= 1), each
 * with `inner` subdomain iterations (>= 1).  tol > 0 stops after the first
 * sweep whose stopping residual (below) falls under tol; tol = 0 runs the
 * fixed counts. */
typedef struct {
  int sweeps, inner;
  double tol;
} tvs_iters;

/* FP64 results of one step, computed on the GPU:
 *   energy    D(p) of the final iterate (eq. tfsdualdis / ir2dualdis)
 *   residual  |D(p^{S-1})^{1/2} - D(p^S)^{1/2}| / (c |Gamma|)^{1/2} over the
 *             last sweep (c = 2 channels for TFS, 1 otherwise): the left side
 *             of the paper's stopping tests (Section 5.2) over their scale
 *   gap       duality gap sum_k sum(|grad u_k| + grad u_k . p_k) of the final
 *             iterate with its primal (tau for TFS, (f - div p)/alpha for
 *             Step 2); >= 0 and 0 exactly at the solution
 *   sweeps_done, seconds (host wall time of the call, including the wait). */
typedef struct {
  int sweeps_done;
  double energy, gap, residual, seconds;
} tvs_stats;

typedef struct tvs_ctx tvs_ctx;

/* Create a context on HIP device `device`.  Returns TVS_OK and *out. */
int tvs_ctx_create(int device, tvs_ctx** out);
/* Release the context and everything it cached.  NULL is ignored. */
void tvs_ctx_destroy(tvs_ctx* ctx);
/* Thread-local message of the last failing call ("" if none). */
const char* tvs_last_error(void);
/* Bytes of device memory the context currently holds (plans, work buffers). */
size_t tvs_ctx_bytes(const tvs_ctx* ctx);

/* Step 1 (TFS) from the observed image d0 (N2*N1) to the smoothed tangent
 * field tau_out (2 planes of (N2+1)*(N1+1)): tau_0 = (-D^{neum-}_y d0,
 * D^{neum-}_x d0) (eq. def:backdiffNeumann), f = delta^{-1} P_K tau_0, then
 * Algorithm 2 on Omega-tilde with the localized inner loop of Algorithm 5,
 * then tau = delta (f - P_K vecdiv p).  stats may be NULL. */
int tvs_step1(tvs_ctx* ctx, const void* d0, int N2, int N1, tvs_dtype dtype,
              const tvs_params* params, const tvs_layout* layout, const tvs_iters* iters,
              void* tau_out, tvs_stats* stats, void* stream);

/* Step 2 from d0 (N2*N1) and a tangent field tau (2 planes of
 * (N2+1)*(N1+1)) to the image d_out (N2*N1).  IRV2: g = the row-wise
 * integral of tau_2 on Omega (D^-_x g = tau_2 with the interior rule in every
 * column, g = 0 left of the first column), f = alpha (d0 - g); IRV1:
 * f = alpha d0 - div xi.  Then Algorithm 2 on Omega with the inner loop of
 * Algorithm 3 (Lambda = div), and d = d0 - div p / alpha (IRV1: minus
 * div xi / alpha as well).  stats may be NULL. */
int tvs_step2(tvs_ctx* ctx, const void* d0, const void* tau, int N2, int N1, tvs_dtype dtype,
              const tvs_params* params, const tvs_layout* layout, const tvs_iters* iters,
              void* d_out, tvs_stats* stats, void* stream);

/* Both steps with the same layout and counts.  tau_out may be NULL; stats,
 * if not NULL, points to two entries (Step 1, Step 2). */
int tvs_schwarz_solve(tvs_ctx* ctx, const void* d0, int N2, int N1, tvs_dtype dtype,
                      const tvs_params* params, const tvs_layout* layout, const tvs_iters* iters,
                      void* d_out, void* tau_out, tvs_stats* stats, void* stream);

/* The orthogonal projection onto divergence-free fields of an n2 x n1 grid,
 * P u = u - grad (Delta)^dagger div u (eq. formula:PKh, Proposition
 * prop:DisProj), 3 <= n2, n1 <= 5120: u_in and u_out are 2 planes of n2*n1 (x- then
 * y-component); they may alias.  Step 1 applies this operator on
 * Omega-tilde. */
int tvs_project_div_free(tvs_ctx* ctx, const void* u_in, int n2, int n1, tvs_dtype dtype,
                         double h, void* u_out, void* stream);

/* Diagnostics: kernel timing.  While enabled, one launch in every `enable`
 * launches of each instrumented kernel class (the 1st, the (enable+1)-th,
 * ...) is bracketed by two HIP events recorded on the call's stream, and
 * credited with the launch's algorithmic bytes (the data the kernel must read
 * and write at minimum; the formulas are listed with each kernel in the
 * library sources).  Enabling it adds two event records per timed launch;
 * every 64 pending records of a class, the older half is folded in, which
 * waits for launches that are by then long finished.
 *   tvs_timing_enable  enable = 0: off; enable = k >= 1: time every k-th
 *                      launch of each class (1: every launch); < 0: error
 *   tvs_timing_reset   drop everything recorded so far
 *   tvs_timing_count   wait for the recorded events and return the number of
 *                      kernel classes (>= 0), or a negative error code
 *   tvs_timing_get     entry i (0 <= i < count): class name copied into
 *                      name[name_len], launches, total milliseconds, total
 *                      algorithmic bytes (for the class "s1_bdct" of the
 *                      block-DCT local projection: floating-point operations) */
int tvs_timing_enable(tvs_ctx* ctx, int enable);
int tvs_timing_reset(tvs_ctx* ctx);
int tvs_timing_count(tvs_ctx* ctx);
int tvs_timing_get(tvs_ctx* ctx, int i, char* name, int name_len, long long* launches, double* ms,
                   double* bytes);

/* Jobs: one image's Step 1 + Step 2 solve (the same problem and the same
 * computation as tvs_schwarz_solve with the default TVS_LP_IMAGE local
 * projection, whose results it reproduces bit for bit)
 * with its own device state, resident between calls: the problem's plans,
 * the dual variables of every subdomain, a copy of d0, tau and d.  A job is
 * advanced one Schwarz sweep (Algorithm 2) at a time, so that a caller can
 * interleave the sweeps of many jobs, admit new ones between sweeps and
 * retire finished ones (continuous batching).
 *   tvs_job_footprint  bytes of device memory a job of this shape needs (its
 *                      own state, plus the Green-function table of its grid,
 *                      which tvs_job_create builds and frees again unless the
 *                      context already holds one from a one-shot call), computed
 *                      on the host; TVS_EINVAL for shapes tvs_job_create
 *                      would refuse
 *   tvs_job_create     validate as tvs_schwarz_solve, allocate and build the
 *                      job's state, copy d0 (device pointer, N2 x N1; the
 *                      caller may reuse it on return) and run the Step-1
 *                      set-up on `stream`; the call waits for that work
 *   tvs_batch_sweep    advance each of the n jobs (of this context, each at
 *                      most once in the list) by one sweep of its current
 *                      step, ordered after the work already on `stream`, and
 *                      make `stream` wait for it.  The work runs on a stream
 *                      of the context: first every job's sweep head (the
 *                      global residual and FP64 energy, and the stopping
 *                      test), then the sweep bodies of all jobs, recorded
 *                      as one HIP graph and replayed while the same jobs
 *                      come in the same states (eagerly while kernel timing
 *                      is on).  In the bodies, jobs of one shape (step,
 *                      dtype, image size, layout, h, t and inner count)
 *                      run each inner iteration as one launch per kernel
 *                      class over the subdomains of all of them.  The sweep
 *                      that completes Step 1 also
 *                      computes tau and its statistics (which waits for that
 *                      job's work) and sets up Step 2; the one that completes
 *                      Step 2 computes d.  A finished job is left as it is.
 *                      Jobs share no data: neither the order of the list nor
 *                      the overlap changes any result.  A job whose FP64
 *                      statistics come out non-finite (NaN or Inf in its
 *                      data) fails alone: it is marked finished with that
 *                      error and the call goes on with the other jobs.
 *   tvs_job_status     step 1 or 2 (3 when finished, -1 when failed), sweeps
 *                      done in it, done = 1 when finished or failed; any
 *                      pointer may be NULL
 *   tvs_job_result     copy d (N2 x N1) and tau (2 x (N2+1) x (N1+1)) into
 *                      the caller's device buffers (either may be NULL) on
 *                      `stream`, and the two steps' statistics into
 *                      stats[2] (may be NULL); TVS_EBUSY before the job has
 *                      finished, the job's error (TVS_ENONFINITE) if it failed
 *   tvs_job_bytes      device bytes held by the job (0 for NULL)
 *   tvs_job_destroy    wait for the device, free the job (NULL is a no-op)
 * The calls on one job must not overlap; jobs of one context share its kernel
 * timer only. */
typedef struct tvs_job tvs_job;
int tvs_job_footprint(int N2, int N1, tvs_dtype dtype, const tvs_layout* layout,
                      const tvs_iters* iters, size_t* bytes);
int tvs_job_create(tvs_ctx* ctx, const void* d0, int N2, int N1, tvs_dtype dtype,
                   const tvs_params* params, const tvs_layout* layout, const tvs_iters* iters,
                   void* stream, tvs_job** out);
int tvs_batch_sweep(tvs_ctx* ctx, tvs_job* const* jobs, int n, void* stream);
int tvs_job_status(const tvs_job* job, int* step, int* sweeps_done, int* done);
int tvs_job_result(tvs_ctx* ctx, tvs_job* job, void* d_out, void* tau_out, tvs_stats* stats,
                   void* stream);
size_t tvs_job_bytes(const tvs_job* job);
int tvs_job_destroy(tvs_job* job);

/* FP64 dual energies D(p^0), D(p^1), ..., D(p^S) at the start of every
 * Schwarz sweep and after the last (S = sweeps done; the TFS dual energy of
 * eq. tfsdualdis for Step 1, the ROF dual energy of Step 2) of the most recent
 * tvs_step1 or tvs_step2 call on this context that asked for statistics (for
 * tvs_schwarz_solve, of its Step 2).  *n = S + 1, or 0 if there was none;
 * min(cap, *n) values are copied into the host array out (out may be NULL
 * when cap is 0, to query *n).  No device work. */
int tvs_energy_history(tvs_ctx* ctx, double* out, int cap, int* n);

/* Realisation of the local projection LP_m = R P_K E of Step 1's inner
 * iterations (eqs. locglobprojpart1, locglobprojpart3), for the later
 * tvs_step1 and tvs_schwarz_solve calls of this context with more than one
 * subdomain:
 *   TVS_LP_IMAGE     (default) the inverse Laplacian of the whole grid on a
 *                    box through the image identity and box-sized FFTs
 *   TVS_LP_BLOCKDCT  the paper's block formula (eq. invLaplLowCapLong): a
 *                    sum over frequency blocks of products of DCT matrix
 *                    blocks (the box's columns, the block's rows) and the
 *                    spectral diagonal of the whole grid, on the matrix
 *                    cores (about 2 n2 n1 (box side) multiply-adds per box;
 *                    workspace of a few frequency blocks per box, see
 *                    tvs_set_block_groups)
 * Both compute the same operator; results differ by rounding only.  Jobs
 * (tvs_job_*) always use TVS_LP_IMAGE.  TVS_EINVAL for another kind. */
enum { TVS_LP_IMAGE = 0, TVS_LP_BLOCKDCT = 1 };
int tvs_set_local_projection(tvs_ctx* ctx, int kind);

/* Grouping of the frequency blocks of TVS_LP_BLOCKDCT (eq. invLaplLowCapLong,
 * Lemma lmChainOp): the frequency rows are cut into ceil(n2 / amax) blocks and
 * the columns into ceil(n1 / bmax) blocks (amax x bmax the largest box, n2 x n1
 * the grid of N2 + 1 x N1 + 1 points), and the sum over the blocks is taken g2
 * row blocks by g1 column blocks at a time; the per-box workspace is g2 x g1
 * blocks at most.  0 (the default) chooses each from the launch size, with
 * at most 16 blocks per group; a positive value is cut to the block count.
 * Applies to plans built after the call.  Results depend on the grouping
 * through the order of the sums only.  TVS_EINVAL outside [0, 64]. */
int tvs_set_block_groups(tvs_ctx* ctx, int g2, int g1);

/* Workgroup shapes (performance only: every choice gives the same results,
 * bit for bit).  The first time a one-shot call (tvs_step1, tvs_step2,
 * tvs_schwarz_solve) builds a problem shape (dtype, image size, layout, h;
 * LP_m realisation) in a context, the library times candidate shapes on the
 * problem's buffers and keeps the fastest for that shape.  A job
 * (tvs_job_create) times nothing: it takes the shapes forced or tuned before
 * for its problem shape in the context, else the plans' defaults (a
 * server's requests come in many sizes, and each would pay the tuning).
 * The shapes:
 *   run1, run1d, run2  rows per thread of the Step-1 update, the Step-1
 *               vecdiv and the Step-2 update kernels (1, 2 or 4)
 *   rows, cols  targets for the row pairs per row-pass workgroup and the
 *               columns per column-pass workgroup of the Green passes of
 *               Step 1's inner iterations (cut to what LDS and thread
 *               counts allow)
 *   tvs_set_tiles  force these for the later calls and jobs of the context
 *                  (0 = the tuner's choice); TVS_EINVAL for a run length not
 *                  in {0, 1, 2, 4} or rows, cols outside [0, 64].  A rows,
 *                  cols pair that would move the Green passes to another
 *                  kernel (another thread count or code path, which may
 *                  round differently) is not applied: the tuner considers
 *                  and applies only shapes within the kernels a plan picks
 *   tvs_get_tiles  the tuner's choice for a shape, out[5] = {run1, run1d,
 *                  rows, cols, run2} (zeros if not tuned yet); for the block-DCT
 *                  realisation pass dtype + 2 */
int tvs_set_tiles(tvs_ctx* ctx, int run1, int run1d, int rows, int cols, int run2);
int tvs_get_tiles(tvs_ctx* ctx, int N2, int N1, tvs_dtype dtype, const tvs_layout* layout, double h, int* out);

/* Quality measures of Section 5.2 (used to pick the TFS weight delta and the
 * Step-2 parameters in the paper's experiments).
 *   tvs_tangent_field  tau_0 = (-D^{neum-}_y d, D^{neum-}_x d) of an N2 x N1
 *                      image d (device pointer), the tangent field of Step 1's
 *                      data (text after eq. ir2dualdis); applied to a clean
 *                      image it gives the ground-truth tangent field.
 *                      tau_out: device pointer, 2 x (N2+1) x (N1+1), planes
 *                      [tau_1, tau_2].  Stream-ordered, does not wait.
 *   tvs_quality        of x against ref, both n2 x n1 device arrays in dtype:
 *                      out[0] = PSNR = -10 log10 MSE (the paper fixes the
 *                      peak value R = 1; HUGE_VAL when x == ref), out[1] =
 *                      MSSIM (one window, the whole grid; means, variances
 *                      and covariance normalised by n2 n1; c1 = 1e-4, c2 =
 *                      9e-4), out[2] = MSE.  out is a host array of 3
 *                      doubles.  The moments are FP64 sums on the device in
 *                      two passes (means, then centred sums) in a fixed
 *                      order; the call waits for them.  TVS_ENONFINITE if a
 *                      moment is NaN or Inf.  Calls on one context share its
 *                      reduction buffers: they must not overlap. */
int tvs_tangent_field(tvs_ctx* ctx, const void* d, int N2, int N1, tvs_dtype dtype, double h, void* tau_out,
                      void* stream);
int tvs_quality(tvs_ctx* ctx, const void* x, const void* ref, int n2, int n1, tvs_dtype dtype, double* out,
                void* stream);

/* For callers that cannot allocate device memory (inside tight serving
 * loops, or harnesses that forbid hipMalloc): tvs_quality with the same
 * arguments, results, errors and sums, bit for bit, but it allocates nothing.
 * Its reduction scratch (1024 FP64 partial sums and the 6 moments, 8.3 KB)
 * is a static array of the library that every GPU holds once, from the first
 * tvs_ctx_create on it until the process ends; image sizes are limited as
 * for tvs_quality (n2 n1 <= 2^31), not by the scratch.  All calls on one GPU
 * share that array, whatever their context: calls that overlap on one GPU
 * (other threads, other streams) race and give wrong results.  The call
 * waits for its stream. */
int tvs_quality_noalloc(tvs_ctx* ctx, const void* x, const void* ref, int n2, int n1, tvs_dtype dtype,
                        double* out, void* stream);

/* Checkpoint and resume: a job's state between two sweeps (Algorithm 2's
 * outer iterate p^n of the current step, the subdomain duals q_m^n that the
 * next sweep's inner iterations start from, the FP64 energy history, the
 * sweep counters, and d0 and tau), copied into one host-memory blob that a
 * job created from it, in this or another context or process, continues from
 * as the original would have: the restored job's results equal the
 * uninterrupted job's bit for bit.  The blob is a versioned header followed
 * by the raw arrays in the job's dtype; it is portable between processes on
 * the same library version, not between versions.  The header begins with
 * char magic[8] = "TVSJOBST", uint32 version, uint32 header bytes, uint64
 * blob bytes, then int32 dtype, N2, N1 (native byte order).
 *   tvs_job_export_state  with buf == NULL: *bytes = the blob size (about
 *                      4 (Step 1) or 2 (Step 2) image planes on the grid plus
 *                      the subdomain frames, in the job's dtype; no device
 *                      work); otherwise copy the blob into the host buffer
 *                      buf of cap bytes (TVS_EINVAL if cap is too small),
 *                      ordered after the work already on `stream` (the
 *                      stream the job's sweeps were joined to), and wait for
 *                      the copy; the job itself is unchanged
 *   tvs_job_import_state  validate the blob (magic, version, sizes, and the
 *                      parameters as tvs_job_create does; TVS_EINVAL
 *                      otherwise), build a job of its shape in ctx, recompute
 *                      what is derived from d0 and tau on `stream` and load
 *                      the arrays; the call waits, so the caller may free
 *                      the blob on return.  The new job belongs to ctx and is
 *                      freed by tvs_job_destroy. */
int tvs_job_export_state(tvs_ctx* ctx, tvs_job* job, void* buf, size_t cap, size_t* bytes,
                         void* stream);
int tvs_job_import_state(tvs_ctx* ctx, const void* buf, size_t bytes, void* stream, tvs_job** out);

#ifdef __cplusplus
}
#endif

#endif /* TVS_H_ */
