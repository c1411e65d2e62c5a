/*
 * suppcg.h -- C ABI of the MI355X (gfx950) SupPCG library, libsuppcg.so.
 *
 * Superiorized preconditioned conjugate gradients for least-squares
 * tomography (Helou, Herman, Lin, Zibetti).  The library solves R x ~ b in the
 * least-squares sense (Section 2, eq. 2.1) through the normal equations
 * R^T R x = R^T b (eq. 2.2) with Algorithm 3 (SupPCG): each iteration perturbs
 * the iterate with Algorithm 1 (S_TV, total-variation superiorization,
 * Section 3.1) and then takes one Algorithm 2 (U_PCG) step, preconditioned by
 * M = F^-1 D F with the ramp-Hamming window of eq. (3.2).
 *
 * Conventions shared by every call:
 *  - Pointers to float/double/int32 data are DEVICE pointers (HBM of the
 *    context's GPU) unless a comment says "host".  The caller owns every data
 *    buffer; the library never frees caller memory.  The context owns its
 *    workspace (padded copies, FFT scratch, reduction partials, scalars), sized
 *    per geometry on first use and freed by sp_ctx_destroy.
 *  - Images are float32 [rows][cols], row-major: pixel (i, j) (0-based, row 0
 *    at the top) is element i*cols + j, as in the paper's TV definition
 *    (Section 3.1).  Its centre is x_j = (j - (cols-1)/2) * pixel,
 *    y_i = ((rows-1)/2 - i) * pixel.
 *  - Data (sinograms) are float32 [n_angles][n_bins], angle-major: ray (a, k)
 *    is element a*n_bins + k.  Ray (a, k) is the line
 *    x cos(theta_a) + y sin(theta_a) = s_k with theta_a = theta0 + a*dtheta and
 *    s_k = (k - (n_bins-1)/2) * bin_spacing + bin_offset (Section 4.1 uses
 *    equally spaced angles in [0, pi) and equally spaced parallel rays).
 *  - R[(a,k),(i,j)] is the length of ray (a, k) inside pixel (i, j); a ray
 *    running exactly along a pixel edge gives each adjacent pixel half a pixel.
 *  - Every call enqueues work on the context's stream and returns before it
 *    finishes, except where noted.  Arguments are validated before anything is
 *    enqueued; on error nothing is enqueued and sp_last_error() describes it.
 *  - Calls on one context are not thread-safe; use one context per thread.
 *  - Accumulation: data are float32; every dot product, norm, TV value and CG
 *    scalar (alpha, beta, p^T h, f) is accumulated and kept in float64, with
 *    fixed-order (deterministic) reductions.  Inside the solvers the iterate
 *    x_k, x_{k+1/2}, the search direction p and the residual r = R x - b are
 *    float64 (their float32 rounding, repeated every iteration and amplified
 *    by the cancellation in R^T r, is what moves a float32 iterate away from
 *    the float64 one); so are R z and R p, through which the solvers take
 *    Algorithm 2's h = A p (z^T h = (R z)^T (R p), p^T h = ||R p||^2; h itself
 *    is never formed).  The gradient g, M g and the TV direction are float32.
 *    Images passed in and out are float32.
 */
#ifndef SUPPCG_H
#define SUPPCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
enum {
    SP_OK = 0,
    SP_ERR_ARG = 1,          /* invalid argument (message in sp_last_error)      */
    SP_ERR_NOT_SPD = 2,      /* preconditioner parameters give an indefinite M   */
    SP_ERR_NONFINITE = 3,    /* a NaN/Inf reached a CG scalar                    */
    SP_ERR_HIP = 4,          /* HIP runtime error                                */
    SP_ERR_ALLOC = 5,        /* device allocation failed                         */
    /* informational results of sp_suppcg_solve (the outputs are valid):        */
    SP_MAXITER = 16,         /* max_iter loop bodies ran, f(x_{k-1/2}) > eps     */
    SP_CONVERGED = 17,       /* stopped because f(x_{k-1/2}) <= eps (Alg. 3)     */
    SP_BREAKDOWN_CONVERGED = 18, /* p^T h == 0: p = 0, the CG step is exact    */
    SP_TRIALS_EXHAUSTED = 19 /* some S_TV inner step accepted no trial          */
};

typedef struct sp_ctx sp_ctx;
typedef struct sp_learned sp_learned;

/* Parallel-beam geometry (Section 4.1).  dtheta <= 0 selects pi / n_angles.
 * Limits: 1 <= rows, cols <= 8192; 1 <= n_angles, n_bins <= 65536;
 * pixel > 0; bin_spacing >= 0.375 pixel. */
typedef struct {
    int32_t rows, cols;
    double pixel;
    int32_t n_angles;
    double theta0, dtheta;
    int32_t n_bins;
    double bin_spacing, bin_offset;
} sp_geometry;

/* Algorithm 1 parameters: K nonascending steps, step-length factor a in (0,1),
 * starting step gamma > 0.  The paper's repeat-until loop has no bound; here
 * an inner step tries at most max_trials step lengths (0 -> 100) and, if none
 * is accepted, leaves the image unchanged while keeping every increment of l.
 * Limits: 0 <= K <= 1000, 0 <= max_trials <= 10000. */
typedef struct {
    int32_t K;
    double a, gamma;
    int32_t max_trials;
} sp_tv_params;

/* Preconditioner (Section 3.2).  SP_PRECOND_RAMP: M = E^T F^-1 D F E with
 * D = h(|omega|), h(w) = (|w| + mu)(rho + (1 - rho) cos w) (eq. 3.2), on the
 * radial frequency of a zero-padded P x P grid, P = 2^ceil(log2(2 max(rows,
 * cols))); requires mu > 0 and 1/2 < rho <= 1 (else SP_ERR_NOT_SPD) and
 * images of at most 2048 pixels a side.
 * SP_PRECOND_NONE: M = I (plain CG).  SP_PRECOND_LEARNED: the network `net`. */
enum { SP_PRECOND_NONE = 0, SP_PRECOND_RAMP = 1, SP_PRECOND_LEARNED = 2 };
typedef struct {
    int32_t kind;
    double mu, rho;
    const sp_learned* net;
} sp_precond;

/* Solver controls.  eps: Algorithm 3's termination level (eps <= 0 disables
 * the test and runs exactly max_iter loop bodies).  The test of step 10,
 * f(x_{k-1/2}) <= eps, is taken at the top of each loop body, so the run that
 * stops has completed its last U_PCG step and x_last holds x_k.
 * flags: SP_FLAG_REPLAY makes
 * each S_TV inner step accept exactly after replay_trials[k*K + i] trials
 * (host array, max_iter*K entries; a value > max_trials means "no trial
 * accepted") instead of testing TV -- used to separate arithmetic differences
 * from control-flow differences. SP_FLAG_GRAPH captures one loop body in a
 * HIP graph and replays it.
 * SP_FLAG_RESUME (sp_suppcg_solve only): skip steps 1-9 and run max_iter more
 * loop bodies from the state the context holds -- left by the previous solve
 * on it, or put there by sp_state_load -- with x0 ignored.  The geometry, the
 * S_TV parameters and the preconditioner must be those the state was made
 * with (else SP_ERR_ARG); b must be the same data.  A run that stopped on the
 * eps test continues (the test is taken again with the new eps); one that
 * stopped on a breakdown or a non-finite value returns that status at once.
 * A run of N bodies and one of N1 followed by a resumed run of N - N1 give
 * bitwise the same images and scalars.
 * SP_FLAG_ASYNC: the call enqueues the whole run and returns SP_OK without
 * waiting; k_out is then a DEVICE int32 pointer (batched: int32[n]) that
 * receives k when the run completes, trace must be NULL, and loop bodies
 * after a stop are enqueued and do nothing.  sp_solve_status gives the
 * statuses once the work is done.  The buffers passed in must stay valid
 * until then. */
enum { SP_FLAG_REPLAY = 1u, SP_FLAG_GRAPH = 2u, SP_FLAG_AUTOTUNE = 4u, SP_FLAG_RESUME = 8u,
       SP_FLAG_ASYNC = 16u };
typedef struct {
    double eps;
    int32_t max_iter;
    uint32_t flags;
    const int32_t* replay_trials; /* host; nullable unless SP_FLAG_REPLAY */
} sp_solve_params;

/* Per-iteration trace (all HOST arrays, capacity `cap` iterations; any pointer
 * may be NULL).  Entry k-1 belongs to loop body k: f_half = f(x_{k+1/2}),
 * tv_half = TV(x_{k+1/2}) as evaluated by the accepted trial, ell = l_{k+1},
 * alpha/beta of U_PCG, s_norm = ||s_k||; trials has cap*K entries. */
typedef struct {
    double* f_half;
    double* tv_half;
    double* alpha;
    double* beta;
    double* s_norm;
    int32_t* ell;
    int32_t* trials;
    int32_t cap;
    double f0;      /* out: f(x_0) */
    double alpha0;  /* out: alpha of the initial step (Alg. 3, step 6) */
    int32_t fallbacks; /* out: 1 if a learned preconditioner was replaced by the
                          Fourier one during the run, else 0 */
    /* DEVICE float32 [g_snap_count][rows][cols] or NULL: row k-1 receives
     * g_{k+1/2} = R^T (R x_{k+1/2} - b), the gradient that loop body k hands to
     * the preconditioner (Algorithm 2, step 1), for k = 1 .. g_snap_count.
     * Rows of bodies that did not run are left untouched. */
    float* g_snap;
    int32_t g_snap_count;
    int32_t bodies;   /* out: loop bodies this call ran (entries written) */
    /* Selective error of every iterate (Section 4.2, eq. 4.1), evaluated on
     * the device inside the loop body: se_ref is the phantom (DEVICE float32
     * [rows][cols]) or NULL to skip; se_axes and se_c give the ellipse S and
     * C as for sp_selective_error.  se (HOST [cap], nullable): se[k-1] =
     * SE(x_{k+1}), the iterate loop body k forms (NaN if its step could not be
     * formed).  se0, se1 (out): SE(x_0) and SE(x_1); NaN on a resumed run,
     * which skips steps 1-9. */
    const float* se_ref;
    double se_axes[2];
    double se_c;
    double* se;
    double se0, se1;
    /* Wall time (HOST [cap], nullable): t_ms[k-1] = milliseconds from the
     * call's first launch to the end of loop body k, from HIP events on the
     * stream between loop bodies (between graph replays with SP_FLAG_GRAPH).
     * t1_ms (out): to the end of steps 1-9 (NaN when t_ms is NULL). */
    double* t_ms;
    double t1_ms;
} sp_trace;

/* ---- context ------------------------------------------------------------ */
/* Creates a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the handle. */
int sp_ctx_create(int device, void* hip_stream, sp_ctx** out);
int sp_ctx_destroy(sp_ctx* ctx);
/* Changes the stream later calls enqueue on. */
int sp_ctx_set_stream(sp_ctx* ctx, void* hip_stream);
/* Host string describing the last failure on ctx; valid until the next call.
 * sp_ctx_last_error is the same call under the context's prefix. */
const char* sp_last_error(const sp_ctx* ctx);
const char* sp_ctx_last_error(const sp_ctx* ctx);
/* Library version string (host, static). */
const char* sp_version(void);

/* ---- operators ------------------------------------------------------------ */
/* y = R x (Section 2: the projection matrix applied to image x).
 * x: [rows][cols] float32 (device, read); y: [n_angles][n_bins] (device, written). */
int sp_project(sp_ctx* ctx, const sp_geometry* g, const float* x, float* y);

/* x = R^T y, the transpose of sp_project's weights, pixel-driven, no atomics
 * (eq. 2.2).  Each (ray, pixel) weight is the same chord length sp_project
 * uses, equal to float64 rounding (bit for bit at axis-parallel angles; R
 * splits oblique rays band by band, R^T evaluates the trapezoid).
 * y: [n_angles][n_bins] (device, read); x: [rows][cols] (device, written). */
int sp_backproject(sp_ctx* ctx, const sp_geometry* g, const float* y, float* x);

/* sp_backproject for callers that cannot allocate device memory (code being
 * captured into a HIP graph, tight serving loops, harnesses that forbid
 * hipMalloc): the same x = R^T y, bit for bit, with the context's workspace
 * replaced by one static 32 MiB scratch array per GPU (the angle table and
 * the padded, wmax-scaled sinogram; held until the process ends).  The call
 * allocates no device or host memory.  It needs n_angles <= 8192 and
 * n_angles * 96 (rounded up to 256) + n_angles * (n_bins + 8) * 4 bytes to
 * fit in the 32 MiB, else SP_ERR_ARG and nothing is enqueued.  Every call on a GPU
 * shares that GPU's array and rewrites it whole; calls that overlap on one
 * GPU (other streams, other contexts, other threads) race and must be
 * ordered by the caller.  y: [n_angles][n_bins], x: [rows][cols] (device). */
int sp_backproject_noalloc(sp_ctx* ctx, const sp_geometry* g, const float* y, float* x);

/* r = R x - b and *f = ||r||^2 (float64, device scalar) -- the primary
 * criterion f(x) = ||Rx - b||^2 of Section 2.  r may equal NULL. */
int sp_residual(sp_ctx* ctx, const sp_geometry* g, const float* x, const float* b,
                float* r, double* f);

/* grad = A x - y = R^T (R x - b), the gradient step 1 of Algorithm 2 forms
 * (A = R^T R, y = R^T b, Section 3.3), computed as the solvers compute it:
 * the residual R x - b is kept in float64 between the two operators.
 * *f = ||R x - b||^2 (float64 device scalar, nullable).
 * x: [rows][cols], b: [n_angles][n_bins], grad: [rows][cols] (device). */
int sp_gradient(sp_ctx* ctx, const sp_geometry* g, const float* x, const float* b, float* grad,
                double* f);

/* z = M g with the preconditioner of Section 3.2 (see sp_precond).
 * g, z: [rows][cols] (device); g and z may alias. */
int sp_precond_apply(sp_ctx* ctx, const sp_geometry* g, const sp_precond* pc,
                     const float* gin, float* z);

/* *tv = TV(x) (Section 3.1), float64 device scalar. */
int sp_tv(sp_ctx* ctx, const sp_geometry* g, const float* x, double* tv);

/* Selective error of Section 4.2, eq. (4.1): SE(x) = C sqrt(sum over S of
 * (x_ij - ref_ij)^2), in float64.  S holds the pixels whose centres (as for R)
 * lie in the closed centred ellipse with semi-axes axes[0] (horizontal:
 * along a row) and axes[1] (vertical), in the geometry's length unit
 * (HOST double[2], both > 0).  C <= 0 selects C = 1 / sqrt(sum over S of
 * ref_ij^2), the relative error inside S (NaN when that sum is 0).  x, ref:
 * DEVICE float32 [rows][cols]; se: DEVICE double, written on the stream. */
int sp_selective_error(sp_ctx* ctx, const sp_geometry* g, const float* x, const float* ref,
                       const double* axes, double C, double* se);

/* t_bar = minus the gradient of TV where defined, 0 elsewhere (Section 3.1);
 * *norm2 = ||t_bar||^2 (float64 device scalar, nullable). */
int sp_tv_grad(sp_ctx* ctx, const sp_geometry* g, const float* x, float* tbar, double* norm2);

/* Algorithm 1: (s, l) = S_TV(x, l, a, gamma, K); writes x_half = x + s
 * (evaluated in float64 on the float32 x, rounded to float32 once).
 * ell: device int32, read and updated in place.  tv_half: device float64,
 * TV(x_half) (nullable).  trials: device int32[K], trials used by each inner
 * step, max_trials + 1 when none was accepted (nullable). */
int sp_tv_perturb(sp_ctx* ctx, const sp_geometry* g, const sp_tv_params* p, const float* x,
                  int32_t* ell, float* x_half, double* tv_half, int32_t* trials);

/* ---- solver ----------------------------------------------------------------- */
/* Algorithm 3, SupPCG(x0, a, gamma, K, eps).  tv = NULL or K = 0 gives plain
 * PCG (CG with SP_PRECOND_NONE).  b: [n_angles][n_bins]; x0: [rows][cols]
 * (NULL = zero image).  x_out receives x_{k-1/2}, the paper's output;
 * x_last (nullable) receives x_k.  *k_out (host) receives k.  Blocks until
 * the run has finished.  Returns SP_MAXITER, SP_CONVERGED,
 * SP_BREAKDOWN_CONVERGED or SP_TRIALS_EXHAUSTED on success (outputs valid),
 * an SP_ERR_* code otherwise. */
int sp_suppcg_solve(sp_ctx* ctx, const sp_geometry* g, const float* b, const float* x0,
                    const sp_tv_params* tv, const sp_precond* pc, const sp_solve_params* sp,
                    float* x_out, float* x_last, int32_t* k_out, sp_trace* trace);

/* ---- checkpoint / resume ------------------------------------------------------
 * The state Algorithm 3 carries from one loop body to the next: x_k,
 * x_{k-1/2}, p_{k-1} (float64), h_{k-1} in the form the solver keeps it,
 * q = R p_{k-1} (n_angles x n_bins float64; h = R^T q), and the scalars p^T h, l_k,
 * k, f(x_{k-1/2}), f(x_0), the stop status and, for a learned preconditioner,
 * whether it has been replaced by the Fourier one, together with the geometry,
 * the S_TV parameters and the preconditioner parameters.  The learned network's
 * weights are not part of it.
 * sp_state_save copies the state the context holds after a single-slice solve
 * (or an sp_state_load) to host memory: with host_blob == NULL it only writes
 * the size needed to *bytes; else *bytes gives the blob's capacity and
 * receives the size written (SP_ERR_ARG if too small or if the context holds
 * no state).  It waits for the context's stream.
 * sp_state_load puts a saved blob into a context (of this library version, on
 * any device) so that a solve with SP_FLAG_RESUME continues from it; it
 * validates the blob and the geometry (SP_ERR_ARG otherwise). */
int sp_state_save(sp_ctx* ctx, void* host_blob, int64_t* bytes);
int sp_state_load(sp_ctx* ctx, const void* host_blob, int64_t bytes);

/* k and status of the slices of the last solve on ctx (count = 1 after
 * sp_suppcg_solve, n after the batched solve): waits for the context's stream;
 * status is SP_MAXITER, SP_CONVERGED, SP_BREAKDOWN_CONVERGED,
 * SP_TRIALS_EXHAUSTED or SP_ERR_NONFINITE.  k and status are host arrays. */
int sp_solve_status(sp_ctx* ctx, int32_t count, int32_t* k, int32_t* status);

/* ---- batched solver -----------------------------------------------------------
 * Algorithm 3 on n independent slices of any mix of geometries, advanced in
 * lockstep: every stage of the loop body is ONE launch whose workgroups walk a
 * table of (slice, block) work items covering all slices, so slices of uneven
 * size share the GPU without a launch per slice.  Per slice the arithmetic,
 * the partial sums and their order are those of sp_suppcg_solve, so every
 * slice's result equals its single-slice solve bit for bit.  Each slice halts
 * on its own (breakdown, non-finite value, eps); the others continue.
 *   geoms[n], b[n] (device [n_angles][n_bins]), x_out[n] (device, x_{k-1/2}):
 *     per-slice arrays of host pointers; x0 (NULL, or n entries each NULL =
 *     zero image) and x_last (NULL, or n entries) likewise.
 *   pc: SP_PRECOND_RAMP or SP_PRECOND_NONE, shared by all slices.
 *   sp->flags: SP_FLAG_GRAPH captures one loop body in a HIP graph and replays
 *     it; SP_FLAG_ASYNC as for sp_suppcg_solve (k_out device int32[n]);
 *     SP_FLAG_AUTOTUNE first tunes the projector launch shapes (sp_tune_shapes)
 *     of every slice geometry the shape table does not hold, then times the
 *     dispatch of the heavy stages (item order: slice-major or grouped by
 *     XCD; grid: one workgroup per item or a persistent 2/4/8 workgroups per
 *     CU) once per batch layout and keeps the fastest; SP_FLAG_REPLAY and
 *     SP_FLAG_RESUME are not supported here.
 *   k_out: host [n].  trace (nullable): host arrays [n][cap] and status[n].
 * Limits: 1 <= n <= 4096; each slice within the single-slice limits.
 * Returns SP_OK when every slice ended without error (per-slice SP_MAXITER /
 * SP_CONVERGED / SP_BREAKDOWN_CONVERGED / SP_TRIALS_EXHAUSTED in
 * trace->status), else the first slice's SP_ERR_* code. */
typedef struct {
    double* f_half;   /* [n][cap] f(x_{k+1/2}) of loop body k */
    double* tv_half;  /* [n][cap] TV(x_{k+1/2}) */
    int32_t* ell;     /* [n][cap] l_{k+1} */
    int32_t cap;
    int32_t* status;  /* [n] */
} sp_batch_trace;

int sp_suppcg_solve_batched(sp_ctx* ctx, int32_t n, const sp_geometry* geoms,
                            const float* const* b, const float* const* x0,
                            const sp_tv_params* tv, const sp_precond* pc,
                            const sp_solve_params* sp, float* const* x_out,
                            float* const* x_last, int32_t* k_out, sp_batch_trace* trace);

/* Launch shapes in use by the batched solver, per stage (prep, project,
 * backproject, FFT rows, FFT columns, TV, vector, per-slice): out[2 s] = item
 * order (0 slice-major, 1 grouped by XCD), out[2 s + 1] = workgroups per CU of
 * the persistent grid (0 = one workgroup per item).  count >= 16. */
int sp_batch_tuning(sp_ctx* ctx, int32_t* out, int32_t count);

/* ---- learned preconditioner ---------------------------------------------------
 * M = C^T diag(softplus(d)) C, with C a stack of `layers` linear 3x3
 * convolutions without bias (cross-correlation, zero "same" padding),
 * 1 -> channels -> ... -> channels, and C^T its exact adjoint; M is symmetric
 * positive semi-definite by construction.  Not in the paper: it replaces the
 * Fourier preconditioner of Section 3.2 in step 2 of Algorithm 2 when passed
 * as sp_precond{SP_PRECOND_LEARNED, mu, rho, net}; (mu, rho) then define the
 * Fourier preconditioner the solver switches to, for the rest of the run, as
 * soon as g^T z <= 0 or g^T z is not finite.
 * Parameters theta (float32, num_params values): W_1 [channels][1][3][3],
 * W_2..W_L [channels][channels][3][3], d [channels]; tap (ky, kx) reads the
 * input at offset (ky - 1, kx - 1).  Supported: channels = 16,
 * 1 <= layers <= 8.  The object owns its parameters, Adam moments and
 * workspace (device memory of the context's GPU). */
int sp_lp_create(sp_ctx* ctx, int32_t layers, int32_t channels, sp_learned** out);
int sp_lp_destroy(sp_learned* net);
int64_t sp_lp_num_params(const sp_learned* net);
/* Copies count = num_params float32 values from / to HOST memory. */
int sp_lp_set_params(sp_ctx* ctx, sp_learned* net, const float* theta, int64_t count);
int sp_lp_get_params(sp_ctx* ctx, const sp_learned* net, float* theta, int64_t count);
/* The same two calls under the names of the network's weights. */
int sp_lp_set_weights(sp_ctx* ctx, sp_learned* net, const float* w, int64_t count);
int sp_lp_get_weights(sp_ctx* ctx, const sp_learned* net, float* w, int64_t count);
/* z = M u for `batch` images u, z: [batch][rows][cols] float32 (device). */
int sp_lp_apply(sp_ctx* ctx, sp_learned* net, int32_t batch, int32_t rows, int32_t cols,
                const float* u, float* z);
/* Training loss over the minibatch idx[0..batch) (device int32, values in
 * [0, nprobe)) of probe pairs Av, v ([nprobe][rows][cols], device):
 * loss = mean_b ||P(M(Av_b) - v_b)||^2 / ||P v_b||^2 -> *loss (device
 * float64), P = restriction to the pixels at least `margin` from every edge
 * (0: all pixels; M reaches 2 * layers pixels, so with that margin the loss on
 * crops of larger images equals the full-size loss on the crop interiors);
 * grad (device float32, num_params) = d loss / d theta.
 * Requires 0 <= margin and 2 * margin < min(rows, cols). */
int sp_lp_loss_grad(sp_ctx* ctx, sp_learned* net, int32_t rows, int32_t cols, const float* Av,
                    const float* v, int32_t nprobe, const int32_t* idx, int32_t batch,
                    int32_t margin, double* loss, float* grad);
/* One Adam step theta -= lr * mhat / (sqrt(vhat) + eps) with gradient grad
 * (device float32); step counts from 1. */
int sp_lp_adam_step(sp_ctx* ctx, sp_learned* net, const float* grad, double lr, double beta1,
                    double beta2, double eps, int32_t step);

/* ---- ART and SupART (Section 3.4) ---------------------------------------------
 * ART for the Bayesian criterion of eq. (2.3), r^2 ||R x - b||^2 +
 * ||x - mu||^2: each step projects (x, u) toward the hyperplane of one ray of
 * the system r R (x - mu) + u = r (b - R mu) with relaxation lambda,
 *   c = lambda (r (b_i - <R_i, x>) - u_i) / (1 + r^2 ||R_i||^2),
 *   u_i += c, x += r c R_i^T;
 * one iteration is a cycle through all rays, angle by angle in increasing
 * index and, within an angle, in q phases (rays k = ph, ph + q, ... for
 * ph = 0 .. q-1, q = floor(2 e / ds + 1e-9) + 1 with e = pixel (|cos| +
 * |sin|) / 2): the rays of a phase touch disjoint pixels and are projected
 * concurrently.  mu is the uniform image at the mean gray level estimated
 * from the data, bin_spacing * sum(b) / (n_angles * rows * cols * pixel^2);
 * x starts at x0 (DEVICE float32 [rows][cols]; NULL: mu) and u at 0; rays with
 * R_i = 0 are skipped.  With tv->K > 0 each iteration first applies
 * Algorithm 1 (SupART, the superiorized step of Section 3.1); tv NULL or K = 0
 * is ART.  r > 0, 0 < lambda < 2.  sp: max_iter iterations (eps is ignored;
 * flags: SP_FLAG_GRAPH only).  x_out (DEVICE float32) receives x after the
 * last cycle.  trace (nullable): ell, tv_half and trials as for the solver
 * (entry k-1: iteration k's S_TV), se[k-1] = SE(x_k) with se0 = SE(x_0), and
 * t_ms[k-1] = milliseconds to the end of iteration k; f_half, alpha, beta,
 * s_norm, g_snap, se1 and t1_ms are not written (se1, t1_ms: NaN).  The
 * iterate is float64 on the device.  Returns SP_MAXITER, or
 * SP_TRIALS_EXHAUSTED if an S_TV inner step accepted no trial. */
int sp_supart_solve(sp_ctx* ctx, const sp_geometry* g, const float* b, const float* x0,
                    const sp_tv_params* tv, double r, double lambda, const sp_solve_params* sp,
                    float* x_out, sp_trace* trace);
/* BlobART (Section 3.4, blob basis): the same ART on the coefficients c of
 * the image x(p) = sum_j c_j b(|p - p_j|), with generalised Kaiser-Bessel
 * blobs b(r) = w^2 I_2(10.4 w) / I_2(10.4), w = sqrt(1 - (r/2)^2), radius 2
 * pixels, centred on the pixel centres; the system matrix entry of ray i and
 * blob j is the blob's line integral at the distance of centre j from ray i,
 * 2 sqrt(2 pi / 10.4) / I_2(10.4) w^(5/2) I_(5/2)(10.4 w) (times the pixel
 * size).  The Bayesian criterion acts on c, whose start is the uniform value
 * whose image is the mean gray level mu; rays of an angle are taken in
 * floor(4 / ds + 1e-9) + 1 phases (ds in pixels).  x_out and the trace's
 * selective errors are the image sampled at the pixel centres.  Otherwise as
 * sp_supart_solve with no S_TV. */
int sp_blobart_solve(sp_ctx* ctx, const sp_geometry* g, const float* b, double r, double lambda,
                     const sp_solve_params* sp, float* x_out, sp_trace* trace);

/* ---- launch shapes ------------------------------------------------------------
 * Two launch shapes of the projector pair can be chosen per geometry: the
 * number of parts R splits each ray's walk into (1, 2, 4 or 8; the parts'
 * float64 sums are added in part order, so the choice changes R's results by
 * rounding) and the pixels per lane of R^T (2 or 4; the results do not
 * depend on it).  By default a rule of the image size and the wave slots
 * picks them.  The choices live in one process-wide table keyed by the whole
 * geometry; every solve, operator and batch of that geometry built after an
 * update uses them, so single and batched solves of a geometry stay bitwise
 * equal (a batch takes 4 pixels per lane for all slices only if all of them
 * agree on it).  Updating the table between the two halves of a resumed run
 * changes R's rounding between them.
 * sp_tune_shapes: times sp_project for each part count (with the default
 * pixels per lane) and then sp_backproject for 2 and 4 pixels per lane on the
 * context's stream, keeps the fastest (the default wins ties within 2%), and
 * stores it; ms (HOST double[6], nullable) receives the best-of-5 times of R
 * at 1, 2, 4, 8 parts and of R^T at 2, 4 pixels per lane.  Synchronises.
 * sp_tuning_set: stores a choice (parts 1..8, px 2 or 4; both 0 erases the
 * entry); SP_ERR_ARG for other values or an invalid geometry.
 * sp_tuning_list: *count = entries; copies up to cap of them to HOST arrays
 * (each nullable).  sp_tuning_clear: erases all entries.  These three touch no
 * device. */
int sp_tune_shapes(sp_ctx* ctx, const sp_geometry* g, int32_t* parts, int32_t* px, double* ms);
int sp_tuning_set(const sp_geometry* g, int32_t parts, int32_t px);
int sp_tuning_list(sp_geometry* geoms, int32_t* parts, int32_t* px, int32_t cap, int32_t* count);
int sp_tuning_clear(void);

/* ---- stored matrices (Section 2, eqs. 2.1-2.2) ---------------------------------
 * R as an explicit sparse matrix: entry (a * n_bins + k, i * cols + j) is the
 * length of ray k of angle a inside pixel (i, j), the same lengths the
 * matrix-free sp_project uses (float32 here, rounded from float64).  Both R
 * (rows by ray) and R^T (rows by pixel) are kept, so each product streams its
 * matrix once, as sliced ELLPACK with 64-row slices: int32 column indices and
 * float32 weights, 8 bytes per stored entry (rows shorter than their slice's
 * longest are padded; the padding is never read).  R and R^T are built from
 * one weight function and are exact transposes; only strictly positive
 * lengths are stored.  Within a row of R the pixels follow the major axis of
 * the ray's walk (image rows when |cos| >= |sin|, else columns); within a row
 * of R^T the rays increase.
 * sp_matrix_build: builds both on the context's device (allocates about
 * 16 bytes per nonzero plus padding; SP_ERR_ALLOC if that fails; SP_ERR_ARG
 * for an invalid geometry or n_angles * n_bins >= 2^31) and synchronises the
 * stream.  The matrix may be used with any context on the same device.
 * sp_matrix_project: y = R x (x DEVICE float32 [rows][cols], y DEVICE float32
 * [n_angles][n_bins]); sp_matrix_backproject: x = R^T y; both enqueue one
 * launch on the context's stream and sum each row in float64 in a fixed
 * order.
 * sp_matrix_info: nonzeros of R and device bytes held by both sides.
 * sp_matrix_export: copies side 0 (R) or 1 (R^T) to HOST arrays in compressed
 * sparse row form, row_ptr [rows + 1], col [nnz], val [nnz] (each nullable);
 * synchronises. */
typedef struct sp_matrix sp_matrix;
int sp_matrix_build(sp_ctx* ctx, const sp_geometry* g, sp_matrix** out);
int sp_matrix_destroy(sp_matrix* m);
int sp_matrix_info(const sp_matrix* m, int64_t* nnz, int64_t* bytes);
int sp_matrix_project(sp_ctx* ctx, const sp_matrix* m, const float* x, float* y);
int sp_matrix_backproject(sp_ctx* ctx, const sp_matrix* m, const float* y, float* x);
int sp_matrix_export(sp_ctx* ctx, const sp_matrix* m, int side, int64_t* row_ptr, int32_t* col,
                     float* val);

/* ---- instrumentation --------------------------------------------------------- */
/* While profiling is enabled on a context, every projector, backprojector,
 * preconditioner, S_TV and loop-body launch made through it is bracketed by
 * HIP events on the context's stream, and sp_suppcg_solve runs its loop
 * eagerly (SP_FLAG_GRAPH is ignored).  sp_profile_read synchronises the stream
 * and returns the summed milliseconds and the number of timed launches of one
 * kind since profiling was last enabled.  Events are created on the host; no
 * device memory is allocated. */
enum { SP_PROF_PROJECT = 0, SP_PROF_BACKPROJECT = 1, SP_PROF_PRECOND = 2, SP_PROF_TV = 3,
       SP_PROF_ITERATION = 4, SP_PROF_STORED_PROJECT = 5, SP_PROF_STORED_BACKPROJECT = 6,
       SP_PROF_KINDS = 7 };
int sp_profile_enable(sp_ctx* ctx, int on);
int sp_profile_read(sp_ctx* ctx, int kind, double* total_ms, int32_t* count);

#ifdef __cplusplus
}
#endif
#endif /* SUPPCG_H */
