/*
 * radonlp.h -- C-ABI of the log-polar Radon transform library for AMD MI355X (gfx950).
 *
 * The Radon transform R and its adjoint, the back-projection R#, are applied as
 * periodic convolutions in log-polar coordinates over M angular partitions, following
 * Andersson, Carlsson and Nikitin, "Fast algorithms and efficient GPU implementations
 * for the Radon transform and the back-projection operator represented as convolution
 * operators" (arXiv 1506.00014): sec. 2 (the transform as a log-polar convolution,
 * eq. logdef, lograd_periodic, Tdef, Radon_all_pb), sec. 3 (kernel coefficients,
 * eq. exprcoef1; sampling, eq. Xgrid, Polargrid, vrho, Lopolargrid_f,
 * Lopolargrid_polar), sec. 4 (cubic B-spline interpolation, eq. Bsplineinterp,
 * wsumn) and sec. 5 (Algorithm 1, fast Radon transform).
 *
 * Conventions shared by every entry point
 *   - Image f: N x N float32, row-major, f[iy][ix] is the value at the node
 *     x = (-1 + ix*2/N, -1 + iy*2/N) (column index = x1, row index = x2); the object
 *     is assumed supported in the unit disc.
 *   - Sinogram g: N_theta x N_s float32, row-major, g[j][k] = R f(theta_j, s_k) with
 *     theta_j = j*pi/N_theta and s_k = -1 + k*2/N_s, and x . theta = x1 cos + x2 sin.
 *   - A batch of B slices is B such arrays back to back.
 *   - All data pointers are DEVICE pointers owned by the caller (for example torch
 *     tensors).  Inputs and outputs must not overlap.  Outputs are fully overwritten.
 *   - Every operation is enqueued asynchronously on the given stream; no call
 *     allocates device memory, synchronises the host, or reads device memory from
 *     the host, except rl_plan_create (which builds and uploads tables),
 *     rl_plan_destroy, rl_plan_autotune and rl_batch_create.  The workspace is caller-provided and must be at least
 *     rl_workspace_bytes(plan, batch, op) bytes, 256-byte aligned; it may be reused
 *     by consecutive calls on the same stream but not by concurrent calls.
 *   - Errors never abort: each call returns an rl_status, and rl_last_error() returns
 *     a message describing the last failure of the calling thread.
 */
#ifndef RADONLP_H
#define RADONLP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RL_OK = 0,
  RL_ERR_INVALID_ARG = 1,    /* null pointer, negative batch, bad enum, overlapping buffers */
  RL_ERR_GEOMETRY = 2,       /* geometry violates a bound of the paper or of this library */
  RL_ERR_WORKSPACE = 3,      /* workspace missing, too small or misaligned */
  RL_ERR_HIP = 4,            /* a HIP runtime call or kernel launch failed */
  RL_ERR_UNSUPPORTED_ARCH = 5, /* current device is not gfx950 */
  RL_ERR_INTERNAL = 6
} rl_status;

/* Operation selector for rl_workspace_bytes (RL_OP_EM: rl_em and, with batch 1, rl_em_norm;
 * RL_OP_BP_LP: radon_bp_lp; RL_OP_FBP_LP: fbp_lp). */
typedef enum {
  RL_OP_FWD = 0,
  RL_OP_ADJ = 1,
  RL_OP_FBP = 2,
  RL_OP_EM = 3,
  RL_OP_BP_LP = 4,
  RL_OP_FBP_LP = 5
} rl_op;

/* Filters of filtered back-projection (sec. 6, eqs. ramp, cosfilt, SLfilt).  The ramp
 * is the Ram-Lak kernel; cosine and Shepp-Logan multiply the ramp's spectrum on the
 * zero-padded s-axis (length lr, the smallest power of two >= 2 n_s and >= 16) at bin k,
 * |k| <= lr / 2, by cos(pi |k| / lr) and sinc(|k| / (2 lr)) (sinc(x) = sin(pi x) / (pi x)):
 * the paper's cos(2 pi sigma / N) and sinc(sigma / N) with sigma = |k| / (lr ds), N = n_s.
 * Other values return RL_ERR_INVALID_ARG. */
typedef enum { RL_FILTER_RAMLAK = 0, RL_FILTER_COSINE = 1, RL_FILTER_SHEPP_LOGAN = 2 } rl_filter;

/*
 * Geometry: every field fixes the discrete operator (changing any of them changes
 * the result).  Bounds, checked by rl_plan_create:
 *   n        image side N, even, 8 <= N <= 8192
 *   n_theta  angles N_theta >= m, <= 16384
 *   n_s      detector bins N_s, 2 <= N_s <= 4096
 *   m        angular partitions M >= 3, beta = pi/M (sec. 2)
 *   n_rho    rho-FFT length 2^a 3^b, a multiple of 4, >= ceil(log a_r / log(1 - 2 a_R / N))
 *            (sec. 3 eq. vrho), <= 8192
 *   k_theta  theta-FFT length >= 2*q_theta*ceil(N_theta/M) (sec. 5, the grid of size
 *            2 N_theta / M, in lattice rows), >= n_sup = q_theta*(n_own - 1) + 5 (the lattice
 *            rows of the owned rows plus two on each side): 8, 12, 16, 24, 32, or 32 times one
 *            of 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64 (the theta pass's four-step splits)
 *   r_dec    fine angular oversampling of the log-polar grid: (Delta theta / q_theta) / r_dec
 *            <= 2 a_R / N (sec. 3, before eq. Lopolargrid_f), <= 32
 *   dec_filter  theta low-pass used to go from the fine grid to the coarse one
 *            (Algorithm 1 step 4; not specified by the paper), its response divided out in
 *            the Fourier multiplier: 0 = cubic B-spline FIR d_n = B(n/r)/r, |n| < 2r;
 *            1 = box of one coarse cell, d_n = 1/r for |n| < r/2 and 1/(2r) at |n| = r/2
 *            (the cell's edges, present for even r).  Other values: RL_ERR_GEOMETRY.
 *   q_theta  coarse lattice spacing Delta theta / q_theta (1: the sinogram's spacing, the grid
 *            Omega_p of sec. 3 eq. Lopolargrid_polar; 2: twice as fine in theta, with the
 *            owned sinogram rows on every other lattice row).  1 or 2; the Algorithm 2 entry
 *            points (radon_bp_lp, fbp_lp) need 1.
 */
typedef struct {
  int32_t n;
  int32_t n_theta;
  int32_t n_s;
  int32_t m;
  int32_t n_rho;
  int32_t k_theta;
  int32_t r_dec;
  int32_t dec_filter;
  int32_t q_theta;
} rl_geom;

typedef struct rl_plan rl_plan;

/* Execution-only launch parameters of a plan.  They change block shapes and schedules, not the
 * operator: with every setting of the first five, every output value is computed by the same
 * arithmetic in the same order (bitwise identical results); adj_walk changes R#'s rounding only
 * (see below).
 *   theta_cols       spectrum columns per block of the theta-convolution pass (1 .. 8, capped
 *                    at 256 / the larger factor of k_theta; 0 = the largest allowed)
 *   theta_xcd_order  1: blocks of the theta pass are ordered so that neighbouring column strips
 *                    (which share cache lines) run on the same XCD (L2); 0: launch order
 *   prefilter_rows   image rows per block of the B-spline prefilter, a multiple of 32 in
 *                    [32, 4096]
 *   fwd_patch_split  1: forward gather tiles whose image box fits the small LDS patch run with
 *                    it (more blocks per CU), the others with the large one; 0: all large
 *   fwd_xcd_order    1: blocks of the forward gather are ordered so that each XCD (with its own
 *                    L2) runs one contiguous run of the tile list (neighbouring tiles read
 *                    overlapping image boxes); 0: launch order
 *   adj_walk         walk of the back-projection's Cartesian splat (both sum each sample's 16
 *                    weighted values in a register footprint that follows the ray and add what it
 *                    leaves behind to the LDS tile): 0 moves the footprint under branches, 1 moves
 *                    it by selects every step (uniform across a wave) and takes e^rho along the
 *                    ray by a running product.  The two add the same FP32 terms up to the last
 *                    bits of the FP64 sample positions, in FP64, in a different order.
 * Defaults (rl_plan_create): 0, 1, 512, 1, 1, 1. */
typedef struct {
  int32_t theta_cols;
  int32_t theta_xcd_order;
  int32_t prefilter_rows;
  int32_t fwd_patch_split;
  int32_t fwd_xcd_order;
  int32_t adj_walk;
} rl_tune;

/* Read / replace the plan's launch parameters.  rl_plan_set_tuning validates *tune
 * (RL_ERR_INVALID_ARG if a field is out of range) and must not run concurrently with calls that
 * use the plan. */
rl_status rl_plan_get_tuning(const rl_plan* plan, rl_tune* out);
rl_status rl_plan_set_tuning(rl_plan* plan, const rl_tune* tune);

/* Workspace bytes rl_plan_autotune needs for `batch` slices. */
size_t rl_tune_workspace_bytes(const rl_plan* plan, int32_t batch);

/* Autotuner: time radon_fwd and radon_adj on `batch` slices of synthetic data (written into the
 * workspace) for candidate values of each field of rl_tune in turn (coordinate descent, each
 * candidate timed with HIP events over three runs after one warm-up, keeping the fastest), and
 * set the best on the plan.  If cache_path is not NULL, the result is first looked up in that
 * file and, when absent, appended to it: one JSON object per line with the key
 * "<arch> rocm=<HIP version> n=.. n_theta=.. n_s=.. m=.. n_rho=.. k_theta=.. r_dec=.. dec_filter=.. q_theta=..
 * batch=..", the four fields and the measured R and R# times.  Synchronous on `stream` (it waits
 * for its own work), not capturable; not concurrent with other calls using the plan.  Errors:
 * RL_ERR_WORKSPACE if ws_bytes < rl_tune_workspace_bytes(plan, batch); RL_ERR_INVALID_ARG for a
 * NULL plan or batch < 1; RL_ERR_INTERNAL if the cache file cannot be written. */
rl_status rl_plan_autotune(rl_plan* plan, int32_t batch, void* d_ws, size_t ws_bytes, hipStream_t stream,
                           const char* cache_path);

/* Fill *out with the default geometry for (n, n_theta, n_s, m) on a coarse lattice q_theta (1 or
 * 2) times finer than the sinogram rows: n_rho and k_theta are the smallest lengths meeting
 * their bounds among the powers of two (smooth = 0) or among the lengths 2^a 3^b the FFTs take
 * (smooth = 1; see n_rho and k_theta above), r_dec the smallest integer meeting its bound,
 * dec_filter = 0.  Host-only; touches no device.  Returns RL_ERR_GEOMETRY if no valid geometry
 * exists within the limits above. */
rl_status rl_geom_default(int32_t n, int32_t n_theta, int32_t n_s, int32_t m, int32_t q_theta, int32_t smooth,
                          rl_geom* out);

/* Validate *geom and build a plan on the current device: partition tables, masks, the
 * Fourier multiplier H = zeta_hat / (B_hat_rho D_hat_theta) of sec. 3 eq. (exprcoef1)
 * computed in FP64 by composite Gauss-Legendre quadrature on the device, and FFT
 * twiddles.  Synchronous and allowed to be slow; not part of any timed path.  The plan
 * owns its device tables (about 12 m n^2 bytes, the per-pixel coordinates Algorithm 2 reads,
 * plus about 70 MB at n = 2048), is immutable after creation and may be used from several
 * streams at once.  On failure *out is set to NULL. */
rl_status rl_plan_create(const rl_geom* geom, rl_plan** out);

/* Release a plan and its device tables.  NULL is a no-op.  The caller must make sure
 * no enqueued work still uses the plan. */
void rl_plan_destroy(rl_plan* plan);

/* Copy the plan's geometry into *out. */
rl_status rl_plan_geometry(const rl_plan* plan, rl_geom* out);

/* Sinogram rows owned by each partition (sec. 2, eq. Radon_all_pb: row j belongs to partition
 * m = [theta_j / beta mod M], rounding half up; the rows that round to M belong to partition 0
 * with theta' = theta - pi and s -> -s).  Writes the largest count, n_own (the coarse rows of
 * the log-polar lattice that carry data), to *n_own and, if rows is not NULL, the count of
 * each of the M partitions to rows[0 .. M-1].  Host-side; RL_ERR_INVALID_ARG on a NULL plan
 * or n_own. */
rl_status rl_plan_rows(const rl_plan* plan, int32_t* n_own, int32_t* rows);

/* Workspace bytes needed by one call of `op` on `batch` slices (0 if batch == 0). */
size_t rl_workspace_bytes(const rl_plan* plan, int32_t batch, rl_op op);

/* Number of fine log-polar samples inside D of one slice, summed over the M partitions
 * (sec. 4, eq. Lopolargrid_f and circle_D): the bicubic interpolations one R or R# performs
 * per slice, for work accounting.  Host-side, from the plan's tables.  Writes *out;
 * RL_ERR_INVALID_ARG on a NULL argument. */
rl_status rl_plan_samples(const rl_plan* plan, int64_t* out);

/* R f: Algorithm 1 (sec. 5).  d_img [batch][n][n] -> d_sino [batch][n_theta][n_s].
 * batch == 0 is a no-op. */
rl_status radon_fwd(const rl_plan* plan, const float* d_img, float* d_sino, int32_t batch,
                    void* d_ws, size_t ws_bytes, hipStream_t stream);

/* R# g, the back-projection (sec. 1, eq. def_Radast), computed as the exact weighted
 * transpose of radon_fwd: for all f, g,  w_S <R f, g> = w_X <f, R# g>  with
 * w_S = (pi/N_theta)(2/N_s) and w_X = (2/N)^2, i.e. R# = (w_S/w_X) R^T.  Each step of
 * Algorithm 1 is transposed (the convolution uses the conjugate multiplier), so the
 * chain mirrors Algorithm 1 in reverse order.  d_sino [batch][n_theta][n_s] ->
 * d_img [batch][n][n]. */
rl_status radon_adj(const rl_plan* plan, const float* d_sino, float* d_img, int32_t batch,
                    void* d_ws, size_t ws_bytes, hipStream_t stream);

/* R^T g, the plain matrix transpose of radon_fwd: (w_X / w_S) * radon_adj.  This is the
 * gradient map of radon_fwd (for a loss L(R f), dL/df = R^T dL/dg), used by the autograd
 * wrapper.  Same arguments, workspace (RL_OP_ADJ) and semantics as radon_adj. */
rl_status radon_transpose(const rl_plan* plan, const float* d_sino, float* d_img, int32_t batch,
                          void* d_ws, size_t ws_bytes, hipStream_t stream);

/* (R#)^T f = (w_S / w_X) R f, the plain matrix transpose of radon_adj: the gradient map of
 * radon_adj (for a loss L(R# g), dL/dg = (R#)^T dL/df), used by the autograd wrapper of R#.
 * It runs the chain of radon_fwd with the factor w_S / w_X folded into its last step.  Same
 * arguments, layouts, workspace (RL_OP_FWD) and errors as radon_fwd. */
rl_status radon_adj_transpose(const rl_plan* plan, const float* d_img, float* d_sino, int32_t batch,
                              void* d_ws, size_t ws_bytes, hipStream_t stream);

/* Bytes of the static device scratch that radon_fwd_noalloc uses as its workspace (128 MiB:
 * one 2048 x 2048 slice at the default geometry needs about 118 MB). */
#define RL_NOALLOC_SCRATCH_BYTES (128u * 1024u * 1024u)

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): radon_fwd with its workspace in a file-scope device array of
 * RL_NOALLOC_SCRATCH_BYTES bytes instead of a caller-provided buffer.  Same arguments (minus the
 * workspace), layouts, results (the same kernels: bitwise equal to radon_fwd), asynchrony and
 * errors as radon_fwd; it calls no hipMalloc / hipFree.  Each GPU holds one copy of the array,
 * from the library's load on that GPU until the process ends; its device address is looked up
 * once per GPU on the first call there.  RL_ERR_WORKSPACE if rl_workspace_bytes(plan, batch,
 * RL_OP_FWD) exceeds RL_NOALLOC_SCRATCH_BYTES.  All calls on one GPU share that GPU's copy:
 * calls that overlap in time on one GPU (other streams, other host threads) race and must be
 * serialised by the caller; calls in order on one stream are safe.  d_img and d_sino are
 * caller-owned device memory as for radon_fwd. */
rl_status radon_fwd_noalloc(const rl_plan* plan, const float* d_img, float* d_sino, int32_t batch,
                            hipStream_t stream);

/* Filtered back-projection f = R# W g (sec. 1 eq. FBP): W is the filter of sec. 6 chosen by
 * `filter`, applied along s: the ramp |sigma| (eq. ramp) as a linear (zero-padded)
 * convolution with the Ram-Lak kernel h_0 = 1/(4 ds^2), h_n = -1/(pi^2 n^2 ds^2) for odd n,
 * 0 for even n != 0 (times ds); cosine and Shepp-Logan as that ramp's spectrum times their
 * window (see rl_filter) on the zero-padded axis, cut back to n_s samples; then radon_adj.
 * d_sino [batch][n_theta][n_s] -> d_img [batch][n][n].  A filter value outside rl_filter
 * returns RL_ERR_INVALID_ARG before any launch. */
rl_status fbp(const rl_plan* plan, const float* d_sino, float* d_img, int32_t batch,
              rl_filter filter, void* d_ws, size_t ws_bytes, hipStream_t stream);

/* Back-projection by the paper's fast algorithm (sec. 5, Algorithm 2; kernel sec. 3 eq.
 * exprcoef2), an approximation of the same integral R# g(x) = int_0^pi g(theta, x.theta)
 * d theta that radon_adj computes as the exact weighted transpose of radon_fwd; the two agree
 * to the method's discretisation error, not to rounding.  Per partition m:
 *   1. spline coefficients of each sinogram row along s, the row extended by zeros beyond
 *      its n_s samples (the lattice rows below lie on sinogram rows, so the prefilter in
 *      theta followed by evaluation there is the identity);
 *   2. the cubic spline of the row at the coarse log-polar lattice: lattice row theta'_i
 *      (the rows m owns), column rho_q, line offset s = (e^rho_q - (1 - a_R) cos theta'_i)/a_R
 *      (negated on rows that wrap past pi); no e^rho weight;
 *   3. periodic convolution on the K x N_rho lattice with zeta#, whose Fourier coefficients
 *      int_{-beta}^{beta} e^{-2 pi i k_theta u / (K dtheta)} (cos u)^{2 pi i k_rho / L} du are
 *      divided by B_hat(k_theta/K) B_hat(k_rho/N_rho) so the result is a spline-coefficient
 *      lattice in both variables;
 *   4. bicubic evaluation of that lattice at the log-polar coordinates of T_m x for every
 *      pixel x with |x| < 1 (node coordinates x = -1 + i dx); pixels with |x| >= 1 are 0;
 * summed over partitions.  d_sino [batch][n_theta][n_s] -> d_img [batch][n][n], row-major
 * float32 on the plan's device; the output is overwritten.  Workspace:
 * rl_workspace_bytes(plan, batch, RL_OP_BP_LP), 256-byte aligned, not overlapping the
 * input or output.  Errors and batch == 0 as radon_adj. */
rl_status radon_bp_lp(const rl_plan* plan, const float* d_sino, float* d_img, int32_t batch, void* d_ws,
                      size_t ws_bytes, hipStream_t stream);

/* FBP through Algorithm 2 (sec. 6 eq. FBP with sec. 5 Algorithm 2): the filter of fbp, then
 * radon_bp_lp.  Arguments and errors as fbp; workspace rl_workspace_bytes(plan, batch,
 * RL_OP_FBP_LP). */
rl_status fbp_lp(const rl_plan* plan, const float* d_sino, float* d_img, int32_t batch, rl_filter filter,
                 void* d_ws, size_t ws_bytes, hipStream_t stream);

/* EM reconstruction (sec. 7, the EM iteration), on radon_fwd and radon_adj:
 *   f <- f R#( chi_C g / R f ) / R# chi_C,
 * chi_C(theta, s) = 1 on the lines through the unit disc (|s| < 1) and 0 elsewhere.  Where
 * the paper is silent: the ratio is 0 on lines with R f <= 0, and the image lives on the
 * unit disc (the support of f, the only part R reads): f is set to 0 at pixels with
 * |x| >= 1 (node coordinates x = -1 + i dx) or where R# chi_C <= 0.
 *
 * rl_em_norm writes the normalisation image R# chi_C, d_norm [n][n] (computed once per
 * plan).  Workspace: rl_workspace_bytes(plan, 1, RL_OP_EM).
 *
 * rl_em runs `iters` EM steps in place on d_img [batch][n][n] (the start image, > 0 on the
 * disc) for the data d_sino [batch][n_theta][n_s] (>= 0) and the normalisation d_norm from
 * rl_em_norm.  Workspace: rl_workspace_bytes(plan, batch, RL_OP_EM); it holds R f and the
 * back-projected ratio between the steps.  batch == 0 or iters == 0 is a no-op; negative
 * values return RL_ERR_INVALID_ARG, as do NULL pointers and an image that overlaps the
 * data, the normalisation or the workspace. */
rl_status rl_em_norm(const rl_plan* plan, float* d_norm, void* d_ws, size_t ws_bytes, hipStream_t stream);
rl_status rl_em(const rl_plan* plan, const float* d_sino, const float* d_norm, float* d_img, int32_t batch,
                int32_t iters, void* d_ws, size_t ws_bytes, hipStream_t stream);

/* Message describing the last failure on the calling thread ("" if none). */
const char* rl_last_error(void);

/* Intermediate stages of radon_fwd for one slice, exported for stage-by-stage parity
 * checks.  stage selects what is written to d_out (float32, device):
 *   RL_STAGE_PREFILTER  c = Q f                                   [n][n]
 *   RL_STAGE_LOGPOLAR   w = e^rho * decimated fine samples         [m][n_own+4][n_rho]
 *   RL_STAGE_CONV       periodic convolution on the owned rows    [m][n_own][n_rho]
 *   RL_STAGE_KERNEL     the multiplier H (complex, interleaved re/im, scaled by
 *                       1/(k_theta n_rho)), independent of d_img  [n_rho/2+1][k_theta/2+1][2]
 * Rows of partitions with fewer owned rows than n_own are zero.  d_out_bytes must hold
 * the stage; the workspace is that of RL_OP_FWD with batch 1. */
typedef enum {
  RL_STAGE_PREFILTER = 0,
  RL_STAGE_LOGPOLAR = 1,
  RL_STAGE_CONV = 2,
  RL_STAGE_KERNEL = 3
} rl_stage;

rl_status rl_debug_stage(const rl_plan* plan, rl_stage stage, const float* d_img, float* d_out,
                         size_t d_out_bytes, void* d_ws, size_t ws_bytes, hipStream_t stream);

/* Kernel timing hooks (for benchmarks).  While recording is on, every kernel the library
 * enqueues is bracketed by a pair of HIP events recorded on the same stream, so the
 * durations are those of the kernels themselves.  rl_profile_start discards earlier
 * records and keeps at most `capacity` new ones (event pairs are created here, host side;
 * no device memory is allocated).  rl_profile_record waits for record i to complete and
 * returns the kernel name (static storage) and its duration in milliseconds.  Not
 * thread-safe; meant for single-threaded benchmark drivers. */
rl_status rl_profile_start(int32_t capacity);
rl_status rl_profile_stop(void);
int32_t rl_profile_count(void);
rl_status rl_profile_record(int32_t i, const char** name, float* ms);

/* ---------------------------------------------------------------- ragged batches
 * A ragged batch is a fixed set of `count` slices of possibly different geometries (sec. 6
 * times stacks of slices; here each slice names one of `nplans` plans, several slices may
 * share one), each with its own image buffer d_imgs[i] ([n][n] of its plan) and sinogram
 * buffer d_sinos[i] ([n_theta][n_s]).  rl_batch_create copies the pointer lists to the device
 * and groups the slices by plan; it is synchronous and allocates.  rl_batch_fwd computes
 * d_sinos[i] = R d_imgs[i] and rl_batch_adj d_imgs[i] = R# d_sinos[i] for every slice, as one
 * batched call per plan whose first and last kernels read and write the slices' own buffers.
 * The calls of the different plans run concurrently, each on a stream the batch owns (default
 * priority), forked from `stream` by an event and joined back to it: when rl_batch_fwd/adj
 * return, all their work is ordered before whatever is enqueued on `stream` next.  They
 * enqueue event records, stream waits and kernels only: no allocation, host synchronisation or
 * host read, so a caller may capture them on `stream` in a HIP graph (the plans' chains become
 * parallel branches) and replay it with new buffer contents.  One batch must not be run by
 * two calls that overlap in time (its streams and events are shared).
 * The buffers stay owned by the caller and must stay valid while the batch is used; input
 * and output buffers must not overlap.  tune_cache (optional, a file path): each plan's launch
 * parameters for the number of slices that use it are taken from that autotuner cache, or
 * found by rl_plan_autotune (with a temporary workspace) and appended to it; the result is set
 * on the plan (see rl_plan_set_tuning; results do not change).  Errors: RL_ERR_INVALID_ARG for
 * NULL lists, count < 0, a plan index out of range or a plan built on another device;
 * RL_ERR_WORKSPACE for a workspace smaller than rl_batch_workspace_bytes(batch, op) or not
 * 256-byte aligned; the autotuner's errors. */
typedef struct rl_batch rl_batch;

rl_status rl_batch_create(const rl_plan* const* plans, int32_t nplans, const int32_t* plan_of_slice,
                          float* const* d_imgs, float* const* d_sinos, int32_t count, const char* tune_cache,
                          rl_batch** out);

/* Workspace bytes rl_batch_fwd (op = RL_OP_FWD) or rl_batch_adj (RL_OP_ADJ) needs: the sum over
 * the plans of rl_workspace_bytes(plan, slices of that plan, op), each rounded up to 256 bytes,
 * since the plans' chains run at once in regions of their own. */
size_t rl_batch_workspace_bytes(const rl_batch* batch, rl_op op);

rl_status rl_batch_fwd(const rl_batch* batch, void* d_ws, size_t ws_bytes, hipStream_t stream);
rl_status rl_batch_adj(const rl_batch* batch, void* d_ws, size_t ws_bytes, hipStream_t stream);

/* d_imgs[i] = the paper's fast back-projection (sec. 5, Algorithm 2; radon_bp_lp) of
 * d_sinos[i] for every slice, in the manner of rl_batch_adj (one batched call per plan, the
 * plans' calls concurrent).  The workspace is rl_batch_workspace_bytes(batch, RL_OP_BP_LP).
 * Errors: those of rl_batch_adj; RL_ERR_GEOMETRY if a plan has q_theta != 1 (nothing is
 * launched). */
rl_status rl_batch_bp_lp(const rl_batch* batch, void* d_ws, size_t ws_bytes, hipStream_t stream);

/* Release a batch (not its buffers or plans).  NULL is a no-op. */
void rl_batch_destroy(rl_batch* batch);

#ifdef __cplusplus
}
#endif

#endif /* RADONLP_H */
