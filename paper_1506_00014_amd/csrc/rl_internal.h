// Internal declarations of the log-polar Radon library (gfx950).  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "radonlp.h"

namespace rl {

constexpr int kHalo = 2;          // coarse rows on each side of a partition's owned rows
constexpr int kThreads = 256;     // threads per block of every hot-path kernel
constexpr int kRowVals = 16;      // complex values per thread in a row FFT (N_rho/2 <= 4096)
constexpr int kColVals = 32;      // complex values per thread in the theta pass
constexpr int kTile = 48;         // image tile side of the adjoint splat
constexpr int kPrefR = 16;        // half-length of the truncated prefilter (|z|^17 ~ 2e-10)
constexpr int kMaxPart = 16;      // largest supported M

// Slice b of a batch: base + b * stride, or tab[b] when a pointer table is given (the slices of
// a ragged batch each live in a buffer of their own).  tab is a device array.
template <class T>
struct Slices {
  T* base;
  T* const* tab;
  size_t stride;
  __host__ __device__ T* at(int b) const { return tab ? tab[b] : base + (size_t)b * stride; }
};
template <class T>
inline Slices<T> dense(T* base, size_t stride) { return Slices<T>{base, nullptr, stride}; }

// Scalars and device tables handed to every kernel by value.
struct DevPlan {
  int n, n_theta, n_s, m, n_rho, k_theta, r;
  int q;                   // coarse lattice rows per sinogram row spacing (q_theta)
  int n_own, n_sup, n_fine, t_min, ld, nc, tw_len, lr;
  double a_R, dx, ds, dtheta, d_rho, rho0, beta;
  double dtheta_c;         // coarse lattice spacing dtheta / q; fine rays dtheta_c / r apart
  double X0[kMaxPart], Y0[kMaxPart];   // image index of T_m^{-1}(0) offsets, per partition
  double phi0[kMaxPart];               // theta' of support row 0, per partition
  int sup_rows[kMaxPart];              // support rows of each partition: the lattice rows of its own
                                       // owned rows plus kHalo on each side (<= n_sup); the lattice
                                       // rows beyond are zero in R and unread by its transpose
  const float2* H;         // [nc + 1][k_theta/2 + 1], zeta_hat/(B_hat D_hat K N_rho)
  const float2* Hbp;       // [nc + 1][k_theta/2 + 1], zeta#_hat/(B_hat_theta B_hat_rho K N_rho)
  const double2* fine_cs;  // [m][n_fine] (cos(phi_t + m beta), sin(phi_t + m beta))
  const int2* fine_q;      // [m][n_fine] inclusive rho-index range inside D (lo > hi: empty)
  const float4* dec;       // [r] weights of the decimation filter for phase p
  const int* own_j;        // [m][n_own] sinogram row, bit 30 set for wrapped rows, -1 if none
  const double* own_cos;   // [m][n_own] cos(theta'_j)
  const float2* tw;        // [tw_len] exp(-2 pi i n / tw_len)
  const float2* twp_rows;  // Stockham pass twiddles of length nc (rho rows), see fft_device.h
  const float2* twp_ramp;  // Stockham pass twiddles of length lr / 2 (ramp filter rows)
  const float2* tw_theta;  // [k_theta] four-step twiddles exp(-2 pi i n2 k1 / k_theta) at
                           // n2 * K1 + k1 (K1 x K2 = k_theta as the theta pass splits it)
  const float* ramp;       // [3][lr/2 + 1] filter multipliers (rl_filter order), include 1/lr
  const float* pref;       // [kPrefR + 1] prefilter taps sqrt(3) z^|k|
  const double* erho;      // [n_rho] e^{rho_q} / (a_R dx): image-index length of the ray at rho_q
  const unsigned* bp_k;    // [m][n][n] Algorithm 2's gather: lattice tap base of T_m x for each
                           // pixel in the unit disc, row (clamped to [1, n_sup - 3]) << 16 |
                           // column + 1 (column clamped to [-1, n_rho - 1])
  const float2* bp_f;      // [m][n][n] the fractions of T_m x past those bases (theta, rho)
  const int4* bp_box;      // [m][gather tiles] lattice box (first row, rows, first column,
                           // columns) the 4 x 4 taps of a 16 x 16-pixel tile's pixels in the
                           // unit disc read; rows = 0: the tile has no such pixel
  const int2* tau;         // [m][n_own][n_s] rho position tau of S_m(theta_j, s_k) on each owned
                           // row: (floor(tau) clamped to [-1, n_rho], bits of the FP32 fraction)
  const float* dtap;       // [4r - 1] decimation taps d_n, n = -(2r-1) .. 2r-1
  const int4* fbox;        // [m][forward tile rows][forward tile columns] image box of each
                           // forward tile: (x0, y0, width, height), width 0 if no sample in D
  const int* ftiles;       // forward blocks (index into fbox of each block's first tile):
                           // ftiles_small whose tiles fit the small patch at its fixed pitch (or
                           // have no sample in D), ftiles_mid that fit the large patch at its
                           // fixed pitch, then the others
  int ftiles_small, ftiles_mid, ftiles_large;
  // splat passes of the adjoint (geometry only, built at plan time), see adjoint.hip
  int adj_ntx;             // tiles per image row
  const int* adj_off;      // [tiles + 1] first pass of each tile
  const int4* adj_pass;    // [passes][3] header of each pass
  const int4* adj_ray;     // [ray slots] (t, first rho, last rho, segment numbers) per slot
};

}  // namespace rl

struct rl_plan {
  rl_geom g;
  int device;
  rl::DevPlan d;
  rl_tune tune;  // execution-only launch parameters (rl_plan_set_tuning / rl_plan_autotune)
  std::vector<int> rows_per_part;
  void* d_mem;  // single device allocation holding all tables
  size_t d_mem_bytes;
  void* d_adj;  // device allocation holding the adjoint splat passes
  size_t d_adj_bytes;
  int64_t n_samples;  // fine log-polar samples inside D of one slice, all partitions
};

namespace rl {

// ---------------------------------------------------------------- error handling
void set_error(const std::string& msg);
rl_status fail(rl_status code, const std::string& msg);
rl_status check_hip(hipError_t e, const char* what);
rl_status check_launch(const char* what);
rl_status check_plan_device(const rl_plan* plan);
// Raise a kernel's dynamic LDS limit above the default 64 KiB on the current device, once:
// later calls with the same or a smaller size make no HIP call, so launches stay capturable.
rl_status ensure_dyn_lds(const void* fn, size_t lds, const char* what);

struct WsLayout {
  size_t off[6];
  size_t total;
};
WsLayout workspace_layout(const rl_plan* plan, int batch, rl_op op);

// Kernel timing hooks: prof_open records a start event (returns a slot or -1), prof_close
// the matching stop event, both on the launch stream.
int prof_open(const char* name, hipStream_t s);
void prof_close(int slot, hipStream_t s);

#define RL_LAUNCH(name, kernel, grid, block, lds, stream, ...)                      \
  do {                                                                            \
    const int rl_slot_ = ::rl::prof_open(name, stream);                           \
    hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);            \
    ::rl::prof_close(rl_slot_, stream);                                           \
  } while (0)

// Launchers (forward.hip / adjoint.hip).
rl_status launch_prefilter(const rl_plan* p, Slices<const float> in, Slices<float> out, int batch, float scale,
                           hipStream_t s);
rl_status launch_cart2lp(const rl_plan* p, const float* c, float* u, int batch, hipStream_t s);
rl_status launch_rfft_rows(const rl_plan* p, const float* in, float2* out, int rows, hipStream_t s);
// Input rows in_off + in_step * i (i < in_rows) and output rows out_off + out_step * o (o < out_rows)
// of the K-row lattice; the other input rows are zero.  H: the multiplier table (nullptr: the
// plan's H of the Radon transform).
rl_status launch_theta_conv(const rl_plan* p, const float2* in, int in_rows, int in_off, int in_step, float2* out,
                            int out_rows, int out_off, int out_step, bool conj, int batch, hipStream_t s,
                            const float2* H = nullptr);
// scale: factor on the output (1 for R)
rl_status launch_irfft_eval(const rl_plan* p, const float2* spec, Slices<float> sino, int batch, double scale,
                            hipStream_t s);
rl_status launch_splat_rfft(const rl_plan* p, Slices<const float> sino, float2* spec, int batch,
                            hipStream_t s);
rl_status launch_irfft_scale(const rl_plan* p, const float2* spec, float* u, int batch,
                             hipStream_t s);
rl_status launch_lp2cart_adj(const rl_plan* p, const float* u, float* cbar, int batch,
                             hipStream_t s);
rl_status launch_ramp(const rl_plan* p, const float* in, float* out, int batch, int filter, hipStream_t s);
rl_status launch_irfft_rows(const rl_plan* p, const float2* spec, float* out, int rows,
                            hipStream_t s);
// The theta pass splits k_theta = K1 K2 (four-step FFT); K1 as a function of k_theta.
constexpr int theta_k1(int k_theta) { return k_theta <= 32 ? k_theta : 32; }
// The theta-FFT lengths the theta pass is instantiated for, as (K, K1, K2) with K = K1 K2 (the
// plan accepts exactly these).
#define RL_THETA_LENGTHS(X)                                                                          \
  X(8, 8, 1) X(12, 12, 1) X(16, 16, 1) X(24, 24, 1) X(32, 32, 1) X(64, 32, 2) X(96, 32, 3) X(128, 32, 4) \
  X(192, 32, 6) X(256, 32, 8) X(384, 32, 12) X(512, 32, 16) X(768, 32, 24) X(1024, 32, 32)          \
  X(1536, 32, 48) X(2048, 32, 64)
// Plan time (host): image boxes of the forward blocks, in the order of the forward grid.
std::vector<int4> build_fwd_boxes(const DevPlan& d, const std::vector<double2>& cs,
                                  const std::vector<int2>& fq, const std::vector<double>& erho);
// Plan time (host): the forward's tile lists (small-patch tiles first; their count in *n_small).
std::vector<int> build_fwd_tiles(const DevPlan& d, const std::vector<int4>& boxes, int* n_small, int* n_mid);
// The operator chains behind radon_fwd and radon_adj / radon_transpose / fbp (arguments
// checked by the caller; ws holds workspace_layout(plan, batch, RL_OP_FWD or op)).
rl_status forward_chain(const rl_plan* plan, Slices<const float> img, Slices<float> sino, int batch, void* ws,
                        int stop_stage, float* stage_out, hipStream_t s, double out_scale);
rl_status adjoint_chain(const rl_plan* plan, Slices<const float> sino, Slices<float> img, int batch, void* ws, rl_op op,
                        bool transpose, hipStream_t s);
// Algorithm 2 (sec. 5): the lattice rows from the sinogram rows, the theta convolution with the
// back-projection kernel, the inverse rho FFT, and the Cartesian gather summed over partitions.
rl_status bp_lp_chain(const rl_plan* plan, Slices<const float> sino, Slices<float> img, int batch, void* ws,
                      rl_op op, hipStream_t s);
// Argument checks shared by the sinogram -> image entry points (op selects the workspace).
rl_status adj_checks(const rl_plan* plan, const void* in, const void* out, int batch, void* ws, size_t ws_bytes,
                     rl_op op);
// Plan time: raise the LDS limit of the Algorithm 2 row kernel (bp.hip).
rl_status prepare_bp_launches(const rl_plan* p);
// Plan time: fill DevPlan::bp_k and bp_f (Algorithm 2's per-pixel lattice coordinates).
rl_status build_bp_geometry(const DevPlan& d, unsigned* k, float2* f, int4* box);
// Gather tiles of Algorithm 2 (16 x 16 pixels) for an n x n image.
int bp_tiles(int n);
// Workspace of rl_em / rl_em_norm (em.hip).
size_t em_workspace_bytes(const rl_plan* plan, int batch);
// Set the plan's launch parameters from the autotuner cache at `path` (tune.hip): false if the
// file has no entry for this plan and batch size.
bool tune_from_cache(rl_plan* plan, int batch, const char* path);
// Plan time: build the adjoint splat passes (allocates plan->d_adj, fills the adj_* fields).
rl_status build_adj_passes(rl_plan* p);
// Plan time: raise the LDS limits of the kernels this plan launches (see ensure_dyn_lds).
rl_status prepare_forward_launches(const rl_plan* p);
rl_status prepare_adjoint_launches(const rl_plan* p);

}  // namespace rl
