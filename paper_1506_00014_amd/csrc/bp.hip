// Back-projection by the paper's fast algorithm (sec. 5, Algorithm 2), and FBP through it.
//
//   k_bp_rows_rfft  one owned lattice row per block: the sinogram row's spline coefficients
//                   along s (FIR sqrt(3) z^|k|, the row extended by zeros), the cubic spline
//                   at the row's log-polar columns (s = (e^rho - (1 - a_R) cos theta')/a_R,
//                   Alg. 2 step 3), then a real FFT along rho
//   k_theta_conv    (shared) with the multiplier H# = zeta#_hat / (B_hat_theta B_hat_rho)
//                   (Alg. 2 step 4, eq. exprcoef2), owned rows in, support rows out
//   k_irfft_rows    (shared) inverse real FFT along rho of every support row
//   k_bp_gather     one thread per pixel: for each partition the bicubic spline of the
//                   lattice at the log-polar coordinates of T_m x (Alg. 2 step 5), summed
//                   over partitions (step 7); pixels with |x| >= 1 are zero
//   k_ramp          (shared) the FBP filter, before k_bp_rows_rfft
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "fft_device.h"
#include "rl_internal.h"

namespace rl {

namespace {

// Coefficients are kept on k = -kBpPad .. n_s + kBpPad - 1: the truncated FIR reaches kPrefR
// samples past the row, and the 4-tap evaluation two more.
constexpr int kBpPad = kPrefR + 2;
constexpr int kGx = 16, kGy = 16;  // pixels per gather block (kGx * kGy == kThreads)
static_assert(kGx * kGy == kThreads, "one pixel per thread");
constexpr int kBch = 8;   // slices per gather thread: the FP64 geometry of a pixel is computed once for them
constexpr int kStageMin = 4;  // calls with at least this many slices stage lattice boxes in LDS
constexpr int kBox = 1024;  // LDS floats of one slice's lattice box in the gather (16 x 16 pixels
                            // need at most 780 at 2048^2, M = 4; larger boxes read global memory)
constexpr int kFirRun = 8;  // consecutive prefilter outputs per thread (inputs held in registers)

// The sinogram row and the lattice row share one region (the first is dead once the
// coefficients are built); the coefficients follow it.
size_t bp_rows_lds(const DevPlan& d) {
  const int nw = d.n_s + 2 * kBpPad;
  return (size_t)(std::max(d.n_rho, nw) + nw) * sizeof(float);
}

}  // namespace

// Block: owned row o of one (slice, partition); writes the row's rho half-spectrum.
__global__ __launch_bounds__(kThreads) void k_bp_rows_rfft(DevPlan P, Slices<const float> sino,
                                                           float2* __restrict__ spec) {
  extern __shared__ float2 sh[];
  const int nc = P.nc, nr = P.n_rho, ns = P.n_s;
  const int o = blockIdx.x;
  const int bm = blockIdx.y;
  const int b = bm / P.m, m = bm - b * P.m;
  const int jw = P.own_j[m * P.n_own + o];
  float2* dst = spec + ((size_t)bm * P.n_own + o) * P.ld;
  if (jw < 0) {  // uniform across the block
    for (int k = threadIdx.x; k <= nc; k += blockDim.x) dst[k] = make_float2(0.f, 0.f);
    return;
  }
  const int j = jw & ((1 << 30) - 1);
  const bool wrap = (jw >> 30) & 1;
  float* x = reinterpret_cast<float*>(sh);  // [n_rho] the lattice row, then its FFT
  const int nw = ns + 2 * kBpPad;
  float* gs = x;                   // [nw] the sinogram row at index k + kBpPad, zeros outside
                                   // (dead once cs is built; x then takes its place)
  float* cs = x + max(nr, nw);     // [nw] its spline coefficients, same indexing
  const float* __restrict__ src = sino.at(b) + (size_t)j * ns;
  row_copy(
      nw,
      [&](int i) { return src[min(max(i - kBpPad, 0), ns - 1)]; },
      [&](int i, float v) { gs[i] = (i >= kBpPad && i < ns + kBpPad) ? v : 0.f; });
  __syncthreads();
  // c_i = sum_{|d| <= kPrefR} pref_|d| g_{i+d}: a thread computes kFirRun consecutive outputs
  // from one window of inputs in registers
  float h[kPrefR + 1];
#pragma unroll
  for (int d = 0; d <= kPrefR; ++d) h[d] = P.pref[d];
  for (int i0 = threadIdx.x * kFirRun; i0 < nw; i0 += blockDim.x * kFirRun) {
    float win[kFirRun + 2 * kPrefR];
#pragma unroll
    for (int u = 0; u < kFirRun + 2 * kPrefR; ++u) {
      const int i = i0 - kPrefR + u;
      win[u] = (i >= 0 && i < nw) ? gs[i] : 0.f;
    }
#pragma unroll
    for (int r = 0; r < kFirRun; ++r) {
      float acc = h[0] * win[r + kPrefR];
#pragma unroll
      for (int d = 1; d <= kPrefR; ++d) acc += h[d] * (win[r + kPrefR - d] + win[r + kPrefR + d]);
      if (i0 + r < nw) cs[i0 + r] = acc;
    }
  }
  __syncthreads();
  const double cth = P.own_cos[m * P.n_own + o];
  const double c0 = (1.0 - P.a_R) * cth, e_scale = P.a_R * P.dx, inv_aR = 1.0 / P.a_R;
  const double inv_ds = 1.0 / P.ds;
  row_copy(nr, [&](int q) { return P.erho[q]; }, [&](int q, double erq) {
    double s = (erq * e_scale - c0) * inv_aR;  // line offset of lattice node (theta', rho_q)
    if (wrap) s = -s;
    const double t = (s + 1.0) * inv_ds;  // index position along s
    float v = 0.f;
    // taps beyond the stored coefficients are zero; the range test also keeps the integer
    // conversion below in range for any t
    if (t > -(double)kBpPad - 2.0 && t < (double)(ns + kBpPad + 1)) {
      const double ft = floor(t);
      const int k0 = (int)ft + kBpPad;
      float w[4];
      bspline_w6((float)(t - ft), w);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int idx = k0 - 1 + a;
        if (idx >= 0 && idx < nw) v += w[a] * cs[idx];
      }
      v *= (1.0f / 6.0f);
    }
    x[q] = v;
  });
  __syncthreads();
  fft_lds<kRowVals, false>(sh, nc, 1, P.twp_rows);
  rfft_post(sh, nc, P.tw, P.tw_len, [&](int k, float2 xv) { dst[k] = xv; });
}

// Block: 16 x 16 pixels (each wave an 8 x 8 sub-tile) of kBch slices.  lat holds the support
// rows [batch][m][n_sup][n_rho] of the convolved lattice (spline coefficients); support row
// kHalo is a partition's first owned row.  Per partition the pixels' lattice coordinates and
// the box their taps cover come from the plan (k_bp_geometry, k_bp_boxes); if the box fits kBox
// floats, the box of each slice is staged in LDS with coalesced loads and the 16 taps are read
// there, otherwise they are read from global memory.
// STAGED = false reads every tap from global memory (no LDS, no barriers): calls with fewer
// than kStageMin slices gain nothing from the staging and lose occupancy to its LDS.
template <bool STAGED>
__global__ __launch_bounds__(kThreads) void k_bp_gather(DevPlan P, const float* __restrict__ lat,
                                                        Slices<float> img, int batch) {
  __shared__ float box[STAGED ? kBch : 1][STAGED ? kBox : 1];
  const int t = (int)threadIdx.x, wv = t >> 6, ln = t & 63;
  const int ix = blockIdx.x * kGx + (ln & 7) + 8 * (wv & 1);
  const int iy = blockIdx.y * kGy + (ln >> 3) + 8 * (wv >> 1);
  const int b0 = blockIdx.z * kBch;
  const int nb = min(kBch, batch - b0);
  const bool in_img = ix < P.n && iy < P.n;
  const bool act = in_img && in_unit_disc(ix, iy, P.n);
  const int nr = P.n_rho;
  const size_t slice = (size_t)P.m * P.n_sup * nr;  // lattice floats of one slice
  float acc[kBch];
#pragma unroll
  for (int bb = 0; bb < kBch; ++bb) acc[bb] = 0.f;
  for (int m = 0; m < P.m; ++m) {
    int kt = 1, kr = 0;
    float wt[4], wr[4];
    if (act) {  // the lattice coordinates of T_m x, built with the plan (k_bp_geometry)
      const size_t gi = ((size_t)m * P.n + iy) * P.n + ix;
      const unsigned kk = P.bp_k[gi];
      const float2 fr = P.bp_f[gi];
      kt = (int)(kk >> 16);
      kr = (int)(kk & 0xffffu) - 1;
      bspline_w6(fr.x, wt);
      bspline_w6(fr.y, wr);
    }
    const float* L0 = lat + (size_t)(b0 * P.m + m) * P.n_sup * nr;  // row 0 of partition m, slice b0
    int r0 = 0, nrow = 0, c0 = 0, ncol = 0;
    if (STAGED) {
      // the tile's lattice box, built with the plan
      const int4 bb = P.bp_box[(size_t)m * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x];
      if (bb.y == 0) continue;  // no pixel of the tile in the disc (uniform)
      __syncthreads();  // the previous partition's box reads are done
      r0 = bb.x;
      nrow = bb.y;
      c0 = bb.z;
      ncol = bb.w;
    }
    if (STAGED && nrow * ncol <= kBox) {  // uniform
      const int nbox = nrow * ncol;
      for (int bb = 0; bb < nb; ++bb) {
        const float* Ls = L0 + bb * slice;
        for (int e = t; e < nbox; e += kThreads) {
          const int r = e / ncol, c = e - r * ncol;
          box[bb][e] = Ls[(size_t)(r0 + r) * nr + wrap1(c0 + c, nr)];
        }
      }
      __syncthreads();
      if (act) {
        const int base = (kt - 1 - r0) * ncol + (kr - 1 - c0);
#pragma unroll
        for (int bb = 0; bb < kBch; ++bb) {
          if (bb < nb) {
            const float* B = box[bb] + base;
            float v = 0.f;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
              const float* Br = B + a * ncol;
              v += wt[a] * (wr[0] * Br[0] + wr[1] * Br[1] + wr[2] * Br[2] + wr[3] * Br[3]);
            }
            acc[bb] += v;
          }
        }
      }
    } else if (act) {
      const float* Lk = L0 + (size_t)(kt - 1) * nr;
      int col[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) col[c] = wrap1(kr - 1 + c, nr);
#pragma unroll
      for (int bb = 0; bb < kBch; ++bb) {
        if (bb < nb) {
          const float* L = Lk + bb * slice;
          float v = 0.f;
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            const float* Lr = L + (size_t)a * nr;
            v += wt[a] * (wr[0] * Lr[col[0]] + wr[1] * Lr[col[1]] + wr[2] * Lr[col[2]] + wr[3] * Lr[col[3]]);
          }
          acc[bb] += v;
        }
      }
    }
  }
  if (in_img) {
#pragma unroll
    for (int bb = 0; bb < kBch; ++bb)
      if (bb < nb) img.at(b0 + bb)[(size_t)iy * P.n + ix] = acc[bb] * (1.0f / 36.0f);
  }
}

// Plan time: the lattice coordinates of T_m x for every pixel x in the unit disc (Alg. 2 step 5):
// y = T_m x = a_R Rot(-m beta) x + (1 - a_R, 0) (eq. Tdef) at angle position T = (atan2(y) -
// phi0_m) / dtheta and log-radius position R = (log |y| - rho0) / d_rho; the gather's 4 x 4 taps
// start one before floor(T), floor(R), with weights from the fractions past them.  |x| < 1 puts
// T in [1, n_own + 2) and R in [-1, n_rho - 1] (T_m maps the unit disc onto D); the clamps only
// guard the gather's loads.
__global__ __launch_bounds__(kThreads) void k_bp_geometry(DevPlan P, unsigned* __restrict__ kout,
                                                          float2* __restrict__ fout) {
  const int ix = blockIdx.x * kGx + (int)threadIdx.x % kGx, iy = blockIdx.y * kGy + (int)threadIdx.x / kGx;
  const int m = blockIdx.z;
  if (ix >= P.n || iy >= P.n) return;
  unsigned kk = (1u << 16) | 1u;  // (pixels outside the disc are never read)
  float2 fr = make_float2(0.f, 0.f);
  if (in_unit_disc(ix, iy, P.n)) {
    const double x1 = -1.0 + ix * P.dx, x2 = -1.0 + iy * P.dx;
    double sm, cm;
    sincospi((double)m / (double)P.m, &sm, &cm);
    const double y1 = P.a_R * (cm * x1 + sm * x2) + (1.0 - P.a_R);
    const double y2 = P.a_R * (cm * x2 - sm * x1);
    const double T = (atan2(y2, y1) - P.phi0[m]) / P.dtheta;
    const double R = (0.5 * log(y1 * y1 + y2 * y2) - P.rho0) / P.d_rho;
    const double ft = floor(T), fq = floor(R);
    const int kt = min(max((int)ft, 1), P.n_sup - 3);
    const int kr = min(max((int)fq, -1), P.n_rho - 1);
    kk = ((unsigned)kt << 16) | (unsigned)(kr + 1);
    fr = make_float2((float)(T - ft), (float)(R - fq));
  }
  const size_t gi = ((size_t)m * P.n + iy) * P.n + ix;
  kout[gi] = kk;
  fout[gi] = fr;
}

// Plan time: each gather tile's lattice box for partition m, from the coordinates above: rows
// min kt - 1 .. max kt + 2 and columns min kr - 1 .. max kr + 2 over its pixels in the disc.
__global__ __launch_bounds__(kThreads) void k_bp_boxes(DevPlan P, const unsigned* __restrict__ kin,
                                                       int4* __restrict__ box) {
  __shared__ int red[4];
  const int t = (int)threadIdx.x, ln = t & 63, wv = t >> 6;
  const int ix = blockIdx.x * kGx + (ln & 7) + 8 * (wv & 1);
  const int iy = blockIdx.y * kGy + (ln >> 3) + 8 * (wv >> 1);
  const int m = blockIdx.z;
  if (t == 0) {
    red[0] = INT_MAX;
    red[1] = INT_MIN;
    red[2] = INT_MAX;
    red[3] = INT_MIN;
  }
  __syncthreads();
  if (ix < P.n && iy < P.n && in_unit_disc(ix, iy, P.n)) {
    const unsigned kk = kin[((size_t)m * P.n + iy) * P.n + ix];
    const int kt = (int)(kk >> 16), kr = (int)(kk & 0xffffu) - 1;
    atomicMin(&red[0], kt);
    atomicMax(&red[1], kt);
    atomicMin(&red[2], kr);
    atomicMax(&red[3], kr);
  }
  __syncthreads();
  if (t == 0) {
    const int4 b = red[0] > red[1] ? make_int4(0, 0, 0, 0)
                                   : make_int4(red[0] - 1, red[1] - red[0] + 4, red[2] - 1, red[3] - red[2] + 4);
    box[((size_t)m * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = b;
  }
}

int bp_tiles(int n) { return ((n + kGx - 1) / kGx) * ((n + kGy - 1) / kGy); }

rl_status build_bp_geometry(const DevPlan& d, unsigned* k, float2* f, int4* box) {
  if (d.n_sup - 3 >= (1 << 16) || d.n_rho + 1 >= (1 << 16))
    return fail(RL_ERR_GEOMETRY, "lattice too large for the packed gather coordinates");
  const dim3 grid((d.n + kGx - 1) / kGx, (d.n + kGy - 1) / kGy, d.m);
  hipLaunchKernelGGL(k_bp_geometry, grid, dim3(kThreads), 0, 0, d, k, f);
  rl_status st = check_launch("k_bp_geometry");
  if (st != RL_OK) return st;
  hipLaunchKernelGGL(k_bp_boxes, grid, dim3(kThreads), 0, 0, d, k, box);
  return check_launch("k_bp_boxes");
}

rl_status prepare_bp_launches(const rl_plan* p) {
  return ensure_dyn_lds((const void*)k_bp_rows_rfft, bp_rows_lds(p->d), "hipFuncSetAttribute(k_bp_rows_rfft)");
}

rl_status bp_lp_chain(const rl_plan* plan, Slices<const float> sino, Slices<float> img, int batch, void* ws,
                      rl_op op, hipStream_t s) {
  const DevPlan& d = plan->d;
  const WsLayout L = workspace_layout(plan, batch, op);
  char* w = (char*)ws;
  float* U = (float*)(w + L.off[1]);
  float2* Bs = (float2*)(w + L.off[2]);
  float2* A = (float2*)(w + L.off[3]);
  rl_status st;
  {
    const size_t lds = bp_rows_lds(d);
    if ((st = ensure_dyn_lds((const void*)k_bp_rows_rfft, lds, "hipFuncSetAttribute(k_bp_rows_rfft)")) != RL_OK)
      return st;
    RL_LAUNCH("k_bp_rows_rfft", k_bp_rows_rfft, dim3(d.n_own, batch * d.m), dim3(kThreads), lds, s, d, sino, A);
    if ((st = check_launch("k_bp_rows_rfft")) != RL_OK) return st;
  }
  if ((st = launch_theta_conv(plan, A, d.n_own, kHalo, 1, Bs, d.n_sup, 0, 1, false, batch, s, d.Hbp)) != RL_OK) return st;
  if ((st = launch_irfft_rows(plan, Bs, U, batch * d.m * d.n_sup, s)) != RL_OK) return st;
  dim3 grid((d.n + kGx - 1) / kGx, (d.n + kGy - 1) / kGy, (batch + kBch - 1) / kBch);
  if (batch >= kStageMin)
    RL_LAUNCH("k_bp_gather", k_bp_gather<true>, grid, dim3(kThreads), 0, s, d, U, img, batch);
  else
    RL_LAUNCH("k_bp_gather", k_bp_gather<false>, grid, dim3(kThreads), 0, s, d, U, img, batch);
  return check_launch("k_bp_gather");
}

}  // namespace rl

using namespace rl;

extern "C" rl_status radon_bp_lp(const rl_plan* plan, const float* d_sino, float* d_img, int32_t batch, void* d_ws,
                                 size_t ws_bytes, hipStream_t stream) {
  if (plan && plan->d.q != 1)
    return fail(RL_ERR_GEOMETRY, "radon_bp_lp needs q_theta = 1 (its lattice rows are the sinogram rows)");
  rl_status st = adj_checks(plan, d_sino, d_img, batch, d_ws, ws_bytes, RL_OP_BP_LP);
  if (st != RL_OK || batch == 0) return st;
  const DevPlan& d = plan->d;
  return bp_lp_chain(plan, dense(d_sino, (size_t)d.n_theta * d.n_s), dense(d_img, (size_t)d.n * d.n), batch, d_ws,
                     RL_OP_BP_LP, stream);
}

extern "C" rl_status fbp_lp(const rl_plan* plan, const float* d_sino, float* d_img, int32_t batch, rl_filter filter,
                            void* d_ws, size_t ws_bytes, hipStream_t stream) {
  if (filter != RL_FILTER_RAMLAK && filter != RL_FILTER_COSINE && filter != RL_FILTER_SHEPP_LOGAN)
    return fail(RL_ERR_INVALID_ARG, "unknown filter");
  if (plan && plan->d.q != 1)
    return fail(RL_ERR_GEOMETRY, "fbp_lp needs q_theta = 1 (its lattice rows are the sinogram rows)");
  rl_status st = adj_checks(plan, d_sino, d_img, batch, d_ws, ws_bytes, RL_OP_FBP_LP);
  if (st != RL_OK || batch == 0) return st;
  const WsLayout L = workspace_layout(plan, batch, RL_OP_FBP_LP);
  float* wg = (float*)((char*)d_ws + L.off[4]);
  if ((st = launch_ramp(plan, d_sino, wg, batch, (int)filter, stream)) != RL_OK) return st;
  const DevPlan& d = plan->d;
  return bp_lp_chain(plan, dense((const float*)wg, (size_t)d.n_theta * d.n_s), dense(d_img, (size_t)d.n * d.n), batch,
                     d_ws, RL_OP_FBP_LP, stream);
}
