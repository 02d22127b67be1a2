// Forward transform R (Algorithm 1 of the paper) and the kernels it shares with the adjoint.
//
//   k_prefilter    c = Q f: separable periodic cubic B-spline prefilter (sec. 4, eq.
//                  Qfrecursive), as the symmetric FIR sqrt(3) z^|k|, |k| <= 16, z = sqrt(3) - 2
//   k_cart2lp      Alg. 1 steps 3-5: bicubic samples of T_m f on the fine log-polar grid
//                  (eq. Tdef, Lopolargrid_f, wsumn), zero outside D (eq. circle_D), theta
//                  low-pass + decimation to the coarse grid (eq. Lopolargrid_polar), times e^rho
//   k_rfft_rows    real FFT along rho of every support row
//   k_theta_conv   FFT along theta, multiply by H = zeta_hat / (B_hat D_hat) (eq. exprcoef1;
//                  Alg. 1 step 6), inverse FFT along theta, kept rows only
//   k_irfft_eval   inverse real FFT along rho, then the 4-tap B-spline evaluation at
//                  S_m(theta_j, s_k) (eq. Sm_def, Radon_all_pb; Alg. 1 step 7), times 1/a_R
#include <hip/hip_runtime.h>

#include "fft_device.h"
#include "rl_internal.h"

namespace rl {

// ------------------------------------------------------------------ prefilter
constexpr int kPSW = 64;                   // output columns per block
constexpr int kPSI = kPSW + 2 * kPrefR;    // input columns per block (96)
constexpr int kPRB = 32;                   // rows per step
constexpr int kPRing = kPRB + 2 * kPrefR;  // row-filtered rows kept (64, a power of two)
constexpr int kPGroups = kPRB * kPSI / 4;  // float4 groups of input per step (768)
static_assert(kPGroups % kThreads == 0, "whole groups per thread");
static_assert(kPRB * (kPSW / 8) == kThreads && kPSW * (kPRB / 8) == kThreads,
              "one run of 8 outputs per thread in each filter pass");

// Block: a strip of kPSW columns and up to `seg` rows of one slice, streamed down in steps
// of kPRB rows.  A step row-filters kPRB new input rows (the periodic 2 kPrefR + 1 taps,
// input staged in LDS) into a ring of the last kPRing row-filtered rows, then column-filters
// the kPRB output rows whose taps the ring now holds.  The first step only fills the ring.
// The next step's input is loaded into registers while the current step computes.
__global__ __launch_bounds__(kThreads) void k_prefilter(Slices<const float> in, Slices<float> out, int n, float scale,
                                                        const float* __restrict__ pref, int seg) {
  __shared__ float tin[kPRB][kPSI + 1];
  __shared__ float ring[kPRing][kPSW + 1];
  __shared__ float q[kPrefR + 1];
  const int b = blockIdx.z;
  const int x0 = blockIdx.x * kPSW;
  const int yseg0 = blockIdx.y * seg, yseg1 = min(yseg0 + seg, n);
  const int base = yseg0 - kPrefR;  // row-filtered row y sits in ring slot (y - base) % kPRing
  const float* __restrict__ src = in.at(b);
  float* __restrict__ dst = out.at(b);
  if (threadIdx.x <= kPrefR) q[threadIdx.x] = pref[threadIdx.x];
  const bool vec_ok = (n & 3) == 0 && x0 - kPrefR >= 0 && x0 - kPrefR + kPSI <= n;  // uniform
  // input rows [ry, ry + kPRB) x columns [x0 - kPrefR, x0 - kPrefR + kPSI), periodic
  auto load = [&](int ry, float4* v) {
#pragma unroll
    for (int u = 0; u < kPGroups / kThreads; ++u) {
      const int g = (int)threadIdx.x + u * kThreads;
      const int ly = g / (kPSI / 4), lg = g - ly * (kPSI / 4);
      int gy = ry + ly;
      if (gy < 0 || gy >= n) gy = ((gy % n) + n) % n;
      const float* srow = src + (size_t)gy * n;
      const int gx = x0 - kPrefR + 4 * lg;
      if (vec_ok) {
        v[u] = *reinterpret_cast<const float4*>(srow + gx);
      } else {
        float t[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          int x = gx + e;
          if (x < 0 || x >= n) x = ((x % n) + n) % n;
          t[e] = srow[x];
        }
        v[u] = make_float4(t[0], t[1], t[2], t[3]);
      }
    }
  };
  float4 v[kPGroups / kThreads];
  load(yseg0 - kPRB + kPrefR, v);  // input rows of the first step
  __syncthreads();
  float qk[kPrefR + 1];
#pragma unroll
  for (int k = 0; k <= kPrefR; ++k) qk[k] = q[k];
  // step at cy computes row-filtered rows [cy + kPrefR, cy + kPrefR + kPRB) and outputs rows
  // [cy, cy + kPRB); the first step (cy = yseg0 - kPRB) only fills the ring
  for (int cy = yseg0 - kPRB; cy < yseg1; cy += kPRB) {
#pragma unroll
    for (int u = 0; u < kPGroups / kThreads; ++u) {
      const int g = (int)threadIdx.x + u * kThreads;
      const int ly = g / (kPSI / 4), lg = g - ly * (kPSI / 4);
      float* d = &tin[ly][4 * lg];
      d[0] = v[u].x;
      d[1] = v[u].y;
      d[2] = v[u].z;
      d[3] = v[u].w;
    }
    __syncthreads();
    if (cy + kPRB < yseg1) load(cy + kPRB + kPrefR, v);  // next step's input, in flight
    {
      // rows: kPRB rows x (kPSW / 8) runs of 8 outputs, one run per thread
      constexpr int R = 8;
      const int row = threadIdx.x / (kPSW / R), seg = threadIdx.x % (kPSW / R);
      float x[R + 2 * kPrefR];
#pragma unroll
      for (int i = 0; i < R + 2 * kPrefR; ++i) x[i] = tin[row][seg * R + i];
      float* rr = ring[(cy + kPrefR + row - base) & (kPRing - 1)];
#pragma unroll
      for (int j = 0; j < R; ++j) {
        float acc = qk[0] * x[j + kPrefR];
#pragma unroll
        for (int k = 1; k <= kPrefR; ++k) acc += qk[k] * (x[j + kPrefR - k] + x[j + kPrefR + k]);
        rr[seg * R + j] = acc;
      }
    }
    __syncthreads();
    if (cy >= yseg0) {  // uniform
      // columns: kPSW columns x (kPRB / 8) runs of 8 outputs, one run per thread
      constexpr int R = kPRB / (kThreads / kPSW);  // 8
      const int col = threadIdx.x % kPSW, run = threadIdx.x / kPSW;
      const int y0 = cy + run * R;
      float y[R + 2 * kPrefR];
#pragma unroll
      for (int i = 0; i < R + 2 * kPrefR; ++i) y[i] = ring[(y0 - kPrefR + i - base) & (kPRing - 1)][col];
#pragma unroll
      for (int j = 0; j < R; ++j) {
        float acc = qk[0] * y[j + kPrefR];
#pragma unroll
        for (int k = 1; k <= kPrefR; ++k) acc += qk[k] * (y[j + kPrefR - k] + y[j + kPrefR + k]);
        const int gy = y0 + j, gx = x0 + col;
        if (gy < yseg1 && gx < n) dst[(size_t)gy * n + gx] = acc * scale;
      }
    }
  }
}

rl_status launch_prefilter(const rl_plan* p, Slices<const float> in, Slices<float> out, int batch, float scale,
                           hipStream_t s) {
  const int n = p->d.n;
  const int seg = p->tune.prefilter_rows;  // a multiple of kPRB
  dim3 grid((n + kPSW - 1) / kPSW, (n + seg - 1) / seg, batch);
  RL_LAUNCH("k_prefilter", k_prefilter, grid, dim3(kThreads), 0, s, in, out, n, scale, p->d.pref, seg);
  return check_launch("k_prefilter");
}

// ------------------------------------------------------------------ cart -> log-polar
constexpr int kFQ = 64;         // rho indices per block: one per lane of a wave
constexpr int kFRows = 8;       // coarse rows per segment (tile)
constexpr int kFSeg = 2;        // segments (vertically adjacent tiles) per block
constexpr int kFPatch = 8448;   // floats of the LDS image patch (large tiles)
constexpr int kFPatchSmall = 5504;  // patch of the small tiles: four blocks per CU fit in LDS
// Row pitches of the patches (odd, so that rows spread over the LDS banks).  A fixed pitch puts
// the 16 taps of a sample at compile-time offsets from one address; a box is staged when its
// width fits the pitch and its height PATCH / PITCH rows.  Pitch 0: the box's own width | 1
// (boxes of wide sectors, M >= 6), staged when that pitch times its height fits PATCH.
constexpr int kFPitch = 93;
constexpr int kFPitchSmall = 77;
constexpr int kFThreads = 512;  // threads per block
static_assert(kFQ == 64, "the sample loop maps rho indices to the lanes of a wave");

// Bicubic sample of the spline coefficients at index position (X, Y); taps read through `tap`.
template <class Tap>
__device__ __forceinline__ float bicubic_at(double X, double Y, int n, Tap tap) {
  const double fx = floor(X), fy = floor(Y);
  float wx[4], wy[4];
  bspline_w6((float)(X - fx), wx);
  bspline_w6((float)(Y - fy), wy);
  const int kx = min(max((int)fx, -1), n), ky = min(max((int)fy, -1), n);
  float v = 0.f;
#pragma unroll
  for (int bb = 0; bb < 4; ++bb) {
    float h = 0.f;
#pragma unroll
    for (int a = 0; a < 4; ++a) h += wx[a] * tap(kx - 1 + a, ky - 1 + bb);
    v += wy[bb] * h;
  }
  return v * (1.0f / 36.0f);
}

// Block: kFQ consecutive rho indices and kFSeg x kFRows coarse rows of one (slice, partition),
// taken as kFSeg segments of kFRows rows (each a tile with its own image box).  Per segment:
// 1) The fine rays feeding its rows sweep an annular sector of the image; the sector's
//    bounding box is staged in LDS (global gathers if it does not fit).  2) Each wave computes
//    the bicubic samples of one fine ray at a time, a lane per rho index, into an LDS buffer;
//    samples outside D are zero.  The last 3r - 1 fine rays of a segment are the first of the
//    next: they are moved to the front of the buffer and not sampled again.  3) Each coarse
//    sample is the decimation filter over the fine rows around it, times e^rho.
template <int PATCH, int PITCH>
__global__ __launch_bounds__(kFThreads) void k_cart2lp(DevPlan P, const int* __restrict__ tiles,
                                                        const float* __restrict__ c, float* __restrict__ u,
                                                        int xcd_order) {
  extern __shared__ float smem[];
  float* patch = smem;
  float* vbuf = smem + PATCH;
  // first tile (m, by, bx) of the block from the plan's list for this patch size; slice from
  // blockIdx.y
  const int gx = (P.n_rho + kFQ - 1) / kFQ, gy = (P.n_sup + kFRows - 1) / kFRows;
  // (list entry, slice) of this block; with xcd_order each XCD takes one contiguous run of
  // them, so tiles that read overlapping image boxes share that XCD's L2
  const int bid = blockIdx.y * gridDim.x + blockIdx.x;
  const int lid = xcd_order ? xcd_block(bid, gridDim.x * gridDim.y) : bid;
  const int b = lid / gridDim.x;
  const int tile0 = tiles[lid - b * gridDim.x];
  const int bx = tile0 % gx, by0 = (tile0 / gx) % gy, m = tile0 / (gx * gy);
  const int bm = b * P.m + m;
  const int q0 = bx * kFQ;
  const int n = P.n, r = P.r;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  const double X0 = P.X0[m], Y0 = P.Y0[m];
  const float* img = c + (size_t)b * n * n;
  const double2* cs = P.fine_cs + (size_t)m * P.n_fine;
  const int2* fq = P.fine_q + (size_t)m * P.n_fine;
  const int nftmax = r * (kFRows + 3) - 1;  // the launch sizes LDS for this many rows
  // LDS copies of the segment's ray table (direction, rho range inside D), of e^rho and of the
  // decimation taps
  double2* scs = reinterpret_cast<double2*>(vbuf + nftmax * kFQ);
  int2* sfq = reinterpret_cast<int2*>(scs + nftmax);
  double* se = reinterpret_cast<double*>(sfq + nftmax);
  float* sdt = reinterpret_cast<float*>(se + kFQ);
  const int qlast = min(q0 + kFQ, P.n_rho) - 1;
  const int nd = 4 * r - 1, nd8 = (nd + 7) & ~7;  // taps, padded with zeros to chunks of 8
  if (threadIdx.x < kFQ) se[threadIdx.x] = q0 + (int)threadIdx.x <= qlast ? P.erho[q0 + threadIdx.x] : 0.0;
  for (int k = threadIdx.x; k < nd8; k += blockDim.x) sdt[k] = k < nd ? P.dtap[k] : 0.f;
  const int ql = lane, q = q0 + lane;
  int kept = 0;  // leading fine rows of vbuf carried over from the previous segment
  // image boxes of the block's tiles (built with the plan; W == 0: no sample inside D), all
  // loaded up front
  int4 boxes[kFSeg];
#pragma unroll
  for (int sg = 0; sg < kFSeg; ++sg) boxes[sg] = P.fbox[tile0 + min(sg, gy - 1 - by0) * gx];
#pragma unroll
  for (int sg = 0; sg < kFSeg; ++sg) {
    const int by = by0 + sg;
    if (by >= gy) break;  // uniform
    const int i0 = by * kFRows;
    const int i1 = min(i0 + kFRows, P.n_sup);
    // fine rows t with |t - r i| < 2r for some i in [i0, i1)
    const int tlo = r * (i0 - 2) + 1, thi = r * (i1 + 1) - 1;
    const int nft = thi - tlo + 1;
    const int tclo = max(tlo, P.t_min), tchi = min(thi, P.t_min + P.n_fine - 1);
    const int4 box = boxes[sg];
    if (sg > 0) __syncthreads();  // the previous segment is done with vbuf, the tables and the patch
    if (box.z == 0) {
      for (int o = threadIdx.x; o < (i1 - i0) * kFQ; o += blockDim.x) {
        const int il = o / kFQ, ql2 = o - il * kFQ;
        if (q0 + ql2 <= qlast) u[((size_t)bm * P.n_sup + i0 + il) * P.n_rho + q0 + ql2] = 0.f;
      }
      kept = 0;
      continue;  // uniform across the block
    }
    // the previous segment's fine rows from r kFRows on are this segment's first `kept` rows
    // (source rows start past the destination's end: no thread overwrites what another reads)
    for (int o = threadIdx.x; o < kept * kFQ; o += blockDim.x) vbuf[o] = vbuf[r * kFRows * kFQ + o];
    // one memory round trip for the segment's inputs: a ray-table entry per thread (address
    // clamped into the table) and every staged group are loaded, unconditionally, before any
    // is stored (a load under a branch would make the branch's join wait for it)
    const int tq = min(max(tlo + (int)threadIdx.x, P.t_min), P.t_min + P.n_fine - 1) - P.t_min;
    const int2 qr_ld = fq[tq];
    const double2 tc_ld = cs[tq];
    const int Xlo = box.x, Ylo = box.y, W = box.z, H = box.w;
    const int pitch = PITCH ? PITCH : (W | 1);
    const bool staged = PITCH ? ((W | 1) <= PITCH && H <= PATCH / PITCH) : pitch * H <= PATCH;
    // groups of four consecutive pixels in flat order, at most PATCH / 4 of them: kU per thread;
    // (ly, lg) advance by the block stride without a division per group.  A group inside the
    // image is one float4 load (rows of 4-aligned groups are 16-byte aligned when n % 4 == 0);
    // a group across the image edge is loaded again below, pixel by pixel with the periodic wrap
    constexpr int kU = (PATCH / 4 + kFThreads - 1) / kFThreads;
    const int Wg = W >> 2, tot = staged ? Wg * H : 0;
    const bool vec_ok = (n & 3) == 0;
    float4 v[kU];
    int dsti[kU];
    bool edge[kU];
    {
      const int wg = max(Wg, 1);
      const int dly = (int)blockDim.x / wg, dlg = (int)blockDim.x - dly * wg;
      int ly = (int)threadIdx.x / wg, lg = (int)threadIdx.x - ly * wg;
#pragma unroll
      for (int uu = 0; uu < kU; ++uu) {
        const bool ok = uu * (int)blockDim.x + (int)threadIdx.x < tot;
        int gyy = Ylo + ly;
        if (gyy < 0 || gyy >= n) gyy = ((gyy % n) + n) % n;
        const int gxx = Xlo + 4 * lg;
        const bool inb = vec_ok && gxx >= 0 && gxx + 3 < n;
        if (vec_ok && staged) {
          const int xc = min(max(gxx, 0), n - 4);
          v[uu] = *reinterpret_cast<const float4*>(img + (size_t)(ok ? gyy : 0) * n + xc);
        }
        dsti[uu] = ok ? ly * pitch + 4 * lg : -1;
        edge[uu] = ok && !inb;
        ly += dly;
        lg += dlg;
        if (lg >= wg) {
          lg -= wg;
          ++ly;
        }
      }
    }
    for (int tl = threadIdx.x; tl < nft; tl += blockDim.x) {
      const int t = tlo + tl;
      const bool in = t >= tclo && t <= tchi;
      int2 qr = make_int2(1, 0);  // empty
      double2 tc = make_double2(0.0, 0.0);
      if (tl == (int)threadIdx.x) {
        if (in) {
          qr = qr_ld;
          tc = tc_ld;
        }
      } else if (in) {  // rows past the block's threads (r > 46 only)
        qr = fq[t - P.t_min];
        tc = cs[t - P.t_min];
      }
      sfq[tl] = qr;
      scs[tl] = tc;
    }
#pragma unroll
    for (int uu = 0; uu < kU; ++uu) {
      if (dsti[uu] < 0) continue;
      float4 w = v[uu];
      if (edge[uu]) {
        const int idx = uu * (int)blockDim.x + (int)threadIdx.x;
        const int ly = idx / Wg, lg = idx - ly * Wg;
        int gyy = Ylo + ly;
        if (gyy < 0 || gyy >= n) gyy = ((gyy % n) + n) % n;
        const float* srow = img + (size_t)gyy * n;
        float tt[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          int x = Xlo + 4 * lg + e;
          if (x < 0 || x >= n) x = ((x % n) + n) % n;
          tt[e] = srow[x];
        }
        w = make_float4(tt[0], tt[1], tt[2], tt[3]);
      }
      float* d = patch + dsti[uu];
      d[0] = w.x;
      d[1] = w.y;
      d[2] = w.z;
      d[3] = w.w;
    }
    __syncthreads();
    // fine samples of rows kept .. nft - 1: a wave takes one ray at a time (its table entries
    // are wave-uniform LDS broadcasts), lane l the rho index q0 + l
    const double E = se[ql];
    if (staged) {
      // two rays per step, branch-free (independent chains for the scheduler): taps are clamped
      // into the patch and samples outside D or past the last ray are zeroed by a select
      auto sample = [&](int tl) -> float {
        const int tr = min(tl, nft - 1);
        const int2 qr = sfq[tr];
        const double2 tc = scs[tr];
        const double X = X0 + E * tc.x, Y = Y0 + E * tc.y;
        const double fx = floor(X), fy = floor(Y);
        float wx[4], wy[4];
        bspline_w6((float)(X - fx), wx);
        bspline_w6((float)(Y - fy), wy);
        const unsigned bxx = min((unsigned)((int)fx - 1 - Xlo), (unsigned)(W - 4));
        const unsigned byy = min((unsigned)((int)fy - 1 - Ylo), (unsigned)(H - 4));
        const float* p0 = patch + __umul24(byy, (unsigned)pitch) + bxx;
        float v = 0.f;
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) {
          const float* pr = p0 + bb * pitch;
          v += wy[bb] * (wx[0] * pr[0] + wx[1] * pr[1] + wx[2] * pr[2] + wx[3] * pr[3]);
        }
        const bool in = tl < nft && q <= qlast && q >= qr.x && q <= qr.y;
        return in ? v * (1.0f / 36.0f) : 0.f;
      };
      for (int tl = kept + wave; tl < nft; tl += 2 * nwave) {
        const float v0 = sample(tl);
        const float v1 = sample(tl + nwave);
        vbuf[tl * kFQ + ql] = v0;
        if (tl + nwave < nft) vbuf[(tl + nwave) * kFQ + ql] = v1;
      }
    } else {
      for (int tl = kept + wave; tl < nft; tl += nwave) {
        const int2 qr = sfq[tl];
        const double2 tc = scs[tl];
        float v = 0.f;
        if (q <= qlast && q >= qr.x && q <= qr.y) {
          const double X = X0 + E * tc.x, Y = Y0 + E * tc.y;
          v = bicubic_at(X, Y, n, [&](int x, int y) { return img[(size_t)wrap1(y, n) * n + wrap1(x, n)]; });
        }
        vbuf[tl * kFQ + ql] = v;
      }
    }
    __syncthreads();
    // decimation: u[i][q] = e^rho_q sum_n d_n v[r i + n][q], the taps in chunks of 8 whose 16 LDS
    // reads all issue before the chunk's adds (past the last tap: row clamped, tap 0)
    for (int o = threadIdx.x; o < (i1 - i0) * kFQ; o += blockDim.x) {
      const int il = o / kFQ, ql2 = o - il * kFQ;
      const int qq = q0 + ql2;
      if (qq > qlast) continue;
      const int i = i0 + il;
      const float* vcol = vbuf + (r * i - (2 * r - 1) - tlo) * kFQ + ql2;
      float acc = 0.f;
      for (int k0 = 0; k0 < nd; k0 += 8) {
        float tv[8], vv[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          tv[j] = sdt[k0 + j];
          vv[j] = vcol[min(k0 + j, nd - 1) * kFQ];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) acc += tv[j] * vv[j];
      }
      const float er = (float)(se[ql2] * (P.a_R * P.dx));
      // lattice rows past this partition's support (partitions own different numbers of rows)
      // are zero: the theta convolution must not see the fine rays beyond its last halo row
      u[((size_t)bm * P.n_sup + i) * P.n_rho + qq] = i < P.sup_rows[m] ? acc * er : 0.f;
    }
    // a full segment's rows r kFRows .. nft - 1 are the next segment's first 3r - 1
    kept = i1 - i0 == kFRows ? 3 * r - 1 : 0;
  }
}

// Image boxes of the forward tiles (plan time, host): for tile (bx, by) of partition m (kFQ rho
// indices, kFRows coarse rows), (Xlo, Ylo, W, H) bounds the image indices of every 4 x 4 tap
// set of its fine samples inside D: the annular sector swept by its rays between e^rho of its
// first and last rho index, widened where the outer arc crosses an axis direction, plus the
// taps' reach.  Xlo and W are multiples of 4 (float4 staging).  W = 0 marks a tile none of
// whose samples lies in D.
std::vector<int4> build_fwd_boxes(const DevPlan& d, const std::vector<double2>& cs_all,
                                  const std::vector<int2>& fq_all, const std::vector<double>& erho) {
  const int gx = (d.n_rho + kFQ - 1) / kFQ, gy = (d.n_sup + kFRows - 1) / kFRows, r = d.r;
  std::vector<int4> out((size_t)d.m * gy * gx, make_int4(0, 0, 0, 0));
  for (int m = 0; m < d.m; ++m) {
    const double2* cs = cs_all.data() + (size_t)m * d.n_fine;
    const int2* fq = fq_all.data() + (size_t)m * d.n_fine;
    for (int by = 0; by < gy; ++by) {
      const int i0 = by * kFRows, i1 = std::min(i0 + kFRows, d.n_sup);
      const int tlo = r * (i0 - 2) + 1, thi = r * (i1 + 1) - 1;
      const int tclo = std::max(tlo, d.t_min), tchi = std::min(thi, d.t_min + d.n_fine - 1);
      for (int bx = 0; bx < gx; ++bx) {
        const int q0 = bx * kFQ, qlast = std::min(q0 + kFQ, d.n_rho) - 1;
        bool inside = false;
        for (int t = tclo; t <= tchi && !inside; ++t) {
          const int2 qr = fq[t - d.t_min];
          inside = qr.x <= qr.y && qr.x <= qlast && qr.y >= q0;
        }
        if (!inside) continue;
        const double Elo = erho[q0], Ehi = erho[qlast];
        const double2 ca = cs[tclo - d.t_min], cb = cs[tchi - d.t_min];
        double xmin = std::min(std::min(Elo * ca.x, Ehi * ca.x), std::min(Elo * cb.x, Ehi * cb.x));
        double xmax = std::max(std::max(Elo * ca.x, Ehi * ca.x), std::max(Elo * cb.x, Ehi * cb.x));
        double ymin = std::min(std::min(Elo * ca.y, Ehi * ca.y), std::min(Elo * cb.y, Ehi * cb.y));
        double ymax = std::max(std::max(Elo * ca.y, Ehi * ca.y), std::max(Elo * cb.y, Ehi * cb.y));
        {
          const double pa = std::atan2(ca.y, ca.x), pb = std::atan2(cb.y, cb.x);
          const double lo = std::min(pa, pb), hi = std::max(pa, pb);
          for (int k = -2; k <= 2; ++k) {
            const double ax = k * (0.5 * M_PI);
            if (ax > lo && ax < hi) {
              const int kk = (k + 4) & 3;
              if (kk == 0) xmax = std::max(xmax, Ehi);
              if (kk == 2) xmin = std::min(xmin, -Ehi);
              if (kk == 1) ymax = std::max(ymax, Ehi);
              if (kk == 3) ymin = std::min(ymin, -Ehi);
            }
          }
        }
        const int Xlo = ((int)std::floor(d.X0[m] + xmin) - 3) & ~3;
        const int Ylo = (int)std::floor(d.Y0[m] + ymin) - 3;
        const int W = (((int)std::floor(d.X0[m] + xmax) + 4 - Xlo + 1) + 3) & ~3;
        const int H = (int)std::floor(d.Y0[m] + ymax) + 4 - Ylo + 1;
        out[((size_t)m * gy + by) * gx + bx] = make_int4(Xlo, Ylo, W, H);
      }
    }
  }
  return out;
}

static size_t cart2lp_lds(const DevPlan& d, int patch) {
  const int nft = d.r * (kFRows + 3) - 1;
  return (size_t)(patch + nft * kFQ) * sizeof(float) + (size_t)nft * (sizeof(double2) + sizeof(int2)) +
         kFQ * sizeof(double) + (size_t)((4 * d.r - 1 + 7) & ~7) * sizeof(float);
}

// The plan lists the blocks whose tiles' image boxes fit the small patch at its pitch (or have
// no sample in D) first, then those that fit the large patch at its pitch, then the others;
// each list runs with its own LDS size and pitch, so that the small blocks, most of them, run
// four per CU.  The timing hooks record the launches as one k_cart2lp interval.
rl_status launch_cart2lp(const rl_plan* p, const float* c, float* u, int batch, hipStream_t s) {
  const DevPlan& d = p->d;
  const int slot = prof_open("k_cart2lp", s);
  rl_status st = RL_OK;
  // with the split off, every tile runs with the large patch at its box's pitch (one launch
  // over the three lists)
  const bool split = p->tune.fwd_patch_split != 0;
  const int n_small = split ? d.ftiles_small : 0, n_mid = split ? d.ftiles_mid : 0;
  const int n_large = d.ftiles_small + d.ftiles_mid + d.ftiles_large - n_small - n_mid;
  if (n_small > 0) {
    hipLaunchKernelGGL((k_cart2lp<kFPatchSmall, kFPitchSmall>), dim3(n_small, batch), dim3(kFThreads),
                       cart2lp_lds(d, kFPatchSmall), s, d, d.ftiles, c, u, p->tune.fwd_xcd_order);
    st = check_launch("k_cart2lp");
  }
  if (st == RL_OK && n_mid > 0) {
    hipLaunchKernelGGL((k_cart2lp<kFPatch, kFPitch>), dim3(n_mid, batch), dim3(kFThreads), cart2lp_lds(d, kFPatch),
                       s, d, d.ftiles + n_small, c, u, p->tune.fwd_xcd_order);
    st = check_launch("k_cart2lp");
  }
  if (st == RL_OK && n_large > 0) {
    hipLaunchKernelGGL((k_cart2lp<kFPatch, 0>), dim3(n_large, batch), dim3(kFThreads), cart2lp_lds(d, kFPatch), s,
                       d, d.ftiles + n_small + n_mid, c, u, p->tune.fwd_xcd_order);
    st = check_launch("k_cart2lp");
  }
  prof_close(slot, s);
  return st;
}

// Plan time (host): the block lists of launch_cart2lp, from the image boxes.  A block takes the
// tiles (m, by, bx) .. (m, by + kFSeg - 1, bx) with by a multiple of kFSeg (fewer at the last
// block row); it is listed, by its first tile, under the largest patch one of its tiles needs.
std::vector<int> build_fwd_tiles(const DevPlan& d, const std::vector<int4>& boxes, int* n_small, int* n_mid) {
  const int gx = (d.n_rho + kFQ - 1) / kFQ, gy = (d.n_sup + kFRows - 1) / kFRows;
  std::vector<int> lists[3];
  for (int m = 0; m < d.m; ++m)
    for (int by = 0; by < gy; by += kFSeg)
      for (int bx = 0; bx < gx; ++bx) {
        const int t0 = (m * gy + by) * gx + bx;
        int cls = 0;
        for (int s = 0; s < kFSeg && by + s < gy; ++s) {
          const int4 bb = boxes[t0 + s * gx];
          const bool fits_small = (bb.z | 1) <= kFPitchSmall && bb.w <= kFPatchSmall / kFPitchSmall;
          const bool fits_mid = (bb.z | 1) <= kFPitch && bb.w <= kFPatch / kFPitch;
          cls = std::max(cls, (bb.z == 0 || fits_small) ? 0 : fits_mid ? 1 : 2);
        }
        lists[cls].push_back(t0);
      }
  *n_small = (int)lists[0].size();
  *n_mid = (int)lists[1].size();
  std::vector<int> out = lists[0];
  out.insert(out.end(), lists[1].begin(), lists[1].end());
  out.insert(out.end(), lists[2].begin(), lists[2].end());
  return out;
}

// ------------------------------------------------------------------ rho FFTs of rows
// in: real rows of length n_rho (stride n_rho); out: half spectra X[0..nc] (stride ld).
__global__ __launch_bounds__(kThreads) void k_rfft_rows(DevPlan P, const float* __restrict__ in,
                                                        float2* __restrict__ out) {
  extern __shared__ float2 sh[];
  const int nc = P.nc;
  const size_t row = blockIdx.x;
  const float2* src = reinterpret_cast<const float2*>(in + row * P.n_rho);
  row_copy<kChunkSmall>(nc, [&](int i) { return src[i]; }, [&](int i, float2 v) { sh[i] = v; });
  __syncthreads();
  fft_lds<kRowVals, false>(sh, nc, 1, P.twp_rows);
  float2* dst = out + row * P.ld;
  rfft_post<kChunkSmall>(sh, nc, P.tw, P.tw_len, [&](int k, float2 x) { dst[k] = x; });
}

rl_status launch_rfft_rows(const rl_plan* p, const float* in, float2* out, int rows, hipStream_t s) {
  const DevPlan& d = p->d;
  RL_LAUNCH("k_rfft_rows", k_rfft_rows, dim3(rows), dim3(kThreads), d.nc * sizeof(float2), s, d, in, out);
  return check_launch("k_rfft_rows");
}

// Inverse of k_rfft_rows without normalisation: out rows of length n_rho.
__global__ __launch_bounds__(kThreads) void k_irfft_rows(DevPlan P, const float2* __restrict__ in,
                                                         float* __restrict__ out) {
  extern __shared__ float2 sh[];
  const int nc = P.nc;
  const size_t row = blockIdx.x;
  const float2* src = in + row * P.ld;
  irfft_pre(sh, nc, P.tw, P.tw_len, [&](int k) { return src[k]; });
  __syncthreads();
  fft_lds<kRowVals, true>(sh, nc, 1, P.twp_rows);
  float2* dst = reinterpret_cast<float2*>(out + row * P.n_rho);
  for (int i = threadIdx.x; i < nc; i += blockDim.x) dst[i] = sh[i];
}

rl_status launch_irfft_rows(const rl_plan* p, const float2* in, float* out, int rows, hipStream_t s) {
  const DevPlan& d = p->d;
  RL_LAUNCH("k_irfft_rows", k_irfft_rows, dim3(rows), dim3(kThreads), d.nc * sizeof(float2), s, d, in, out);
  return check_launch("k_irfft_rows");
}

// ------------------------------------------------------------------ theta convolution
// Four-step FFT of length K = K1 K2 along theta for CW spectrum columns of one
// (slice, partition), with the multiplier applied between the forward and inverse K2-point
// stages, so that the whole convolution makes two LDS round trips:
//   A   thread (n2, c): x[n1] = in[K2 n1 + n2]; K1-point FFT over n1; times W_K^{n2 k1} -> LDS
//   B   thread (k1, c): K2-point FFT over n2 (-> k = k1 + K1 k2); times H (or conj H);
//       inverse K2-point FFT -> LDS
//   A'  thread (n2, c): times W_K^{-n2 k1}; inverse K1-point FFT -> out rows K2 n1 + n2
// Rows outside the input range are zero; only the requested output rows are written.  The
// twiddles W_K^{n2 k1} are copied to LDS once per block (n2-major, as stage A reads them).
template <int K1, int K2>
__global__ __launch_bounds__(kThreads) void k_theta_conv(DevPlan P, const float2* __restrict__ in, int in_rows,
                                                         int in_off, int in_step, float2* __restrict__ out,
                                                         int out_rows, int out_off, int out_step, int conj, int cw,
                                                         int xcd_order) {
  extern __shared__ float2 sh[];
  constexpr int K = K1 * K2;
  constexpr int RS = K2 + 1;           // padded stride between k1 rows
  constexpr int CS = K1 * RS + 1;      // padded stride between columns
  const int nkt = K / 2 + 1, ncol = P.nc + 1;
  // the four-step twiddles W_K^{n2 k1}, copied once per block behind the columns' buffers
  float2* twl = sh + ((cw * CS + 1) & ~1);
  {
    const float4* src4 = reinterpret_cast<const float4*>(P.tw_theta);
    float4* dst4 = reinterpret_cast<float4*>(twl);
    for (int i = threadIdx.x; i < K / 2; i += blockDim.x) dst4[i] = src4[i];
  }
  // neighbouring column strips share 128-byte lines: keep them on one XCD
  const int bid = blockIdx.y * gridDim.x + blockIdx.x;
  const int lid = xcd_order ? xcd_block(bid, gridDim.x * gridDim.y) : bid;
  const int bm = lid / gridDim.x;
  const int col0 = (lid - bm * gridDim.x) * cw;
  const float2* src = in + (size_t)bm * in_rows * P.ld;
  // stage A
  {
    const int c = threadIdx.x % cw, n2 = threadIdx.x / cw;
    const int col = col0 + c;
    const bool act = n2 < K2 && col < ncol;
    float2 x[K1];
    if (act) {
#pragma unroll
      for (int n1 = 0; n1 < K1; ++n1) {
        // lattice row K2 n1 + n2 holds input row ir if it is in_off + in_step * ir
        const int lr = K2 * n1 + n2 - in_off;
        const int ir = in_step == 1 ? lr : lr >> 1;
        const bool hit = lr >= 0 && (in_step == 1 || (lr & 1) == 0) && ir < in_rows;
        // (a 24-bit product: rows and their stride are far below 2^24)
        x[n1] = hit ? src[__umul24((unsigned)ir, (unsigned)P.ld) + col] : make_float2(0.f, 0.f);
      }
      reg_fft<K1, false>(x, P.tw, P.tw_len);
    }
    __syncthreads();  // the twiddle copy is complete
    if (act) {
      float2* T = sh + c * CS;
      const float4* tq = reinterpret_cast<const float4*>(twl + n2 * K1);
#pragma unroll
      for (int k1 = 0; k1 < K1; k1 += 2) {
        const float4 t = tq[k1 / 2];
        const float2 w0 = make_float2(t.x, t.y), w1 = make_float2(t.z, t.w);
        T[k1 * RS + n2] = (k1 == 0 || n2 == 0) ? x[k1] : cmul(x[k1], w0);
        T[(k1 + 1) * RS + n2] = n2 == 0 ? x[k1 + 1] : cmul(x[k1 + 1], w1);
      }
    }
  }
  __syncthreads();
  // stage B
  {
    const int c = threadIdx.x % cw, k1 = threadIdx.x / cw;
    const int col = col0 + c;
    if (k1 < K1 && col < ncol) {
      float2* T = sh + c * CS + k1 * RS;
      float2 y[K2];
#pragma unroll
      for (int n2 = 0; n2 < K2; ++n2) y[n2] = T[n2];
      reg_fft<K2, false>(y, P.tw, P.tw_len);
      const float2* Hc = P.H + (size_t)col * nkt;
#pragma unroll
      for (int k2 = 0; k2 < K2; ++k2) {
        const int kt = k1 + K1 * k2;
        float2 h = Hc[kt <= K / 2 ? kt : K - kt];
        if (conj) h.y = -h.y;
        y[k2] = cmul(y[k2], h);
      }
      reg_fft<K2, true>(y, P.tw, P.tw_len);
#pragma unroll
      for (int n2 = 0; n2 < K2; ++n2) T[n2] = y[n2];
    }
  }
  __syncthreads();
  // stage A'
  {
    const int c = threadIdx.x % cw, n2 = threadIdx.x / cw;
    const int col = col0 + c;
    if (n2 < K2 && col < ncol) {
      const float2* T = sh + c * CS;
      const float4* tq = reinterpret_cast<const float4*>(twl + n2 * K1);
      float2 x[K1];
#pragma unroll
      for (int k1 = 0; k1 < K1; k1 += 2) {
        const float4 t = tq[k1 / 2];
        const float2 w0 = make_float2(t.x, -t.y), w1 = make_float2(t.z, -t.w);
        const float2 v0 = T[k1 * RS + n2], v1 = T[(k1 + 1) * RS + n2];
        x[k1] = (k1 == 0 || n2 == 0) ? v0 : cmul(v0, w0);
        x[k1 + 1] = n2 == 0 ? v1 : cmul(v1, w1);
      }
      reg_fft<K1, true>(x, P.tw, P.tw_len);
      float2* dst = out + (size_t)bm * out_rows * P.ld;
#pragma unroll
      for (int n1 = 0; n1 < K1; ++n1) {
        const int lr = K2 * n1 + n2 - out_off;
        const int orow = out_step == 1 ? lr : lr >> 1;
        if (lr >= 0 && (out_step == 1 || (lr & 1) == 0) && orow < out_rows)
          dst[__umul24((unsigned)orow, (unsigned)P.ld) + col] = x[n1];
      }
    }
  }
}

// Columns per block of the theta pass: at most 256 / max(K1, K2) (one thread per column and row
// of each stage), 8 at most (the default), or the plan's tuned value if it fits.
template <int K1, int K2>
static int theta_cw(int tuned) {
  const int cap = max(1, min(8, kThreads / max(K1, K2)));
  return (tuned >= 1 && tuned <= cap) ? tuned : cap;
}

template <int K1, int K2>
static size_t theta_lds(int cw) {
  return ((size_t)cw * (K1 * (K2 + 1) + 1) + 1 + K1 * K2) * sizeof(float2);
}

template <int K1, int K2>
static rl_status theta_prepare() {
  // the largest LDS any column count needs
  return ensure_dyn_lds((const void*)k_theta_conv<K1, K2>, theta_lds<K1, K2>(theta_cw<K1, K2>(0)),
                        "hipFuncSetAttribute(k_theta_conv)");
}

rl_status prepare_forward_launches(const rl_plan* p) {
  rl_status st = ensure_dyn_lds((const void*)k_cart2lp<kFPatchSmall, kFPitchSmall>, cart2lp_lds(p->d, kFPatchSmall),
                                "hipFuncSetAttribute(k_cart2lp)");
  if (st != RL_OK) return st;
  st = ensure_dyn_lds((const void*)k_cart2lp<kFPatch, kFPitch>, cart2lp_lds(p->d, kFPatch),
                      "hipFuncSetAttribute(k_cart2lp)");
  if (st != RL_OK) return st;
  st = ensure_dyn_lds((const void*)k_cart2lp<kFPatch, 0>, cart2lp_lds(p->d, kFPatch), "hipFuncSetAttribute(k_cart2lp)");
  if (st != RL_OK) return st;
  switch (p->d.k_theta) {
#define RL_THETA_CASE(K, K1, K2) \
  case K: return theta_prepare<K1, K2>();
    RL_THETA_LENGTHS(RL_THETA_CASE)
#undef RL_THETA_CASE
    default: return fail(RL_ERR_INTERNAL, "unsupported k_theta");
  }
}

template <int K1, int K2>
static rl_status launch_theta_conv_t(const rl_plan* p, const float2* in, int in_rows, int in_off, int in_step,
                                     float2* out, int out_rows, int out_off, int out_step, bool conj, int batch,
                                     hipStream_t s, const float2* H) {
  if ((in_step != 1 && in_step != 2) || (out_step != 1 && out_step != 2))
    return fail(RL_ERR_INTERNAL, "theta pass row step must be 1 or 2");
  DevPlan d = p->d;
  if (H) d.H = H;
  const int cw = theta_cw<K1, K2>(p->tune.theta_cols);
  const size_t lds = theta_lds<K1, K2>(cw);
  rl_status st = ensure_dyn_lds((const void*)k_theta_conv<K1, K2>, lds, "hipFuncSetAttribute(k_theta_conv)");
  if (st != RL_OK) return st;
  dim3 grid((d.nc + 1 + cw - 1) / cw, batch * d.m);
  RL_LAUNCH("k_theta_conv", (k_theta_conv<K1, K2>), grid, dim3(kThreads), lds, s, d, in, in_rows, in_off, in_step,
            out, out_rows, out_off, out_step, conj ? 1 : 0, cw, p->tune.theta_xcd_order);
  return check_launch("k_theta_conv");
}

rl_status launch_theta_conv(const rl_plan* p, const float2* in, int in_rows, int in_off, int in_step, float2* out,
                            int out_rows, int out_off, int out_step, bool conj, int batch, hipStream_t s,
                            const float2* H) {
  switch (p->d.k_theta) {
#define RL_THETA_CASE(K, K1, K2) \
  case K:                        \
    return launch_theta_conv_t<K1, K2>(p, in, in_rows, in_off, in_step, out, out_rows, out_off, out_step, conj, batch, s, H);
    RL_THETA_LENGTHS(RL_THETA_CASE)
#undef RL_THETA_CASE
    default: return fail(RL_ERR_INTERNAL, "unsupported k_theta");
  }
}

// ------------------------------------------------------------------ inverse rho FFT + evaluation
// Block: one owned row of one (slice, partition); writes sinogram row j.
__global__ __launch_bounds__(kThreads) void k_irfft_eval(DevPlan P, const float2* __restrict__ spec,
                                                         Slices<float> sino, float scale) {
  extern __shared__ float2 sh[];
  const int o = blockIdx.x;
  const int bm = blockIdx.y;
  const int b = bm / P.m, m = bm - b * P.m;
  const int jw = P.own_j[m * P.n_own + o];
  if (jw < 0) return;  // uniform across the block
  const int j = jw & ((1 << 30) - 1);
  const int nc = P.nc, nr = P.n_rho;
  const float2* src = spec + ((size_t)bm * P.n_own + o) * P.ld;
  irfft_pre<kChunkSmall>(sh, nc, P.tw, P.tw_len, [&](int k) { return src[k]; });
  __syncthreads();
  fft_lds<kRowVals, true>(sh, nc, 1, P.twp_rows);
  const float* x = reinterpret_cast<const float*>(sh);
  const float inv_aR = (float)(scale / (6.0 * P.a_R));  // 1/a_R, the weights' 1/6, the output scale
  float* __restrict__ dst = sino.at(b) + (size_t)j * P.n_s;
  const int2* tr = P.tau + ((size_t)m * P.n_own + o) * P.n_s;  // rho position of each sample
  row_copy<kChunkSmall>(
      P.n_s, [&](int k) { return tr[k]; },
      [&](int k, int2 t) {
        float w[4];
        bspline_w6(__int_as_float(t.y), w);
        const int kq = t.x;
        float acc = 0.f;
#pragma unroll
        for (int a = 0; a < 4; ++a) acc += w[a] * x[wrap1(kq - 1 + a, nr)];
        dst[k] = acc * inv_aR;
      });
}

rl_status launch_irfft_eval(const rl_plan* p, const float2* spec, Slices<float> sino, int batch, double scale,
                            hipStream_t s) {
  const DevPlan& d = p->d;
  dim3 grid(d.n_own, batch * d.m);
  RL_LAUNCH("k_irfft_eval", k_irfft_eval, grid, dim3(kThreads), d.nc * sizeof(float2), s, d, spec, sino,
            (float)scale);
  return check_launch("k_irfft_eval");
}

}  // namespace rl

using namespace rl;

namespace {

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

rl_status common_checks(const rl_plan* plan, const void* in, const void* out, int batch, void* ws, size_t ws_bytes,
                        rl_op op, size_t in_bytes, size_t out_bytes) {
  if (!plan) return fail(RL_ERR_INVALID_ARG, "plan is NULL");
  if (batch < 0) return fail(RL_ERR_INVALID_ARG, "batch is negative");
  if (batch == 0) return RL_OK;
  if (!in || !out) return fail(RL_ERR_INVALID_ARG, "input or output pointer is NULL");
  if (overlaps(in, in_bytes, out, out_bytes)) return fail(RL_ERR_INVALID_ARG, "input and output overlap");
  const size_t need = rl_workspace_bytes(plan, batch, op);
  if (!ws || ws_bytes < need)
    return fail(RL_ERR_WORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes, need " + std::to_string(need));
  if (((uintptr_t)ws) & 255) return fail(RL_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (overlaps(ws, need, in, in_bytes) || overlaps(ws, need, out, out_bytes))
    return fail(RL_ERR_INVALID_ARG, "workspace overlaps input or output");
  return check_plan_device(plan);
}

}  // namespace

namespace rl {

rl_status forward_chain(const rl_plan* plan, Slices<const float> img, Slices<float> sino, int batch, void* ws,
                        int stop_stage, float* stage_out, hipStream_t s, double out_scale) {
  const DevPlan& d = plan->d;
  const WsLayout L = workspace_layout(plan, batch, RL_OP_FWD);
  char* w = (char*)ws;
  float* c = (float*)(w + L.off[0]);
  float* u = (float*)(w + L.off[1]);
  float2* A = (float2*)(w + L.off[2]);
  float2* Bs = (float2*)(w + L.off[3]);
  rl_status st;
  const size_t nn = (size_t)d.n * d.n;
  if ((st = launch_prefilter(plan, img, dense(stop_stage == RL_STAGE_PREFILTER ? stage_out : c, nn), batch, 1.0f, s)) !=
      RL_OK)
    return st;
  if (stop_stage == RL_STAGE_PREFILTER) return RL_OK;
  if ((st = launch_cart2lp(plan, c, stop_stage == RL_STAGE_LOGPOLAR ? stage_out : u, batch, s)) != RL_OK) return st;
  if (stop_stage == RL_STAGE_LOGPOLAR) return RL_OK;
  if ((st = launch_rfft_rows(plan, u, A, batch * d.m * d.n_sup, s)) != RL_OK) return st;
  if ((st = launch_theta_conv(plan, A, d.n_sup, 0, 1, Bs, d.n_own, kHalo, d.q, false, batch, s)) != RL_OK) return st;
  if (stop_stage == RL_STAGE_CONV) return launch_irfft_rows(plan, Bs, stage_out, batch * d.m * d.n_own, s);
  return launch_irfft_eval(plan, Bs, sino, batch, out_scale, s);
}

}  // namespace rl

namespace {

rl_status fwd_entry(const rl_plan* plan, const float* d_img, float* d_sino, int32_t batch, void* d_ws,
                    size_t ws_bytes, hipStream_t stream, double out_scale) {
  rl_status st = RL_OK;
  if (plan) {
    const size_t ib = (size_t)batch * plan->d.n * plan->d.n * sizeof(float);
    const size_t ob = (size_t)batch * plan->d.n_theta * plan->d.n_s * sizeof(float);
    st = common_checks(plan, d_img, d_sino, batch, d_ws, ws_bytes, RL_OP_FWD, ib, ob);
  } else {
    st = fail(RL_ERR_INVALID_ARG, "plan is NULL");
  }
  if (st != RL_OK || batch == 0) return st;
  const DevPlan& d = plan->d;
  return forward_chain(plan, dense(d_img, (size_t)d.n * d.n), dense(d_sino, (size_t)d.n_theta * d.n_s), batch, d_ws,
                       -1, nullptr, stream, out_scale);
}

}  // namespace

extern "C" rl_status radon_fwd(const rl_plan* plan, const float* d_img, float* d_sino, int32_t batch, void* d_ws,
                               size_t ws_bytes, hipStream_t stream) {
  return fwd_entry(plan, d_img, d_sino, batch, d_ws, ws_bytes, stream, 1.0);
}

extern "C" rl_status radon_adj_transpose(const rl_plan* plan, const float* d_img, float* d_sino, int32_t batch,
                                         void* d_ws, size_t ws_bytes, hipStream_t stream) {
  if (!plan) return fail(RL_ERR_INVALID_ARG, "plan is NULL");
  const DevPlan& d = plan->d;
  return fwd_entry(plan, d_img, d_sino, batch, d_ws, ws_bytes, stream, (d.dtheta * d.ds) / (d.dx * d.dx));
}

extern "C" rl_status rl_debug_stage(const rl_plan* plan, rl_stage stage, const float* d_img, float* d_out,
                                    size_t d_out_bytes, void* d_ws, size_t ws_bytes, hipStream_t stream) {
  if (!plan || !d_out) return fail(RL_ERR_INVALID_ARG, "NULL argument");
  const DevPlan& d = plan->d;
  size_t need = 0;
  switch (stage) {
    case RL_STAGE_PREFILTER: need = (size_t)d.n * d.n * sizeof(float); break;
    case RL_STAGE_LOGPOLAR: need = (size_t)d.m * d.n_sup * d.n_rho * sizeof(float); break;
    case RL_STAGE_CONV: need = (size_t)d.m * d.n_own * d.n_rho * sizeof(float); break;
    case RL_STAGE_KERNEL: need = (size_t)(d.nc + 1) * (d.k_theta / 2 + 1) * sizeof(float2); break;
    default: return fail(RL_ERR_INVALID_ARG, "unknown stage");
  }
  if (d_out_bytes < need) return fail(RL_ERR_INVALID_ARG, "d_out too small for the stage");
  rl_status st = check_plan_device(plan);
  if (st != RL_OK) return st;
  if (stage == RL_STAGE_KERNEL)
    return check_hip(hipMemcpyAsync(d_out, d.H, need, hipMemcpyDeviceToDevice, stream), "copy kernel table");
  if (!d_img) return fail(RL_ERR_INVALID_ARG, "d_img is NULL");
  const size_t ib = (size_t)d.n * d.n * sizeof(float);
  st = common_checks(plan, d_img, d_out, 1, d_ws, ws_bytes, RL_OP_FWD, ib, need);
  if (st != RL_OK) return st;
  return forward_chain(plan, dense(d_img, ib / sizeof(float)), dense((float*)nullptr, 0), 1, d_ws, (int)stage, d_out,
                       stream, 1.0);
}
