// Back-projection R# as the exact weighted transpose of Algorithm 1, and FBP.
//
//   k_splat_rfft   transpose of the polar evaluation (Alg. 1 step 7): each log-polar rho
//                  node gathers the sinogram samples whose 4-tap B-spline footprint covers
//                  it (same taps and weights as the forward), times 1/a_R; then a real FFT
//                  along rho
//   k_theta_conv   (shared with the forward) with the conjugate multiplier
//   k_irfft_scale  inverse real FFT along rho of every support row, times e^rho (step 5)
//   k_lp2cart_adj  transpose of steps 3-4: per 48x48 image tile, every fine log-polar
//                  sample whose bicubic footprint meets the tile is rebuilt from the coarse
//                  rows by the decimation filter and spread into LDS with the same 16
//                  weights the forward gathers with; partitions are summed in the tile
//   k_prefilter    (shared) Q is symmetric, times w_S / w_X
//   k_ramp         FBP filter along s (sec. 6, eqs. ramp, cosfilt, SLfilt) as a zero-padded
//                  real FFT times the filter's multiplier
#include <hip/hip_runtime.h>

#include "fft_device.h"
#include "rl_internal.h"

namespace rl {

// ------------------------------------------------------------------ transpose of step 7
// One owned row per block.  The forward evaluation reads, for every sinogram sample k, the
// four periodic taps kq_k - 1 .. kq_k + 2 (kq_k = floor(tau_k)) of the log-polar row; its
// transpose adds w_a(tau_k) g_k / a_R to tap a.  Each thread adds the taps of its samples to
// an FP64 row in LDS (FP64 LDS atomics are fast on this target; where tau moves by more than
// one rho step from sample to sample, as usual, the lanes of one add hit distinct entries).  The row is
// then converted to FP32 in place and real-FFT'd.
__global__ __launch_bounds__(kThreads) void k_splat_rfft(DevPlan P, Slices<const float> sino,
                                                         float2* __restrict__ spec) {
  extern __shared__ double acc[];  // n_rho entries; reused as the FP32 FFT buffer
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
  const float inv_aR = (float)(1.0 / (6.0 * P.a_R));  // 1/a_R and the weights' 1/6
  const float* __restrict__ src = sino.at(b) + (size_t)j * ns;
  const int2* tr = P.tau + ((size_t)m * P.n_own + o) * ns;  // rho position of each sample
  for (int q = threadIdx.x; q < nr; q += blockDim.x) acc[q] = 0.0;
  __syncthreads();
  struct Sample {
    float g;
    int2 t;
  };
  row_copy(
      ns, [&](int k) { return Sample{src[k], tr[k]}; },
      [&](int, Sample sm) {
        const float g = sm.g * inv_aR;
        const int kq = sm.t.x;
        float w[4];
        bspline_w6(__int_as_float(sm.t.y), w);
#pragma unroll
        for (int a = 0; a < 4; ++a) atomicAdd(&acc[wrap1(kq - 1 + a, nr)], (double)(w[a] * g));
      });
  __syncthreads();
  // FP64 -> FP32 in place: every thread reads its entries before any is overwritten
  constexpr int kPer = 2 * kRowVals;  // n_rho <= kPer * blockDim.x (checked at plan time)
  float v[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int q = threadIdx.x + i * blockDim.x;
    v[i] = q < nr ? (float)acc[q] : 0.f;
  }
  __syncthreads();
  float* xs = reinterpret_cast<float*>(acc);
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int q = threadIdx.x + i * blockDim.x;
    if (q < nr) xs[q] = v[i];
  }
  __syncthreads();
  float2* sh = reinterpret_cast<float2*>(acc);
  fft_lds<kRowVals, false>(sh, nc, 1, P.twp_rows);
  rfft_post(sh, nc, P.tw, P.tw_len, [&](int k, float2 x) { dst[k] = x; });
}

rl_status prepare_adjoint_launches(const rl_plan* p) {
  return ensure_dyn_lds((const void*)k_splat_rfft, (size_t)p->d.n_rho * sizeof(double),
                        "hipFuncSetAttribute(k_splat_rfft)");
}

rl_status launch_splat_rfft(const rl_plan* p, Slices<const float> sino, float2* spec, int batch, hipStream_t s) {
  const DevPlan& d = p->d;
  const size_t lds = (size_t)d.n_rho * sizeof(double);
  dim3 grid(d.n_own, batch * d.m);
  rl_status st = ensure_dyn_lds((const void*)k_splat_rfft, lds, "hipFuncSetAttribute(k_splat_rfft)");
  if (st != RL_OK) return st;
  RL_LAUNCH("k_splat_rfft", k_splat_rfft, grid, dim3(kThreads), lds, s, d, sino, spec);
  return check_launch("k_splat_rfft");
}

// ------------------------------------------------------------------ inverse rho FFT, times e^rho
__global__ __launch_bounds__(kThreads) void k_irfft_scale(DevPlan P, const float2* __restrict__ spec,
                                                          float* __restrict__ u) {
  extern __shared__ float2 sh[];
  const int nc = P.nc;
  const size_t row = blockIdx.x;
  const float2* src = spec + row * P.ld;
  irfft_pre<kChunkSmall>(sh, nc, P.tw, P.tw_len, [&](int k) { return src[k]; });
  __syncthreads();
  fft_lds<kRowVals, true>(sh, nc, 1, P.twp_rows);
  const float* x = reinterpret_cast<const float*>(sh);
  float* dst = u + row * P.n_rho;
  const double e_scale = P.a_R * P.dx;
  row_copy<kChunkSmall>(
      P.n_rho, [&](int q) { return P.erho[q]; }, [&](int q, double e) { dst[q] = x[q] * (float)(e * e_scale); });
}

rl_status launch_irfft_scale(const rl_plan* p, const float2* spec, float* u, int batch, hipStream_t s) {
  const DevPlan& d = p->d;
  RL_LAUNCH("k_irfft_scale", k_irfft_scale, dim3(batch * d.m * d.n_sup), dim3(kThreads), d.nc * sizeof(float2), s, d, spec,
                     u);
  return check_launch("k_irfft_scale");
}

// ------------------------------------------------------------------ transpose of steps 3-4
__device__ __forceinline__ int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Block: one kTile x kTile image tile.  For every partition, the fine log-polar rays that
// cross the tile are listed first (one thread per ray): a ray t is the half-line
// x* + E (cos psi_t, sin psi_t) in image-index coordinates (x* = T_m^{-1}(0),
// E = e^rho / (a_R dx)).  A slab test against the tile grown by two pixels gives a range of
// rho indices (intersected with the ray's range inside D), which is then trimmed at both
// ends to exactly the samples whose 4 x 4 bicubic footprint meets the tile (the footprint
// origin floor(X) moves monotonically along a ray, so those samples are contiguous).  The
// ranges are cut into segments of one length (and a shorter last one per ray), long enough
// that every thread walks at most one, and numbered by a scan with the rays taken kRayGap
// apart (rays t, t + kRayGap, ... first), full segments before the shorter ones, so that
// the threads of a wave, which walk consecutive segments in lockstep, mostly have equal
// work and sit on rays kRayGap apart or a segment length apart on one ray: their footprints
// are then mostly disjoint and each LDS add of a wave spreads over the banks.  Each sample is rebuilt from the coarse rows by the transposed
// decimation filter; its 16 weighted values are summed in registers into the walking
// thread's 4 x 4 footprint.  Along a ray the footprint origin floor(X), floor(Y) advances by
// at most one pixel per sample for the usual geometries, so the footprint is kept oriented
// along the ray's direction and, when it advances, only its trailing column or row is added
// to the LDS tile (any other move adds all of it).  The FP64 LDS tile has a halo of kAHalo
// pixels that holds every footprint, so the adds need no bounds tests.
constexpr int kAThreads = 512;  // threads of the adjoint splat
constexpr int kARows = 128;     // rays listed per pass
constexpr int kSegMin = 8;      // shortest segment (rho indices)
constexpr int kRayGap = 2;      // rays of one lane group are kRayGap apart (2, 4, 8, 16 timed: 2 fastest)
constexpr int kASlots = kARows + kRayGap;  // ray slots per pass (groups padded to equal size)
constexpr int kAHalo = 4;       // halo of the LDS tile: footprints reach 3 pixels before and 2 after,
                                // one more on each side covers the range's rounding
constexpr int kAW = kTile + 2 * kAHalo;  // LDS tile side
constexpr int kAP = kAW + 1;             // LDS tile pitch (odd)
constexpr int kUCap = 4096;     // floats of the LDS copy of the coarse rows a pass reads
constexpr int kECap = 256;      // rho indices of the LDS copy of e^rho
// The tile side, the two caps and the block's register budget (waves_per_eu below) are sized
// together: 51.8 KB of LDS and at most 80 VGPRs let three 512-thread blocks share a CU (six
// waves per SIMD; measured, 53 192 bytes of LDS per block still ran three per CU, 53 384 did
// not).  64 x 64 tiles (74 KB) ran two blocks per CU, 25% slower.
constexpr int kSplatLds = 8 * kAW * kAP + 4 * (5 * kASlots + 1) + 2 * 16 * kASlots + 4 * kUCap + 8 * kECap +
                          2 * kAThreads;  // the splat's __shared__ arrays, in bytes
static_assert(kSplatLds + 256 <= 53248, "the splat's LDS must leave room for three blocks per CU");

// In-place exclusive scan of buf[0..nitems), nitems <= 3 * 64, by the first wave alone (no
// block barriers inside); returns the total to that wave.  Callers synchronise around it.
__device__ __forceinline__ int wave_exclusive_scan(int* buf, int nitems) {
  const int lane = threadIdx.x & 63;
  int v[3], s = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int k = 3 * lane + i;
    v[i] = k < nitems ? buf[k] : 0;
    s += v[i];
  }
  int incl = s;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  int run = incl - s;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int k = 3 * lane + i;
    if (k < nitems) buf[k] = run;
    run += v[i];
  }
  return __shfl(incl, 63, 64);
}

// Everything one thread needs to walk one segment of a ray.
struct SegWalk {
  double X0, Y0;       // x* in image-index coordinates
  double cx, cy;       // ray direction
  int qbeg, qend;      // rho indices of the segment (inclusive)
  int ux0, ux1, uy0, uy1;  // tile [ux0, ux1) x [uy0, uy1) in unwrapped index coordinates
  float dw[4];         // decimation weights of the coarse rows (0 for rows outside the support)
  int roff[4];         // offsets of those rows in the row store read
};

// Walk one segment: rebuild every sample from the coarse rows, sum its bicubic weights into
// the register footprint, and add to the LDS tile what the footprint leaves behind.  Rows
// and e^rho come from their LDS copies, indexed from rho index qlo.
__device__ __forceinline__ void splat_walk(const SegWalk& sw, double* acc, const float* rows, const double* erho,
                                           int qlo) {
  // footprint in the ray's orientation: w[j][i] is the pixel i columns and j rows from the
  // trailing corner (x = kx - 1 + i or kx + 2 - i as the ray runs towards +x or -x; likewise
  // for y), so it always advances by dropping w[.][0] or w[0][.]; weights in that order are
  // the cubic B-spline weights at the fraction measured from the other side (the weights are
  // symmetric: w_k(a) = w_{3-k}(1 - a))
  const bool xp = sw.cx >= 0.0, yp = sw.cy >= 0.0;
  const int cstep = xp ? 1 : -1, rstep = yp ? kAP : -kAP;
  auto corner = [&](int kx, int ky) {
    const int x = xp ? kx - 1 : kx + 2, y = yp ? ky - 1 : ky + 2;
    return (y - sw.uy0 + kAHalo) * kAP + (x - sw.ux0 + kAHalo);
  };
  float w[4][4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) w[j][i] = 0.f;
  int ckx = 0, cky = 0;
  for (int q = sw.qbeg; q <= sw.qend; ++q) {
    const int qi = q - qlo;
    const double E = erho[qi];
    // (dw carries the weights' 1/36)
    const float V = sw.dw[0] * rows[sw.roff[0] + qi] + sw.dw[1] * rows[sw.roff[1] + qi] +
                    sw.dw[2] * rows[sw.roff[2] + qi] + sw.dw[3] * rows[sw.roff[3] + qi];
    const double X = sw.X0 + E * sw.cx, Y = sw.Y0 + E * sw.cy;
    const double fx = floor(X), fy = floor(Y);
    // the trimmed range keeps kx in [ux0 - 2, ux1] and ky in [uy0 - 2, uy1], give or take the
    // trim's rounding (one pixel, with zero weight on the tile); the clamp only keeps the adds
    // inside the halo should that ever fail
    const int kx = min(max((int)fx, sw.ux0 - 3), sw.ux1 + 1), ky = min(max((int)fy, sw.uy0 - 3), sw.uy1 + 1);
    if (q == sw.qbeg) {
      ckx = kx;
      cky = ky;
    } else {
      const int dx = xp ? kx - ckx : ckx - kx, dy = yp ? ky - cky : cky - ky;
      if ((unsigned)dx > 1u || (unsigned)dy > 1u) {
        const int o = corner(ckx, cky);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            atomicAdd(acc + o + j * rstep + i * cstep, (double)w[j][i]);
            w[j][i] = 0.f;
          }
        ckx = kx;
        cky = ky;
      } else {
        if (dx) {
          const int o = corner(ckx, cky);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            atomicAdd(acc + o + j * rstep, (double)w[j][0]);
            w[j][0] = w[j][1];
            w[j][1] = w[j][2];
            w[j][2] = w[j][3];
            w[j][3] = 0.f;
          }
          ckx = kx;
        }
        if (dy) {
          const int o = corner(ckx, cky);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            atomicAdd(acc + o + i * cstep, (double)w[0][i]);
            w[0][i] = w[1][i];
            w[1][i] = w[2][i];
            w[2][i] = w[3][i];
            w[3][i] = 0.f;
          }
          cky = ky;
        }
      }
    }
    const float ax = (float)(X - fx), ay = (float)(Y - fy);
    float wx[4], wy[4];
    bspline_w6(xp ? ax : 1.0f - ax, wx);
    bspline_w6(yp ? ay : 1.0f - ay, wy);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float vy = V * wy[j];
#pragma unroll
      for (int i = 0; i < 4; ++i) w[j][i] += vy * wx[i];
    }
  }
  if (sw.qend >= sw.qbeg) {
    const int o = corner(ckx, cky);
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) atomicAdd(acc + o + j * rstep + i * cstep, (double)w[j][i]);
  }
}

// The same walk with the footprint moves made uniform across a wave.  Coordinates are mirrored
// so that every ray runs towards +x and +y (X' = sx X, Y' = sy Y with sx, sy the signs of the
// ray direction; B is even, so the mirrored taps carry the same weights): the footprint then
// only ever drops its column i = 0 or its row j = 0.  Each step every lane shifts its
// registers by selects (a move of 0 keeps them), and only the flush of the dropped column or
// row (four FP64 LDS atomics) sits under a branch, so the registers need no copies at the
// branches' joins.  The coarse rows come from the interleaved copy: the four rows of the ray
// at rho index q are consecutive.
struct SegWalk2 {
  double X0, Y0;           // x* in mirrored image-index coordinates (sx X0, sy Y0)
  double cx, cy;           // |ray direction|
  int qbeg, qend;          // rho indices of the segment (inclusive)
  int lox, hix, loy, hiy;  // range of the footprint origin (mirrored), as in splat_walk
  int cstep, rstep;        // LDS index steps of one mirrored column (sx) and row (sy kAP)
  int obase;               // LDS index of mirrored pixel (c, r) is obase + sx c + sy kAP r
  float dw[4];             // decimation weights (with the bicubic weights' 1/36)
  int rrow;                // offset of the ray's first coarse row in an interleaved rho step
};

// One row of the register footprint (named members, so that the moves below stay selects on
// registers and never become indexed loads from a private array).
struct Row4 {
  float c0, c1, c2, c3;
};

// b where lane mask m has this lane's bit, else a: one v_cndmask_b32.  Written as an
// instruction so that the compiler keeps it a select instead of merging it into the branch
// on the same condition (which brings back register copies at the branch's join).
__device__ __forceinline__ float lane_select(float a, float b, unsigned long long m) {
  float r;
  asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(m));
  return r;
}

__device__ __forceinline__ void splat_walk_bf(const SegWalk2& sw, double* acc, const float* rows, int rstride,
                                              const double* erho, int qlo) {
  if (sw.qend < sw.qbeg) return;
  const int cs = sw.cstep, rs = sw.rstep;
  Row4 r0 = {0.f, 0.f, 0.f, 0.f}, r1 = r0, r2 = r0, r3 = r0;
  int ckx, cky;
  {
    const double E = erho[sw.qbeg - qlo];
    const double X = sw.X0 + E * sw.cx, Y = sw.Y0 + E * sw.cy;
    ckx = min(max((int)floor(X), sw.lox), sw.hix);
    cky = min(max((int)floor(Y), sw.loy), sw.hiy);
  }
  const float* rp = rows + (sw.qbeg - qlo) * rstride + sw.rrow;
  for (int q = sw.qbeg; q <= sw.qend; ++q, rp += rstride) {
    const double E = erho[q - qlo];
    const float V = sw.dw[0] * rp[0] + sw.dw[1] * rp[1] + sw.dw[2] * rp[2] + sw.dw[3] * rp[3];
    const double X = sw.X0 + E * sw.cx, Y = sw.Y0 + E * sw.cy;
    const double fx = floor(X), fy = floor(Y);
    const int kx = min(max((int)fx, sw.lox), sw.hix);
    const int ky = min(max((int)fy, sw.loy), sw.hiy);
    // a step moves the origin by at most one pixel per axis forward (samples are less than a
    // pixel apart along a ray); anything else (only the clamp could cause it) flushes all
    if (((unsigned)(kx - ckx) | (unsigned)(ky - cky)) > 1u) {
      const int o = sw.obase + cs * (ckx - 1) + rs * (cky - 1);
      const Row4* rr[4] = {&r0, &r1, &r2, &r3};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        atomicAdd(acc + o + j * rs, (double)rr[j]->c0);
        atomicAdd(acc + o + j * rs + cs, (double)rr[j]->c1);
        atomicAdd(acc + o + j * rs + 2 * cs, (double)rr[j]->c2);
        atomicAdd(acc + o + j * rs + 3 * cs, (double)rr[j]->c3);
      }
      r0 = Row4{0.f, 0.f, 0.f, 0.f};
      r1 = r0;
      r2 = r0;
      r3 = r0;
      ckx = kx;
      cky = ky;
    }
    const bool mx = kx != ckx, my = ky != cky;
    if (mx) {  // drop column 0
      const int o = sw.obase + cs * (ckx - 1) + rs * (cky - 1);
      atomicAdd(acc + o, (double)r0.c0);
      atomicAdd(acc + o + rs, (double)r1.c0);
      atomicAdd(acc + o + 2 * rs, (double)r2.c0);
      atomicAdd(acc + o + 3 * rs, (double)r3.c0);
    }
    const unsigned long long bx = __builtin_amdgcn_ballot_w64(mx), by = __builtin_amdgcn_ballot_w64(my);
    const float zero = 0.f;
#define RL_SHIFT_X(r)                   \
  r.c0 = lane_select(r.c0, r.c1, bx);   \
  r.c1 = lane_select(r.c1, r.c2, bx);   \
  r.c2 = lane_select(r.c2, r.c3, bx);   \
  r.c3 = lane_select(r.c3, zero, bx);
    RL_SHIFT_X(r0)
    RL_SHIFT_X(r1)
    RL_SHIFT_X(r2)
    RL_SHIFT_X(r3)
#undef RL_SHIFT_X
    if (my) {  // drop row 0
      const int o = sw.obase + cs * (kx - 1) + rs * (cky - 1);
      atomicAdd(acc + o, (double)r0.c0);
      atomicAdd(acc + o + cs, (double)r0.c1);
      atomicAdd(acc + o + 2 * cs, (double)r0.c2);
      atomicAdd(acc + o + 3 * cs, (double)r0.c3);
    }
#define RL_SHIFT_Y(c)                   \
  r0.c = lane_select(r0.c, r1.c, by);   \
  r1.c = lane_select(r1.c, r2.c, by);   \
  r2.c = lane_select(r2.c, r3.c, by);   \
  r3.c = lane_select(r3.c, zero, by);
    RL_SHIFT_Y(c0)
    RL_SHIFT_Y(c1)
    RL_SHIFT_Y(c2)
    RL_SHIFT_Y(c3)
#undef RL_SHIFT_Y
    ckx = kx;
    cky = ky;
    float wx[4], wy[4];
    bspline_w6((float)(X - fx), wx);
    bspline_w6((float)(Y - fy), wy);
#define RL_ACC(r, j)                         \
  {                                          \
    const float vy = V * wy[j];              \
    r.c0 = fmaf(vy, wx[0], r.c0);            \
    r.c1 = fmaf(vy, wx[1], r.c1);            \
    r.c2 = fmaf(vy, wx[2], r.c2);            \
    r.c3 = fmaf(vy, wx[3], r.c3);            \
  }
    RL_ACC(r0, 0)
    RL_ACC(r1, 1)
    RL_ACC(r2, 2)
    RL_ACC(r3, 3)
#undef RL_ACC
  }
  const int o = sw.obase + cs * (ckx - 1) + rs * (cky - 1);
  const Row4 rr[4] = {r0, r1, r2, r3};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    atomicAdd(acc + o + j * rs, (double)rr[j].c0);
    atomicAdd(acc + o + j * rs + cs, (double)rr[j].c1);
    atomicAdd(acc + o + j * rs + 2 * cs, (double)rr[j].c2);
    atomicAdd(acc + o + j * rs + 3 * cs, (double)rr[j].c3);
  }
}

// The walk above for a wave whose lanes all run their rays in one quadrant: with the mirror
// signs SX, SY known at compile time, the LDS element of the footprint's trailing corner is
// kept as a running index (advanced by SX or SY kAP when the footprint moves), and every add
// of a dropped column or row, or of the whole footprint, is one DS instruction at an immediate
// offset from a single address (the lowest of the group; `pin` keeps the compiler from
// folding that address back into a base with negative offsets).  Same terms, same FP64
// additions as splat_walk_bf.
__device__ __forceinline__ int pin(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// p[i0], p[i0 + S], p[i0 + 2 S], p[i0 + 3 S] += a, b, c, d (S of either sign)
template <int S>
__device__ __forceinline__ void add_line(double* acc, int i0, float a, float b, float c, float d) {
  constexpr int lo = S < 0 ? 3 * S : 0;  // offset of the lowest element from i0
  const int base = pin(i0 + lo);
  atomicAdd(acc + base + (0 - lo), (double)a);
  atomicAdd(acc + base + (S - lo), (double)b);
  atomicAdd(acc + base + (2 * S - lo), (double)c);
  atomicAdd(acc + base + (3 * S - lo), (double)d);
}

// the whole footprint: element i0 + j RS + i CS gets row j, column i
template <int CS, int RS>
__device__ __forceinline__ void add_block(double* acc, int i0, const Row4& r0, const Row4& r1, const Row4& r2,
                                          const Row4& r3) {
  constexpr int lo = (CS < 0 ? 3 * CS : 0) + (RS < 0 ? 3 * RS : 0);
  const int base = pin(i0 + lo);
  const Row4* rr[4] = {&r0, &r1, &r2, &r3};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    atomicAdd(acc + base + (j * RS - lo), (double)rr[j]->c0);
    atomicAdd(acc + base + (j * RS + CS - lo), (double)rr[j]->c1);
    atomicAdd(acc + base + (j * RS + 2 * CS - lo), (double)rr[j]->c2);
    atomicAdd(acc + base + (j * RS + 3 * CS - lo), (double)rr[j]->c3);
  }
}

template <int SX, int SY>
__device__ __forceinline__ void splat_walk_fixed(const SegWalk2& sw, double* acc, const float* rows, int rstride,
                                                 const double* erho, int qlo, double eratio) {
  if (sw.qend < sw.qbeg) return;
  constexpr int CS = SX, RS = SY * kAP;
  Row4 r0 = {0.f, 0.f, 0.f, 0.f}, r1 = r0, r2 = r0, r3 = r0;
  int ckx, cky;
  {
    const double E = erho[sw.qbeg - qlo];
    const double X = sw.X0 + E * sw.cx, Y = sw.Y0 + E * sw.cy;
    ckx = min(max((int)floor(X), sw.lox), sw.hix);
    cky = min(max((int)floor(Y), sw.loy), sw.hiy);
  }
  int ci = sw.obase + CS * (ckx - 1) + RS * (cky - 1);  // element of the trailing corner
  const float* rp = rows + (sw.qbeg - qlo) * rstride + sw.rrow;
  // e^rho of the next step by one product (eratio = e^{Delta rho}) instead of an LDS read:
  // a read issued after the previous step's adds would wait for them (LDS operations of a
  // wave complete in order); over a segment the product drifts by ~1e-14 relative
  double Er = erho[sw.qbeg - qlo];
  for (int q = sw.qbeg; q <= sw.qend; ++q, rp += rstride) {
    const double E = Er;
    Er *= eratio;
    const float V = sw.dw[0] * rp[0] + sw.dw[1] * rp[1] + sw.dw[2] * rp[2] + sw.dw[3] * rp[3];
    const double X = sw.X0 + E * sw.cx, Y = sw.Y0 + E * sw.cy;
    const double fx = floor(X), fy = floor(Y);
    const int kx = min(max((int)fx, sw.lox), sw.hix);
    const int ky = min(max((int)fy, sw.loy), sw.hiy);
    if (((unsigned)(kx - ckx) | (unsigned)(ky - cky)) > 1u) {  // (see splat_walk_bf)
      add_block<CS, RS>(acc, ci, r0, r1, r2, r3);
      r0 = Row4{0.f, 0.f, 0.f, 0.f};
      r1 = r0;
      r2 = r0;
      r3 = r0;
      ckx = kx;
      cky = ky;
      ci = sw.obase + CS * (kx - 1) + RS * (ky - 1);
    }
    const bool mx = kx != ckx, my = ky != cky;
    if (mx) add_line<RS>(acc, ci, r0.c0, r1.c0, r2.c0, r3.c0);  // drop column 0
    const unsigned long long bx = __builtin_amdgcn_ballot_w64(mx), by = __builtin_amdgcn_ballot_w64(my);
    const float zero = 0.f;
#define RL_SHIFT_X(r)                   \
  r.c0 = lane_select(r.c0, r.c1, bx);   \
  r.c1 = lane_select(r.c1, r.c2, bx);   \
  r.c2 = lane_select(r.c2, r.c3, bx);   \
  r.c3 = lane_select(r.c3, zero, bx);
    RL_SHIFT_X(r0)
    RL_SHIFT_X(r1)
    RL_SHIFT_X(r2)
    RL_SHIFT_X(r3)
#undef RL_SHIFT_X
    ci += mx ? CS : 0;
    if (my) add_line<CS>(acc, ci, r0.c0, r0.c1, r0.c2, r0.c3);  // drop row 0
#define RL_SHIFT_Y(c)                   \
  r0.c = lane_select(r0.c, r1.c, by);   \
  r1.c = lane_select(r1.c, r2.c, by);   \
  r2.c = lane_select(r2.c, r3.c, by);   \
  r3.c = lane_select(r3.c, zero, by);
    RL_SHIFT_Y(c0)
    RL_SHIFT_Y(c1)
    RL_SHIFT_Y(c2)
    RL_SHIFT_Y(c3)
#undef RL_SHIFT_Y
    ci += my ? RS : 0;
    ckx = kx;
    cky = ky;
    float wx[4], wy[4];
    bspline_w6((float)(X - fx), wx);
    bspline_w6((float)(Y - fy), wy);
#define RL_ACC(r, j)                         \
  {                                          \
    const float vy = V * wy[j];              \
    r.c0 = fmaf(vy, wx[0], r.c0);            \
    r.c1 = fmaf(vy, wx[1], r.c1);            \
    r.c2 = fmaf(vy, wx[2], r.c2);            \
    r.c3 = fmaf(vy, wx[3], r.c3);            \
  }
    RL_ACC(r0, 0)
    RL_ACC(r1, 1)
    RL_ACC(r2, 2)
    RL_ACC(r3, 3)
#undef RL_ACC
  }
  add_block<CS, RS>(acc, ci, r0, r1, r2, r3);
}

// ---- splat passes, built once per plan
// A pass is one partition m, one periodic shift (sx, sy) of one tile and up to kARows fine
// rays ta .. ta + nrows - 1, laid out in ray slots (slot of ray k: (k % kRayGap) * ng +
// k / kRayGap, ng = ceil(nrows / kRayGap); slots past the last ray are empty).  Header, three
// int4: (m, sx, sy, nslot), (cg0, cg1, qlo, qhi), (seglen, segments, first slot record, full
// segments); one int4 per slot: (t, first rho index, last rho index, first full segment |
// rank of its shorter segment << 16), the shorter segments numbered by decreasing length
// after all full ones (kNoShort: the ray's range is a whole number of full ones).  The kernel below
// computes them (one block per tile): COUNT only counts passes and slots per tile, WRITE
// stores them at the offsets the host derives from the counts.
constexpr int kBThreads = 256;  // threads of the pass builder (>= kASlots)
constexpr int kNoShort = 0x7fff;  // slot record: the slot has no shorter segment

template <bool WRITE>
__global__ __launch_bounds__(kBThreads) void k_adj_build(DevPlan P, int2* __restrict__ counts,
                                                         const int2* __restrict__ offs, int4* __restrict__ passes,
                                                         int4* __restrict__ rays) {
  __shared__ int rq0[kASlots];
  __shared__ int rqb[kASlots];
  __shared__ int rpre[kASlots + 1];
  __shared__ int rpart[kASlots + 1];
  __shared__ int rplen[kASlots];  // length of each slot's shorter segment (0: none)
  __shared__ int qext[4];
  const int n = P.n, r = P.r;
  const int tile = blockIdx.y * gridDim.x + blockIdx.x;
  const int tx0 = blockIdx.x * kTile, ty0 = blockIdx.y * kTile;
  const int txe = min(tx0 + kTile, n), tye = min(ty0 + kTile, n);
  int npass = 0, nrec = 0;
  const int pass0 = WRITE ? offs[tile].x : 0, rec0 = WRITE ? offs[tile].y : 0;
  for (int m = 0; m < P.m; ++m) {
    const double cb = cos(m * P.beta), sb = sin(m * P.beta);
    const double2* cs = P.fine_cs + (size_t)m * P.n_fine;
    const int2* fq = P.fine_q + (size_t)m * P.n_fine;
    const double X0 = P.X0[m], Y0 = P.Y0[m];
    for (int sy = -1; sy <= 1; ++sy) {
      for (int sx = -1; sx <= 1; ++sx) {
        const int ux0 = tx0 + sx * n, ux1 = txe + sx * n;
        const int uy0 = ty0 + sy * n, uy1 = tye + sy * n;
        // samples whose taps reach the tile have X in [ux0 - 2, ux1 + 1); inside D, X in (0, n)
        const int Xa = max(ux0 - 2, 0), Xb = min(ux1 + 1, n);
        const int Ya = max(uy0 - 2, 0), Yb = min(uy1 + 1, n);
        if (Xa >= Xb || Ya >= Yb) continue;  // uniform across the block
        {
          const double x1a = -1.0 + Xa * P.dx, x1b = -1.0 + Xb * P.dx;
          const double x2a = -1.0 + Ya * P.dx, x2b = -1.0 + Yb * P.dx;
          const double ex = fmax(fmax(x1a, -x1b), 0.0), ey = fmax(fmax(x2a, -x2b), 0.0);
          if (ex * ex + ey * ey >= 1.0) continue;  // rectangle misses the unit disc
        }
        // angular extent of the rectangle seen from x* (which lies outside it), padded by a ray
        double phmin = 1e30, phmax = -1e30;
        for (int c = 0; c < 4; ++c) {
          const double dX = ((c & 1) ? Xb : Xa) - X0, dY = ((c & 2) ? Yb : Ya) - Y0;
          const double ph = atan2(-sb * dX + cb * dY, cb * dX + sb * dY);
          phmin = fmin(phmin, ph);
          phmax = fmax(phmax, ph);
        }
        const double fstep = P.dtheta_c / r;
        const int ta = max(P.t_min, (int)floor((phmin - P.phi0[m]) / fstep) - 1);
        const int tb = min(P.t_min + P.n_fine - 1, (int)ceil((phmax - P.phi0[m]) / fstep) + 1);
        for (int tc = ta; tc <= tb; tc += kARows) {
          const int nrows = min(kARows, tb - tc + 1);
          const int ng = (nrows + kRayGap - 1) / kRayGap;  // slots per group
          const int nslot = ng * kRayGap;
          if (threadIdx.x == 0) {
            qext[0] = 0x7fffffff;
            qext[1] = -0x7fffffff;
          }
          __syncthreads();
          // rho range of each ray inside the grown tile (slab test) and inside D
          for (int sl = threadIdx.x; sl < nslot; sl += blockDim.x) {
            const int k = (sl % ng) * kRayGap + sl / ng;  // ray of slot sl
            int qa = 0, qb = -1;
            if (k < nrows) {
              const int ti = tc + k - P.t_min;
              const int2 qr = fq[ti];
              const double2 tcs = cs[ti];
              if (qr.x <= qr.y) {
                double elo = 0.0, ehi = 1e300;
                bool ok = true;
                if (fabs(tcs.x) > 1e-15) {
                  const double e1 = (Xa - X0) / tcs.x, e2 = (Xb - X0) / tcs.x;
                  elo = fmax(elo, fmin(e1, e2));
                  ehi = fmin(ehi, fmax(e1, e2));
                } else {
                  ok = ok && X0 >= Xa && X0 <= Xb;
                }
                if (fabs(tcs.y) > 1e-15) {
                  const double e1 = (Ya - Y0) / tcs.y, e2 = (Yb - Y0) / tcs.y;
                  elo = fmax(elo, fmin(e1, e2));
                  ehi = fmin(ehi, fmax(e1, e2));
                } else {
                  ok = ok && Y0 >= Ya && Y0 <= Yb;
                }
                // samples whose footprint meets the tile: floor(X) in [ux0 - 2, ux1] and floor(Y)
                // in [uy0 - 2, uy1], i.e. the point inside the grown tile [Xa, Xb] x [Ya, Yb]
                // (within D, X and Y lie in (0, n), so the clip to [0, n] changes nothing):
                // E in [elo, ehi], rho indices from ceil(tau(elo)) to floor(tau(ehi)).  Rounding
                // can only misplace a sample within ~1e-9 pixel of a footprint edge, where its
                // weight on the tile is zero; the tile's halo holds such a footprint
                if (ok && elo <= ehi && ehi > 0.0) {
                  const double scale = P.a_R * P.dx;
                  const double tlo = log(fmax(elo * scale, 1e-300)) / P.d_rho + P.n_rho - 1;
                  const double thi = log(ehi * scale) / P.d_rho + P.n_rho - 1;
                  qa = (int)fmax(ceil(tlo), (double)qr.x);
                  qb = (int)fmin(floor(thi), (double)qr.y);
                }
              }
            }
            const int cnt = max(qb - qa + 1, 0);
            if (cnt > 0) {
              atomicMin(&qext[0], qa);
              atomicMax(&qext[1], qb);
            }
            rq0[sl] = qa;
            rqb[sl] = qb;
            rpre[sl] = cnt;
          }
          __syncthreads();
          // segment length: long enough that every thread of the splat walks at most one
          // segment (sum over rays of ceil(cnt / len) <= samples / len + rays <= kAThreads)
          if (threadIdx.x < 64) {
            int ssum = 0, nray = 0;
            for (int i = threadIdx.x; i < nslot; i += 64) {
              ssum += rpre[i];
              nray += rpre[i] > 0;
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
              ssum += __shfl_xor(ssum, off, 64);
              nray += __shfl_xor(nray, off, 64);
            }
            const int len = max(kSegMin, (ssum + (kAThreads - nray) - 1) / (kAThreads - nray));
            // a ray's range is cut into full segments of len samples and at most one shorter
            // one; the full segments of all rays are numbered first, so that the waves that
            // walk them have no idle lanes, then the shorter ones by decreasing length, so that
            // each wave of them walks segments of similar lengths
            for (int i = threadIdx.x; i < nslot; i += 64) {
              const int c = rpre[i];
              rpre[i] = c / len;
              rpart[i] = (c % len) != 0;
              rplen[i] = c % len;
            }
            const int nfull = wave_exclusive_scan(rpre, nslot);
            const int npart = wave_exclusive_scan(rpart, nslot);
            if (threadIdx.x == 0) {
              rpre[nslot] = nfull;
              rpart[nslot] = npart;
              qext[2] = len;
              qext[3] = nfull;
            }
          }
          __syncthreads();
          const int total = rpre[nslot] + rpart[nslot];
          if (total > 0) {  // uniform
            if (WRITE) {
              // rank of each shorter segment: longer ones first, equal lengths in slot order
              // (kNoShort: the slot has none); rpart is free again after the totals above
              for (int sl = threadIdx.x; sl < nslot; sl += blockDim.x) {
                const int pl = rplen[sl];
                int rank = kNoShort;
                if (pl > 0) {
                  rank = 0;
                  for (int j = 0; j < nslot; ++j) {
                    const int pj = rplen[j];
                    rank += pj > pl || (pj == pl && j < sl);
                  }
                }
                rpart[sl] = rank;
              }
              __syncthreads();
              const int cg0 = max(floordiv(tc, r) - 1, 0);
              const int cg1 = min(floordiv(tc + nrows - 1, r) + 2, P.n_sup - 1);
              if (threadIdx.x == 0) {
                int4* h = passes + 3 * (size_t)(pass0 + npass);
                h[0] = make_int4(m, sx, sy, nslot);
                h[1] = make_int4(cg0, cg1, qext[0], qext[1]);
                h[2] = make_int4(qext[2], total, rec0 + nrec, qext[3]);
              }
              for (int sl = threadIdx.x; sl < nslot; sl += blockDim.x) {
                const int k = (sl % ng) * kRayGap + sl / ng;
                rays[rec0 + nrec + sl] =
                    make_int4(tc + min(k, nrows - 1), rq0[sl], rqb[sl], rpre[sl] | (rpart[sl] << 16));
              }
            }
            ++npass;
            nrec += nslot;
          }
          __syncthreads();
        }
      }
    }
  }
  if (!WRITE && threadIdx.x == 0) counts[tile] = make_int2(npass, nrec);
}

rl_status build_adj_passes(rl_plan* p) {
  DevPlan& d = p->d;
  const int nt = (d.n + kTile - 1) / kTile;
  const int tiles = nt * nt;
  int2* dcnt = nullptr;
  rl_status st;
  if ((st = check_hip(hipMalloc(&dcnt, sizeof(int2) * tiles), "hipMalloc(pass counts)")) != RL_OK) return st;
  hipLaunchKernelGGL(k_adj_build<false>, dim3(nt, nt), dim3(kBThreads), 0, 0, d, dcnt, nullptr, nullptr, nullptr);
  std::vector<int2> cnt(tiles);
  if ((st = check_launch("k_adj_build")) != RL_OK ||
      (st = check_hip(hipMemcpy(cnt.data(), dcnt, sizeof(int2) * tiles, hipMemcpyDeviceToHost), "copy pass counts")) !=
          RL_OK) {
    (void)hipFree(dcnt);
    return st;
  }
  // offsets: tile t's passes start at offs[t].x, its slot records at offs[t].y
  std::vector<int2> offs(tiles);
  std::vector<int> toff(tiles + 1);
  long long np = 0, nr = 0;
  for (int t = 0; t < tiles; ++t) {
    offs[t] = make_int2((int)np, (int)nr);
    toff[t] = (int)np;
    np += cnt[t].x;
    nr += cnt[t].y;
  }
  toff[tiles] = (int)np;
  if (np >= (1ll << 30) || nr >= (1ll << 30)) {
    (void)hipFree(dcnt);
    return fail(RL_ERR_GEOMETRY, "adjoint splat tables too large");
  }
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t o_off = 0, o_pass = al(sizeof(int) * (tiles + 1)), o_ray = o_pass + al(sizeof(int4) * 3 * (np + 1));
  const size_t bytes = o_ray + al(sizeof(int4) * (nr + 1)) + al(sizeof(int2) * tiles);
  const size_t o_offs = bytes - al(sizeof(int2) * tiles);
  char* mem = nullptr;
  if ((st = check_hip(hipMalloc(&mem, bytes), "hipMalloc(adjoint passes)")) != RL_OK) {
    (void)hipFree(dcnt);
    return st;
  }
  (void)hipFree(dcnt);
  if ((st = check_hip(hipMemcpy(mem + o_off, toff.data(), sizeof(int) * (tiles + 1), hipMemcpyHostToDevice),
                      "upload pass offsets")) != RL_OK ||
      (st = check_hip(hipMemcpy(mem + o_offs, offs.data(), sizeof(int2) * tiles, hipMemcpyHostToDevice),
                      "upload pass offsets")) != RL_OK) {
    (void)hipFree(mem);
    return st;
  }
  hipLaunchKernelGGL(k_adj_build<true>, dim3(nt, nt), dim3(kBThreads), 0, 0, d, nullptr, (const int2*)(mem + o_offs),
                     (int4*)(mem + o_pass), (int4*)(mem + o_ray));
  if ((st = check_launch("k_adj_build")) != RL_OK ||
      (st = check_hip(hipDeviceSynchronize(), "k_adj_build")) != RL_OK) {
    (void)hipFree(mem);
    return st;
  }
  d.adj_ntx = nt;
  d.adj_off = (const int*)(mem + o_off);
  d.adj_pass = (const int4*)(mem + o_pass);
  d.adj_ray = (const int4*)(mem + o_ray);
  p->d_adj = mem;
  p->d_adj_bytes = bytes;
  return RL_OK;
}

// ---- the splat
// Block: one kTile x kTile image tile of one slice.  For every pass of the tile (built at
// plan time, above), the pass's ray slots are read into LDS, the coarse rows cg - 1 .. cg + 2
// of its rays are copied to LDS with e^rho for one window of rho indices at a time (one
// window usually covers the pass), and every thread walks at most one segment.  The FP64
// tile (with its halo) collects all partitions and is written once.
template <bool BF>
__global__ __launch_bounds__(kAThreads) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_lp2cart_adj(
    DevPlan P, const float* __restrict__ U, float* __restrict__ cbar) {
  // FP64: LDS float atomics are slow on this target.
  __shared__ double acc[kAW * kAP];
  __shared__ int rq0[kASlots];
  __shared__ int rpre[kASlots + 1];   // first full segment of each slot
  __shared__ int rppre[kASlots];      // index of the slot's shorter segment among them
  __shared__ int rcnt[kASlots];
  __shared__ int rcg[kASlots];
  __shared__ float4 rdw[kASlots];
  __shared__ double2 rcs[kASlots];
  __shared__ __align__(16) float us[kUCap];  // coarse rows [cg0, cg0 + nur) x rho [wq4, wq4 + span)
  __shared__ double es[kECap];               // e^{rho_q} / (a_R dx) for q in [wq4, wq4 + span)
  // slot of each segment of the pass (a pass has at most kAThreads segments: the builder picks
  // the segment length so that every thread walks at most one)
  __shared__ short segslot[kAThreads];
  const int n = P.n, r = P.r;
  // (tile, slice) of this block: with at least one slice per XCD, each XCD takes one contiguous
  // run of them in slice, tile-row, tile order, so that neighbouring tiles, which copy
  // overlapping coarse rows, share its L2 (HBM fetch 5.1 -> 2.2 GB per launch of 64 slices at
  // 2048^2); with fewer slices, runs of one image's tiles would give the XCDs unequal work
  const int nbt = gridDim.x * gridDim.y;
  const int bid = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  const int lid = gridDim.z >= kXcds ? xcd_block(bid, nbt * gridDim.z) : bid;
  const int b = lid / nbt, tl = lid - b * nbt;
  const int tyi = tl / gridDim.x, txi = tl - tyi * gridDim.x;
  const int tx0 = txi * kTile, ty0 = tyi * kTile;
  const double eratio = exp(P.d_rho);  // ratio of consecutive e^rho
  const int tile = tyi * P.adj_ntx + txi;
  for (int i = threadIdx.x; i < kAW * kAP; i += blockDim.x) acc[i] = 0.0;
  const int txe = min(tx0 + kTile, n), tye = min(ty0 + kTile, n);
  const int pbeg = P.adj_off[tile], pend = P.adj_off[tile + 1];
  for (int pi = pbeg; pi < pend; ++pi) {
    const int4 h0 = P.adj_pass[3 * pi], h1 = P.adj_pass[3 * pi + 1], h2 = P.adj_pass[3 * pi + 2];
    const int m = h0.x, nslot = h0.w;
    const int ux0 = tx0 + h0.y * n, ux1 = txe + h0.y * n;
    const int uy0 = ty0 + h0.z * n, uy1 = tye + h0.z * n;
    const int cg0 = h1.x, cg1 = h1.y, qlo = h1.z, qhi = h1.w;
    const int seglen = h2.x, total = h2.y, nfull = h2.w;
    const int4* rec = P.adj_ray + h2.z;
    const double2* cs = P.fine_cs + (size_t)m * P.n_fine;
    const float* Ub = U + (size_t)(b * P.m + m) * P.n_sup * P.n_rho;
    const double X0 = P.X0[m], Y0 = P.Y0[m];
    __syncthreads();  // the previous pass's walk is done with the LDS slots
    for (int sl = threadIdx.x; sl < nslot; sl += blockDim.x) {
      const int4 e = rec[sl];
      const int cg = floordiv(e.x, r);
      rq0[sl] = e.y;
      rcnt[sl] = e.z;
      rpre[sl] = e.w & 0xffff;
      rppre[sl] = e.w >> 16;
      rcs[sl] = cs[e.x - P.t_min];
      rcg[sl] = cg;
      rdw[sl] = P.dec[e.x - r * cg];
    }
    if (threadIdx.x == 0) rpre[nslot] = nfull;
    __syncthreads();
    // segment -> slot: slot sl holds full segments rpre[sl] .. rpre[sl + 1] - 1 and, unless
    // rppre[sl] is kNoShort, the shorter segment nfull + rppre[sl]
    for (int sl = threadIdx.x; sl < nslot; sl += blockDim.x) {
      const int f1 = min(rpre[sl + 1], kAThreads);
      for (int j = rpre[sl]; j < f1; ++j) segslot[j] = (short)sl;
      if (rppre[sl] != kNoShort && nfull + rppre[sl] < kAThreads) segslot[nfull + rppre[sl]] = (short)sl;
    }
    // (the barrier before the first window's walk publishes segslot)
    // rho windows of the row copies; a window starts at a multiple of 4 and spans a multiple
    // of 4, so rows are copied as float4 (n_rho is a multiple of 4).  The branch-free walk
    // reads an interleaved copy [rho][row] of the rows rlo .. rhi, which covers every ray's rows
    // cg - 1 .. cg + 2 (the pass header clamps cg0, cg1 to the support; where it did, the copy
    // reaches three rows below 0 or four above the last lattice row), rows outside the
    // partition's support copied as zeros
    const int rlo = BF ? (cg0 == 0 ? -3 : cg0) : cg0;
    const int rhi = BF ? (cg1 == P.n_sup - 1 ? P.n_sup + 3 : cg1) : cg1;
    const int nur = rhi - rlo + 1;
    const int wlen = max(4, (min(kECap, kUCap / nur) - 4) & ~3);  // nur <= kARows / r + 11
    for (int wq = qlo; wq <= qhi; wq += wlen) {
      const int wq4 = wq & ~3;
      const int wend = min(wq + wlen - 1, qhi);  // last rho index walked in this window
      const int span = (wend - wq4 + 4) & ~3;    // copied: [wq4, wq4 + span)
      if (wq > qlo) __syncthreads();  // the previous window's walk is done with the copies
      if (BF) {
        // group i: rho group g = i / nur, row rr = i % nur (consecutive threads, consecutive rows)
        const int sg = span >> 2, tot = nur * sg;
        const int srows = P.sup_rows[m];
        for (int i = threadIdx.x; i < tot; i += kAThreads) {
          const int g = i / nur, rr = i - g * nur;
          const int row = rlo + rr;
          const float4 v = (row >= 0 && row < srows)
                               ? *reinterpret_cast<const float4*>(Ub + (size_t)row * P.n_rho + wq4 + 4 * g)
                               : make_float4(0.f, 0.f, 0.f, 0.f);
          float* d = us + 4 * g * nur + rr;
          d[0] = v.x;
          d[nur] = v.y;
          d[2 * nur] = v.z;
          d[3 * nur] = v.w;
        }
        if (threadIdx.x < span) es[threadIdx.x] = P.erho[wq4 + threadIdx.x];
      } else {
        constexpr int kIt = (kUCap / 4 + kAThreads - 1) / kAThreads;
        const int sg = span >> 2, tot = nur * sg;
        // group i = threadIdx.x + it * kAThreads is (row, g) = divmod(i, sg); both advance by
        // the block stride without a division per group
        const int drow = kAThreads / sg, dg = kAThreads - drow * sg;
        int row = (int)threadIdx.x / sg, g = (int)threadIdx.x - row * sg;
        float4 tmp[kIt];
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
          const int i = threadIdx.x + it * kAThreads;
          tmp[it] = i < tot ? *reinterpret_cast<const float4*>(Ub + (size_t)(cg0 + row) * P.n_rho + wq4 + 4 * g)
                            : make_float4(0.f, 0.f, 0.f, 0.f);
          row += drow;
          g += dg;
          if (g >= sg) {
            g -= sg;
            ++row;
          }
        }
        const double e = threadIdx.x < span ? P.erho[wq4 + threadIdx.x] : 0.0;
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
          const int i = threadIdx.x + it * kAThreads;
          if (i < tot) reinterpret_cast<float4*>(us)[i] = tmp[it];
        }
        if (threadIdx.x < span) es[threadIdx.x] = e;
      }
      __syncthreads();
      // walk whole segments (clipped to the window)
      for (int idx = threadIdx.x; idx < min(total, kAThreads); idx += blockDim.x) {
        // segments [0, nfull) are full ones, the rest the shorter last ones of their rays
        const bool full = idx < nfull;
        const int j = full ? idx : idx - nfull;
        const int k = segslot[idx];
        const int q0 = rq0[k] + (full ? j - rpre[k] : rpre[k + 1] - rpre[k]) * seglen;
        if (BF) {
          SegWalk2 sw;
          const double2 tcs = rcs[k];
          const bool xp = tcs.x >= 0.0, yp = tcs.y >= 0.0;
          sw.X0 = xp ? X0 : -X0;
          sw.Y0 = yp ? Y0 : -Y0;
          sw.cx = fabs(tcs.x);
          sw.cy = fabs(tcs.y);
          sw.qbeg = max(q0, wq);
          sw.qend = min(min(q0 + seglen - 1, rcnt[k]), wend);
          // footprint origins kx in [ux0 - 3, ux1 + 1] (columns kx - 1 .. kx + 2); mirrored,
          // the columns -kx' + 1 .. -kx' - 2 give kx' in [-ux1 - 2, -ux0 + 2]
          sw.lox = xp ? ux0 - 3 : -ux1 - 2;
          sw.hix = xp ? ux1 + 1 : -ux0 + 2;
          sw.loy = yp ? uy0 - 3 : -uy1 - 2;
          sw.hiy = yp ? uy1 + 1 : -uy0 + 2;
          sw.cstep = xp ? 1 : -1;
          sw.rstep = yp ? kAP : -kAP;
          sw.obase = (kAHalo - uy0) * kAP + (kAHalo - ux0);
          const float4 dw = rdw[k];
          sw.dw[0] = dw.x * (1.0f / 36.0f);
          sw.dw[1] = dw.y * (1.0f / 36.0f);
          sw.dw[2] = dw.z * (1.0f / 36.0f);
          sw.dw[3] = dw.w * (1.0f / 36.0f);
          sw.rrow = rcg[k] - 1 - rlo;
          // lanes that all run their rays in one quadrant take the walk with compile-time
          // mirror signs (wave-uniform branch); a wave with mixed quadrants the general one
          const unsigned long long act = __builtin_amdgcn_ballot_w64(true);
          const unsigned long long bxp = __builtin_amdgcn_ballot_w64(xp), byp = __builtin_amdgcn_ballot_w64(yp);
          if ((bxp == 0 || bxp == act) && (byp == 0 || byp == act)) {
            const bool wx = __builtin_amdgcn_readfirstlane((int)xp) != 0;
            const bool wy = __builtin_amdgcn_readfirstlane((int)yp) != 0;
            if (wx) {
              if (wy) splat_walk_fixed<1, 1>(sw, acc, us, nur, es, wq4, eratio);
              else splat_walk_fixed<1, -1>(sw, acc, us, nur, es, wq4, eratio);
            } else {
              if (wy) splat_walk_fixed<-1, 1>(sw, acc, us, nur, es, wq4, eratio);
              else splat_walk_fixed<-1, -1>(sw, acc, us, nur, es, wq4, eratio);
            }
          } else {
            splat_walk_bf(sw, acc, us, nur, es, wq4);
          }
          continue;
        }
        SegWalk sw;
        sw.X0 = X0;
        sw.Y0 = Y0;
        const double2 tcs = rcs[k];
        sw.cx = tcs.x;
        sw.cy = tcs.y;
        sw.qbeg = max(q0, wq);
        sw.qend = min(min(q0 + seglen - 1, rcnt[k]), wend);
        sw.ux0 = ux0;
        sw.ux1 = ux1;
        sw.uy0 = uy0;
        sw.uy1 = uy1;
        const int cg = rcg[k];
        const float4 dw = rdw[k];
        const float dwv[4] = {dw.x, dw.y, dw.z, dw.w};
        // coarse rows cg-1 .. cg+2 feed this ray; a row outside the support gets weight 0
        // and reads a copied row instead
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = cg - 1 + i;
          const bool ok = row >= 0 && row < P.sup_rows[m];
          sw.dw[i] = ok ? dwv[i] * (1.0f / 36.0f) : 0.f;
          sw.roff[i] = (min(max(row, cg0), cg1) - cg0) * span;
        }
        splat_walk(sw, acc, us, es, wq4);
      }
    }
  }
  __syncthreads();
  float* dst = cbar + (size_t)b * n * n;
  for (int i = threadIdx.x; i < kTile * kTile; i += blockDim.x) {
    const int ly = i / kTile, lx = i % kTile;
    if (ty0 + ly < n && tx0 + lx < n)
      dst[(size_t)(ty0 + ly) * n + tx0 + lx] = (float)acc[(ly + kAHalo) * kAP + lx + kAHalo];
  }
}

rl_status launch_lp2cart_adj(const rl_plan* p, const float* U, float* cbar, int batch, hipStream_t s) {
  const DevPlan& d = p->d;
  dim3 grid((d.n + kTile - 1) / kTile, (d.n + kTile - 1) / kTile, batch);
  if (p->tune.adj_walk)
    RL_LAUNCH("k_lp2cart_adj", k_lp2cart_adj<true>, grid, dim3(kAThreads), 0, s, d, U, cbar);
  else
    RL_LAUNCH("k_lp2cart_adj", k_lp2cart_adj<false>, grid, dim3(kAThreads), 0, s, d, U, cbar);
  return check_launch("k_lp2cart_adj");
}

// ------------------------------------------------------------------ FBP filter
// One sinogram row per block: zero-pad to lr, real FFT, multiply by the real multiplier of
// the filter (the Ram-Lak ramp, times the cosine or Shepp-Logan window), inverse real FFT,
// keep the first n_s samples.  The multiplier is applied pairwise (k, lr/2 - k) in place
// between the two packings.
__global__ __launch_bounds__(kThreads) void k_ramp(DevPlan P, const float* __restrict__ in, float* __restrict__ out,
                                                   int filter) {
  extern __shared__ float2 sh[];
  const int ncr = P.lr / 2, ns = P.n_s;
  const size_t row = blockIdx.x;
  float* xs = reinterpret_cast<float*>(sh);
  const float* src = in + row * ns;
  row_copy(
      P.lr, [&](int i) { return src[min(i, ns - 1)]; }, [&](int i, float v) { xs[i] = i < ns ? v : 0.f; });
  __syncthreads();
  fft_lds<kRowVals, false>(sh, ncr, 1, P.twp_ramp);
  const int step = P.tw_len / P.lr;
  const float* mult = P.ramp + (size_t)filter * (ncr + 1);
  for (int k = threadIdx.x; k <= ncr / 2; k += blockDim.x) {
    const int km = ncr - k;
    const float2 a = sh[k];
    const float2 bz = sh[k == 0 ? 0 : km];
    // forward packing -> X[k], X[km]
    auto post = [&](float2 za, float2 zb, int kk) {
      const float2 e = cscale(cadd(za, cconj(zb)), 0.5f);
      const float2 o = cscale(csub(za, cconj(zb)), 0.5f);
      const float2 w = P.tw[kk * step];
      const float2 t = cmul(w, o);
      return make_float2(e.x + t.y, e.y - t.x);
    };
    float2 Xk = post(a, bz, k);
    float2 Xm = post(bz, a, km);
    Xk = cscale(Xk, mult[k]);
    Xm = cscale(Xm, mult[km]);
    // inverse packing from (Y[k], Y[km])
    auto pre = [&](float2 ya, float2 yb, int kk) {
      const float2 bb = cconj(yb);
      const float2 e = cadd(ya, bb), dd = csub(ya, bb);
      float2 w = P.tw[kk * step];
      w.y = -w.y;
      const float2 oo = cmul(dd, w);
      return make_float2(e.x - oo.y, e.y + oo.x);
    };
    const float2 Zk = pre(Xk, Xm, k);
    if (k == 0) {
      sh[0] = Zk;
    } else {
      const float2 Zm = pre(Xm, Xk, km);
      sh[k] = Zk;
      sh[km] = Zm;
    }
  }
  __syncthreads();
  fft_lds<kRowVals, true>(sh, ncr, 1, P.twp_ramp);
  float* dst = out + row * ns;
  for (int i = threadIdx.x; i < ns; i += blockDim.x) dst[i] = xs[i];
}

rl_status launch_ramp(const rl_plan* p, const float* in, float* out, int batch, int filter, hipStream_t s) {
  const DevPlan& d = p->d;
  RL_LAUNCH("k_ramp", k_ramp, dim3(batch * d.n_theta), dim3(kThreads), (size_t)(d.lr / 2) * sizeof(float2), s, d, in,
            out, filter);
  return check_launch("k_ramp");
}

}  // namespace rl

using namespace rl;

namespace {

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

}  // namespace

namespace rl {

rl_status adj_checks(const rl_plan* plan, const void* in, const void* out, int batch, void* ws, size_t ws_bytes,
                     rl_op op) {
  if (!plan) return fail(RL_ERR_INVALID_ARG, "plan is NULL");
  if (batch < 0) return fail(RL_ERR_INVALID_ARG, "batch is negative");
  if (batch == 0) return RL_OK;
  if (!in || !out) return fail(RL_ERR_INVALID_ARG, "input or output pointer is NULL");
  const size_t ib = (size_t)batch * plan->d.n_theta * plan->d.n_s * sizeof(float);
  const size_t ob = (size_t)batch * plan->d.n * plan->d.n * sizeof(float);
  if (overlaps(in, ib, out, ob)) return fail(RL_ERR_INVALID_ARG, "input and output overlap");
  const size_t need = rl_workspace_bytes(plan, batch, op);
  if (!ws || ws_bytes < need)
    return fail(RL_ERR_WORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes, need " + std::to_string(need));
  if (((uintptr_t)ws) & 255) return fail(RL_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (overlaps(ws, need, in, ib) || overlaps(ws, need, out, ob))
    return fail(RL_ERR_INVALID_ARG, "workspace overlaps input or output");
  return check_plan_device(plan);
}


rl_status adjoint_chain(const rl_plan* plan, Slices<const float> sino, Slices<float> img, int batch, void* ws, rl_op op,
                        bool transpose, hipStream_t s) {
  const DevPlan& d = plan->d;
  const WsLayout L = workspace_layout(plan, batch, op);
  char* w = (char*)ws;
  float* cbar = (float*)(w + L.off[0]);
  float* U = (float*)(w + L.off[1]);
  float2* Bs = (float2*)(w + L.off[2]);
  float2* A = (float2*)(w + L.off[3]);
  rl_status st;
  if ((st = launch_splat_rfft(plan, sino, A, batch, s)) != RL_OK) return st;
  if ((st = launch_theta_conv(plan, A, d.n_own, kHalo, d.q, Bs, d.n_sup, 0, 1, true, batch, s)) != RL_OK) return st;
  if ((st = launch_irfft_scale(plan, Bs, U, batch, s)) != RL_OK) return st;
  if ((st = launch_lp2cart_adj(plan, U, cbar, batch, s)) != RL_OK) return st;
  const double scale = transpose ? 1.0 : (d.dtheta * d.ds) / (d.dx * d.dx);  // w_S / w_X for R#
  return launch_prefilter(plan, dense((const float*)cbar, (size_t)d.n * d.n), img, batch, (float)scale, s);
}

}  // namespace rl

extern "C" rl_status radon_adj(const rl_plan* plan, const float* d_sino, float* d_img, int32_t batch, void* d_ws,
                               size_t ws_bytes, hipStream_t stream) {
  rl_status st = adj_checks(plan, d_sino, d_img, batch, d_ws, ws_bytes, RL_OP_ADJ);
  if (st != RL_OK || batch == 0) return st;
  const DevPlan& d = plan->d;
  return adjoint_chain(plan, dense(d_sino, (size_t)d.n_theta * d.n_s), dense(d_img, (size_t)d.n * d.n), batch, d_ws,
                       RL_OP_ADJ, false, stream);
}

extern "C" rl_status radon_transpose(const rl_plan* plan, const float* d_sino, float* d_img, int32_t batch,
                                     void* d_ws, size_t ws_bytes, hipStream_t stream) {
  rl_status st = adj_checks(plan, d_sino, d_img, batch, d_ws, ws_bytes, RL_OP_ADJ);
  if (st != RL_OK || batch == 0) return st;
  const DevPlan& d = plan->d;
  return adjoint_chain(plan, dense(d_sino, (size_t)d.n_theta * d.n_s), dense(d_img, (size_t)d.n * d.n), batch, d_ws,
                       RL_OP_ADJ, true, stream);
}

extern "C" rl_status fbp(const rl_plan* plan, const float* d_sino, float* d_img, int32_t batch, rl_filter filter,
                         void* d_ws, size_t ws_bytes, hipStream_t stream) {
  if (filter != RL_FILTER_RAMLAK && filter != RL_FILTER_COSINE && filter != RL_FILTER_SHEPP_LOGAN)
    return fail(RL_ERR_INVALID_ARG, "unknown filter");
  rl_status st = adj_checks(plan, d_sino, d_img, batch, d_ws, ws_bytes, RL_OP_FBP);
  if (st != RL_OK || batch == 0) return st;
  const WsLayout L = workspace_layout(plan, batch, RL_OP_FBP);
  float* wg = (float*)((char*)d_ws + L.off[4]);
  if ((st = launch_ramp(plan, d_sino, wg, batch, (int)filter, stream)) != RL_OK) return st;
  const DevPlan& d = plan->d;
  return adjoint_chain(plan, dense((const float*)wg, (size_t)d.n_theta * d.n_s), dense(d_img, (size_t)d.n * d.n), batch,
                       d_ws, RL_OP_FBP, false, stream);
}
