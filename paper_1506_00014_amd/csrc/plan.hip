// Plan construction: geometry checks, partition/mask tables, the Fourier multiplier of the
// log-polar kernel (computed on the device in FP64), twiddles; error reporting; workspace.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fft_device.h"
#include "rl_internal.h"

namespace rl {

namespace {
thread_local std::string g_last_error;

int next_pow2(long x) {
  int p = 1;
  while (p < x) p *= 2;
  return p;
}
bool is_pow2(long x) { return x > 0 && (x & (x - 1)) == 0; }
// 2^a 3^b: the FFT lengths the Stockham and register FFTs handle
bool is_smooth23(long x) {
  if (x <= 0) return false;
  while (x % 3 == 0) x /= 3;
  return is_pow2(x);
}
// theta-FFT lengths with a four-step split K1 x K2 the theta pass is built for: K <= 32 with at
// most one factor 3, or 32 K2 with K2 in {2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64}
bool theta_length_ok(long k) {
  if (k < 8 || k > 2048 || !is_smooth23(k)) return false;
  if (k <= 32) return k % 9 != 0;
  if (k % 32 != 0) return false;
  const long k2 = k / 32;
  return k2 % 9 != 0 && k2 <= 64;
}
long lcm_l(long a, long b) {
  long x = a, y = b;
  while (y) {
    const long t = x % y;
    x = y;
    y = t;
  }
  return a / x * b;
}

void partition_constants(int m, double* a_R, double* a_r) {
  // sec. 2, eq. (aconst), beta = pi / M
  const double beta = M_PI / m;
  const double sh = std::sin(0.5 * beta), ch = std::cos(0.5 * beta);
  *a_R = sh / (1.0 + sh);
  *a_r = (ch - sh) / (1.0 + sh);
}

long rho_bound(int n, int m) {
  // sec. 3, eq. (vrho)
  double a_R, a_r;
  partition_constants(m, &a_R, &a_r);
  return (long)std::ceil(std::log(a_r) / std::log(1.0 - 2.0 * a_R / n));
}

long r_bound(int n, int n_theta, int m, int q) {
  // Delta theta_c / r <= 2 a_R / N (sec. 3, the angular step before eq. Lopolargrid_f), with
  // Delta theta_c = Delta theta / q the coarse lattice spacing
  double a_R, a_r;
  partition_constants(m, &a_R, &a_r);
  return (long)std::ceil((M_PI / ((double)n_theta * q)) / (2.0 * a_R / n) - 1e-12);
}

// Lattice rows spanned by n consecutive owned rows on a lattice q times finer than the sinogram.
int lattice_rows(int n, int q) { return n > 0 ? q * (n - 1) + 1 : 0; }

// Ownership of sinogram row j (eq. Radon_all_pb, rounding half up, exact in integers):
// partition, wrap flag, and nu with theta'_j = pi nu / (N_theta M).
void owner(int j, int n_theta, int m, int* part, bool* wrap, long* nu) {
  const long mm = (2L * j * m + n_theta) / (2L * n_theta);
  *nu = (long)j * m - mm * n_theta;
  *wrap = (mm == m);
  *part = *wrap ? 0 : (int)mm;
}

struct OwnedRow {
  int j;
  bool wrap;
  long nu;
};

std::vector<std::vector<OwnedRow>> partition_rows(int n_theta, int m) {
  std::vector<std::vector<OwnedRow>> rows(m);
  for (int j = 0; j < n_theta; ++j) {
    int p;
    bool w;
    long nu;
    owner(j, n_theta, m, &p, &w, &nu);
    rows[p].push_back({j, w, nu});
  }
  for (auto& r : rows)
    std::sort(r.begin(), r.end(), [](const OwnedRow& a, const OwnedRow& b) { return a.nu < b.nu; });
  return rows;
}

double bspline(double x) {
  // cubic cardinal B-spline, sec. 4 (the definition before eq. Bcoeff)
  const double a = std::fabs(x);
  if (a < 1.0) return (3.0 * a * a * a - 6.0 * a * a + 4.0) / 6.0;
  if (a < 2.0) return (2.0 - a) * (2.0 - a) * (2.0 - a) / 6.0;
  return 0.0;
}

// Taps of the theta low-pass of Algorithm 1 step 4 (the paper leaves it open), n = -(2r-1) ..
// 2r-1, sum 1: kind 0 the cubic B-spline d_n = B(n/r)/r; kind 1 the box of one coarse cell
// sampled by the trapezoid rule on the fine rows (1/r inside, 1/(2r) on the cell's two edges,
// which fall on fine rows when r is even).
double dec_tap(int kind, int n, int r) {
  if (std::abs(n) >= 2 * r) return 0.0;
  if (kind == 0) return bspline((double)n / r) / r;
  if (2 * std::abs(n) < r) return 1.0 / r;
  return 2 * std::abs(n) == r ? 0.5 / r : 0.0;
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton's method on the Legendre recurrence.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// zeta_hat(kt, kr) = sum_nodes amp_n exp(-2 pi i (kt u_n / P + kr lc_n / L)),
// amp = w / cos u, lc = log cos u (sec. 3 eq. exprcoef1 by composite Gauss-Legendre).
// Block: 16 x 16 outputs; nodes staged 64 at a time together with their phasors.
constexpr int kZT = 16;
constexpr int kZN = 64;

__global__ __launch_bounds__(256) void k_zeta_hat(double2* __restrict__ out, const double* __restrict__ u,
                                                  const double* __restrict__ amp,
                                                  const double* __restrict__ lc, int n_nodes, int nkt,
                                                  int nkr, double invP, double invL) {
  __shared__ double2 et[kZT][kZN];
  __shared__ double2 er[kZN][kZT + 1];
  const int tx = threadIdx.x % kZT, ty = threadIdx.x / kZT;
  const int kt0 = blockIdx.x * kZT, kr0 = blockIdx.y * kZT;
  double2 acc = make_double2(0.0, 0.0);
  for (int n0 = 0; n0 < n_nodes; n0 += kZN) {
    for (int idx = threadIdx.x; idx < kZT * kZN; idx += blockDim.x) {
      const int a = idx / kZN, n = idx % kZN;
      const int node = n0 + n;
      double s, c;
      // theta phasor, turns reduced before the sine to keep the argument small
      double turns = (double)(kt0 + a) * u[node] * invP;
      turns -= rint(turns);
      sincospi(-2.0 * turns, &s, &c);
      et[a][n] = make_double2(amp[node] * c, amp[node] * s);
      double turns2 = (double)(kr0 + a) * lc[node] * invL;
      turns2 -= rint(turns2);
      sincospi(-2.0 * turns2, &s, &c);
      er[n][a] = make_double2(c, s);
    }
    __syncthreads();
#pragma unroll 8
    for (int n = 0; n < kZN; ++n) {
      const double2 a = et[tx][n], b = er[n][ty];
      acc.x += a.x * b.x - a.y * b.y;
      acc.y += a.x * b.y + a.y * b.x;
    }
    __syncthreads();
  }
  const int kt = kt0 + tx, kr = kr0 + ty;
  if (kt < nkt && kr < nkr) out[(size_t)kt * nkr + kr] = acc;
}

rl_status validate(const rl_geom& g) {
  if (g.n < 8 || g.n > 8192 || (g.n & 1))
    return fail(RL_ERR_GEOMETRY, "n must be even and in [8, 8192]");
  if (g.m < 3 || g.m > kMaxPart) return fail(RL_ERR_GEOMETRY, "m must be in [3, 16]");
  if (g.n_theta < g.m || g.n_theta > 16384)
    return fail(RL_ERR_GEOMETRY, "n_theta must be in [m, 16384]");
  if (g.n_s < 2 || g.n_s > 4096) return fail(RL_ERR_GEOMETRY, "n_s must be in [2, 4096]");
  if (!is_smooth23(g.n_rho) || g.n_rho % 4 != 0 || g.n_rho < 16 || g.n_rho > 8192)
    return fail(RL_ERR_GEOMETRY, "n_rho must be 2^a 3^b, a multiple of 4, in [16, 8192]");
  if (g.n_rho < rho_bound(g.n, g.m))
    return fail(RL_ERR_GEOMETRY, "n_rho below the sampling bound ceil(log a_r / log(1 - 2 a_R / N))");
  int n_own = 0;
  {
    auto rows = partition_rows(g.n_theta, g.m);
    for (auto& r : rows) n_own = std::max<int>(n_own, (int)r.size());
  }
  if (!theta_length_ok(g.k_theta))
    return fail(RL_ERR_GEOMETRY,
                "k_theta must be in [8, 2048]: 2^a 3^b up to 32 with at most one factor 3, or 32 times one of "
                "2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64");
  if (g.q_theta != 1 && g.q_theta != 2) return fail(RL_ERR_GEOMETRY, "q_theta must be 1 or 2");
  if (g.k_theta < 2 * g.q_theta * ((g.n_theta + g.m - 1) / g.m) ||
      g.k_theta < lattice_rows(n_own, g.q_theta) + 2 * kHalo)
    return fail(RL_ERR_GEOMETRY,
                "k_theta must be >= 2 q_theta ceil(n_theta/m) and >= q_theta (n_own - 1) + 5");
  if (g.r_dec < r_bound(g.n, g.n_theta, g.m, g.q_theta) || g.r_dec > 32)
    return fail(RL_ERR_GEOMETRY, "r_dec must satisfy (dtheta / q_theta) / r_dec <= 2 a_R / n and be <= 32");
  if (g.dec_filter != 0 && g.dec_filter != 1)
    return fail(RL_ERR_GEOMETRY, "dec_filter must be 0 (cubic B-spline) or 1 (box)");
  return RL_OK;
}

// rho position of every sample of every owned sinogram row (eq. Sm_def): tau = (log(a_R s +
// (1 - a_R) cos theta') - rho_0) / d_rho, s -> -s on the wrapped rows.  Stored as floor(tau)
// (clamped to [-1, n_rho]) and the FP32 fraction, which the 4-tap evaluation and its
// transpose read instead of recomputing the logarithm.
__global__ __launch_bounds__(256) void k_tau_table(DevPlan P, int2* __restrict__ tab) {
  const int o = blockIdx.x, m = blockIdx.y;
  const int jw = P.own_j[m * P.n_own + o];
  int2* row = tab + ((size_t)m * P.n_own + o) * P.n_s;
  if (jw < 0) {
    for (int k = threadIdx.x; k < P.n_s; k += blockDim.x) row[k] = make_int2(0, 0);
    return;
  }
  const bool wrap = (jw >> 30) & 1;
  const double cth = P.own_cos[m * P.n_own + o];
  const double aR = P.a_R;
  for (int k = threadIdx.x; k < P.n_s; k += blockDim.x) {
    double s = -1.0 + k * P.ds;
    if (wrap) s = -s;
    // On the rows at theta' = +-beta/2 the edge sample lands on tau = -1 exactly, which rounding
    // can put just below -1.  Clamping tau itself (not only its floor) keeps the base index and
    // the fraction consistent, so the four taps stay where the unrounded tau puts them.
    const double tau = fmin(fmax((log(aR * s + (1.0 - aR) * cth) - P.rho0) / P.d_rho, -1.0), (double)P.n_rho);
    const double ft = floor(tau);
    row[k] = make_int2((int)ft, __float_as_int((float)(tau - ft)));
  }
}

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

rl_status fail(rl_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

rl_status check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return RL_OK;
  return fail(RL_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

rl_status check_launch(const char* what) { return check_hip(hipGetLastError(), what); }

rl_status ensure_dyn_lds(const void* fn, size_t lds, const char* what) {
  if (lds <= 65536) return RL_OK;
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, size_t> done;  // (kernel, device) -> limit set
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(RL_ERR_HIP, "hipGetDevice failed");
  std::lock_guard<std::mutex> lock(mu);
  size_t& have = done[std::make_pair(fn, dev)];
  if (have >= lds) return RL_OK;
  rl_status st = check_hip(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds), what);
  if (st == RL_OK) have = lds;
  return st;
}

rl_status check_plan_device(const rl_plan* plan) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(RL_ERR_HIP, "hipGetDevice failed");
  if (dev != plan->device)
    return fail(RL_ERR_INVALID_ARG, "plan was built on device " + std::to_string(plan->device) +
                                        " but the current device is " + std::to_string(dev));
  return RL_OK;
}

// ---------------------------------------------------------------- kernel timing hooks
namespace {
struct Profiler {
  bool on = false;
  int capacity = 0;
  int used = 0;
  std::vector<hipEvent_t> start, stop;
  std::vector<const char*> names;
} g_prof;
}  // namespace

int prof_open(const char* name, hipStream_t s) {
  if (!g_prof.on || g_prof.used >= g_prof.capacity) return -1;
  const int slot = g_prof.used++;
  g_prof.names[slot] = name;
  (void)hipEventRecord(g_prof.start[slot], s);
  return slot;
}

void prof_close(int slot, hipStream_t s) {
  if (slot >= 0) (void)hipEventRecord(g_prof.stop[slot], s);
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

WsLayout workspace_layout(const rl_plan* plan, int batch, rl_op op) {
  WsLayout L{};
  const DevPlan& d = plan->d;
  const size_t B = (size_t)batch, M = (size_t)d.m;
  const size_t img = align256(B * d.n * d.n * sizeof(float));
  const size_t lp = align256(B * M * d.n_sup * d.n_rho * sizeof(float));
  const size_t spec_sup = align256(B * M * d.n_sup * d.ld * sizeof(float2));
  const size_t spec_own = align256(B * M * d.n_own * d.ld * sizeof(float2));
  const size_t sino = align256(B * d.n_theta * d.n_s * sizeof(float));
  size_t sizes[6] = {0, 0, 0, 0, 0, 0};
  if (batch > 0) {
    if (op == RL_OP_FWD) {
      sizes[0] = img;       // prefiltered image
      sizes[1] = lp;        // log-polar samples
      sizes[2] = spec_sup;  // rho spectra of the support rows
      sizes[3] = spec_own;  // convolved spectra of the owned rows
    } else {
      sizes[0] = img;       // spline-coefficient accumulator
      sizes[1] = lp;        // log-polar adjoint samples
      sizes[2] = spec_sup;  // convolved spectra of the support rows
      sizes[3] = spec_own;  // rho spectra of the owned rows
      if (op == RL_OP_FBP || op == RL_OP_FBP_LP) sizes[4] = sino;  // filtered sinogram
      if (op == RL_OP_BP_LP || op == RL_OP_FBP_LP) sizes[0] = 0;  // Algorithm 2 writes the image directly
    }
  }
  size_t off = 0;
  for (int i = 0; i < 6; ++i) {
    L.off[i] = off;
    off += sizes[i];
  }
  L.total = off;
  return L;
}

}  // namespace rl

using namespace rl;

extern "C" rl_status rl_geom_default(int32_t n, int32_t n_theta, int32_t n_s, int32_t m, int32_t q_theta,
                                    int32_t smooth, rl_geom* out) {
  if (!out) return fail(RL_ERR_INVALID_ARG, "out is NULL");
  if (n < 8 || (n & 1) || n > 8192 || m < 3 || m > kMaxPart || n_theta < m || n_s < 2 || (q_theta != 1 && q_theta != 2) ||
      (smooth != 0 && smooth != 1))
    return fail(RL_ERR_GEOMETRY, "no default geometry for these sizes");
  rl_geom g{};
  g.n = n;
  g.n_theta = n_theta;
  g.n_s = n_s;
  g.m = m;
  int n_own = 0;
  auto rows = partition_rows(n_theta, m);
  for (auto& r : rows) n_own = std::max<int>(n_own, (int)r.size());
  const long kmin = std::max<long>(2L * q_theta * ((n_theta + m - 1) / m), lattice_rows(n_own, q_theta) + 2 * kHalo);
  if (smooth) {
    long nr = std::max(16L, rho_bound(n, m));
    while (nr <= 8192 && !(is_smooth23(nr) && nr % 4 == 0)) ++nr;
    long kt = std::max(8L, kmin);
    while (kt <= 2048 && !theta_length_ok(kt)) ++kt;
    g.n_rho = (int)nr;
    g.k_theta = (int)kt;
  } else {
    g.n_rho = std::max(16, next_pow2(rho_bound(n, m)));
    g.k_theta = std::max(8, next_pow2(kmin));
  }
  g.r_dec = (int)r_bound(n, n_theta, m, q_theta);
  g.dec_filter = 0;
  g.q_theta = q_theta;
  rl_status st = validate(g);
  if (st != RL_OK) return st;
  *out = g;
  return RL_OK;
}

extern "C" rl_status rl_plan_create(const rl_geom* geom, rl_plan** out) {
  if (!out) return fail(RL_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!geom) return fail(RL_ERR_INVALID_ARG, "geom is NULL");
  const rl_geom g = *geom;
  rl_status st = validate(g);
  if (st != RL_OK) return st;

  int dev = 0;
  if ((st = check_hip(hipGetDevice(&dev), "hipGetDevice")) != RL_OK) return st;
  hipDeviceProp_t prop;
  if ((st = check_hip(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties")) != RL_OK) return st;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(RL_ERR_UNSUPPORTED_ARCH, std::string("device is ") + prop.gcnArchName + ", need gfx950");

  rl_plan* plan = new rl_plan();
  plan->g = g;
  plan->device = dev;
  plan->tune = rl_tune{0, 1, 512, 1, 1, 1};
  DevPlan& d = plan->d;
  std::memset(&d, 0, sizeof(d));
  d.n = g.n;
  d.n_theta = g.n_theta;
  d.n_s = g.n_s;
  d.m = g.m;
  d.n_rho = g.n_rho;
  d.k_theta = g.k_theta;
  d.r = g.r_dec;
  d.q = g.q_theta;
  double a_R, a_r;
  partition_constants(g.m, &a_R, &a_r);
  const double L = -std::log(a_r);
  d.a_R = a_R;
  d.beta = M_PI / g.m;
  d.dx = 2.0 / g.n;
  d.ds = 2.0 / g.n_s;
  d.dtheta = M_PI / g.n_theta;
  d.dtheta_c = d.dtheta / g.q_theta;
  d.d_rho = L / g.n_rho;
  d.rho0 = (1.0 - g.n_rho) * d.d_rho;
  auto rows = partition_rows(g.n_theta, g.m);
  int n_own = 0;
  for (auto& r : rows) n_own = std::max<int>(n_own, (int)r.size());
  d.n_own = n_own;
  d.n_sup = lattice_rows(n_own, g.q_theta) + 2 * kHalo;
  const int r = g.r_dec;
  d.t_min = -(2 * r - 1);
  d.n_fine = r * (d.n_sup - 1) + 4 * r - 1;
  d.nc = g.n_rho / 2;
  d.ld = d.nc + 8;
  d.lr = std::max(16, next_pow2(2L * g.n_s));
  // one twiddle table serves every FFT length (the rho rows, the theta pass, the ramp filter)
  d.tw_len = (int)lcm_l(lcm_l(g.n_rho, g.k_theta), d.lr);
  plan->rows_per_part.resize(g.m);
  for (int p = 0; p < g.m; ++p) {
    plan->rows_per_part[p] = (int)rows[p].size();
    const double mb = p * d.beta;
    d.X0[p] = (1.0 - (1.0 - a_R) * std::cos(mb) / a_R) / d.dx;
    d.Y0[p] = (1.0 - (1.0 - a_R) * std::sin(mb) / a_R) / d.dx;
    d.phi0[p] = M_PI * (double)rows[p][0].nu / ((double)g.n_theta * g.m) - kHalo * d.dtheta_c;
    d.sup_rows[p] = lattice_rows((int)rows[p].size(), g.q_theta) + 2 * kHalo;
  }

  // ---------------- host tables
  const int M = g.m, NF = d.n_fine;
  std::vector<double2> fine_cs((size_t)M * NF);
  std::vector<int2> fine_q((size_t)M * NF);
  int64_t n_samples = 0;
  const double eps = 1e-9;  // samples within eps (in e^rho) of the boundary of D count as outside
  for (int p = 0; p < M; ++p) {
    for (int ti = 0; ti < NF; ++ti) {
      const double phi = d.phi0[p] + (double)(d.t_min + ti) * (d.dtheta_c / r);
      fine_cs[(size_t)p * NF + ti] = make_double2(std::cos(phi + p * d.beta), std::sin(phi + p * d.beta));
      // the ray of angle phi meets D (eq. circle_D) for e^rho in (c - root, c + root)
      const double disc = a_R * a_R - (1.0 - a_R) * (1.0 - a_R) * std::sin(phi) * std::sin(phi);
      int2 qr = make_int2(1, 0);
      if (disc > 0.0) {
        const double c = (1.0 - a_R) * std::cos(phi), root = std::sqrt(disc);
        const double lo = c - root + eps, hi = c + root - eps;
        if (hi > lo) {
          const long qlo = (long)std::floor(std::log(lo) / d.d_rho + g.n_rho - 1) + 1;
          const long qhi = (long)std::ceil(std::log(hi) / d.d_rho + g.n_rho - 1) - 1;
          if (qhi >= qlo) qr = make_int2((int)std::max(0L, qlo), (int)std::min<long>(g.n_rho - 1, qhi));
        }
      }
      fine_q[(size_t)p * NF + ti] = qr;
      if (qr.y >= qr.x) n_samples += qr.y - qr.x + 1;
    }
  }
  std::vector<float4> dec(r);
  {
    auto dn = [&](int n) { return dec_tap(g.dec_filter, n, r); };
    for (int p = 0; p < r; ++p)
      dec[p] = make_float4((float)dn(p + r), (float)dn(p), (float)dn(p - r), (float)dn(p - 2 * r));
  }
  std::vector<float> dtap(4 * r - 1);
  for (int k = 0; k < 4 * r - 1; ++k) {
    const int nn = k - (2 * r - 1);
    dtap[k] = (float)dec_tap(g.dec_filter, nn, r);
  }
  std::vector<int> own_j((size_t)M * n_own, -1);
  std::vector<double> own_cos((size_t)M * n_own, 1.0);
  for (int p = 0; p < M; ++p)
    for (size_t o = 0; o < rows[p].size(); ++o) {
      const auto& R = rows[p][o];
      own_j[(size_t)p * n_own + o] = R.j | (R.wrap ? (1 << 30) : 0);
      own_cos[(size_t)p * n_own + o] = std::cos(M_PI * (double)R.nu / ((double)g.n_theta * g.m));
    }
  std::vector<float2> tw(d.tw_len);
  for (int i = 0; i < d.tw_len; ++i) {
    const double a = -2.0 * M_PI * (double)i / d.tw_len;
    tw[i] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  // Stockham pass twiddles (entries of tw, so the passes multiply by the same values)
  auto pass_twiddles = [&](int N) {
    std::vector<float2> out;
    for (int Ns = 1; Ns < N;) {
      const int R = stockham_radix(N / Ns), RP = stockham_slots(R), step = d.tw_len / (R * Ns);
      for (int k = 0; k < Ns; ++k)
        for (int r = 1; r <= RP; ++r) out.push_back(r < R ? tw[(size_t)r * k * step] : make_float2(0.f, 0.f));
      Ns *= R;
    }
    return out;
  };
  const std::vector<float2> twp_rows = pass_twiddles(d.nc), twp_ramp = pass_twiddles(d.lr / 2);
  std::vector<float2> tw_theta(g.k_theta);
  {
    const int K1 = theta_k1(g.k_theta), K2 = g.k_theta / K1, step = d.tw_len / g.k_theta;
    for (int n2 = 0; n2 < K2; ++n2)
      for (int k1 = 0; k1 < K1; ++k1) tw_theta[(size_t)n2 * K1 + k1] = tw[(size_t)n2 * k1 * step];
  }
  // Ram-Lak kernel (times ds) on a cyclic grid of length lr, and its DFT / lr (real, even),
  // times the window of each filter of rl_filter: table f at ramp[f * (lr / 2 + 1) + k]
  std::vector<float> ramp(3 * (d.lr / 2 + 1));
  {
    const int lr = d.lr;
    std::vector<double> h(lr, 0.0);
    const double ds = d.ds;
    h[0] = 1.0 / (4.0 * ds);
    for (int n = 1; n < g.n_s; ++n) {
      if (n & 1) {
        const double v = -1.0 / (M_PI * M_PI * (double)n * n * ds);
        h[n] = v;
        h[lr - n] = v;
      }
    }
    for (int k = 0; k <= lr / 2; ++k) {
      double acc = h[0];
      for (int n = 1; n < g.n_s; n += 2) acc += 2.0 * h[n] * std::cos(2.0 * M_PI * (double)((long)k * n % lr) / lr);
      const double r0 = acc / lr, t = M_PI * k / (2.0 * lr);
      ramp[k] = (float)r0;
      ramp[(lr / 2 + 1) + k] = (float)(r0 * std::cos(M_PI * k / lr));
      ramp[2 * (lr / 2 + 1) + k] = (float)(k == 0 ? r0 : r0 * std::sin(t) / t);
    }
  }
  std::vector<double> erho(g.n_rho);
  for (int q = 0; q < g.n_rho; ++q) erho[q] = std::exp((double)(q - g.n_rho + 1) * d.d_rho) / (a_R * d.dx);
  std::vector<float> pref(kPrefR + 1);
  {
    const double z = std::sqrt(3.0) - 2.0;
    for (int k = 0; k <= kPrefR; ++k) pref[k] = (float)(std::sqrt(3.0) * std::pow(z, k));
  }

  const std::vector<int4> fbox = build_fwd_boxes(d, fine_cs, fine_q, erho);
  int n_small_tiles = 0, n_mid_tiles = 0;
  const std::vector<int> ftiles = build_fwd_tiles(d, fbox, &n_small_tiles, &n_mid_tiles);

  // ---------------- kernel table: zeta_hat on the device in FP64
  const int nkt = g.k_theta / 2 + 1, nkr = g.n_rho / 2 + 1;
  const double P = g.k_theta * d.dtheta_c;
  std::vector<double> xg, wg;
  gauss_legendre(16, xg, wg);
  const double max_rate = 2.0 * M_PI * (nkt - 1) / P + 2.0 * M_PI * (nkr - 1) / L * std::tan(d.beta);
  const int n_panels = std::max(8, (int)std::ceil(2.0 * d.beta * max_rate / 6.0));
  int n_nodes = n_panels * 16;
  const int n_nodes_pad = (n_nodes + kZN - 1) / kZN * kZN;
  // zeta_hat (eq. exprcoef1): amplitude w / cos u, phase log cos u; zeta#_hat (eq. exprcoef2):
  // amplitude w, phase -log cos u (the integrand's (cos u)^{2 pi i k_rho / L})
  std::vector<double> u(n_nodes_pad, 0.0), amp(n_nodes_pad, 0.0), lcv(n_nodes_pad, 0.0);
  std::vector<double> amp2(n_nodes_pad, 0.0), lcv2(n_nodes_pad, 0.0);
  const double hw = d.beta / n_panels;
  for (int pi = 0; pi < n_panels; ++pi) {
    const double mid = -d.beta + (2.0 * pi + 1.0) * hw;
    for (int i = 0; i < 16; ++i) {
      const double x = mid + hw * xg[i];
      u[pi * 16 + i] = x;
      amp[pi * 16 + i] = hw * wg[i] / std::cos(x);
      lcv[pi * 16 + i] = std::log(std::cos(x));
      amp2[pi * 16 + i] = hw * wg[i];
      lcv2[pi * 16 + i] = -std::log(std::cos(x));
    }
  }

  // one device allocation for everything
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t off = 0;
  const size_t o_H = off; off += al(sizeof(float2) * (size_t)nkr * nkt);
  const size_t o_Hb = off; off += al(sizeof(float2) * (size_t)nkr * nkt);
  const size_t o_cs = off; off += al(sizeof(double2) * fine_cs.size());
  const size_t o_q = off; off += al(sizeof(int2) * fine_q.size());
  const size_t o_dec = off; off += al(sizeof(float4) * dec.size());
  const size_t o_oj = off; off += al(sizeof(int) * own_j.size());
  const size_t o_oc = off; off += al(sizeof(double) * own_cos.size());
  const size_t o_tw = off; off += al(sizeof(float2) * tw.size());
  const size_t o_tpr = off; off += al(sizeof(float2) * twp_rows.size());
  const size_t o_tpl = off; off += al(sizeof(float2) * twp_ramp.size());
  const size_t o_tth = off; off += al(sizeof(float2) * tw_theta.size());
  const size_t o_rp = off; off += al(sizeof(float) * ramp.size());
  const size_t o_pf = off; off += al(sizeof(float) * pref.size());
  const size_t o_er = off; off += al(sizeof(double) * erho.size());
  const size_t o_dt = off; off += al(sizeof(float) * dtap.size());
  const size_t o_ta = off; off += al(sizeof(int2) * (size_t)M * n_own * g.n_s);
  const size_t o_fb = off; off += al(sizeof(int4) * fbox.size());
  const size_t o_ft = off; off += al(sizeof(int) * ftiles.size());
  const size_t n_px = (size_t)M * g.n * g.n;  // Algorithm 2's per-pixel lattice coordinates
  const size_t o_bk = off; off += al(sizeof(unsigned) * n_px);
  const size_t o_bf = off; off += al(sizeof(float2) * n_px);
  const size_t o_bb = off; off += al(sizeof(int4) * (size_t)M * bp_tiles(g.n));
  const size_t table_bytes = off;
  // scratch for the quadrature (freed before returning)
  const size_t s_u = 0, s_a = al(sizeof(double) * n_nodes_pad), s_l = 2 * s_a, s_a2 = 3 * s_a, s_l2 = 4 * s_a;
  const size_t s_z = 5 * s_a, s_z2 = s_z + al(sizeof(double2) * (size_t)nkt * nkr);
  const size_t scratch = s_z2 + al(sizeof(double2) * (size_t)nkt * nkr);

  char* mem = nullptr;
  char* tmp = nullptr;
  std::vector<double2> zeta((size_t)nkt * nkr), zeta2((size_t)nkt * nkr);
  auto cleanup = [&](rl_status code) {
    if (tmp) (void)hipFree(tmp);
    if (code != RL_OK) {
      if (mem) (void)hipFree(mem);
      delete plan;
    }
    return code;
  };
  if ((st = check_hip(hipMalloc(&mem, table_bytes), "hipMalloc(tables)")) != RL_OK) return cleanup(st);
  if ((st = check_hip(hipMalloc(&tmp, scratch), "hipMalloc(quadrature scratch)")) != RL_OK) return cleanup(st);
  if ((st = check_hip(hipMemcpy(tmp + s_u, u.data(), sizeof(double) * n_nodes_pad, hipMemcpyHostToDevice), "copy nodes")) != RL_OK) return cleanup(st);
  if ((st = check_hip(hipMemcpy(tmp + s_a, amp.data(), sizeof(double) * n_nodes_pad, hipMemcpyHostToDevice), "copy weights")) != RL_OK) return cleanup(st);
  if ((st = check_hip(hipMemcpy(tmp + s_l, lcv.data(), sizeof(double) * n_nodes_pad, hipMemcpyHostToDevice), "copy logcos")) != RL_OK) return cleanup(st);
  if ((st = check_hip(hipMemcpy(tmp + s_a2, amp2.data(), sizeof(double) * n_nodes_pad, hipMemcpyHostToDevice), "copy weights")) != RL_OK) return cleanup(st);
  if ((st = check_hip(hipMemcpy(tmp + s_l2, lcv2.data(), sizeof(double) * n_nodes_pad, hipMemcpyHostToDevice), "copy logcos")) != RL_OK) return cleanup(st);
  {
    dim3 grid((nkt + kZT - 1) / kZT, (nkr + kZT - 1) / kZT);
    hipLaunchKernelGGL(k_zeta_hat, grid, dim3(256), 0, 0, (double2*)(tmp + s_z), (const double*)(tmp + s_u),
                       (const double*)(tmp + s_a), (const double*)(tmp + s_l), n_nodes_pad, nkt, nkr, 1.0 / P,
                       1.0 / L);
    if ((st = check_launch("k_zeta_hat")) != RL_OK) return cleanup(st);
    hipLaunchKernelGGL(k_zeta_hat, grid, dim3(256), 0, 0, (double2*)(tmp + s_z2), (const double*)(tmp + s_u),
                       (const double*)(tmp + s_a2), (const double*)(tmp + s_l2), n_nodes_pad, nkt, nkr, 1.0 / P,
                       1.0 / L);
    if ((st = check_launch("k_zeta_hat")) != RL_OK) return cleanup(st);
  }
  if ((st = check_hip(hipMemcpy(zeta.data(), tmp + s_z, sizeof(double2) * zeta.size(), hipMemcpyDeviceToHost), "copy zeta")) != RL_OK) return cleanup(st);
  if ((st = check_hip(hipMemcpy(zeta2.data(), tmp + s_z2, sizeof(double2) * zeta2.size(), hipMemcpyDeviceToHost), "copy zeta#")) != RL_OK) return cleanup(st);

  // H = zeta_hat / (B_hat(kr/N_rho) D_hat(kt) K N_rho), stored [kr][kt]; real part at the rho Nyquist bin
  std::vector<float2> H((size_t)nkr * nkt);
  {
    std::vector<double> dhat(nkt);
    for (int kt = 0; kt < nkt; ++kt) {
      double acc = 0.0;
      for (int n = -(2 * r - 1); n <= 2 * r - 1; ++n)
        acc += dec_tap(g.dec_filter, n, r) * std::cos(2.0 * M_PI * kt * n / ((double)r * g.k_theta));
      dhat[kt] = acc;
    }
    const double norm = 1.0 / ((double)g.k_theta * g.n_rho);
    for (int kr = 0; kr < nkr; ++kr) {
      const double bh = 2.0 / 3.0 + std::cos(2.0 * M_PI * kr / g.n_rho) / 3.0;
      for (int kt = 0; kt < nkt; ++kt) {
        double2 z = zeta[(size_t)kt * nkr + kr];
        const double s = norm / (bh * dhat[kt]);
        double re = z.x * s, im = z.y * s;
        if (kr == nkr - 1) im = 0.0;
        H[(size_t)kr * nkt + kt] = make_float2((float)re, (float)im);
      }
    }
  }
  // H# = zeta#_hat / (B_hat(kt/K) B_hat(kr/N_rho) K N_rho) (Alg. 2 step 4), same layout and
  // Nyquist treatment
  std::vector<float2> Hb((size_t)nkr * nkt);
  {
    const double norm = 1.0 / ((double)g.k_theta * g.n_rho);
    for (int kr = 0; kr < nkr; ++kr) {
      const double bh = 2.0 / 3.0 + std::cos(2.0 * M_PI * kr / g.n_rho) / 3.0;
      for (int kt = 0; kt < nkt; ++kt) {
        const double bt = 2.0 / 3.0 + std::cos(2.0 * M_PI * kt / g.k_theta) / 3.0;
        const double2 z = zeta2[(size_t)kt * nkr + kr];
        const double s = norm / (bh * bt);
        Hb[(size_t)kr * nkt + kt] = make_float2((float)(z.x * s), kr == nkr - 1 ? 0.f : (float)(z.y * s));
      }
    }
  }
  struct Up {
    size_t off;
    const void* src;
    size_t bytes;
  } ups[] = {
      {o_H, H.data(), sizeof(float2) * H.size()},
      {o_Hb, Hb.data(), sizeof(float2) * Hb.size()},
      {o_cs, fine_cs.data(), sizeof(double2) * fine_cs.size()},
      {o_q, fine_q.data(), sizeof(int2) * fine_q.size()},
      {o_dec, dec.data(), sizeof(float4) * dec.size()},
      {o_oj, own_j.data(), sizeof(int) * own_j.size()},
      {o_oc, own_cos.data(), sizeof(double) * own_cos.size()},
      {o_tw, tw.data(), sizeof(float2) * tw.size()},
      {o_tpr, twp_rows.data(), sizeof(float2) * twp_rows.size()},
      {o_tpl, twp_ramp.data(), sizeof(float2) * twp_ramp.size()},
      {o_tth, tw_theta.data(), sizeof(float2) * tw_theta.size()},
      {o_rp, ramp.data(), sizeof(float) * ramp.size()},
      {o_pf, pref.data(), sizeof(float) * pref.size()},
      {o_er, erho.data(), sizeof(double) * erho.size()},
      {o_dt, dtap.data(), sizeof(float) * dtap.size()},
      {o_fb, fbox.data(), sizeof(int4) * fbox.size()},
      {o_ft, ftiles.data(), sizeof(int) * ftiles.size()},
  };
  for (auto& up : ups)
    if ((st = check_hip(hipMemcpy(mem + up.off, up.src, up.bytes, hipMemcpyHostToDevice), "upload table")) != RL_OK)
      return cleanup(st);
  d.H = (const float2*)(mem + o_H);
  d.Hbp = (const float2*)(mem + o_Hb);
  d.fine_cs = (const double2*)(mem + o_cs);
  d.fine_q = (const int2*)(mem + o_q);
  d.dec = (const float4*)(mem + o_dec);
  d.own_j = (const int*)(mem + o_oj);
  d.own_cos = (const double*)(mem + o_oc);
  d.tw = (const float2*)(mem + o_tw);
  d.twp_rows = (const float2*)(mem + o_tpr);
  d.twp_ramp = (const float2*)(mem + o_tpl);
  d.tw_theta = (const float2*)(mem + o_tth);
  d.ramp = (const float*)(mem + o_rp);
  d.pref = (const float*)(mem + o_pf);
  d.erho = (const double*)(mem + o_er);
  d.dtap = (const float*)(mem + o_dt);
  d.tau = (const int2*)(mem + o_ta);
  d.fbox = (const int4*)(mem + o_fb);
  d.ftiles = (const int*)(mem + o_ft);
  d.ftiles_small = n_small_tiles;
  d.ftiles_mid = n_mid_tiles;
  d.ftiles_large = (int)ftiles.size() - n_small_tiles - n_mid_tiles;
  d.bp_k = (const unsigned*)(mem + o_bk);
  d.bp_f = (const float2*)(mem + o_bf);
  d.bp_box = (const int4*)(mem + o_bb);
  hipLaunchKernelGGL(k_tau_table, dim3(n_own, M), dim3(256), 0, 0, d, (int2*)(mem + o_ta));
  if ((st = check_launch("k_tau_table")) != RL_OK) return cleanup(st);
  if ((st = build_bp_geometry(d, (unsigned*)(mem + o_bk), (float2*)(mem + o_bf), (int4*)(mem + o_bb))) != RL_OK) return cleanup(st);
  if ((st = check_hip(hipDeviceSynchronize(), "k_tau_table")) != RL_OK) return cleanup(st);
  plan->d_mem = mem;
  plan->d_mem_bytes = table_bytes;
  plan->n_samples = n_samples;
  plan->d_adj = nullptr;
  plan->d_adj_bytes = 0;
  if ((st = build_adj_passes(plan)) != RL_OK) {
    plan->d_mem = nullptr;  // freed by cleanup
    return cleanup(st);
  }
  if ((st = prepare_forward_launches(plan)) != RL_OK || (st = prepare_adjoint_launches(plan)) != RL_OK ||
      (st = prepare_bp_launches(plan)) != RL_OK) {
    if (plan->d_adj) (void)hipFree(plan->d_adj);
    plan->d_mem = nullptr;
    return cleanup(st);
  }
  cleanup(RL_OK);
  *out = plan;
  return RL_OK;
}

extern "C" void rl_plan_destroy(rl_plan* plan) {
  if (!plan) return;
  if (plan->d_mem) (void)hipFree(plan->d_mem);
  if (plan->d_adj) (void)hipFree(plan->d_adj);
  delete plan;
}

extern "C" rl_status rl_plan_samples(const rl_plan* plan, int64_t* out) {
  if (!plan || !out) return fail(RL_ERR_INVALID_ARG, "NULL argument");
  *out = plan->n_samples;
  return RL_OK;
}

extern "C" rl_status rl_plan_rows(const rl_plan* plan, int32_t* n_own, int32_t* rows) {
  if (!plan || !n_own) return fail(RL_ERR_INVALID_ARG, "NULL argument");
  *n_own = plan->d.n_own;
  if (rows)
    for (int p = 0; p < plan->d.m; ++p) rows[p] = plan->rows_per_part[p];
  return RL_OK;
}

extern "C" rl_status rl_plan_geometry(const rl_plan* plan, rl_geom* out) {
  if (!plan || !out) return fail(RL_ERR_INVALID_ARG, "NULL argument");
  *out = plan->g;
  return RL_OK;
}

extern "C" size_t rl_workspace_bytes(const rl_plan* plan, int32_t batch, rl_op op) {
  if (!plan || batch <= 0) return 0;
  if (op == RL_OP_EM) return em_workspace_bytes(plan, batch);
  if (op != RL_OP_FWD && op != RL_OP_ADJ && op != RL_OP_FBP && op != RL_OP_BP_LP && op != RL_OP_FBP_LP) return 0;
  return workspace_layout(plan, batch, op).total;
}

extern "C" const char* rl_last_error(void) { return g_last_error.c_str(); }

extern "C" rl_status rl_profile_start(int32_t capacity) {
  if (capacity < 0) return fail(RL_ERR_INVALID_ARG, "negative capacity");
  g_prof.on = false;
  while ((int)g_prof.start.size() < capacity) {
    hipEvent_t a, b;
    rl_status st = check_hip(hipEventCreate(&a), "hipEventCreate");
    if (st != RL_OK) return st;
    st = check_hip(hipEventCreate(&b), "hipEventCreate");
    if (st != RL_OK) {
      (void)hipEventDestroy(a);
      return st;
    }
    g_prof.start.push_back(a);
    g_prof.stop.push_back(b);
  }
  g_prof.names.assign(g_prof.start.size(), "");
  g_prof.capacity = capacity;
  g_prof.used = 0;
  g_prof.on = true;
  return RL_OK;
}

extern "C" rl_status rl_profile_stop(void) {
  g_prof.on = false;
  return RL_OK;
}

extern "C" int32_t rl_profile_count(void) { return g_prof.used; }

extern "C" rl_status rl_profile_record(int32_t i, const char** name, float* ms) {
  if (i < 0 || i >= g_prof.used || !name || !ms) return fail(RL_ERR_INVALID_ARG, "bad profile record index");
  rl_status st = check_hip(hipEventSynchronize(g_prof.stop[i]), "hipEventSynchronize");
  if (st != RL_OK) return st;
  *name = g_prof.names[i];
  return check_hip(hipEventElapsedTime(ms, g_prof.start[i], g_prof.stop[i]), "hipEventElapsedTime");
}
