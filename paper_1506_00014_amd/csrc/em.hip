// EM reconstruction (sec. 7, the EM iteration) on the library's R and R#:
//   f <- f R#( chi_C g / R f ) / R# chi_C
// chi_C(theta, s) = 1 on the lines through the unit disc (|s| < 1), the ratio is 0 on lines
// with R f <= 0, and the image lives on the unit disc (R reads no sample outside it): f is
// set to 0 at pixels with |x| >= 1 or R# chi_C <= 0.
//   k_em_chi     chi_C on the sinogram grid
//   k_em_ratio   chi_C g / R f, in place over R f
//   k_em_update  f * back / norm on the disc, 0 elsewhere
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "fft_device.h"
#include "rl_internal.h"

namespace rl {

namespace {

constexpr int kEThreads = 256;

__device__ __forceinline__ bool through_disc(int k, double ds) { return fabs(-1.0 + k * ds) < 1.0; }

__global__ __launch_bounds__(kEThreads) void k_em_chi(float* __restrict__ sino, size_t count, int n_s, double ds) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    sino[i] = through_disc((int)(i % n_s), ds) ? 1.f : 0.f;
}

__global__ __launch_bounds__(kEThreads) void k_em_ratio(const float* __restrict__ g, float* __restrict__ rf,
                                                        size_t count, int n_s, double ds) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const float r = rf[i];
    rf[i] = (through_disc((int)(i % n_s), ds) && r > 0.f) ? g[i] / r : 0.f;
  }
}

__global__ __launch_bounds__(kEThreads) void k_em_update(float* __restrict__ f, const float* __restrict__ back,
                                                         const float* __restrict__ norm, size_t count, int n) {
  const size_t nn = (size_t)n * n;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const size_t p = i % nn;
    const float w = norm[p];
    f[i] = (in_unit_disc((int)(p % n), (int)(p / n), n) && w > 0.f) ? f[i] * back[i] / w : 0.f;
  }
}

dim3 grid_for(size_t count) {
  const size_t b = (count + kEThreads - 1) / kEThreads;
  return dim3((unsigned)(b < 65536 ? (b ? b : 1) : 65536));
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

struct EmLayout {
  size_t chain, rf, back, total;
};

EmLayout em_layout(const rl_plan* p, int batch) {
  const DevPlan& d = p->d;
  EmLayout L;
  const size_t wf = workspace_layout(p, batch, RL_OP_FWD).total, wa = workspace_layout(p, batch, RL_OP_ADJ).total;
  L.chain = 0;
  L.rf = al256(wf > wa ? wf : wa);
  L.back = L.rf + al256((size_t)batch * d.n_theta * d.n_s * sizeof(float));
  L.total = L.back + al256((size_t)batch * d.n * d.n * sizeof(float));
  return L;
}

rl_status ws_check(const rl_plan* plan, int batch, void* ws, size_t ws_bytes) {
  const size_t need = em_layout(plan, batch).total;
  if (!ws || ws_bytes < need)
    return fail(RL_ERR_WORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes, need " + std::to_string(need));
  if (((uintptr_t)ws) & 255) return fail(RL_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  return RL_OK;
}

}  // namespace

size_t em_workspace_bytes(const rl_plan* plan, int batch) { return em_layout(plan, batch).total; }

}  // namespace rl

using namespace rl;

extern "C" rl_status rl_em_norm(const rl_plan* plan, float* d_norm, void* d_ws, size_t ws_bytes, hipStream_t stream) {
  if (!plan) return fail(RL_ERR_INVALID_ARG, "plan is NULL");
  if (!d_norm) return fail(RL_ERR_INVALID_ARG, "norm pointer is NULL");
  rl_status st = ws_check(plan, 1, d_ws, ws_bytes);
  if (st != RL_OK) return st;
  const DevPlan& d = plan->d;
  const EmLayout L = em_layout(plan, 1);
  if (overlaps(d_ws, L.total, d_norm, (size_t)d.n * d.n * sizeof(float)))
    return fail(RL_ERR_INVALID_ARG, "workspace overlaps the output");
  if ((st = check_plan_device(plan)) != RL_OK) return st;
  float* chi = (float*)((char*)d_ws + L.rf);
  const size_t cs = (size_t)d.n_theta * d.n_s;
  hipLaunchKernelGGL(k_em_chi, grid_for(cs), dim3(kEThreads), 0, stream, chi, cs, d.n_s, d.ds);
  if ((st = check_launch("k_em_chi")) != RL_OK) return st;
  return adjoint_chain(plan, dense((const float*)chi, cs), dense(d_norm, (size_t)d.n * d.n), 1, (char*)d_ws + L.chain,
                       RL_OP_ADJ, false, stream);
}

extern "C" rl_status rl_em(const rl_plan* plan, const float* d_sino, const float* d_norm, float* d_img, int32_t batch,
                           int32_t iters, void* d_ws, size_t ws_bytes, hipStream_t stream) {
  if (!plan) return fail(RL_ERR_INVALID_ARG, "plan is NULL");
  if (batch < 0 || iters < 0) return fail(RL_ERR_INVALID_ARG, "batch and iters must be >= 0");
  if (batch == 0 || iters == 0) return RL_OK;
  if (!d_sino || !d_norm || !d_img) return fail(RL_ERR_INVALID_ARG, "sino, norm or image pointer is NULL");
  const DevPlan& d = plan->d;
  const size_t sb = (size_t)batch * d.n_theta * d.n_s * sizeof(float), ib = (size_t)batch * d.n * d.n * sizeof(float),
               nb = (size_t)d.n * d.n * sizeof(float);
  if (overlaps(d_sino, sb, d_img, ib) || overlaps(d_norm, nb, d_img, ib))
    return fail(RL_ERR_INVALID_ARG, "the image overlaps the data or the normalisation");
  rl_status st = ws_check(plan, batch, d_ws, ws_bytes);
  if (st != RL_OK) return st;
  const EmLayout L = em_layout(plan, batch);
  if (overlaps(d_ws, L.total, d_sino, sb) || overlaps(d_ws, L.total, d_img, ib) || overlaps(d_ws, L.total, d_norm, nb))
    return fail(RL_ERR_INVALID_ARG, "workspace overlaps an argument");
  if ((st = check_plan_device(plan)) != RL_OK) return st;
  char* w = (char*)d_ws;
  float* rf = (float*)(w + L.rf);
  float* back = (float*)(w + L.back);
  const size_t cs = (size_t)batch * d.n_theta * d.n_s, ci = (size_t)batch * d.n * d.n;
  for (int it = 0; it < iters; ++it) {
    if ((st = forward_chain(plan, dense((const float*)d_img, (size_t)d.n * d.n), dense(rf, (size_t)d.n_theta * d.n_s),
                            batch, w + L.chain, -1, nullptr, stream, 1.0)) != RL_OK)
      return st;
    hipLaunchKernelGGL(k_em_ratio, grid_for(cs), dim3(kEThreads), 0, stream, d_sino, rf, cs, d.n_s, d.ds);
    if ((st = check_launch("k_em_ratio")) != RL_OK) return st;
    if ((st = adjoint_chain(plan, dense((const float*)rf, (size_t)d.n_theta * d.n_s), dense(back, (size_t)d.n * d.n),
                            batch, w + L.chain, RL_OP_ADJ, false, stream)) != RL_OK)
      return st;
    hipLaunchKernelGGL(k_em_update, grid_for(ci), dim3(kEThreads), 0, stream, d_img, back, d_norm, ci, d.n);
    if ((st = check_launch("k_em_update")) != RL_OK) return st;
  }
  return RL_OK;
}
