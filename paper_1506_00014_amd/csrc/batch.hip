// Ragged batches: slices of several geometries in one call per plan.  The slices of a plan
// are gathered from their buffers into a contiguous block of the workspace, transformed by
// one batched call, and the results scattered back.  Everything after rl_batch_create is a
// kernel launch on the caller's stream (graph-capturable).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "rl_internal.h"

namespace rl {
namespace {

// dst[s][i] = src[s][i] (gather: src through a pointer list) or dst[s][i] = src[s][i]
// (scatter: dst through a pointer list), slice s = blockIdx.y.
__global__ __launch_bounds__(kThreads) void k_gather(const float* const* __restrict__ src, float* __restrict__ dst,
                                                     size_t elems, int vec4) {
  const float* s = src[blockIdx.y];
  float* d = dst + (size_t)blockIdx.y * elems;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (vec4) {
    for (size_t i = t0; i < elems / 4; i += stride)
      reinterpret_cast<float4*>(d)[i] = reinterpret_cast<const float4*>(s)[i];
  } else {
    for (size_t i = t0; i < elems; i += stride) d[i] = s[i];
  }
}

__global__ __launch_bounds__(kThreads) void k_scatter(const float* __restrict__ src, float* const* __restrict__ dst,
                                                      size_t elems, int vec4) {
  const float* s = src + (size_t)blockIdx.y * elems;
  float* d = dst[blockIdx.y];
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (vec4) {
    for (size_t i = t0; i < elems / 4; i += stride)
      reinterpret_cast<float4*>(d)[i] = reinterpret_cast<const float4*>(s)[i];
  } else {
    for (size_t i = t0; i < elems; i += stride) d[i] = s[i];
  }
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace
}  // namespace rl

using namespace rl;

struct rl_batch {
  struct Group {
    const rl_plan* plan;
    int first, count;    // slices [first, first + count) of the device pointer lists
    size_t img_elems, sino_elems;
    bool img_vec4, sino_vec4;  // all buffers 16-byte aligned and whole float4 rows
  };
  int device;
  int count;
  std::vector<Group> groups;
  float** d_ptrs;  // [2][count]: image pointers, then sinogram pointers, in group order
};

namespace {

size_t group_ws(const rl_batch::Group& g, rl_op op) {
  const size_t io = al256(sizeof(float) * g.img_elems * g.count) + al256(sizeof(float) * g.sino_elems * g.count);
  return io + rl_workspace_bytes(g.plan, g.count, op);
}

// Gather the group's inputs, run `op` on them as one batch, scatter the outputs.
rl_status run_group(const rl_batch* b, const rl_batch::Group& g, bool fwd, char* ws, size_t ws_bytes,
                    hipStream_t s) {
  float* imgs = reinterpret_cast<float*>(ws);
  float* sinos = reinterpret_cast<float*>(ws + al256(sizeof(float) * g.img_elems * g.count));
  char* rest = ws + al256(sizeof(float) * g.img_elems * g.count) + al256(sizeof(float) * g.sino_elems * g.count);
  const size_t rest_bytes = ws_bytes - (size_t)(rest - ws);
  float** img_ptrs = b->d_ptrs + g.first;
  float** sino_ptrs = b->d_ptrs + b->count + g.first;
  auto blocks = [](size_t elems) { return dim3((unsigned)std::min<size_t>((elems / 4 + kThreads - 1) / kThreads + 1, 1024)); };
  rl_status st;
  if (fwd) {
    dim3 gi = blocks(g.img_elems);
    gi.y = g.count;
    RL_LAUNCH("k_gather", k_gather, gi, dim3(kThreads), 0, s, (const float* const*)img_ptrs, imgs, g.img_elems,
              g.img_vec4 ? 1 : 0);
    if ((st = check_launch("k_gather")) != RL_OK) return st;
    if ((st = radon_fwd(g.plan, imgs, sinos, g.count, rest, rest_bytes, s)) != RL_OK) return st;
    dim3 go = blocks(g.sino_elems);
    go.y = g.count;
    RL_LAUNCH("k_scatter", k_scatter, go, dim3(kThreads), 0, s, sinos, sino_ptrs, g.sino_elems, g.sino_vec4 ? 1 : 0);
    return check_launch("k_scatter");
  }
  dim3 gi = blocks(g.sino_elems);
  gi.y = g.count;
  RL_LAUNCH("k_gather", k_gather, gi, dim3(kThreads), 0, s, (const float* const*)sino_ptrs, sinos, g.sino_elems,
            g.sino_vec4 ? 1 : 0);
  if ((st = check_launch("k_gather")) != RL_OK) return st;
  if ((st = radon_adj(g.plan, sinos, imgs, g.count, rest, rest_bytes, s)) != RL_OK) return st;
  dim3 go = blocks(g.img_elems);
  go.y = g.count;
  RL_LAUNCH("k_scatter", k_scatter, go, dim3(kThreads), 0, s, imgs, img_ptrs, g.img_elems, g.img_vec4 ? 1 : 0);
  return check_launch("k_scatter");
}

rl_status batch_run(const rl_batch* b, bool fwd, void* d_ws, size_t ws_bytes, hipStream_t s) {
  if (!b) return fail(RL_ERR_INVALID_ARG, "batch is NULL");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(RL_ERR_HIP, "hipGetDevice failed");
  if (dev != b->device) return fail(RL_ERR_INVALID_ARG, "batch was created on another device");
  if (b->count == 0) return RL_OK;
  const size_t need = rl_batch_workspace_bytes(b, fwd ? RL_OP_FWD : RL_OP_ADJ);
  if (!d_ws || ws_bytes < need) return fail(RL_ERR_WORKSPACE, "workspace smaller than rl_batch_workspace_bytes");
  if (((uintptr_t)d_ws & 255) != 0) return fail(RL_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  for (const auto& g : b->groups) {
    rl_status st = run_group(b, g, fwd, static_cast<char*>(d_ws), ws_bytes, s);
    if (st != RL_OK) return st;
  }
  return RL_OK;
}

}  // namespace

extern "C" rl_status rl_batch_create(const rl_plan* const* plans, int32_t nplans, const int32_t* plan_of_slice,
                                     float* const* d_imgs, float* const* d_sinos, int32_t count,
                                     const char* tune_cache, rl_batch** out) {
  if (!out) return fail(RL_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (tune_cache) return fail(RL_ERR_INVALID_ARG, "tune_cache is reserved and must be NULL");
  if (count < 0 || nplans < 0) return fail(RL_ERR_INVALID_ARG, "negative count");
  if (count > 0 && (!plans || !plan_of_slice || !d_imgs || !d_sinos))
    return fail(RL_ERR_INVALID_ARG, "NULL list");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(RL_ERR_HIP, "hipGetDevice failed");
  for (int i = 0; i < count; ++i) {
    const int p = plan_of_slice[i];
    if (p < 0 || p >= nplans || !plans[p]) return fail(RL_ERR_INVALID_ARG, "plan index out of range or NULL plan");
    if (plans[p]->device != dev) return fail(RL_ERR_INVALID_ARG, "plan built on another device");
    if (!d_imgs[i] || !d_sinos[i]) return fail(RL_ERR_INVALID_ARG, "NULL slice buffer");
  }
  auto* b = new rl_batch;
  b->device = dev;
  b->count = count;
  b->d_ptrs = nullptr;
  std::vector<float*> ptrs(2 * (size_t)count);
  int k = 0;
  for (int p = 0; p < nplans; ++p) {
    rl_batch::Group g;
    g.plan = plans[p];
    g.first = k;
    g.count = 0;
    g.img_vec4 = g.sino_vec4 = true;
    for (int i = 0; i < count; ++i) {
      if (plan_of_slice[i] != p) continue;
      ptrs[k] = d_imgs[i];
      ptrs[count + k] = d_sinos[i];
      g.img_vec4 = g.img_vec4 && ((uintptr_t)d_imgs[i] & 15) == 0;
      g.sino_vec4 = g.sino_vec4 && ((uintptr_t)d_sinos[i] & 15) == 0;
      ++k;
      ++g.count;
    }
    if (g.count == 0) continue;
    g.img_elems = (size_t)g.plan->d.n * g.plan->d.n;
    g.sino_elems = (size_t)g.plan->d.n_theta * g.plan->d.n_s;
    g.img_vec4 = g.img_vec4 && g.img_elems % 4 == 0;
    g.sino_vec4 = g.sino_vec4 && g.sino_elems % 4 == 0;
    b->groups.push_back(g);
  }
  if (count > 0) {
    rl_status st = check_hip(hipMalloc((void**)&b->d_ptrs, sizeof(float*) * ptrs.size()), "hipMalloc(batch)");
    if (st == RL_OK)
      st = check_hip(hipMemcpy(b->d_ptrs, ptrs.data(), sizeof(float*) * ptrs.size(), hipMemcpyHostToDevice),
                     "upload batch pointers");
    if (st != RL_OK) {
      if (b->d_ptrs) (void)hipFree(b->d_ptrs);
      delete b;
      return st;
    }
  }
  *out = b;
  return RL_OK;
}

extern "C" size_t rl_batch_workspace_bytes(const rl_batch* batch, rl_op op) {
  if (!batch) return 0;
  size_t need = 0;
  for (const auto& g : batch->groups) need = std::max(need, group_ws(g, op));
  return need;
}

extern "C" rl_status rl_batch_fwd(const rl_batch* batch, void* d_ws, size_t ws_bytes, hipStream_t stream) {
  return batch_run(batch, true, d_ws, ws_bytes, stream);
}

extern "C" rl_status rl_batch_adj(const rl_batch* batch, void* d_ws, size_t ws_bytes, hipStream_t stream) {
  return batch_run(batch, false, d_ws, ws_bytes, stream);
}

extern "C" void rl_batch_destroy(rl_batch* batch) {
  if (!batch) return;
  if (batch->d_ptrs) (void)hipFree(batch->d_ptrs);
  delete batch;
}
