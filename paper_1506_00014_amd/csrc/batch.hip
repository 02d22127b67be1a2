// Ragged batches: slices of several geometries.  The slices of one plan run as one batched
// call of its operator chain whose first and last kernels address each slice's own buffer
// through a device table of pointers (built once by rl_batch_create), so no slice is copied.
// The chains of the plans run concurrently: each on a stream of its own (created with the
// batch, default priority), forked from the caller's stream by an event and joined back to it
// by one event per chain, each chain in its own region of the workspace.  Everything after
// rl_batch_create is event records, stream waits and kernel launches, so a call captured on
// the caller's stream becomes one graph with the chains as parallel branches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "rl_internal.h"

using namespace rl;

struct rl_batch {
  struct Group {
    const rl_plan* plan;
    int first, count;    // slices [first, first + count) of the device pointer lists
  };
  int device;
  int count;
  std::vector<Group> groups;
  float** d_ptrs;  // [2][count]: image pointers, then sinogram pointers, in group order
  std::vector<hipStream_t> streams;  // one per group
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> joins;     // one per group
};

namespace {

size_t group_ws(const rl_batch::Group& g, rl_op op) {
  return (rl_workspace_bytes(g.plan, g.count, op) + 255) & ~(size_t)255;
}

// Run `op` (RL_OP_FWD: R, RL_OP_ADJ: R#, RL_OP_BP_LP: Algorithm 2) on the group's slices as
// one batch, reading and writing the slices in place.
rl_status run_group(const rl_batch* b, const rl_batch::Group& g, rl_op op, void* ws, hipStream_t s) {
  float* const* img_tab = b->d_ptrs + g.first;
  float* const* sino_tab = b->d_ptrs + b->count + g.first;
  if (op == RL_OP_FWD)
    return forward_chain(g.plan, Slices<const float>{nullptr, img_tab, 0}, Slices<float>{nullptr, sino_tab, 0},
                         g.count, ws, -1, nullptr, s, 1.0);
  if (op == RL_OP_BP_LP)
    return bp_lp_chain(g.plan, Slices<const float>{nullptr, sino_tab, 0}, Slices<float>{nullptr, img_tab, 0}, g.count,
                       ws, RL_OP_BP_LP, s);
  return adjoint_chain(g.plan, Slices<const float>{nullptr, sino_tab, 0}, Slices<float>{nullptr, img_tab, 0}, g.count,
                       ws, RL_OP_ADJ, false, s);
}

rl_status batch_run(const rl_batch* b, rl_op op, void* d_ws, size_t ws_bytes, hipStream_t s) {
  if (!b) return fail(RL_ERR_INVALID_ARG, "batch is NULL");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(RL_ERR_HIP, "hipGetDevice failed");
  if (dev != b->device) return fail(RL_ERR_INVALID_ARG, "batch was created on another device");
  if (b->count == 0) return RL_OK;
  if (op == RL_OP_BP_LP)
    for (const auto& g : b->groups)
      if (g.plan->d.q != 1)
        return fail(RL_ERR_GEOMETRY, "rl_batch_bp_lp needs q_theta = 1 (its lattice rows are the sinogram rows)");
  const size_t need = rl_batch_workspace_bytes(b, op);
  if (!d_ws || ws_bytes < need) return fail(RL_ERR_WORKSPACE, "workspace smaller than rl_batch_workspace_bytes");
  if (((uintptr_t)d_ws & 255) != 0) return fail(RL_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  rl_status st = check_hip(hipEventRecord(b->fork, s), "hipEventRecord(batch fork)");
  size_t off = 0;
  for (size_t i = 0; i < b->groups.size() && st == RL_OK; ++i) {
    const auto& g = b->groups[i];
    hipStream_t gs = b->streams[i];
    st = check_hip(hipStreamWaitEvent(gs, b->fork, 0), "hipStreamWaitEvent(batch fork)");
    if (st != RL_OK) break;
    st = run_group(b, g, op, (char*)d_ws + off, gs);
    // a chain that was forked is joined back even when one of its launches failed
    rl_status jt = check_hip(hipEventRecord(b->joins[i], gs), "hipEventRecord(batch join)");
    if (jt == RL_OK) jt = check_hip(hipStreamWaitEvent(s, b->joins[i], 0), "hipStreamWaitEvent(batch join)");
    if (st == RL_OK) st = jt;
    off += group_ws(g, op);
  }
  return st;
}

}  // namespace

extern "C" rl_status rl_batch_create(const rl_plan* const* plans, int32_t nplans, const int32_t* plan_of_slice,
                                     float* const* d_imgs, float* const* d_sinos, int32_t count,
                                     const char* tune_cache, rl_batch** out) {
  if (!out) return fail(RL_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
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
    for (int i = 0; i < count; ++i) {
      if (plan_of_slice[i] != p) continue;
      ptrs[k] = d_imgs[i];
      ptrs[count + k] = d_sinos[i];
      ++k;
      ++g.count;
    }
    if (g.count == 0) continue;
    b->groups.push_back(g);
  }
  {
    // the chains' streams (default priority, not synchronising with the null stream) and events
    rl_status st = check_hip(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming), "hipEventCreate(batch)");
    for (size_t i = 0; i < b->groups.size() && st == RL_OK; ++i) {
      hipStream_t gs = nullptr;
      hipEvent_t ev = nullptr;
      st = check_hip(hipStreamCreateWithFlags(&gs, hipStreamNonBlocking), "hipStreamCreate(batch)");
      if (st == RL_OK) b->streams.push_back(gs);
      if (st == RL_OK) st = check_hip(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate(batch)");
      if (st == RL_OK) b->joins.push_back(ev);
    }
    if (st != RL_OK) {
      rl_batch_destroy(b);
      return st;
    }
  }
  if (count > 0) {
    rl_status st = check_hip(hipMalloc((void**)&b->d_ptrs, sizeof(float*) * ptrs.size()), "hipMalloc(batch)");
    if (st == RL_OK)
      st = check_hip(hipMemcpy(b->d_ptrs, ptrs.data(), sizeof(float*) * ptrs.size(), hipMemcpyHostToDevice),
                     "upload batch pointers");
    if (st != RL_OK) {
      rl_batch_destroy(b);
      return st;
    }
  }
  if (tune_cache) {
    // launch parameters of each plan for its slice count: from the cache, else tuned now (with a
    // temporary workspace, on the null stream) and appended to it
    for (const auto& g : b->groups) {
      rl_plan* p = const_cast<rl_plan*>(g.plan);  // only its execution-only launch parameters change
      if (tune_from_cache(p, g.count, tune_cache)) continue;
      const size_t need = rl_tune_workspace_bytes(p, g.count);
      void* tmp = nullptr;
      rl_status st = check_hip(hipMalloc(&tmp, need), "hipMalloc(autotune workspace)");
      if (st == RL_OK) st = rl_plan_autotune(p, g.count, tmp, need, nullptr, tune_cache);
      if (tmp) (void)hipFree(tmp);
      if (st != RL_OK) {
        rl_batch_destroy(b);
        return st;
      }
    }
  }
  *out = b;
  return RL_OK;
}

extern "C" size_t rl_batch_workspace_bytes(const rl_batch* batch, rl_op op) {
  if (!batch) return 0;
  size_t need = 0;  // the chains run concurrently: one region each
  for (const auto& g : batch->groups) need += group_ws(g, op);
  return need;
}

extern "C" rl_status rl_batch_fwd(const rl_batch* batch, void* d_ws, size_t ws_bytes, hipStream_t stream) {
  return batch_run(batch, RL_OP_FWD, d_ws, ws_bytes, stream);
}

extern "C" rl_status rl_batch_adj(const rl_batch* batch, void* d_ws, size_t ws_bytes, hipStream_t stream) {
  return batch_run(batch, RL_OP_ADJ, d_ws, ws_bytes, stream);
}

extern "C" rl_status rl_batch_bp_lp(const rl_batch* batch, void* d_ws, size_t ws_bytes, hipStream_t stream) {
  return batch_run(batch, RL_OP_BP_LP, d_ws, ws_bytes, stream);
}

extern "C" void rl_batch_destroy(rl_batch* batch) {
  if (!batch) return;
  if (batch->d_ptrs) (void)hipFree(batch->d_ptrs);
  for (hipStream_t gs : batch->streams) (void)hipStreamDestroy(gs);
  for (hipEvent_t ev : batch->joins) (void)hipEventDestroy(ev);
  if (batch->fork) (void)hipEventDestroy(batch->fork);
  delete batch;
}
