// radon_fwd_noalloc: radon_fwd with its workspace in a file-scope device array instead of a
// caller-provided buffer, for callers that cannot allocate device memory.
//
// The array `scratch` below is one copy per GPU, created when the code object is loaded on that
// GPU and held until the process ends.  In host code its name is only a host-side stand-in:
// the device address of each GPU's copy is looked up once per GPU with hipGetSymbolAddress
// (with that GPU current) and only that address is handed to the kernels.  The forward chain
// overwrites every workspace word it reads, so nothing in the array has to start at zero.
// Every call on one GPU uses that GPU's single copy: calls that overlap in time on one GPU
// (several streams, several host threads) race on it and must be serialised by the caller.
#include <mutex>

#include "rl_internal.h"

namespace {

static_assert(RL_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size must keep 256-byte alignment");

static __device__ __align__(256) unsigned char scratch[RL_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of each GPU's copy (nullptr until looked up)

// Device address of the current GPU's copy of `scratch`, looked up on the first call per GPU.
rl_status scratch_address(void** out) {
  int dev = -1;
  rl_status st = rl::check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (st != RL_OK) return st;
  if (dev < 0 || dev >= kMaxDevices) return rl::fail(RL_ERR_INTERNAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    st = rl::check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (st != RL_OK) return st;
    if (!p || (reinterpret_cast<uintptr_t>(p) & 255))
      return rl::fail(RL_ERR_INTERNAL, "scratch array has no 256-byte aligned device address");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return RL_OK;
}

}  // namespace

extern "C" rl_status radon_fwd_noalloc(const rl_plan* plan, const float* d_img, float* d_sino, int32_t batch,
                                       hipStream_t stream) {
  if (!plan) return rl::fail(RL_ERR_INVALID_ARG, "plan is NULL");
  if (batch < 0) return rl::fail(RL_ERR_INVALID_ARG, "batch is negative");
  if (batch == 0) return RL_OK;
  const size_t need = rl_workspace_bytes(plan, batch, RL_OP_FWD);
  if (need > (size_t)RL_NOALLOC_SCRATCH_BYTES)
    return rl::fail(RL_ERR_WORKSPACE, "radon_fwd_noalloc: " + std::to_string(batch) + " slices of this plan need " +
                                          std::to_string(need) + " bytes of workspace, more than the " +
                                          std::to_string((size_t)RL_NOALLOC_SCRATCH_BYTES) +
                                          "-byte static scratch; use radon_fwd with a workspace or fewer slices");
  rl_status st = rl::check_plan_device(plan);
  if (st != RL_OK) return st;
  void* ws = nullptr;
  if ((st = scratch_address(&ws)) != RL_OK) return st;
  return radon_fwd(plan, d_img, d_sino, batch, ws, (size_t)RL_NOALLOC_SCRATCH_BYTES, stream);
}
