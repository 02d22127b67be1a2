// Autotuner of the execution-only launch parameters (rl_tune) and its cache file.
//
// Each field of rl_tune changes block shapes or schedules only (results are bitwise the same),
// so the tuner may pick any candidate: it times radon_fwd and radon_adj on synthetic slices for
// the candidates of one field at a time (coordinate descent) and keeps the fastest.  The cache
// holds one JSON object per line, keyed by the device architecture, the HIP version, the
// geometry and the batch size.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "rl_internal.h"

namespace rl {
namespace {

// Deterministic fill of the tuner's input buffers: a smooth pattern plus a hash, in [0, 1).
__global__ void k_tune_fill(float* x, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    unsigned h = (unsigned)i * 2654435761u;
    h ^= h >> 15;
    x[i] = (float)(h & 0xffffff) * (1.0f / 16777216.0f);
  }
}

bool tune_valid(const rl_tune& t) {
  return t.theta_cols >= 0 && t.theta_cols <= 8 && (t.theta_xcd_order == 0 || t.theta_xcd_order == 1) &&
         t.prefilter_rows >= 32 && t.prefilter_rows <= 4096 && t.prefilter_rows % 32 == 0 &&
         (t.fwd_patch_split == 0 || t.fwd_patch_split == 1) && (t.fwd_xcd_order == 0 || t.fwd_xcd_order == 1) &&
         (t.adj_walk == 0 || t.adj_walk == 1);
}

std::string cache_key(const rl_plan* p, int batch) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
  }
  int rt = 0;
  (void)hipRuntimeGetVersion(&rt);
  const rl_geom& g = p->g;
  std::ostringstream k;
  k << arch << " rocm=" << rt << " n=" << g.n << " n_theta=" << g.n_theta << " n_s=" << g.n_s << " m=" << g.m
    << " n_rho=" << g.n_rho << " k_theta=" << g.k_theta << " r_dec=" << g.r_dec << " dec_filter=" << g.dec_filter << " q_theta=" << g.q_theta
    << " batch=" << batch;
  return k.str();
}

bool json_int(const std::string& line, const char* field, int* out) {
  const std::string pat = std::string("\"") + field + "\":";
  const size_t at = line.find(pat);
  if (at == std::string::npos) return false;
  const char* s = line.c_str() + at + pat.size();
  char* end = nullptr;
  const long v = std::strtol(s, &end, 10);
  if (end == s) return false;
  *out = (int)v;
  return true;
}

// Look the key up in the cache file: true and *out set if a valid entry is found.
bool cache_lookup(const char* path, const std::string& key, rl_tune* out) {
  std::ifstream in(path);
  if (!in) return false;
  const std::string want = "\"key\": \"" + key + "\"";
  std::string line;
  bool found = false;
  while (std::getline(in, line)) {
    if (line.find(want) == std::string::npos) continue;
    rl_tune t;
    if (json_int(line, "theta_cols", &t.theta_cols) && json_int(line, "theta_xcd_order", &t.theta_xcd_order) &&
        json_int(line, "prefilter_rows", &t.prefilter_rows) && json_int(line, "fwd_patch_split", &t.fwd_patch_split) &&
        json_int(line, "fwd_xcd_order", &t.fwd_xcd_order) && json_int(line, "adj_walk", &t.adj_walk) &&
        tune_valid(t)) {
      *out = t;  // the last valid entry wins
      found = true;
    }
  }
  return found;
}

bool cache_append(const char* path, const std::string& key, const rl_tune& t, float ms_fwd, float ms_adj) {
  std::FILE* f = std::fopen(path, "a");
  if (!f) return false;
  const int n = std::fprintf(f,
                             "{\"key\": \"%s\", \"theta_cols\": %d, \"theta_xcd_order\": %d, \"prefilter_rows\": %d, "
                             "\"fwd_patch_split\": %d, \"fwd_xcd_order\": %d, \"adj_walk\": %d, \"ms_fwd\": %.4f, "
                             "\"ms_adj\": %.4f}\n",
                             key.c_str(), t.theta_cols, t.theta_xcd_order, t.prefilter_rows, t.fwd_patch_split, t.fwd_xcd_order,
                             t.adj_walk,
                             ms_fwd, ms_adj);
  return std::fclose(f) == 0 && n > 0;
}

struct TuneRun {
  rl_plan* p;
  int batch;
  float* img;
  float* sino;
  void* ws;
  size_t ws_bytes;
  hipStream_t s;
  hipEvent_t e0, e1;

  // mean ms of one call of radon_fwd (fwd) or radon_adj over three runs after one warm-up
  rl_status time_op(bool fwd, float* ms) {
    auto call = [&]() {
      return fwd ? radon_fwd(p, img, sino, batch, ws, ws_bytes, s) : radon_adj(p, sino, img, batch, ws, ws_bytes, s);
    };
    rl_status st = call();
    if (st != RL_OK) return st;
    if ((st = check_hip(hipEventRecord(e0, s), "hipEventRecord")) != RL_OK) return st;
    for (int i = 0; i < 3; ++i)
      if ((st = call()) != RL_OK) return st;
    if ((st = check_hip(hipEventRecord(e1, s), "hipEventRecord")) != RL_OK) return st;
    if ((st = check_hip(hipEventSynchronize(e1), "hipEventSynchronize")) != RL_OK) return st;
    float t = 0.f;
    if ((st = check_hip(hipEventElapsedTime(&t, e0, e1), "hipEventElapsedTime")) != RL_OK) return st;
    *ms = t / 3.0f;
    return RL_OK;
  }

  rl_status time_both(float* fwd, float* adj) {
    rl_status st = time_op(true, fwd);
    return st == RL_OK ? time_op(false, adj) : st;
  }
};

}  // namespace

bool tune_from_cache(rl_plan* plan, int batch, const char* path) {
  rl_tune t;
  if (!path || !cache_lookup(path, cache_key(plan, batch), &t)) return false;
  plan->tune = t;
  return true;
}

}  // namespace rl

using namespace rl;

extern "C" rl_status rl_plan_get_tuning(const rl_plan* plan, rl_tune* out) {
  if (!plan || !out) return fail(RL_ERR_INVALID_ARG, "NULL argument");
  *out = plan->tune;
  return RL_OK;
}

extern "C" rl_status rl_plan_set_tuning(rl_plan* plan, const rl_tune* tune) {
  if (!plan || !tune) return fail(RL_ERR_INVALID_ARG, "NULL argument");
  if (!tune_valid(*tune)) return fail(RL_ERR_INVALID_ARG, "launch parameter out of range");
  plan->tune = *tune;
  return RL_OK;
}

extern "C" size_t rl_tune_workspace_bytes(const rl_plan* plan, int32_t batch) {
  if (!plan || batch < 1) return 0;
  const DevPlan& d = plan->d;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t chain = std::max(rl_workspace_bytes(plan, batch, RL_OP_FWD), rl_workspace_bytes(plan, batch, RL_OP_ADJ));
  return al(sizeof(float) * (size_t)batch * d.n * d.n) + al(sizeof(float) * (size_t)batch * d.n_theta * d.n_s) + chain;
}

extern "C" rl_status rl_plan_autotune(rl_plan* plan, int32_t batch, void* d_ws, size_t ws_bytes, hipStream_t stream,
                                      const char* cache_path) {
  if (!plan) return fail(RL_ERR_INVALID_ARG, "plan is NULL");
  if (batch < 1) return fail(RL_ERR_INVALID_ARG, "batch must be >= 1");
  const size_t need = rl_tune_workspace_bytes(plan, batch);
  if (!d_ws || ws_bytes < need)
    return fail(RL_ERR_WORKSPACE, "autotune workspace of " + std::to_string(ws_bytes) + " bytes, need " +
                                      std::to_string(need));
  if (((uintptr_t)d_ws) & 255) return fail(RL_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  rl_status st = check_plan_device(plan);
  if (st != RL_OK) return st;
  const std::string key = cache_key(plan, batch);
  if (cache_path) {
    rl_tune t;
    if (cache_lookup(cache_path, key, &t)) {
      plan->tune = t;
      return RL_OK;
    }
  }
  const DevPlan& d = plan->d;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t ni = (size_t)batch * d.n * d.n, ns = (size_t)batch * d.n_theta * d.n_s;
  char* w = (char*)d_ws;
  TuneRun run{plan, batch, (float*)w, (float*)(w + al(sizeof(float) * ni)), w + al(sizeof(float) * ni) +
              al(sizeof(float) * ns), ws_bytes - al(sizeof(float) * ni) - al(sizeof(float) * ns), stream,
              nullptr, nullptr};
  hipLaunchKernelGGL(k_tune_fill, dim3(1024), dim3(256), 0, stream, run.img, ni);
  hipLaunchKernelGGL(k_tune_fill, dim3(1024), dim3(256), 0, stream, run.sino, ns);
  if ((st = check_launch("k_tune_fill")) != RL_OK) return st;
  if ((st = check_hip(hipEventCreate(&run.e0), "hipEventCreate")) != RL_OK) return st;
  if ((st = check_hip(hipEventCreate(&run.e1), "hipEventCreate")) != RL_OK) {
    (void)hipEventDestroy(run.e0);
    return st;
  }
  const rl_tune start = plan->tune;
  rl_tune best = start;
  float best_f = 0.f, best_a = 0.f;
  st = run.time_both(&best_f, &best_a);
  // candidates of each field (coordinate descent); the objective is the sum of the R and R# times
  const std::vector<std::vector<int>> cands = {{1, 2, 4, 8}, {0, 1}, {128, 256, 512, 1024}, {0, 1}, {0, 1}, {0, 1}};
  for (size_t f = 0; f < cands.size() && st == RL_OK; ++f) {
    for (int v : cands[f]) {
      rl_tune t = best;
      int* field = f == 0   ? &t.theta_cols
                   : f == 1 ? &t.theta_xcd_order
                   : f == 2 ? &t.prefilter_rows
                   : f == 3 ? &t.fwd_patch_split
                   : f == 4 ? &t.fwd_xcd_order
                            : &t.adj_walk;
      if (*field == v) continue;
      *field = v;
      plan->tune = t;
      float tf = 0.f, ta = 0.f;
      if ((st = run.time_both(&tf, &ta)) != RL_OK) break;
      if (tf + ta < best_f + best_a) {
        best = t;
        best_f = tf;
        best_a = ta;
      }
    }
  }
  (void)hipEventDestroy(run.e0);
  (void)hipEventDestroy(run.e1);
  if (st != RL_OK) {
    plan->tune = start;
    return st;
  }
  plan->tune = best;
  if (cache_path && !cache_append(cache_path, key, best, best_f, best_a))
    return fail(RL_ERR_INTERNAL, std::string("cannot append to the tune cache ") + cache_path);
  return RL_OK;
}
