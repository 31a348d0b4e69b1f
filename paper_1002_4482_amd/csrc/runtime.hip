// Host runtime shared by all entry points: option defaults, error strings,
// device properties, workspace and phase timers.
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "pj_internal.hpp"

namespace pj {

static thread_local std::string g_last_hip_error;

void set_last_hip_error(hipError_t e, const char* what, const char* file, int line) {
  g_last_hip_error = std::string(hipGetErrorName(e)) + " (" + hipGetErrorString(e) + ") in " +
                     what + " at " + file + ":" + std::to_string(line);
}

static std::mutex g_dev_mu;
static std::unordered_map<int, DeviceInfo> g_dev;

const DeviceInfo& device_info() {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_dev_mu);
  auto it = g_dev.find(dev);
  if (it != g_dev.end()) return it->second;
  DeviceInfo d;
  d.device = dev;
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) == hipSuccess) {
    d.cus = p.multiProcessorCount;
    d.max_threads_per_cu = p.maxThreadsPerMultiProcessor;
    d.lds_per_block = p.sharedMemPerBlock;
    d.arch = p.gcnArchName;
  }
  return g_dev.emplace(dev, d).first->second;
}

static std::mutex g_occ_mu;
static std::unordered_map<uint64_t, int> g_occ;

int persistent_grid(const void* kernel, int block, size_t lds_bytes) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  uint64_t key = (uint64_t)(uintptr_t)kernel ^ ((uint64_t)block << 48) ^ ((uint64_t)dev << 60) ^
                 ((uint64_t)lds_bytes << 20);
  {
    std::lock_guard<std::mutex> lk(g_occ_mu);
    auto it = g_occ.find(key);
    if (it != g_occ.end()) return it->second;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds_bytes) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  int grid = per_cu * device_info().cus;
  std::lock_guard<std::mutex> lk(g_occ_mu);
  g_occ[key] = grid;
  return grid;
}

int workspace_acquire(Workspace& ws, size_t bytes, const pj_opts* opts, hipStream_t stream) {
  ws.used = 0;
  ws.stream = stream;
  if (opts && opts->workspace) {
    if (opts->workspace_bytes < bytes) return PJ_EINVAL;
    ws.base = static_cast<char*>(opts->workspace);
    ws.size = opts->workspace_bytes;
    ws.owned = false;
    return PJ_OK;
  }
  static std::once_flag pool_once;
  std::call_once(pool_once, [] {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) return;
    for (int d = 0; d < ndev; ++d) {
      hipMemPool_t pool;
      if (hipDeviceGetDefaultMemPool(&pool, d) == hipSuccess) {
        uint64_t keep = UINT64_MAX;  // keep freed blocks cached in the pool
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
      }
    }
  });
  void* p = nullptr;
  size_t want = bytes < 256 ? 256 : bytes;
  hipError_t e = hipMallocAsync(&p, want, stream);
  if (e != hipSuccess) {
    set_last_hip_error(e, "hipMallocAsync(workspace)", __FILE__, __LINE__);
    return e == hipErrorOutOfMemory ? PJ_ENOMEM : PJ_EHIP;
  }
  ws.base = static_cast<char*>(p);
  ws.size = want;
  ws.owned = true;
  return PJ_OK;
}

int workspace_release(Workspace& ws) {
  if (ws.owned && ws.base) {
    PJ_HIP(hipFreeAsync(ws.base, ws.stream));
  }
  ws.base = nullptr;
  ws.owned = false;
  return PJ_OK;
}

// Pinned words are carved from 4 KiB pinned pages that are never freed (a
// flag copy must not wait for the allocation of a page).
static std::mutex g_pin_mu;
static std::vector<int32_t*> g_pin_free;

PinnedWord::PinnedWord() {
  std::lock_guard<std::mutex> lk(g_pin_mu);
  if (g_pin_free.empty()) {
    int32_t* page = nullptr;
    if (hipHostMalloc((void**)&page, 4096, hipHostMallocDefault) != hipSuccess) return;
    for (int i = 0; i < 4096 / 64; ++i) g_pin_free.push_back(page + i * 16);  // 64 B apart
  }
  p_ = g_pin_free.back();
  g_pin_free.pop_back();
}

PinnedWord::~PinnedWord() {
  if (!p_) return;
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pin_free.push_back(p_);
}

int PhaseTimer::begin(bool enable, hipStream_t s) {
  on = enable;
  stream = s;
  n = 0;
  if (!on) return PJ_OK;
  hipEvent_t e = nullptr;
  PJ_HIP(hipEventCreate(&e));
  ev.push_back(e);
  PJ_HIP(hipEventRecord(e, stream));
  return PJ_OK;
}

void PhaseTimer::mark(const char* phase_name) {
  if (!on) return;
  int p = 0;
  while (p < n && strcmp(name[p], phase_name) != 0) ++p;
  if (p == n) {
    if (n >= PJ_MAX_PHASES) return;
    name[n++] = phase_name;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    on = false;  // finish() reports what was recorded so far
    return;
  }
  ev.push_back(e);
  phase_of.push_back(p);
  (void)hipEventRecord(e, stream);
}

int PhaseTimer::finish(pj_stats* st) {
  if (ev.empty()) return PJ_OK;
  PJ_HIP(hipEventSynchronize(ev.back()));
  if (st) {
    float acc[PJ_MAX_PHASES] = {};
    for (size_t j = 0; j < phase_of.size(); ++j) {
      float ms = 0.f;
      PJ_HIP(hipEventElapsedTime(&ms, ev[j], ev[j + 1]));
      acc[phase_of[j]] += ms;
    }
    st->nphases = n;
    for (int i = 0; i < n; ++i) {
      st->phase_ms[i] = acc[i];
      snprintf(st->phase_name[i], sizeof st->phase_name[i], "%s", name[i]);
    }
  }
  return PJ_OK;
}

PhaseTimer::~PhaseTimer() {
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
}

pj_opts resolved_opts(const pj_opts* in) {
  pj_opts o;
  pj_opts_init(&o);
  if (in) o = *in;
  if (o.block <= 0) o.block = 256;
  o.block = (o.block + 63) / 64 * 64;
  if (o.block > 1024) o.block = 1024;
  if (o.spacing <= 0) o.spacing = 16;
  if (o.spacing_up <= 0) o.spacing_up = 4;
  if (o.cutoff <= 0) o.cutoff = 16384;
  if (o.cutoff < 64) o.cutoff = 64;
  if (o.cutoff > 16384) o.cutoff = 16384;
  if (o.max_walk <= 0) o.max_walk = 1024;
  if (o.max_walk < 16) o.max_walk = 16;
  if (o.rounds_per_check <= 0) o.rounds_per_check = 2;
  return o;
}

}  // namespace pj

extern "C" {

void pj_opts_init(pj_opts* o) {
  if (!o) return;
  *o = pj_opts{};
  o->seed = 0x5EED1002449ull;
}

const char* pj_strerror(int code) {
  switch (code) {
    case PJ_OK: return "ok";
    case PJ_EINVAL: return "invalid argument";
    case PJ_ENOMEM: return "out of device memory";
    case PJ_EHIP: return "HIP runtime error";
    case PJ_EBADLIST: return "input is not one linked list per instance";
    case PJ_ENOCONV: return "connected components did not converge within the round guard";
    case PJ_EBUDGET: return "request exceeds the HBM budget";
    case PJ_ENOTFOUND: return "unknown request id";
    case PJ_EBUSY: return "request not finished";
    case PJ_ESHUTDOWN: return "server shutting down";
    case PJ_ESCRATCH: return "input needs more workspace than the no-allocation scratch holds";
    default: return "unknown status";
  }
}

const char* pj_last_hip_error(void) { return pj::g_last_hip_error.c_str(); }

int pj_version(void) { return 10000; }

}  // extern "C"
