// List ranking that allocates nothing: pj_list_rank_noalloc runs the same
// plan and kernels as pj_list_rank_ex, with its workspace (the control block,
// the level tables and the splitter ranks) carved from a fixed device array
// of this file instead of the device memory pool.
//
// `scratch` is a device symbol: in host code its name is only a stand-in, so
// host code never passes it to a kernel or a copy.  The first call on each
// device, with that device current, looks up the array's device address with
// hipGetSymbolAddress and keeps it per device (each GPU holds its own copy of
// the array at its own address); every later use goes through that address.
// The kernels receive it as the workspace they take in pj_list_rank_ex, and
// they write every word of it before reading it (the pool's memory is
// recycled with old contents too), so the previous call's contents never
// reach a result.
#include <mutex>

#include "pj_internal.hpp"

namespace pj {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array, looked up once per device.
int scratch_address(void** out) {
  int dev = 0;
  PJ_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return PJ_EINVAL;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    PJ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return PJ_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PJ_OK;
}

}  // namespace
}  // namespace pj

extern "C" {

size_t pj_list_rank_noalloc_max_bytes(void) { return pj::kScratchBytes; }

int pj_list_rank_noalloc(const int32_t* succ, int64_t n, int32_t* rank, const pj_opts* opts,
                         pj_stream_t stream) {
  if (n < 0) return PJ_EINVAL;
  pj_opts o;
  pj_opts_init(&o);
  if (opts) o = *opts;
  // options that allocate (a caller workspace is not needed here, the graph
  // cache, the phase timers) or read a status back through host memory
  if (o.workspace || o.workspace_bytes || o.use_graph || o.stats || (o.validate && !o.d_status))
    return PJ_EINVAL;
  // host-side size check before anything touches the device
  if (pj::list_rank_workspace(n, 1, &o, true) > pj::kScratchBytes) return PJ_ESCRATCH;
  if (n == 0 && !o.d_status) return PJ_OK;
  void* ws = nullptr;
  PJ_TRY(pj::scratch_address(&ws));
  o.workspace = ws;
  o.workspace_bytes = pj::kScratchBytes;
  return pj::list_rank_impl(succ, nullptr, 1, nullptr, n, rank, &o, (hipStream_t)stream);
}

}  // extern "C"
