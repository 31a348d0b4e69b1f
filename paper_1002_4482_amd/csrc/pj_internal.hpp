// Internal helpers shared by the gfx950 kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "ptrjump.h"

namespace pj {

constexpr int kWave = 64;

// ------------------------------------------------------------------ errors
// Device-side error bits, OR-ed into a control word and turned into
// PJ_EBADLIST / PJ_ENOCONV at the end of a call.
enum : int32_t {
  kErrRange = 1,     // a successor outside its instance
  kErrTails = 2,     // an instance without exactly one tail
  kErrHead = 4,      // head by index sum is not a node
  kErrOverflow = 8,  // too many cut points: a cycle without splitters
  kErrBase = 16,     // the splitter list is not a list (branch or cycle)
  kErrTotal = 32,    // sublists do not cover every node exactly once
  kErrCheck = 64,    // the full output check failed
  kErrNoConv = 128,  // components: round guard reached
  kErrSplitter = 256,  // a caller-chosen splitter out of range or repeated
};

void set_last_hip_error(hipError_t e, const char* what, const char* file, int line);

#define PJ_HIP(expr)                                                   \
  do {                                                                 \
    hipError_t pj_e_ = (expr);                                         \
    if (pj_e_ != hipSuccess) {                                         \
      ::pj::set_last_hip_error(pj_e_, #expr, __FILE__, __LINE__);      \
      return PJ_EHIP;                                                  \
    }                                                                  \
  } while (0)

#define PJ_TRY(expr)             \
  do {                           \
    int pj_rc_ = (expr);         \
    if (pj_rc_ != PJ_OK) return pj_rc_; \
  } while (0)

// ------------------------------------------------------------ device info
struct DeviceInfo {
  int device = -1;
  int cus = 256;
  int max_threads_per_cu = 2048;
  size_t lds_per_block = 65536;
  std::string arch;
};
const DeviceInfo& device_info();

// Number of workgroups of `block` threads that fill the current device for a
// kernel (cached by kernel address).
int persistent_grid(const void* kernel, int block, size_t lds_bytes);

// ---------------------------------------------------------------- workspace
// A bump allocator over one device buffer, either the caller's or one taken
// stream-ordered from the device memory pool for the duration of the call.
// Bump allocator over one workspace.  A workspace the library allocated is
// freed (stream-ordered) by workspace_release, or by the destructor when an
// error path returns early.
struct Workspace {
  char* base = nullptr;
  size_t size = 0;
  size_t used = 0;
  bool owned = false;
  hipStream_t stream = nullptr;

  Workspace() = default;
  Workspace(const Workspace&) = delete;
  Workspace& operator=(const Workspace&) = delete;
  ~Workspace() {
    if (owned && base) (void)hipFreeAsync(base, stream);
  }

  template <typename T>
  T* take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    if (used + bytes > size) return nullptr;
    T* p = reinterpret_cast<T*>(base + used);
    used += bytes;
    return p;
  }
};

// Round a byte count up to the 256-byte granule used by Workspace::take.
inline size_t ws_bytes(size_t count, size_t elem) { return (count * elem + 255) & ~size_t(255); }

int workspace_acquire(Workspace& ws, size_t bytes, const pj_opts* opts, hipStream_t stream);
int workspace_release(Workspace& ws);

// One pinned host word for a device-to-host flag copy, from a process-wide
// pool (released on destruction; the pool never shrinks, and holds as many
// words as calls ever ran at once).
class PinnedWord {
 public:
  PinnedWord();
  ~PinnedWord();
  PinnedWord(const PinnedWord&) = delete;
  PinnedWord& operator=(const PinnedWord&) = delete;
  int32_t* get() const { return p_; }

 private:
  int32_t* p_ = nullptr;
};

// ------------------------------------------------------------ phase timing
// Device time per named phase.  Each mark closes the interval since the last
// one and adds it to the phase of that name, so a phase marked once per round
// or per level accumulates over all of them (at most PJ_MAX_PHASES names).
struct PhaseTimer {
  bool on = false;
  hipStream_t stream = nullptr;
  int n = 0;                             // distinct phase names
  const char* name[PJ_MAX_PHASES] = {};
  std::vector<hipEvent_t> ev;            // ev[0] = begin, ev[j + 1] closes mark j
  std::vector<int> phase_of;             // phase index of mark j
  int begin(bool enable, hipStream_t s);
  void mark(const char* phase_name);
  int finish(pj_stats* st);              // synchronises, fills phase times
  ~PhaseTimer();
};

// Resolve option defaults.
pj_opts resolved_opts(const pj_opts* in);

// List ranking entry shared by the plain, batched, graph and tuning paths.
// d_off == nullptr means one list of n_single nodes.
// weight != nullptr: weighted ranks (exclusive prefix sums of the weights).
int list_rank_impl(const int32_t* succ, const int64_t* d_off, int64_t L, const int64_t* h_off,
                   int64_t n_single, int32_t* rank, const pj_opts* user, hipStream_t stream,
                   const int32_t* weight = nullptr);
size_t list_rank_workspace(int64_t n0, int64_t L, const pj_opts* user, bool single,
                           bool weighted = false);
int list_rank_default_spacing(int64_t n, bool single);
int level0_spacing(int requested, int64_t n0, bool single, int32_t* planned);

// Tuned ruling-set parameters for a problem of n0 nodes in L lists, if the
// tune cache holds an entry for its size class; fills the zero fields of o.
void apply_tuned(pj_opts& o, int64_t n0, int64_t L);

// Frees the captured components graphs (synchronises the device).
void cc_graph_cache_clear();

// Batched list ranking through the captured-graph cache (h_off required).
int graph_batched(const int32_t* succ, const int64_t* d_off, int64_t L, const int64_t* h_off,
                  int32_t* rank, const pj_opts& user, hipStream_t stream);

// ---------------------------------------------------------- device helpers
// 32-bit finaliser of MurmurHash3 (Appleby), used as a counter-based hash to
// place one splitter per block of node ids.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x85ebca6bu;
  x ^= x >> 13;
  x *= 0xc2b2ae35u;
  x ^= x >> 16;
  return x;
}

__host__ __device__ __forceinline__ uint32_t level_seed(uint64_t seed, int level) {
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(level + 1);  // SplitMix64 step
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return (uint32_t)(z ^ (z >> 31));
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Number of active lanes below this one in `mask`.
__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T u = __shfl_xor(v, o, kWave);
    v = u < v ? u : v;
  }
  return v;
}

// Index of the instance owning global position g: largest l with off[l] <= g
// (off is non-decreasing, off[0] == 0, off[L] > g).
__device__ __forceinline__ int find_instance(const int64_t* __restrict__ off, int L, int64_t g) {
  int lo = 0, hi = L - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Device-scope relaxed atomic store: written through to the device-coherent
// level, so a store from one XCD is not lost behind another XCD's
// write-back L2 when several workgroups write the same word.
__device__ __forceinline__ void publish(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Device-scope relaxed load: sees what `publish` wrote from any XCD.
__device__ __forceinline__ int32_t load_coherent(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Raises a per-round flag (change or stagnant-root flag) from a workgroup-
// wide OR.  Thousands of waves raise the same word in one kernel; a
// write-through store per wave would serialise on that word, so a workgroup
// stores at most once, and not at all once a coherent load shows it set.
// Every thread of the workgroup must call it.
__device__ __forceinline__ void raise_flag(int32_t* flag, bool mine) {
  if (__syncthreads_or(mine) && threadIdx.x == 0 &&
      __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
    publish(flag, 1);
}

}  // namespace pj
