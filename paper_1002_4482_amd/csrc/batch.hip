// Batched list ranking as one replayed hipGraph, and the autotuner that picks
// the ruling-set parameters (splitter spacing per level, LDS cutoff).
//
// Graph replay: the whole launch sequence of a batched solve (init, head find,
// the persistent walks of every level, the base ranking and the expansions)
// is captured once per (buffers, sizes, options) on a private stream with a
// workspace the cache owns, and later calls launch the instantiated graph on
// the caller's stream: one hipGraphLaunch instead of ~15 kernel launches.
//
// Tuning: candidate parameter sets are timed with HIP events on the caller's
// input; the fastest is stored in a cache keyed by (gfx arch, size class of
// the node count, size class of the list count).  Calls that leave a
// parameter at zero take it from the cache.  The cache can be saved to and
// loaded from a text file (and is loaded from $PJ_TUNE_CACHE on first use).
#include <algorithm>
#include <array>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "pj_internal.hpp"

namespace pj {
namespace {

int bits_for(int64_t v) {
  int b = 0;
  while ((int64_t(1) << b) < v) ++b;
  return b;
}

// ------------------------------------------------------------ tune cache
struct Tuned {
  int spacing, spacing_up, cutoff, max_walk, block;
  float ms;
};
using TuneKey = std::tuple<std::string, int, int>;

std::mutex g_tune_mu;
std::map<TuneKey, Tuned> g_tune;
bool g_tune_env_loaded = false;
int64_t g_tune_gen = 0;  // bumped on every change, part of the graph cache key

int load_locked(const char* path) {
  FILE* f = fopen(path, "r");
  if (!f) return PJ_EINVAL;
  char arch[128];
  int nb, lb;
  Tuned t;
  while (fscanf(f, "%127s %d %d %d %d %d %d %d %f", arch, &nb, &lb, &t.spacing, &t.spacing_up,
                &t.cutoff, &t.max_walk, &t.block, &t.ms) == 9)
    g_tune[TuneKey(arch, nb, lb)] = t;
  ++g_tune_gen;
  fclose(f);
  return PJ_OK;
}

TuneKey tune_key(int64_t n0, int64_t L) {
  return TuneKey(device_info().arch, bits_for(std::max<int64_t>(n0, 1)),
                 bits_for(std::max<int64_t>(L, 1)));
}

// ----------------------------------------------------------- graph cache
using GraphKey = std::array<int64_t, 19>;
struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  void* ws = nullptr;
  uint64_t last_used = 0;
};
std::mutex g_graph_mu;
std::map<GraphKey, GraphEntry> g_graphs;
uint64_t g_graph_clock = 0;
constexpr size_t kMaxGraphs = 8;
std::map<int, hipStream_t> g_capture_stream;

void drop_entry(GraphEntry& e) {
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (e.ws) (void)hipFree(e.ws);
  e.exec = nullptr;
  e.ws = nullptr;
}

}  // namespace

void apply_tuned(pj_opts& o, int64_t n0, int64_t L) {
  if (o.spacing > 0 && o.spacing_up > 0 && o.cutoff > 0 && o.max_walk > 0 && o.block > 0) return;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (!g_tune_env_loaded) {
    g_tune_env_loaded = true;
    if (const char* p = getenv("PJ_TUNE_CACHE")) (void)load_locked(p);
  }
  if (g_tune.empty()) return;
  auto it = g_tune.find(tune_key(n0, L));
  if (it == g_tune.end()) return;
  const Tuned& t = it->second;
  if (o.spacing <= 0) o.spacing = t.spacing;
  if (o.spacing_up <= 0) o.spacing_up = t.spacing_up;
  if (o.cutoff <= 0) o.cutoff = t.cutoff;
  if (o.max_walk <= 0) o.max_walk = t.max_walk;
  if (o.block <= 0) o.block = t.block;
}

int graph_batched(const int32_t* succ, const int64_t* d_off, int64_t L, const int64_t* h_off,
                  int32_t* rank, const pj_opts& user, hipStream_t stream) {
  int64_t n0 = h_off[L];
  // The captured plan depends on the offsets only through the node total, the
  // list count and (Wyllie) the round count ceil(log2) of the largest list;
  // the kernels read the offsets' contents at replay time.
  int64_t max_size = 0;
  for (int64_t l = 0; l < L; ++l) max_size = std::max(max_size, h_off[l + 1] - h_off[l]);
  int dev = 0;
  PJ_HIP(hipGetDevice(&dev));
  GraphKey key{dev,
               (int64_t)(uintptr_t)succ,
               (int64_t)(uintptr_t)d_off,
               (int64_t)(uintptr_t)rank,
               (int64_t)(uintptr_t)user.d_status,
               L,
               n0,
               user.algo,
               user.spacing,
               user.spacing_up,
               user.cutoff,
               user.max_walk,
               user.to_tail,
               user.validate,
               (int64_t)user.seed,
               user.block,
               0,
               bits_for(std::max<int64_t>(max_size, 1)),
               user.level0_state};
  {
    std::lock_guard<std::mutex> tl(g_tune_mu);
    key[16] = g_tune_gen;  // zero parameters may resolve differently after a retune
  }
  std::lock_guard<std::mutex> lk(g_graph_mu);
  auto it = g_graphs.find(key);
  if (it == g_graphs.end()) {
    if (g_graphs.size() >= kMaxGraphs) {  // evict the least recently used
      auto lru = g_graphs.begin();
      for (auto j = g_graphs.begin(); j != g_graphs.end(); ++j)
        if (j->second.last_used < lru->second.last_used) lru = j;
      drop_entry(lru->second);
      g_graphs.erase(lru);
    }
    hipStream_t& cap = g_capture_stream[dev];
    if (!cap) PJ_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    GraphEntry e;
    pj_opts o = user;
    o.use_graph = 0;
    o.stats = nullptr;
    o.h_offsets = h_off;
    const size_t bytes = std::max<size_t>(list_rank_workspace(n0, L, &o, false), 256);
    PJ_HIP(hipMalloc(&e.ws, bytes));
    o.workspace = e.ws;
    o.workspace_bytes = bytes;
    hipGraph_t graph = nullptr;
    hipError_t he = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (he != hipSuccess) {
      drop_entry(e);
      set_last_hip_error(he, "hipStreamBeginCapture", __FILE__, __LINE__);
      return PJ_EHIP;
    }
    const int rc = list_rank_impl(succ, d_off, L, h_off, 0, rank, &o, cap);
    he = hipStreamEndCapture(cap, &graph);
    if (rc != PJ_OK || he != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      drop_entry(e);
      if (rc != PJ_OK) return rc;
      set_last_hip_error(he, "hipStreamEndCapture", __FILE__, __LINE__);
      return PJ_EHIP;
    }
    he = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (he != hipSuccess) {
      drop_entry(e);
      set_last_hip_error(he, "hipGraphInstantiate", __FILE__, __LINE__);
      return PJ_EHIP;
    }
    it = g_graphs.emplace(key, e).first;
  }
  it->second.last_used = ++g_graph_clock;
  PJ_HIP(hipGraphLaunch(it->second.exec, stream));
  return PJ_OK;
}

}  // namespace pj

extern "C" {

int pj_tune_list_rank(const int32_t* succ, const int64_t* offsets, int64_t L,
                      const int64_t* h_offsets, int64_t n, pj_opts* best, float* best_ms,
                      pj_stream_t stream) {
  hipStream_t s = (hipStream_t)stream;
  const bool single = offsets == nullptr;
  if (single) L = 1;
  if (L < 1 || (!single && !h_offsets)) return PJ_EINVAL;
  const int64_t n0 = single ? n : h_offsets[L];
  if (n0 < 0 || n0 >= INT32_MAX || (n0 > 0 && !succ)) return PJ_EINVAL;
  // scratch output and timing events, released on every return path
  struct Scratch {
    hipStream_t s;
    int32_t* out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Scratch() {
      if (out) (void)hipFreeAsync(out, s);
      (void)hipStreamSynchronize(s);
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } scratch{s};
  PJ_HIP(hipMallocAsync((void**)&scratch.out, (size_t)std::max<int64_t>(n0, 1) * 4, s));
  PJ_HIP(hipEventCreate(&scratch.e0));
  PJ_HIP(hipEventCreate(&scratch.e1));
  int32_t* out = scratch.out;
  hipEvent_t e0 = scratch.e0, e1 = scratch.e1;
  // Coordinate descent from the library defaults: first-level spacing, then
  // recursion spacing, LDS cutoff and workgroup size, each swept with the
  // others held at their best so far (1 warm-up and 3 timed solves each).
  pj::Tuned cur{0, 4, 16384, 1024, 256, 1e30f};
  cur.spacing = pj::list_rank_default_spacing(n0, single);
  const std::vector<int> sweeps[4] = {{8, 16, 32, 64, 128, 256},
                                      {4, 8, 16},
                                      {2048, 4096, 8192, 16384},
                                      {128, 256, 512, 1024}};
  int rc = PJ_OK;
  auto time_one = [&](const pj::Tuned& t, float* ms_out) -> int {
    pj_opts o;
    pj_opts_init(&o);
    o.algo = PJ_ALGO_RULING_SET;
    o.spacing = t.spacing;
    o.spacing_up = t.spacing_up;
    o.cutoff = t.cutoff;
    o.max_walk = t.max_walk;
    o.block = t.block;
    o.h_offsets = h_offsets;
    auto run = [&] {
      return single ? pj::list_rank_impl(succ, nullptr, 1, nullptr, n0, out, &o, s)
                    : pj::list_rank_impl(succ, offsets, L, h_offsets, 0, out, &o, s);
    };
    int r = run();  // warm-up
    if (r != PJ_OK) return r;
    PJ_HIP(hipEventRecord(e0, s));
    for (int k = 0; k < 3 && r == PJ_OK; ++k) r = run();
    PJ_HIP(hipEventRecord(e1, s));
    PJ_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    PJ_HIP(hipEventElapsedTime(&ms, e0, e1));
    *ms_out = ms / 3.f;
    return r;
  };
  rc = time_one(cur, &cur.ms);
  for (int dim = 0; dim < 4 && rc == PJ_OK; ++dim) {
    for (int v : sweeps[dim]) {
      pj::Tuned t = cur;
      int* field = dim == 0 ? &t.spacing : dim == 1 ? &t.spacing_up : dim == 2 ? &t.cutoff : &t.block;
      if (*field == v) continue;
      *field = v;
      rc = time_one(t, &t.ms);
      if (rc != PJ_OK) break;
      if (t.ms < cur.ms) cur = t;
    }
  }
  const pj::Tuned bestt = cur;
  if (rc != PJ_OK) return rc;
  {
    std::lock_guard<std::mutex> lk(pj::g_tune_mu);
    pj::g_tune[pj::tune_key(n0, L)] = bestt;
    ++pj::g_tune_gen;
  }
  if (best) {
    pj_opts_init(best);
    best->algo = PJ_ALGO_RULING_SET;
    best->spacing = bestt.spacing;
    best->spacing_up = bestt.spacing_up;
    best->cutoff = bestt.cutoff;
    best->max_walk = bestt.max_walk;
    best->block = bestt.block;
  }
  if (best_ms) *best_ms = bestt.ms;
  return PJ_OK;
}

int pj_tune_save(const char* path) {
  if (!path) return PJ_EINVAL;
  std::lock_guard<std::mutex> lk(pj::g_tune_mu);
  FILE* f = fopen(path, "w");
  if (!f) return PJ_EINVAL;
  for (auto& kv : pj::g_tune) {
    const auto& t = kv.second;
    fprintf(f, "%s %d %d %d %d %d %d %d %.4f\n", std::get<0>(kv.first).c_str(),
            std::get<1>(kv.first), std::get<2>(kv.first), t.spacing, t.spacing_up, t.cutoff,
            t.max_walk, t.block, t.ms);
  }
  fclose(f);
  return PJ_OK;
}

int pj_tune_load(const char* path) {
  if (!path) return PJ_EINVAL;
  std::lock_guard<std::mutex> lk(pj::g_tune_mu);
  return pj::load_locked(path);
}

void pj_tune_clear(void) {
  std::lock_guard<std::mutex> lk(pj::g_tune_mu);
  pj::g_tune.clear();
  ++pj::g_tune_gen;
}

int pj_tune_lookup(int64_t n, int64_t L, pj_opts* out) {
  if (!out) return PJ_EINVAL;
  pj_opts o;
  pj_opts_init(&o);
  pj::apply_tuned(o, n, L);
  if (o.spacing <= 0) return PJ_ENOTFOUND;
  *out = o;
  return PJ_OK;
}

void pj_graph_cache_clear(void) {
  {
    std::lock_guard<std::mutex> lk(pj::g_graph_mu);
    for (auto& kv : pj::g_graphs) pj::drop_entry(kv.second);
    pj::g_graphs.clear();
  }
  pj::cc_graph_cache_clear();
}

}  // extern "C"
