// Serving loop: continuous batching of list-ranking and components requests
// under an HBM budget.
//
// Requests carry host input and output arrays.  A scheduler thread admits
// waiting requests in arrival order into a "tick" while the tick's exact
// device footprint (inputs, outputs, offset tables, statuses and the
// workspace of the two batched solves) fits in the unused part of the budget.
// Requests are sized into two classes: a large one (at least `large_items`
// list nodes, or graph vertices plus pairs) gets a tick of its own, and at
// most max_inflight - 1 large ticks are admitted at once, so one worker is
// always left for ticks of small requests, which never wait behind a large
// solve and its host copies.
// Each tick goes to one of `max_inflight` worker threads, each owning a HIP
// stream: the worker copies the inputs in, runs one batched list ranking and
// one batched components solve over all of the tick's requests, copies the
// results out, and retires the tick, which frees its memory for the next
// admissions.  Ticks on different workers overlap on the device, and requests
// that arrive while ticks run join the next tick as soon as a worker and
// memory are free.  Results do not depend on how requests were batched (the
// outputs are canonical), so every result is the same alone or in the mix.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pj_internal.hpp"

namespace pj {
namespace {

using Clock = std::chrono::steady_clock;

double seconds_since(Clock::time_point t0) {
  return std::chrono::duration<double>(Clock::now() - t0).count();
}

struct Request {
  uint64_t id = 0;
  int kind = 0;  // 0 list ranking, 1 components
  const int32_t* in0 = nullptr;
  const int32_t* in1 = nullptr;
  int64_t n = 0, m = 0;
  int32_t* out = nullptr;
  double t_submit = 0, t_done = 0;
  int32_t status = PJ_EBUSY;
  bool done = false;
  bool large = false;     // size class (see Server::large_items)
  size_t lr_ws1 = 0;      // list ranking: workspace of a solve of this list alone
};

// Running totals of a tick's requests, from which its footprint follows.
struct TickSize {
  int64_t lr_n = 0, lr_L = 0, cc_n = 0, cc_m = 0, cc_G = 0;
  size_t lr_ws1 = 0;  // largest single-list workspace
  void add(const Request* r) {
    if (r->kind == 0) {
      lr_n += r->n;
      ++lr_L;
      lr_ws1 = std::max(lr_ws1, r->lr_ws1);
    } else {
      cc_n += r->n;
      cc_m += r->m;
      ++cc_G;
    }
  }
};

struct Tick {
  std::vector<Request*> reqs;
  size_t bytes = 0;
  bool large = false;
};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

struct HostStage;

struct Server {
  // configuration
  size_t budget = 0;
  int max_inflight = 3;
  int max_batch = 256;
  int device = 0;
  int64_t large_items = int64_t(1) << 22;
  pj_opts opts{};
  // state
  std::mutex mu;
  std::condition_variable cv_sched;   // wakes the scheduler
  std::condition_variable cv_work;    // wakes workers
  std::condition_variable cv_done;    // wakes waiters
  std::deque<Request*> pending;
  std::deque<Tick*> ready;            // formed ticks waiting for a worker
  std::unordered_map<uint64_t, Request*> reqs;
  size_t used = 0, used_peak = 0;
  int busy_workers = 0, inflight_peak = 0;
  int large_inflight = 0;              // large ticks ready or running
  int64_t pending_large = 0;           // large requests not yet admitted
  int64_t large_ticks = 0;
  bool stopping = false;
  uint64_t next_id = 1;
  Clock::time_point t0 = Clock::now();
  double first_submit = -1, last_done = 0;
  int64_t submitted = 0, completed = 0, failed = 0, ticks = 0, budget_waits = 0;
  int64_t items_done = 0;
  std::vector<double> lat_ms;
  std::thread sched;
  std::vector<std::thread> workers;

  // Options of a tick's solves (statuses always written, nothing validated
  // on the host, the tick's own workspace).
  pj_opts solve_opts() const {
    pj_opts o = opts;
    o.workspace = nullptr;
    o.stats = nullptr;
    o.validate = 0;
    o.use_graph = 0;
    o.d_status = (int32_t*)1;
    return o;
  }

  // Workspace bytes of a tick's list ranking: the batched solve, and, should
  // a malformed list make the worker re-solve the tick's lists one by one,
  // the largest single-list solve (the same region serves both).
  size_t lr_workspace(const TickSize& z) const {
    if (z.lr_L == 0) return 0;
    const pj_opts o = solve_opts();
    const size_t batched = pj_list_rank_workspace_bytes(z.lr_n, z.lr_L, &o);
    return align256(z.lr_L > 1 ? std::max(batched, z.lr_ws1) : batched);
  }

  // Exact device bytes of a tick with these totals (must match run_tick's carve).
  size_t tick_bytes(const TickSize& z) const {
    size_t b = 0;
    const pj_opts o = solve_opts();
    if (z.lr_L) {
      b += align256(z.lr_n * 4) * 2 + align256((z.lr_L + 1) * 8) + align256(z.lr_L * 4);
      b += lr_workspace(z);
    }
    if (z.cc_G) {
      b += align256(z.cc_m * 4) * 2 + align256(z.cc_n * 4) + 2 * align256((z.cc_G + 1) * 8) +
           align256(z.cc_G * 4);
      b += align256(pj_cc_workspace_bytes(z.cc_n, z.cc_m, z.cc_G, &o));
    }
    return b;
  }

  size_t tick_bytes(const std::vector<Request*>& rs) const {
    TickSize z;
    for (auto* r : rs) z.add(r);
    return tick_bytes(z);
  }

  // A large tick may be admitted while another worker stays free for small ones.
  bool large_slot_free() const { return max_inflight < 2 || large_inflight < max_inflight - 1; }

  // Some tick can be formed now (memory aside).
  bool can_form() const {
    if (pending.empty() || busy_workers + (int)ready.size() >= max_inflight) return false;
    const int64_t small = (int64_t)pending.size() - pending_large;
    return small > 0 || (pending_large > 0 && large_slot_free());
  }

  void scheduler_loop();
  void worker_loop(int idx);
  int run_tick(Tick* t, hipStream_t s, HostStage& stage);
  void finish_tick(Tick* t, bool ok);
};

void Server::scheduler_loop() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    // Leave the wait only when there is something to do: a tick can be formed,
    // or the server is stopping with nothing left to admit.  (A predicate that
    // is true while nothing can be done would spin with the lock held and keep
    // the workers from retiring their ticks.)
    cv_sched.wait(lk, [&] { return (stopping && pending.empty()) || can_form(); });
    if (pending.empty()) break;  // stopping, everything admitted
    // The oldest large request goes first if it is older than every small
    // one and a large slot is free; otherwise a tick of small requests in
    // arrival order (large ones skipped) while the footprint fits.
    auto first_large = pending.end(), first_small = pending.end();
    for (auto it = pending.begin(); it != pending.end(); ++it) {
      if ((*it)->large) {
        if (first_large == pending.end()) first_large = it;
      } else if (first_small == pending.end()) {
        first_small = it;
      }
      if (first_large != pending.end() && first_small != pending.end()) break;
    }
    const bool pick_large = first_large != pending.end() && large_slot_free() &&
                            (first_small == pending.end() || (*first_large)->id < (*first_small)->id);
    Tick* t = new Tick;
    t->large = pick_large;
    const size_t free_bytes = budget - used;
    TickSize z;
    if (pick_large) {
      z.add(*first_large);
      const size_t b = tick_bytes(z);
      if (b <= free_bytes) {
        t->reqs.push_back(*first_large);
        t->bytes = b;
        pending.erase(first_large);
        --pending_large;
      }
    } else {
      for (auto it = first_small; it != pending.end() && (int)t->reqs.size() < max_batch;) {
        if ((*it)->large) {
          ++it;
          continue;
        }
        TickSize z2 = z;
        z2.add(*it);
        const size_t b = tick_bytes(z2);
        if (b > free_bytes) break;
        z = z2;
        t->reqs.push_back(*it);
        t->bytes = b;
        it = pending.erase(it);
      }
    }
    if (t->reqs.empty()) {
      // The chosen request must wait for memory held by admitted ticks.  It
      // fits the whole budget (checked at submit), so some tick holds memory
      // and will release it; stopping changes nothing here.
      delete t;
      ++budget_waits;
      cv_sched.wait(lk, [&] { return budget - used != free_bytes; });
      continue;
    }
    used += t->bytes;
    used_peak = std::max(used_peak, used);
    ++ticks;
    if (t->large) {
      ++large_inflight;
      ++large_ticks;
    }
    ready.push_back(t);
    cv_work.notify_one();
  }
}

// A worker's pinned host staging for tick tables and statuses, kept across
// ticks (pinning memory per tick costs more than a small tick's solve).  A
// tick ends with a stream synchronisation, so the next tick may reuse it.
struct HostStage {
  char* p = nullptr;
  size_t cap = 0;
  HostStage() = default;
  HostStage(const HostStage&) = delete;
  HostStage& operator=(const HostStage&) = delete;
  ~HostStage() {
    if (p) (void)hipHostFree(p);
  }
  char* get(size_t bytes) {
    if (bytes > cap) {
      if (p) (void)hipHostFree(p);
      p = nullptr;
      cap = 0;
      size_t c = 64 << 10;
      while (c < bytes) c *= 2;
      if (hipHostMalloc((void**)&p, c, hipHostMallocDefault) != hipSuccess) {
        p = nullptr;
        return nullptr;
      }
      cap = c;
    }
    return p;
  }
};

void Server::worker_loop(int idx) {
  (void)idx;
  (void)hipSetDevice(device);
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
  HostStage stage;
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_work.wait(lk, [&] { return !ready.empty() || (stopping && pending.empty()); });
    if (ready.empty()) {
      if (stopping && pending.empty() && busy_workers == 0) break;
      if (stopping && pending.empty()) break;
      continue;
    }
    Tick* t = ready.front();
    ready.pop_front();
    ++busy_workers;
    inflight_peak = std::max(inflight_peak, busy_workers);
    lk.unlock();
    const int rc = s ? run_tick(t, s, stage) : PJ_EHIP;
    lk.lock();
    finish_tick(t, rc == PJ_OK);
    --busy_workers;
    used -= t->bytes;
    if (t->large) --large_inflight;
    delete t;
    cv_sched.notify_all();
    cv_done.notify_all();
  }
  if (s) (void)hipStreamDestroy(s);
}

// Called with the lock held.
void Server::finish_tick(Tick* t, bool ok) {
  const double now = seconds_since(t0);
  for (auto* r : t->reqs) {
    if (!ok && r->status == PJ_OK) r->status = PJ_EHIP;
    r->done = true;
    r->t_done = now;
    last_done = now;
    if (r->status == PJ_OK) {
      ++completed;
      items_done += r->kind == 0 ? r->n : r->m;
      lat_ms.push_back((r->t_done - r->t_submit) * 1e3);
    } else {
      ++failed;
    }
  }
}

int Server::run_tick(Tick* t, hipStream_t s, HostStage& stage) {
  std::vector<Request*> lr, cc;
  for (auto* r : t->reqs) (r->kind == 0 ? lr : cc).push_back(r);
  const int64_t L = (int64_t)lr.size(), G = (int64_t)cc.size();
  std::vector<int64_t> loff(L + 1, 0), voff(G + 1, 0), eoff(G + 1, 0);
  for (int64_t i = 0; i < L; ++i) loff[i + 1] = loff[i] + lr[i]->n;
  for (int64_t i = 0; i < G; ++i) {
    voff[i + 1] = voff[i] + cc[i]->n;
    eoff[i + 1] = eoff[i] + cc[i]->m;
  }
  // host staging for tables and statuses (pinned so copies stay asynchronous)
  const size_t hbytes = (L + 1 + 2 * (G + 1)) * 8 + (L + G) * 4 + 64;
  char* hst = stage.get(hbytes);
  if (!hst) return PJ_ENOMEM;
  int64_t* h_loff = reinterpret_cast<int64_t*>(hst);
  int64_t* h_voff = h_loff + (L + 1);
  int64_t* h_eoff = h_voff + (G + 1);
  int32_t* h_lst = reinterpret_cast<int32_t*>(h_eoff + (G + 1));
  int32_t* h_cst = h_lst + L;
  std::copy(loff.begin(), loff.end(), h_loff);
  std::copy(voff.begin(), voff.end(), h_voff);
  std::copy(eoff.begin(), eoff.end(), h_eoff);

  char* d = nullptr;
  char* lr_ws = nullptr;  // the list-ranking workspace inside the tick's memory
  size_t lr_ws_bytes = 0;
  int rc = PJ_OK;
  hipError_t he = hipMallocAsync((void**)&d, std::max<size_t>(t->bytes, 256), s);
  if (he != hipSuccess) {
    set_last_hip_error(he, "hipMallocAsync(tick)", __FILE__, __LINE__);
    return PJ_ENOMEM;
  }
  size_t at = 0;
  auto take = [&](size_t b) {
    char* p = d + at;
    at += align256(b);
    return p;
  };
  pj_opts o = opts;
  o.stats = nullptr;
  o.use_graph = 0;
  o.validate = 0;
  if (L > 0) {
    const int64_t N = loff[L];
    int32_t* d_succ = (int32_t*)take(N * 4);
    int32_t* d_rank = (int32_t*)take(N * 4);
    int64_t* d_off = (int64_t*)take((L + 1) * 8);
    int32_t* d_st = (int32_t*)take(L * 4);
    o.d_status = d_st;
    TickSize z;
    for (auto* r : t->reqs) z.add(r);
    lr_ws_bytes = lr_workspace(z);
    lr_ws = take(lr_ws_bytes);
    o.workspace = lr_ws;
    o.workspace_bytes = lr_ws_bytes;
    o.h_offsets = h_loff;
    for (int64_t i = 0; i < L && rc == PJ_OK; ++i)
      if (lr[i]->n)
        if (hipMemcpyAsync(d_succ + loff[i], lr[i]->in0, lr[i]->n * 4, hipMemcpyHostToDevice, s) !=
            hipSuccess)
          rc = PJ_EHIP;
    if (rc == PJ_OK && hipMemcpyAsync(d_off, h_loff, (L + 1) * 8, hipMemcpyHostToDevice, s) !=
                           hipSuccess)
      rc = PJ_EHIP;
    if (rc == PJ_OK) rc = pj_list_rank_batched_ex(d_succ, d_off, L, d_rank, &o, (pj_stream_t)s);
    for (int64_t i = 0; i < L && rc == PJ_OK; ++i)
      if (lr[i]->n)
        if (hipMemcpyAsync(lr[i]->out, d_rank + loff[i], lr[i]->n * 4, hipMemcpyDeviceToHost, s) !=
            hipSuccess)
          rc = PJ_EHIP;
    if (rc == PJ_OK &&
        hipMemcpyAsync(h_lst, d_st, L * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
      rc = PJ_EHIP;
  }
  if (G > 0 && rc == PJ_OK) {
    const int64_t V = voff[G], M = eoff[G];
    int32_t* d_src = (int32_t*)take(M * 4);
    int32_t* d_dst = (int32_t*)take(M * 4);
    int32_t* d_lab = (int32_t*)take(V * 4);
    int64_t* d_voff = (int64_t*)take((G + 1) * 8);
    int64_t* d_eoff = (int64_t*)take((G + 1) * 8);
    int32_t* d_st = (int32_t*)take(G * 4);
    pj_opts oc = opts;
    oc.stats = nullptr;
    oc.validate = 0;
    oc.d_status = d_st;
    const size_t wsb = pj_cc_workspace_bytes(V, M, G, &oc);
    oc.workspace = take(wsb);
    oc.workspace_bytes = align256(wsb);
    oc.h_offsets = h_voff;
    oc.h_edge_offsets = h_eoff;
    for (int64_t i = 0; i < G && rc == PJ_OK; ++i) {
      if (cc[i]->m) {
        if (hipMemcpyAsync(d_src + eoff[i], cc[i]->in0, cc[i]->m * 4, hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipMemcpyAsync(d_dst + eoff[i], cc[i]->in1, cc[i]->m * 4, hipMemcpyHostToDevice, s) !=
                hipSuccess)
          rc = PJ_EHIP;
      }
    }
    if (rc == PJ_OK &&
        (hipMemcpyAsync(d_voff, h_voff, (G + 1) * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
         hipMemcpyAsync(d_eoff, h_eoff, (G + 1) * 8, hipMemcpyHostToDevice, s) != hipSuccess))
      rc = PJ_EHIP;
    if (rc == PJ_OK)
      rc = pj_connected_components_batched_ex(d_src, d_dst, d_voff, d_eoff, G, d_lab, &oc,
                                              (pj_stream_t)s);
    for (int64_t i = 0; i < G && rc == PJ_OK; ++i)
      if (cc[i]->n)
        if (hipMemcpyAsync(cc[i]->out, d_lab + voff[i], cc[i]->n * 4, hipMemcpyDeviceToHost, s) !=
            hipSuccess)
          rc = PJ_EHIP;
    if (rc == PJ_OK &&
        hipMemcpyAsync(h_cst, d_st, G * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
      rc = PJ_EHIP;
  }
  if (at > std::max<size_t>(t->bytes, 256)) rc = PJ_EINVAL;  // accounting mismatch
  if (hipStreamSynchronize(s) != hipSuccess && rc == PJ_OK) rc = PJ_EHIP;
  // A malformed list can raise an error the batched solve cannot pin on one
  // list.  Then each list of the tick is solved again on its own (from the
  // tick's buffers and its workspace, sized for the largest single solve),
  // so only the malformed requests fail.
  bool lr_bad = false;
  for (int64_t i = 0; i < L && rc == PJ_OK; ++i) lr_bad |= h_lst[i] != PJ_OK;
  if (rc == PJ_OK && lr_bad && L > 1) {
    int32_t* d_succ = (int32_t*)d;
    int32_t* d_rank = (int32_t*)(d + align256(loff[L] * 4));
    int32_t* d_st = (int32_t*)(d + 2 * align256(loff[L] * 4) + align256((L + 1) * 8));
    pj_opts o1 = opts;
    o1.stats = nullptr;
    o1.use_graph = 0;
    o1.validate = 0;
    o1.workspace = lr_ws;
    o1.workspace_bytes = lr_ws_bytes;
    for (int64_t i = 0; i < L && rc == PJ_OK; ++i) {
      o1.d_status = d_st + i;
      rc = pj_list_rank_ex(d_succ + loff[i], lr[i]->n, d_rank + loff[i], &o1, (pj_stream_t)s);
      if (rc == PJ_OK && lr[i]->n &&
          hipMemcpyAsync(lr[i]->out, d_rank + loff[i], lr[i]->n * 4, hipMemcpyDeviceToHost, s) !=
              hipSuccess)
        rc = PJ_EHIP;
    }
    if (rc == PJ_OK &&
        hipMemcpyAsync(h_lst, d_st, L * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
      rc = PJ_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess && rc == PJ_OK) rc = PJ_EHIP;
  }
  (void)hipFreeAsync(d, s);
  (void)hipStreamSynchronize(s);
  for (int64_t i = 0; i < L; ++i) lr[i]->status = rc == PJ_OK ? h_lst[i] : rc;
  for (int64_t i = 0; i < G; ++i) cc[i]->status = rc == PJ_OK ? h_cst[i] : rc;
  return PJ_OK;
}

}  // namespace pj

extern "C" {

struct pj_server {
  pj::Server s;
};

int pj_server_create(const pj_server_config* cfg, pj_server** out) {
  if (!out) return PJ_EINVAL;
  *out = nullptr;
  auto* w = new pj_server;
  pj::Server& s = w->s;
  if (cfg) {
    s.budget = cfg->hbm_budget;
    if (cfg->max_inflight > 0) s.max_inflight = cfg->max_inflight;
    if (cfg->max_batch > 0) s.max_batch = cfg->max_batch;
    s.opts = cfg->opts;
    s.device = cfg->device;
    if (cfg->large_items > 0) s.large_items = cfg->large_items;
  } else {
    pj_opts_init(&s.opts);
    s.device = -1;
  }
  if (s.budget == 0) s.budget = size_t(16) << 30;
  if (s.device < 0 && hipGetDevice(&s.device) != hipSuccess) s.device = 0;
  s.opts.stats = nullptr;
  s.opts.workspace = nullptr;
  s.opts.d_status = nullptr;
  s.opts.d_splitters = nullptr;
  s.opts.n_splitters = 0;
  s.t0 = pj::Clock::now();
  s.sched = std::thread([&s] { s.scheduler_loop(); });
  for (int i = 0; i < s.max_inflight; ++i) s.workers.emplace_back([&s, i] { s.worker_loop(i); });
  *out = w;
  return PJ_OK;
}

static int submit(pj_server* w, int kind, const int32_t* a, const int32_t* b, int64_t n,
                  int64_t m, int32_t* out, uint64_t* id) {
  if (!w || !id || n < 0 || m < 0 || n >= INT32_MAX) return PJ_EINVAL;
  if ((n > 0 && (!out || (kind == 0 && !a))) || (m > 0 && (!a || !b))) return PJ_EINVAL;
  pj::Server& s = w->s;
  auto* r = new pj::Request;
  r->kind = kind;
  r->in0 = a;
  r->in1 = b;
  r->n = n;
  r->m = m;
  r->out = out;
  r->large = (kind == 0 ? n : n + m) >= s.large_items;
  if (kind == 0) {
    const pj_opts o = s.solve_opts();
    r->lr_ws1 = pj_list_rank_workspace_bytes(n, 1, &o);
  }
  std::lock_guard<std::mutex> lk(s.mu);
  if (s.stopping) {
    delete r;
    return PJ_ESHUTDOWN;
  }
  if (s.tick_bytes(std::vector<pj::Request*>{r}) > s.budget) {
    delete r;
    return PJ_EBUDGET;
  }
  r->id = s.next_id++;
  r->t_submit = pj::seconds_since(s.t0);
  if (s.first_submit < 0) s.first_submit = r->t_submit;
  s.reqs[r->id] = r;
  s.pending.push_back(r);
  if (r->large) ++s.pending_large;
  ++s.submitted;
  *id = r->id;
  s.cv_sched.notify_one();
  return PJ_OK;
}

int pj_server_submit_list_rank(pj_server* w, const int32_t* h_succ, int64_t n, int32_t* h_rank,
                               uint64_t* id) {
  return submit(w, 0, h_succ, nullptr, n, 0, h_rank, id);
}

int pj_server_submit_cc(pj_server* w, const int32_t* h_src, const int32_t* h_dst, int64_t n,
                        int64_t m, int32_t* h_label, uint64_t* id) {
  return submit(w, 1, h_src, h_dst, n, m, h_label, id);
}

static int collect(pj::Server& s, uint64_t id, int32_t* status, double* latency_ms) {
  auto it = s.reqs.find(id);
  if (it == s.reqs.end()) return PJ_ENOTFOUND;
  pj::Request* r = it->second;
  if (!r->done) return PJ_EBUSY;
  if (status) *status = r->status;
  if (latency_ms) *latency_ms = (r->t_done - r->t_submit) * 1e3;
  s.reqs.erase(it);
  delete r;
  return PJ_OK;
}

int pj_server_poll(pj_server* w, uint64_t id, int32_t* status, double* latency_ms) {
  if (!w) return PJ_EINVAL;
  std::lock_guard<std::mutex> lk(w->s.mu);
  return collect(w->s, id, status, latency_ms);
}

int pj_server_wait(pj_server* w, uint64_t id, int32_t* status, double* latency_ms,
                   int64_t timeout_us) {
  if (!w) return PJ_EINVAL;
  pj::Server& s = w->s;
  std::unique_lock<std::mutex> lk(s.mu);
  auto ready = [&] {
    auto it = s.reqs.find(id);
    return it == s.reqs.end() || it->second->done;
  };
  if (timeout_us < 0) s.cv_done.wait(lk, ready);
  else if (!s.cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) return PJ_EBUSY;
  return collect(s, id, status, latency_ms);
}

int pj_server_drain(pj_server* w) {
  if (!w) return PJ_EINVAL;
  pj::Server& s = w->s;
  std::unique_lock<std::mutex> lk(s.mu);
  s.cv_done.wait(lk, [&] {
    return s.pending.empty() && s.ready.empty() && s.busy_workers == 0;
  });
  return PJ_OK;
}

int pj_server_get_stats(pj_server* w, pj_server_stats* out) {
  if (!w || !out) return PJ_EINVAL;
  pj::Server& s = w->s;
  std::lock_guard<std::mutex> lk(s.mu);
  *out = pj_server_stats{};
  out->submitted = s.submitted;
  out->completed = s.completed;
  out->failed = s.failed;
  out->ticks = s.ticks;
  out->inflight_peak = s.inflight_peak;
  out->budget_waits = s.budget_waits;
  out->large_ticks = s.large_ticks;
  out->bytes_peak = s.used_peak;
  out->bytes_in_use = s.used;
  std::vector<double> l = s.lat_ms;
  if (!l.empty()) {
    std::sort(l.begin(), l.end());
    auto q = [&](double p) {
      const size_t i = std::min(l.size() - 1, (size_t)(p * (double)(l.size() - 1) + 0.5));
      return l[i];
    };
    out->p50_ms = q(0.50);
    out->p99_ms = q(0.99);
    out->max_ms = l.back();
    double sum = 0;
    for (double v : l) sum += v;
    out->mean_ms = sum / (double)l.size();
  }
  if (s.first_submit >= 0 && s.last_done > s.first_submit) {
    out->wall_s = s.last_done - s.first_submit;
    out->req_per_s = (double)s.completed / out->wall_s;
    out->items_per_s = (double)s.items_done / out->wall_s;
  }
  return PJ_OK;
}

int pj_server_destroy(pj_server* w) {
  if (!w) return PJ_EINVAL;
  pj::Server& s = w->s;
  {
    std::lock_guard<std::mutex> lk(s.mu);
    s.stopping = true;
  }
  s.cv_sched.notify_all();
  s.cv_work.notify_all();
  if (s.sched.joinable()) s.sched.join();
  // the scheduler has handed out every pending request; wake idle workers
  {
    std::lock_guard<std::mutex> lk(s.mu);
  }
  s.cv_work.notify_all();
  for (auto& t : s.workers)
    if (t.joinable()) t.join();
  for (auto& kv : s.reqs) delete kv.second;
  s.reqs.clear();
  delete w;
  return PJ_OK;
}

}  // extern "C"
