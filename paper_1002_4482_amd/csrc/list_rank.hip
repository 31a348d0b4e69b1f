// List ranking on gfx950: Wyllie pointer jumping and the random-splitter
// (sparse ruling set) method with recursive ranking of the splitter list.
//
// One code path serves a single list and a batch of lists: a single list is
// a batch with L = 1.  Global node ids run over the concatenation; the
// successors of level 0 are local to their list.
//
// Ruling set, per level l (Section 3.2, "Parallel Random Splitter"):
//   * splitters: one node per block of 2^log2B consecutive ids, at an offset
//     drawn by a counter-based hash (so "is y a splitter" is arithmetic, with
//     no mark array), plus one virtual splitter per list standing at its head;
//   * walk (the paper's RS3): persistent lanes take splitters from a work
//     counter and follow successors until the next splitter or the tail,
//     writing (sublist id, weight before the node) per node and
//     (next splitter, sublist weight) per splitter.  A walk longer than
//     max_walk nodes is cut and the cut node becomes a new splitter, which
//     bounds every loop even on malformed input;
//   * the splitter lists (one per input list, head = its virtual splitter)
//     form level l+1, weighted by sublist length, and are ranked the same way
//     (the recursion replacing the paper's single-block RS4) until a level is
//     small enough for one workgroup, which ranks it in LDS by pointer
//     jumping (the paper's single-kernel Wyllie);
//   * expand (the paper's RS5): rank[x] = rank of its splitter + its weight
//     offset, a coalesced pass per level.
// The rank counted here is the distance from the head; the paper's RS5
// subtracts from the splitter rank because it counts toward the tail.
#include <algorithm>
#include <cmath>
#include <vector>

#include "pj_internal.hpp"

namespace pj {
namespace {

constexpr int kMaxCutoff = 16384;
constexpr int kBaseThreads = 1024;
constexpr int kPerThread = kMaxCutoff / kBaseThreads;

struct LevelCtl {
  int32_t n;     // nodes at this level (level 0: written by init)
  int32_t r;     // static splitters of this level (written by its walk)
  int32_t dyn;   // cut points requested at this level (may exceed the cap)
  int32_t work;  // work counter of the persistent walk
};

struct LrCtl {
  LevelCtl lv[PJ_MAX_LEVELS + 2];
  int32_t err;
  int32_t pad;
  unsigned long long base_total;  // total weight seen by the base ranking
  unsigned long long near;        // single list: successors within kNear ids
};

// A successor within kNear ids of its node counts as local (see lr_walk).
constexpr int kNear = 64;

// Node count of level `level` >= 1: static + virtual + granted cut points of
// the level below.
__device__ __forceinline__ int level_nodes(const LrCtl* ctl, int level, int L, int cap_prev) {
  if (level == 0) return ctl->lv[0].n;
  const LevelCtl& p = ctl->lv[level - 1];
  return p.r + L + min(p.dyn, cap_prev);
}

__device__ __forceinline__ uint32_t splitter_offset(uint32_t block, uint32_t seed, uint32_t bsize) {
  uint32_t h = mix32(block * 0x9E3779B9u ^ seed);
  return (uint32_t)(((uint64_t)h * bsize) >> 32);
}

// Is id y the static splitter of its block?
__device__ __forceinline__ bool is_static(int y, int N, int log2B, uint32_t seed) {
  int b = y >> log2B;
  int start = b << log2B;
  int bsize = min(1 << log2B, N - start);
  return (uint32_t)(y - start) == splitter_offset((uint32_t)b, seed, (uint32_t)bsize);
}

__device__ __forceinline__ void store_pair(int2* p, int a, int b) { *p = make_int2(a, b); }

// ------------------------------------------------------------------ init
__global__ void lr_init(LrCtl* ctl, int n0, unsigned long long* lsum, int32_t* ltails,
                        int32_t* lerr, int L, int64_t* off_single) {
  int tid = blockIdx.x * blockDim.x + threadIdx.x;
  int stride = gridDim.x * blockDim.x;
  int32_t* c = reinterpret_cast<int32_t*>(ctl);
  for (int i = tid; i < (int)(sizeof(LrCtl) / 4); i += stride) c[i] = 0;
  for (int i = tid; i < L; i += stride) {
    lsum[i] = 0ull;
    ltails[i] = 0;
    lerr[i] = 0;
  }
  if (tid == 0) {
    ctl->lv[0].n = n0;
    if (off_single) {
      off_single[0] = 0;
      off_single[1] = n0;
    }
  }
}

// ------------------------------------------------------------- head find
// Head of each list by the index-sum identity: the nodes with a predecessor
// are exactly the non-tail successors, so
//   head = size(size-1)/2 - sum of non-tail successors.
// The same coalesced pass counts tails and flags out-of-range successors.
template <bool kCopy>
__global__ void __launch_bounds__(256) lr_headfind_single(const int32_t* __restrict__ succ, int n,
                                                          int32_t* __restrict__ copy,
                                                          unsigned long long* lsum,
                                                          int32_t* ltails, int32_t* lerr,
                                                          unsigned long long* lnear) {
  unsigned long long acc = 0;
  int tails = 0, bad = 0, near = 0;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  const bool vec = ((reinterpret_cast<uintptr_t>(succ) | reinterpret_cast<uintptr_t>(copy)) & 15) == 0;
  const int n4 = vec ? (n >> 2) : 0;
  const int4* s4 = reinterpret_cast<const int4*>(succ);
  for (int q = tid; q < n4; q += stride) {
    const int4 v = s4[q];
    if (kCopy) reinterpret_cast<int4*>(copy)[q] = v;
    int i = q << 2;
    int vs[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      int s = vs[t];
      bool tail = (s == -1) | (s == i + t);
      bool range = (unsigned)s < (unsigned)n;
      tails += tail;
      bad |= (!tail & !range);
      acc += (!tail & range) ? (unsigned long long)s : 0ull;
      near += (!tail & range) & ((unsigned)(s - (i + t) + kNear) <= 2u * kNear);
    }
  }
  for (int i = (n4 << 2) + tid; i < n; i += stride) {
    int s = succ[i];
    if (kCopy) copy[i] = s;
    bool tail = (s == -1) | (s == i);
    bool range = (unsigned)s < (unsigned)n;
    tails += tail;
    bad |= (!tail & !range);
    acc += (!tail & range) ? (unsigned long long)s : 0ull;
    near += (!tail & range) & ((unsigned)(s - i + kNear) <= 2u * kNear);
  }
  acc = wave_sum(acc);
  tails = wave_sum(tails);
  bad = wave_sum(bad);
  near = wave_sum(near);
  // one atomic per workgroup: atomics on a single address serialise
  __shared__ unsigned long long s_acc[256 / kWave];
  __shared__ int s_tails[256 / kWave], s_bad[256 / kWave], s_near[256 / kWave];
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) {
    s_acc[w] = acc;
    s_tails[w] = tails;
    s_bad[w] = bad;
    s_near[w] = near;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x / kWave); ++i) {
      acc += s_acc[i];
      tails += s_tails[i];
      bad += s_bad[i];
      near += s_near[i];
    }
    if (acc) atomicAdd(lsum, acc);
    if (tails) atomicAdd(ltails, tails);
    if (bad) atomicOr(lerr, kErrRange);
    if (near && lnear) atomicAdd(lnear, (unsigned long long)near);
  }
}

// Batched form: each wave owns chunks of 64*kChunk consecutive positions and
// tracks the owning list while it advances.
constexpr int kHfChunk = 16;
template <bool kCopy>
__global__ void __launch_bounds__(256) lr_headfind_batched(const int32_t* __restrict__ succ,
                                                           const int64_t* __restrict__ off, int L,
                                                           int n, int32_t* __restrict__ copy,
                                                           unsigned long long* lsum,
                                                           int32_t* ltails, int32_t* lerr) {
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int nwaves = (gridDim.x * blockDim.x) / kWave;
  const int lane = lane_id();
  const int chunk = kWave * kHfChunk;
  // each wave owns a contiguous run of chunks: one search of the offset
  // table per wave, then every lane follows the list boundaries forward
  const int64_t nchunks = ((int64_t)n + chunk - 1) / chunk;
  const int64_t per = (nchunks + nwaves - 1) / nwaves;
  const int64_t ci0 = (int64_t)wave * per;
  const int64_t ci1 = ci0 + per < nchunks ? ci0 + per : nchunks;
  int l = ci0 < ci1 ? find_instance(off, L, ci0 * chunk) : 0;
  for (int64_t ci = ci0; ci < ci1; ++ci) {
    const int64_t c0 = ci * chunk;
    int64_t lend = off[l + 1];
    int64_t lbase = off[l];
    unsigned long long acc = 0;
    int tails = 0;
    // all loads (and the copy) of the chunk first: the flushes below hold
    // atomics that would otherwise keep each load waiting for the last
    int sv[kHfChunk];
#pragma unroll
    for (int t = 0; t < kHfChunk; ++t) {
      const int64_t g = c0 + t * kWave + lane;
      sv[t] = g < n ? succ[g] : 0;
    }
    if (kCopy) {
#pragma unroll
      for (int t = 0; t < kHfChunk; ++t) {
        const int64_t g = c0 + t * kWave + lane;
        if (g < n) copy[g] = sv[t];
      }
    }
    for (int t = 0; t < kHfChunk; ++t) {
      int64_t g = c0 + t * kWave + lane;
      if (g >= n) break;
      if (g >= lend) {  // moved into a later list: flush
        if (acc) atomicAdd(&lsum[l], acc);
        if (tails) atomicAdd(&ltails[l], tails);
        acc = 0;
        tails = 0;
        while (off[l + 1] <= g) ++l;
        lbase = off[l];
        lend = off[l + 1];
      }
      const int s = sv[t];
      int x = (int)(g - lbase);
      int size = (int)(lend - lbase);
      bool tail = (s == -1) | (s == x);
      bool range = (unsigned)s < (unsigned)size;
      tails += tail;
      if (!tail & !range) atomicOr(&lerr[l], kErrRange);
      acc += (!tail & range) ? (unsigned long long)s : 0ull;
    }
    // wave-combine when the whole wave ended in one list
    int l0 = __shfl(l, 0);
    if (__ballot(l != l0) == 0) {
      acc = wave_sum(acc);
      tails = wave_sum(tails);
      if (lane == 0) {
        if (acc) atomicAdd(&lsum[l], acc);
        if (tails) atomicAdd(&ltails[l], tails);
      }
    } else {
      if (acc) atomicAdd(&lsum[l], acc);
      if (tails) atomicAdd(&ltails[l], tails);
    }
  }
}

// ------------------------------------------------------------------ walk
struct WalkArgs {
  const int32_t* succ0;              // level 0: local successors
  const int32_t* weight0;            // level 0, weighted call: node weights (unpacked form)
  const int2* link_in;               // level >= 1: {next, weight} per node
  const int64_t* off;                // level 0: list offsets (L+1)
  const unsigned long long* lsum;    // level 0: head-find sums
  const int32_t* ltails;             // level 0: tail counts
  int32_t* lerr;                     // per-list error bits
  int2* state;                       // {sublist id, weight before node} per node
  int32_t* work;                     // level 0 packed form: successor copy, overwritten
                                     // in place by (sublist id << kbits | offset)
  int2* link_out;                    // {next splitter, sublist weight} per splitter
  LrCtl* ctl;
  int L;
  int level;
  int log2B;
  int log2B_far; // level 0, single list, > 0: the block size used instead of
                 // 2^log2B when fewer than half the successors are local,
  int kbits_far; // with these offset bits and cut length
  int max_walk_far;
  int max_walk;
  int cap;       // cut points this level may create
  int cap_prev;  // cut points the level below could create
  int kbits;     // level 0 packed form: bits of the in-sublist offset
  uint32_t seed;
};

// kPacked (level 0): the successors are read from a.work, a copy made by the
// head-find pass, and each visited slot is overwritten with the node's packed
// state.  The read and the write then touch the same cache line, which costs
// far less than a write to a second random line.
constexpr int kWalkBurst = 16;
constexpr int kWalkChunk = 64;  // items a wave takes at a time

template <bool kLevel0, bool kBatched, bool kPacked>
__global__ void __launch_bounds__(1024) lr_walk(WalkArgs a) {
  LrCtl* ctl = a.ctl;
  const int N = level_nodes(ctl, a.level, a.L, a.cap_prev);
  // Splitter spacing for level 0 of a single list chosen on the device from
  // the head-find pass: when most successors are local (sequential-like
  // layouts), the lanes of a wave walk neighbouring sublists and share cache
  // lines, and short sublists (spacing 2^log2B) pay; when they are random,
  // every step is its own line and fewer, longer sublists (2^log2B_far) make
  // the final scatter's splitter-rank gathers hit in L2.  The plan is sized
  // for the smaller spacing.
  const bool far =
      kLevel0 && a.log2B_far > 0 && 2ull * ctl->near <= (unsigned long long)N;
  const int log2B = far ? a.log2B_far : a.log2B;
  const int kbits = far ? a.kbits_far : a.kbits;
  const int max_walk = far ? a.max_walk_far : a.max_walk;
  const int r = (int)(((int64_t)N + (1 << log2B) - 1) >> log2B);
  const int head_base = kLevel0 ? 0 : ctl->lv[a.level - 1].r;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->lv[a.level].r = r;
  const int items = r + a.L;
  int* dyn = &ctl->lv[a.level].dyn;
  const uint32_t seed = a.seed;
  // Work distribution.  One list, and the recursion levels: each workgroup
  // owns a contiguous range of items (static splitters, then the virtual
  // splitters at the list heads) and hands them to its lanes through an LDS
  // counter.  A batch's level 0 (kChunks): its thousands of list heads come
  // last and would all fall to the last workgroups, so each wave walks
  // chunks of kWalkChunk items instead, first the chunk of its own index,
  // then chunks taken from a device-wide counter with one atomic per chunk
  // (4096 lists of 2^6..2^20 nodes: 17.1 -> 15.7 ms for the walk; for one
  // list the counter costs more than it balances: the sequential 2^26 list,
  // 8 M sublists, 0.6 -> 1.5 ms).  A counter hit at every refill of every
  // wave would serialise at the memory side.
  constexpr bool kChunks = kLevel0 && kBatched;
  __shared__ int wg_next;
  int wg_hi = items;
  if (!kChunks) {
    const int per = (int)(((int64_t)items + gridDim.x - 1) / gridDim.x);
    const int wg_lo = min(items, (int)((int64_t)blockIdx.x * per));
    wg_hi = min(items, wg_lo + per);
    if (threadIdx.x == 0) wg_next = wg_lo;
    __syncthreads();
  }
  const int nwaves = (int)(((int64_t)gridDim.x * blockDim.x) / kWave);
  const int wave_id = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  int chunk_lo = (int)min<int64_t>(items, (int64_t)wave_id * kWalkChunk);
  int chunk_hi = (int)min<int64_t>(items, (int64_t)chunk_lo + kWalkChunk);
  bool drained = false;  // the device-wide counter has passed the last item
  int* counter = &ctl->lv[a.level].work;
  const int64_t dyn_base = (int64_t)nwaves * kWalkChunk;

  int sid = -1;       // sublist being walked, -1 = idle
  int x = 0;          // current node
  int k = 0;          // weight of the sublist before x
  int steps = 0;
  int64_t base = 0;   // level 0: first id of the lane's list
  int size = N;       // level 0: size of the lane's list
  int lid = 0;        // level 0: list index
  bool retired = false;
  int errbits = 0;

  while (true) {
    const bool need = (sid < 0) & !retired;
    const uint64_t needm = __ballot(need);
    if (needm) {
      int first, avail;
      if (kChunks) {
        if (chunk_lo >= chunk_hi && !drained) {  // the wave's chunk is used up
          int got = 0;
          if (lane_id() == 0) got = atomicAdd(counter, kWalkChunk);
          got = __shfl(got, 0);
          const int64_t lo = dyn_base + got;
          drained = lo >= items;
          chunk_lo = drained ? items : (int)lo;
          chunk_hi = drained ? items : (int)min<int64_t>(items, lo + kWalkChunk);
        }
        first = chunk_lo;
        avail = chunk_hi - chunk_lo;
        chunk_lo += min(avail, __popcll(needm));
      } else {
        const int leader = __builtin_ctzll(needm);
        int f = 0;
        if (lane_id() == leader) f = atomicAdd(&wg_next, __popcll(needm));
        first = __shfl(f, leader);
        avail = max(0, wg_hi - first);
      }
      // lanes past the end of the chunk (or range) wait for the next chunk,
      // or retire once there is none
      const int rank_in = lanes_below(needm);
      if (need && rank_in >= avail) {
        retired = kChunks ? drained : true;
      } else if (need) {
        const int item = first + rank_in;
        if (item < r) {  // static splitter
          const int start = item << log2B;
          const int bsize = min(1 << log2B, N - start);
          x = start + (int)splitter_offset((uint32_t)item, seed, (uint32_t)bsize);
          if (kLevel0 && kBatched) {
            lid = find_instance(a.off, a.L, x);
            base = a.off[lid];
            size = (int)(a.off[lid + 1] - base);
          }
          sid = item;
          k = 0;
          steps = 0;
        } else {  // virtual splitter standing at the head of list l
          const int l = item - r;
          int h;
          bool ok = true;
          if (kLevel0) {
            if (kBatched) {
              base = a.off[l];
              size = (int)(a.off[l + 1] - base);
            } else {
              base = 0;
              size = N;
            }
            lid = l;
            if (size == 0) {
              ok = false;  // empty list: a weightless one-node list above
            } else {
              const unsigned long long tri =
                  (unsigned long long)size * (unsigned long long)(size - 1) / 2ull;
              const long long hl = (long long)(tri - a.lsum[l]);
              if (a.ltails[l] != 1 || hl < 0 || hl >= size) {
                atomicOr(&a.lerr[l], a.ltails[l] != 1 ? kErrTails : kErrHead);
                ok = false;
              }
              h = (int)(base + hl);
            }
          } else {
            h = head_base + l;
            if (h >= N) {
              errbits |= kErrBase;
              ok = false;
            }
          }
          if (!ok) {
            store_pair(&a.link_out[item], -1, 0);
          } else if (is_static(h, N, log2B, seed)) {
            store_pair(&a.link_out[item], h >> log2B, 0);
          } else {
            x = h;
            sid = item;
            k = 0;
            steps = 0;
          }
        }
      }
    }
    if (__ballot(!retired) == 0) break;
    // Up to kWalkBurst steps before looking for new work: when the steps hit
    // in cache (local layouts) the work-distribution code, not memory, would
    // otherwise set the pace; random layouts do not notice either way.
    for (int rep = 0; rep < kWalkBurst && sid >= 0; ++rep) {
      int y, w;
      bool tail;
      if (kLevel0) {
        const int s = kPacked ? a.work[x] : a.succ0[x];
        const int xl = (int)(x - base);
        tail = (s == -1) | (s == xl);
        if (!tail && (unsigned)s >= (unsigned)size) {
          atomicOr(&a.lerr[lid], kErrRange);
          tail = true;
        }
        y = (int)(base + s);
        w = (!kPacked && a.weight0) ? a.weight0[x] : 1;
      } else {
        const int2 in = a.link_in[x];
        tail = in.x == -1;
        if (!tail && (unsigned)in.x >= (unsigned)N) {
          errbits |= kErrBase;
          tail = true;
        }
        y = in.x;
        w = in.y;
      }
      if (kLevel0 && kPacked) a.work[x] = (sid << kbits) | k;
      else store_pair(&a.state[x], sid, k);
      k += w;
      if (tail) {
        store_pair(&a.link_out[sid], -1, k);
        sid = -1;
      } else if (is_static(y, N, log2B, seed)) {
        store_pair(&a.link_out[sid], y >> log2B, k);
        sid = -1;
      } else if (++steps >= max_walk) {
        const int t = atomicAdd(dyn, 1);
        if (t >= a.cap) {
          errbits |= kErrOverflow;
          store_pair(&a.link_out[sid], -1, k);
          sid = -1;
        } else {
          const int nid = r + a.L + t;
          store_pair(&a.link_out[sid], nid, k);
          sid = nid;
          k = 0;
          steps = 0;
          x = y;
        }
      } else {
        x = y;
      }
    }
  }
  if (errbits) atomicOr(&ctl->err, errbits);
}

// ------------------------------------------------- caller-chosen splitters
// Level 0 of one list with the splitters chosen by the caller (Section 3.2's
// random-versus-even comparison).  "Is y a splitter" is then no longer
// arithmetic: lr_mark_splitters overwrites each splitter's slot of the
// successor copy with the mark -(2 + splitter index) and keeps the
// successor it replaced, and the walk learns that it reached a splitter from
// the word it reads at the next node anyway.  Distinct ids leave exactly one
// mark per splitter; a repeated id or one out of range raises kErrSplitter.
__global__ void __launch_bounds__(256) lr_mark_splitters(int32_t* __restrict__ work,
                                                         const int32_t* __restrict__ splitters,
                                                         int r, int n, int32_t* __restrict__ ssucc,
                                                         int32_t* lerr) {
  bool bad = false;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < r; s += gridDim.x * blockDim.x) {
    const int x = splitters[s];
    int old = -1;
    if ((unsigned)x >= (unsigned)n) {
      bad = true;
    } else {
      old = atomicExch(&work[x], -(2 + s));
      bad |= old <= -2;  // a second mark of one node
    }
    ssucc[s] = old;
  }
  if (__ballot(bad) && lane_id() == 0) atomicOr(lerr, kErrSplitter);
}

// The level-0 walk over marked splitters (one list, packed state).  A lane
// holds the node x it has reached and x's successor word sx, read one step
// earlier: it writes x's packed state over sx's slot, then reads the word of
// the successor, which tells whether that node is a splitter (a mark) or
// gives the next successor.  A splitter's own slot keeps its mark, which is
// its state (its sublist, offset 0) for the final scatter: the walker that
// arrives from its predecessor may read the mark at any time during the
// kernel.  Work distribution and cuts as in lr_walk.
__global__ void __launch_bounds__(1024) lr_walk_marked(WalkArgs a,
                                                       const int32_t* __restrict__ splitters,
                                                       const int32_t* __restrict__ ssucc, int r) {
  LrCtl* ctl = a.ctl;
  const int N = ctl->lv[0].n;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->lv[0].r = r;
  const int items = r + 1;  // chosen splitters, then the virtual one at the head
  int* dyn = &ctl->lv[0].dyn;
  __shared__ int wg_next;
  const int per = (int)(((int64_t)items + gridDim.x - 1) / gridDim.x);
  const int wg_lo = min(items, (int)((int64_t)blockIdx.x * per));
  const int wg_hi = min(items, wg_lo + per);
  if (threadIdx.x == 0) wg_next = wg_lo;
  __syncthreads();

  int sid = -1, x = 0, sx = 0, k = 0, steps = 0;
  bool at_mark = false;  // x is a chosen splitter: its slot keeps the mark
  bool retired = false;
  int errbits = 0;
  while (true) {
    const bool need = (sid < 0) & !retired;
    const uint64_t needm = __ballot(need);
    if (needm) {
      const int leader = __builtin_ctzll(needm);
      int first = 0;
      if (lane_id() == leader) first = atomicAdd(&wg_next, __popcll(needm));
      first = __shfl(first, leader);
      if (need) {
        const int item = first + lanes_below(needm);
        if (item >= wg_hi) {
          retired = true;
        } else if (item < r) {  // a chosen splitter
          const int y = splitters[item];
          if ((unsigned)y >= (unsigned)N) {  // reported by the marking pass
            store_pair(&a.link_out[item], -1, 0);
          } else {
            sid = item;
            x = y;
            sx = ssucc[item];
            k = 0;
            steps = 0;
            at_mark = true;
          }
        } else {  // the virtual splitter at the head
          const unsigned long long tri =
              (unsigned long long)N * (unsigned long long)(N - 1) / 2ull;
          const long long h = (long long)(tri - a.lsum[0]);
          if (a.ltails[0] != 1 || h < 0 || h >= N) {
            atomicOr(&a.lerr[0], a.ltails[0] != 1 ? kErrTails : kErrHead);
            store_pair(&a.link_out[item], -1, 0);
          } else {
            const int v = a.work[(int)h];
            if (v <= -2) {  // the head is a chosen splitter itself
              store_pair(&a.link_out[item], -(v + 2), 0);
            } else {
              sid = item;
              x = (int)h;
              sx = v;
              k = 0;
              steps = 0;
              at_mark = false;
            }
          }
        }
      }
    }
    if (__ballot(!retired) == 0) break;
    for (int rep = 0; rep < kWalkBurst && sid >= 0; ++rep) {
      bool tail = (sx == -1) | (sx == x);
      if (!tail && (unsigned)sx >= (unsigned)N) {
        atomicOr(&a.lerr[0], kErrRange);
        tail = true;
      }
      if (!at_mark) a.work[x] = (sid << a.kbits) | k;
      at_mark = false;
      ++k;
      if (tail) {
        store_pair(&a.link_out[sid], -1, k);
        sid = -1;
        continue;
      }
      const int y = sx;
      const int v = a.work[y];
      if (v <= -2) {
        // (an index past the level's nodes only comes from a malformed input
        // word, which the head-find pass has reported; level 1 bounds it)
        store_pair(&a.link_out[sid], -(v + 2), k);
        sid = -1;
      } else if (++steps >= a.max_walk) {
        const int t = atomicAdd(dyn, 1);
        if (t >= a.cap) {
          errbits |= kErrOverflow;
          store_pair(&a.link_out[sid], -1, k);
          sid = -1;
        } else {
          const int nid = r + 1 + t;
          store_pair(&a.link_out[sid], nid, k);
          sid = nid;
          k = 0;
          steps = 0;
          x = y;
          sx = v;
        }
      } else {
        x = y;
        sx = v;
      }
    }
  }
  if (errbits) atomicOr(&ctl->err, errbits);
}

// Longest level-0 sublist (stats only): the largest weight among the level-1
// nodes, which for unit weights is the node count of each sublist piece.
__global__ void __launch_bounds__(256) lr_sublist_max(const int2* __restrict__ link,
                                                      const LrCtl* ctl, int L, int cap0,
                                                      int32_t* out) {
  const int N1 = level_nodes(ctl, 1, L, cap0);
  int mx = 0;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < N1; j += gridDim.x * blockDim.x)
    mx = max(mx, link[j].y);
  mx = -wave_min(-mx);
  if (lane_id() == 0 && mx > 0) atomicMax(out, mx);
}

// ------------------------------------------------------------ base: LDS
// Ranks a weighted forest of at most kMaxCutoff nodes in one workgroup:
// predecessor links are built in LDS, then pointer jumping along them sums
// the weights of all earlier nodes (exclusive prefix from each head).  The
// heads must be exactly the ids head_base .. head_base + L - 1.
__global__ void __launch_bounds__(kBaseThreads) lr_base_lds(const int2* __restrict__ link,
                                                            int32_t* __restrict__ srank,
                                                            LrCtl* ctl, int level, int L,
                                                            int cap_prev) {
  __shared__ int lnk[kMaxCutoff];
  __shared__ int pre[kMaxCutoff];
  __shared__ int nheads;
  __shared__ int bad;
  __shared__ unsigned long long total;
  const int N = level_nodes(ctl, level, L, cap_prev);
  const int head_base = ctl->lv[level - 1].r;
  const int tid = threadIdx.x;
  if (tid == 0) {
    nheads = 0;
    bad = 0;
    total = 0ull;
  }
  if (N > kMaxCutoff) {
    if (tid == 0) atomicOr(&ctl->err, kErrBase);
    return;
  }
  for (int j = tid; j < N; j += kBaseThreads) lnk[j] = -1;
  __syncthreads();
  // All global loads of a phase are issued before any is used: one
  // workgroup alone cannot hide their latency otherwise.
  unsigned long long mytotal = 0;
  {
    int2 in[kPerThread];
#pragma unroll
    for (int t = 0; t < kPerThread; ++t) {
      const int j = tid + t * kBaseThreads;
      in[t] = j < N ? link[j] : make_int2(-1, 0);
    }
#pragma unroll
    for (int t = 0; t < kPerThread; ++t) {
      const int j = tid + t * kBaseThreads;
      if (j >= N) continue;
      mytotal += (unsigned)in[t].y;
      if (in[t].x >= 0 && in[t].x < N) {
        if (atomicExch(&lnk[in[t].x], j) != -1) bad = 1;
      } else if (in[t].x != -1) {
        bad = 1;
      }
    }
  }
  __syncthreads();
  int myheads = 0;
  {
    int pw[kPerThread];
#pragma unroll
    for (int t = 0; t < kPerThread; ++t) {
      const int j = tid + t * kBaseThreads;
      const int p = j < N ? lnk[j] : -1;
      pw[t] = p >= 0 ? link[p].y : 0;
      if (j < N && p < 0) {
        ++myheads;
        if (j < head_base || j >= head_base + L) bad = 1;
      }
    }
#pragma unroll
    for (int t = 0; t < kPerThread; ++t) {
      const int j = tid + t * kBaseThreads;
      if (j < N) pre[j] = pw[t];
    }
  }
  if (myheads) atomicAdd(&nheads, myheads);
  mytotal = wave_sum(mytotal);
  if (lane_id() == 0 && mytotal) atomicAdd(&total, mytotal);
  __syncthreads();
  int rounds = 0;
  while ((1 << rounds) < N) ++rounds;
  int pa[kPerThread], la[kPerThread];
  for (int it = 0; it < rounds; ++it) {
#pragma unroll
    for (int t = 0; t < kPerThread; ++t) {
      const int j = tid + t * kBaseThreads;
      la[t] = -1;
      pa[t] = 0;
      if (j < N) {
        const int p = lnk[j];
        if (p >= 0) {
          pa[t] = pre[p];
          la[t] = lnk[p];
        } else {
          la[t] = -2;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kPerThread; ++t) {
      const int j = tid + t * kBaseThreads;
      if (j < N && la[t] != -2) {
        pre[j] += pa[t];
        lnk[j] = la[t];
      }
    }
    __syncthreads();
  }
  for (int j = tid; j < N; j += kBaseThreads) {
    if (lnk[j] != -1) bad = 1;
    srank[j] = pre[j];
  }
  __syncthreads();
  if (tid == 0) {
    if (bad || nheads != L) atomicOr(&ctl->err, kErrBase);
    ctl->base_total = total;
  }
}

// ---------------------------------------------------- base: device-wide
// The same predecessor pointer jumping for forests too large for one
// workgroup, one launch per round; (prefix, link) pairs are packed into one
// 64-bit word so a gather reads a consistent pair.
__device__ __forceinline__ unsigned long long pack_pl(int prefix, int lnk) {
  return ((unsigned long long)(unsigned)prefix << 32) | (unsigned)lnk;
}

__global__ void wide_clear(int32_t* lnk, const LrCtl* ctl, int level, int L, int cap_prev) {
  const int N = level_nodes(ctl, level, L, cap_prev);
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < N; j += gridDim.x * blockDim.x)
    lnk[j] = -1;
}

__global__ void wide_pred(const int2* __restrict__ link, int32_t* lnk, LrCtl* ctl, int level,
                          int L, int cap_prev) {
  const int N = level_nodes(ctl, level, L, cap_prev);
  int bad = 0;
  unsigned long long tot = 0;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < N; j += gridDim.x * blockDim.x) {
    const int2 in = link[j];
    tot += (unsigned)in.y;
    if (in.x >= 0 && in.x < N) {
      if (atomicExch(&lnk[in.x], j) != -1) bad = 1;
    } else if (in.x != -1) {
      bad = 1;
    }
  }
  tot = wave_sum(tot);
  if (lane_id() == 0 && tot) atomicAdd(&ctl->base_total, tot);
  if (bad) atomicOr(&ctl->err, kErrBase);
}

__global__ void wide_init(const int2* __restrict__ link, const int32_t* __restrict__ lnk,
                          unsigned long long* pl, LrCtl* ctl, int level, int L, int cap_prev) {
  const int N = level_nodes(ctl, level, L, cap_prev);
  const int head_base = ctl->lv[level - 1].r;
  int bad = 0;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < N; j += gridDim.x * blockDim.x) {
    const int p = lnk[j];
    if (p < 0 && (j < head_base || j >= head_base + L)) bad = 1;
    pl[j] = pack_pl(p >= 0 ? link[p].y : 0, p);
  }
  if (bad) atomicOr(&ctl->err, kErrBase);
}

__global__ void wide_jump(unsigned long long* pl, const LrCtl* ctl, int level, int L,
                          int cap_prev) {
  const int N = level_nodes(ctl, level, L, cap_prev);
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < N; j += gridDim.x * blockDim.x) {
    const unsigned long long v = pl[j];
    const int p = (int)(unsigned)v;
    if (p < 0) continue;
    const unsigned long long q = pl[p];
    const int pre = (int)(v >> 32) + (int)(q >> 32);
    pl[j] = pack_pl(pre, (int)(unsigned)q);
  }
}

__global__ void wide_final(const unsigned long long* __restrict__ pl, int32_t* srank, LrCtl* ctl,
                           int level, int L, int cap_prev) {
  const int N = level_nodes(ctl, level, L, cap_prev);
  int bad = 0;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < N; j += gridDim.x * blockDim.x) {
    const unsigned long long v = pl[j];
    if ((int)(unsigned)v != -1) bad = 1;
    srank[j] = (int)(v >> 32);
  }
  if (bad) atomicOr(&ctl->err, kErrBase);
}

// ---------------------------------------------------------------- expand
// rank of node x = rank of its splitter + weight before x in its sublist.
__global__ void __launch_bounds__(256) lr_expand(const int2* __restrict__ state,
                                                 const int32_t* __restrict__ srank_up,
                                                 int32_t* __restrict__ out, LrCtl* ctl, int level,
                                                 int L, int cap_prev, int cap_here) {
  const int N = level_nodes(ctl, level, L, cap_prev);
  const int Nup = level_nodes(ctl, level + 1, L, cap_here);
  int bad = 0;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < N; j += gridDim.x * blockDim.x) {
    const int2 s = state[j];
    int v = 0;
    if ((unsigned)s.x < (unsigned)Nup) v = srank_up[s.x] + s.y;
    else bad = 1;
    out[j] = v;
  }
  if (bad) atomicOr(&ctl->err, kErrTotal);
}

// Level 0: write the output ranks (from the head, or to the tail).
constexpr int kExpandPer = 4;
template <bool kBatched, bool kToTail, bool kPacked>
__global__ void __launch_bounds__(256) lr_expand0(const int2* __restrict__ state,
                                                  const int32_t* __restrict__ srank_up,
                                                  int32_t* rank,
                                                  const int64_t* __restrict__ off, LrCtl* ctl,
                                                  int L, int cap_here, int kbits_near,
                                                  int kbits_far) {
  const int N = ctl->lv[0].n;
  // the walk's choice of packing (see lr_walk), from the same count
  const int kbits = kbits_far > 0 && 2ull * ctl->near <= (unsigned long long)N ? kbits_far
                                                                                 : kbits_near;
  const int Nup = level_nodes(ctl, 1, L, cap_here);
  int bad = 0;
  // kExpandPer nodes per thread per pass, loads first: the splitter-rank
  // gathers of one thread are in flight together.  The packed words are read
  // once and overwritten, so they are streamed past the cache (nontemporal)
  // and the gathered splitter ranks keep it.
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j0 < N;
       j0 += kExpandPer * stride) {
    int2 s[kExpandPer];
#pragma unroll
    for (int u = 0; u < kExpandPer; ++u) {
      const int64_t j = j0 + u * stride;
      s[u] = make_int2(-1, 0);
      if (j < N) {
        if (kPacked) {
          // a packed (sublist, offset) word, or the mark -(2 + splitter) that
          // a caller-chosen splitter keeps (its sublist, offset 0)
          const int w = __builtin_nontemporal_load(&rank[j]);
          s[u] = w >= 0 ? make_int2((int)((unsigned)w >> kbits), w & ((1 << kbits) - 1))
                        : make_int2(-(w + 2), 0);
        } else {
          s[u] = state[j];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kExpandPer; ++u) {
      const int64_t j = j0 + u * stride;
      if (j >= N) break;
      int v = 0;
      if ((unsigned)s[u].x < (unsigned)Nup) v = srank_up[s[u].x] + s[u].y;
      else bad = 1;
      if (kToTail) {
        int size = N;
        if (kBatched) {
          const int l = find_instance(off, L, j);
          size = (int)(off[l + 1] - off[l]);
        }
        v = size - 1 - v;
      }
      __builtin_nontemporal_store(v, &rank[j]);
    }
  }
  if (bad) atomicOr(&ctl->err, kErrTotal);
}

// ------------------------------------------------ per-node batched passes
// Calls f(g, l, base, size) for every node g of a batch, with l its list.
// Each wave owns a contiguous run of chunks of kWave * kListedPer nodes: one
// search of the offset table per wave, then every lane follows the list
// boundaries forward (a search per node costs a chain of dependent loads).
// Lanes of a wave touch consecutive nodes, so accesses stay coalesced.
constexpr int kListedPer = 16;
template <class F>
__device__ __forceinline__ void for_each_listed(const int64_t* __restrict__ off, int L, int64_t n,
                                                F f) {
  constexpr int64_t kChunk = kWave * kListedPer;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int nwaves = (gridDim.x * blockDim.x) / kWave;
  const int lane = lane_id();
  const int64_t nchunks = (n + kChunk - 1) / kChunk;
  const int64_t per = (nchunks + nwaves - 1) / nwaves;
  const int64_t ci0 = (int64_t)wave * per;
  const int64_t ci1 = ci0 + per < nchunks ? ci0 + per : nchunks;
  if (ci0 >= ci1) return;
  int l = find_instance(off, L, ci0 * kChunk);
  int64_t base = off[l], end = off[l + 1];
  for (int64_t ci = ci0; ci < ci1; ++ci)
    for (int t = 0; t < kListedPer; ++t) {
      const int64_t g = ci * kChunk + t * kWave + lane;
      if (g >= n) break;
      while (g >= end) {  // later lists (empty ones skipped)
        ++l;
        base = end;
        end = off[l + 1];
      }
      f(g, l, base, (int)(end - base));
    }
}

// --------------------------------------------------------------- Wyllie
// Pointer jumping (Section 3.1) on packed (distance to tail, next) pairs:
// one 64-bit read of the node's own pair, one 64-bit gather of its next's
// pair, one 64-bit write.  Updating in place is safe: a gather that sees a
// pair already advanced in this round still holds a consistent
// (distance, next) relation, only a longer jump.
__device__ __forceinline__ unsigned long long pack_dn(int dist, int next) {
  return ((unsigned long long)(unsigned)dist << 32) | (unsigned)next;
}

template <bool kBatched>
__global__ void __launch_bounds__(1024) wy_init(const int32_t* __restrict__ succ,
                                                const int64_t* __restrict__ off, int L, int n,
                                                unsigned long long* __restrict__ pair,
                                                int32_t* lerr) {
  auto one = [&](int64_t g, int l, int64_t base, int size) {
    const int s = succ[g];
    const int xl = (int)(g - base);
    bool tail = (s == -1) | (s == xl);
    if (!tail && (unsigned)s >= (unsigned)size) {
      atomicOr(&lerr[l], kErrRange);
      tail = true;
    }
    pair[g] = tail ? pack_dn(0, -1) : pack_dn(1, (int)(base + s));
  };
  if (kBatched) {
    for_each_listed(off, L, n, one);
  } else {
    const int stride = gridDim.x * blockDim.x;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n; g += stride) one(g, 0, 0, n);
  }
}

__global__ void __launch_bounds__(1024) wy_jump(unsigned long long* __restrict__ pair, int n) {
  const int stride = gridDim.x * blockDim.x;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n; g += stride) {
    const unsigned long long v = pair[g];
    const int nx = (int)(unsigned)v;
    if (nx < 0) continue;
    const unsigned long long q = pair[nx];
    pair[g] = pack_dn((int)(v >> 32) + (int)(q >> 32), (int)(unsigned)q);
  }
}

template <bool kBatched, bool kToTail>
__global__ void __launch_bounds__(1024) wy_final(const unsigned long long* __restrict__ pair,
                                                 const int64_t* __restrict__ off, int L, int n,
                                                 int32_t* __restrict__ rank, int32_t* lerr) {
  auto one = [&](int64_t g, int l, int64_t, int size) {
    const unsigned long long v = pair[g];
    const int dist = (int)(v >> 32);
    if ((int)(unsigned)v != -1) atomicOr(&lerr[l], kErrBase);
    rank[g] = kToTail ? dist : size - 1 - dist;
  };
  if (kBatched) {
    for_each_listed(off, L, n, one);
  } else {
    const int stride = gridDim.x * blockDim.x;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n; g += stride) one(g, 0, 0, n);
  }
}

// ------------------------------------------------------- small one-group
// A whole batch of at most kMaxCutoff nodes ranked by one workgroup:
// predecessor links in LDS, pointer jumping along them with unit weights.
// succ is read before any rank is written (in place allowed).  With weights,
// a node's own term is its predecessor's weight instead of 1.
__global__ void __launch_bounds__(kBaseThreads) lr_small(const int32_t* succ,
                                                         const int32_t* weight,
                                                         const int64_t* __restrict__ off, int L,
                                                         int n, int32_t* rank,
                                                         int to_tail, int32_t* ltails,
                                                         int32_t* lerr) {
  __shared__ int lnk[kMaxCutoff];
  __shared__ int pre[kMaxCutoff];
  const int tid = threadIdx.x;
  for (int j = tid; j < n; j += kBaseThreads) lnk[j] = -1;
  __syncthreads();
  // Thread t reads the kPerThread consecutive ids from t * kPerThread, all
  // loads first, and follows the list boundaries forward (one search of the
  // offset table per thread).
  const int j0 = tid * kPerThread;
  if (j0 < n) {
    int sv[kPerThread];
    if (j0 + kPerThread <= n && (reinterpret_cast<uintptr_t>(succ) & 15) == 0) {
      const int4* s4 = reinterpret_cast<const int4*>(succ + j0);
#pragma unroll
      for (int q = 0; q < kPerThread / 4; ++q) {
        const int4 v = s4[q];
        sv[4 * q] = v.x;
        sv[4 * q + 1] = v.y;
        sv[4 * q + 2] = v.z;
        sv[4 * q + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int t = 0; t < kPerThread; ++t) sv[t] = j0 + t < n ? succ[j0 + t] : -1;
    }
    int l = find_instance(off, L, j0);
    int base = (int)off[l], end = (int)off[l + 1];
    for (int t = 0; t < kPerThread; ++t) {
      const int j = j0 + t;
      if (j >= n) break;
      while (j >= end) {
        ++l;
        base = end;
        end = (int)off[l + 1];
      }
      const int s = sv[t];
      const bool tail = (s == -1) | (s == j - base);
      if (tail) {
        atomicAdd(&ltails[l], 1);
      } else if ((unsigned)s >= (unsigned)(end - base)) {
        atomicOr(&lerr[l], kErrRange);
      } else if (atomicExch(&lnk[base + s], j) != -1) {
        atomicOr(&lerr[l], kErrBase);
      }
    }
  }
  __syncthreads();
  for (int j = tid; j < n; j += kBaseThreads) {
    const int p = lnk[j];
    pre[j] = p >= 0 ? (weight ? weight[p] : 1) : 0;
  }
  __syncthreads();
  int rounds = 0;
  while ((1 << rounds) < n) ++rounds;
  int pa[kPerThread], la[kPerThread];
  for (int it = 0; it < rounds; ++it) {
#pragma unroll
    for (int t = 0; t < kPerThread; ++t) {
      const int j = tid + t * kBaseThreads;
      la[t] = -2;
      pa[t] = 0;
      if (j < n) {
        const int p = lnk[j];
        if (p >= 0) {
          pa[t] = pre[p];
          la[t] = lnk[p];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kPerThread; ++t) {
      const int j = tid + t * kBaseThreads;
      if (j < n && la[t] != -2) {
        pre[j] += pa[t];
        lnk[j] = la[t];
      }
    }
    __syncthreads();
  }
  if (j0 < n) {
    int l = find_instance(off, L, j0);
    int base = (int)off[l], end = (int)off[l + 1];
    for (int t = 0; t < kPerThread; ++t) {
      const int j = j0 + t;
      if (j >= n) break;
      while (j >= end) {
        ++l;
        base = end;
        end = (int)off[l + 1];
      }
      if (lnk[j] != -1) atomicOr(&lerr[l], kErrBase);
      const int v = pre[j];
      rank[j] = to_tail ? end - base - 1 - v : v;
    }
  }
}

// ------------------------------------------------------------ full check
// Complete check of the output (validate = 1): per list, ranks are a
// permutation of 0..size-1 and rank[succ[i]] = rank[i] + 1 off the tail.
__global__ void chk_clear(int32_t* cnt, int n) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
    cnt[j] = 0;
}

template <bool kBatched>
__global__ void chk_count(const int32_t* __restrict__ succ, const int32_t* __restrict__ rank,
                          const int64_t* __restrict__ off, int L, int n, int to_tail,
                          int32_t* cnt, int32_t* lerr) {
  auto one = [&](int64_t g, int l, int64_t base, int size) {
    int r = rank[g];
    if (to_tail) r = size - 1 - r;
    if ((unsigned)r >= (unsigned)size) {
      atomicOr(&lerr[l], kErrCheck);
      return;
    }
    atomicAdd(&cnt[base + r], 1);
    const int s = succ[g];
    const int xl = (int)(g - base);
    if (s == -1 || s == xl) return;
    if ((unsigned)s >= (unsigned)size) {
      atomicOr(&lerr[l], kErrCheck);
      return;
    }
    int rs = rank[base + s];
    if (to_tail) rs = size - 1 - rs;
    if (rs != r + 1) atomicOr(&lerr[l], kErrCheck);
  };
  // a grid-stride sweep, not for_each_listed: all waves then work in one
  // window of the batch, whose ranks the random gathers above find in cache
  // (contiguous runs per wave were slower: 27.7 against 17.6 ms on 4096 lists)
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n; g += gridDim.x * blockDim.x) {
    if (kBatched) {
      const int l = find_instance(off, L, g);
      one(g, l, off[l], (int)(off[l + 1] - off[l]));
    } else {
      one(g, 0, 0, n);
    }
  }
}

template <bool kBatched>
__global__ void chk_perm(const int32_t* __restrict__ cnt, const int64_t* __restrict__ off, int L,
                         int n, int32_t* lerr) {
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n; g += gridDim.x * blockDim.x) {
    if (cnt[g] != 1) {
      const int l = kBatched ? find_instance(off, L, g) : 0;
      atomicOr(&lerr[l], kErrCheck);
    }
  }
}

// Weighted calls with a status: the level sums are weights, not node counts,
// so the coverage check by the base total does not apply.  Instead every
// state word starts as "no sublist", and an expansion that meets one (a node
// no walk reached: a cycle beside the list) reports it.
__global__ void __launch_bounds__(256) lr_state_clear(int2* __restrict__ state, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    state[i] = make_int2(-1, 0);
}

// ---------------------------------------------------------------- status
__global__ void lr_status(const LrCtl* ctl, const int32_t* lerr, const int32_t* ltails,
                          const int64_t* off, int L, int n0, int check_total, int check_tails,
                          int32_t* status) {
  const bool global_bad = ctl && (ctl->err != 0 ||
                                  (check_total && ctl->base_total != (unsigned long long)n0));
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < L; l += gridDim.x * blockDim.x) {
    const int64_t size = off[l + 1] - off[l];
    bool bad = global_bad || lerr[l] != 0;
    if (check_tails && size > 0 && ltails[l] != 1) bad = true;
    status[l] = (lerr[l] & kErrSplitter) ? PJ_EINVAL : bad ? PJ_EBADLIST : PJ_OK;
  }
}

// ------------------------------------------------------------------ host
inline int ilog2(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

inline int grid_for(int64_t n, int block, int cap) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

struct Plan {
  int algo = PJ_ALGO_RULING_SET;
  bool small = false;
  int levels = 0;          // walk levels
  int base_kind = 1;       // 1 LDS, 2 device-wide
  int64_t bound[PJ_MAX_LEVELS + 2] = {};
  int log2B[PJ_MAX_LEVELS + 1] = {};
  int cap[PJ_MAX_LEVELS + 1] = {};
  int wide_rounds = 0;
  int wy_rounds = 0;
  bool packed = false;     // level 0 state packed into the output buffer
  int kbits = 0;           // offset bits of the packed state
  int max_walk0 = 0;       // cut length at level 0
  int log2B_far = 0;       // > 0: level 0 may pick this on the device (see lr_walk),
  int kbits_far = 0;       // with these offset bits (packed form)
  int max_walk_far = 0;    // and this cut length
  int64_t chosen = 0;      // > 0: level 0 uses this many caller-chosen splitters
};

// rank may be succ itself (in place: the successors are overwritten by the
// ranks, the way Section 3.2 reuses the device successor array for the
// output); any other overlap is rejected.  The full output check reads succ
// after the ranks are written, so it needs two arrays.
inline int check_alias(const int32_t* succ, const int32_t* rank, int64_t n, bool validate) {
  if (n <= 0) return PJ_OK;
  const uintptr_t s0 = (uintptr_t)succ, r0 = (uintptr_t)rank;
  const uintptr_t bytes = (uintptr_t)n * sizeof(int32_t);
  if (s0 == r0) return validate ? PJ_EINVAL : PJ_OK;
  if (s0 < r0 + bytes && r0 < s0 + bytes) return PJ_EINVAL;
  return PJ_OK;
}

inline int bits_for(int64_t v) {  // bits to hold values 0..v-1
  int b = 0;
  while ((int64_t(1) << b) < v) ++b;
  return b;
}

// pack = false keeps level 0 in the separate (sublist, offset) state, which
// weighted calls need (an offset is then a weight sum, not a step count).
// chosen > 0: level 0 has that many caller-chosen splitters (never the
// one-workgroup path, so that they are used).
Plan make_plan(int64_t n0, int64_t L, int64_t max_size, const pj_opts& o, bool pack = true,
               int64_t chosen = 0) {
  Plan p;
  p.algo = o.algo == PJ_ALGO_WYLLIE ? PJ_ALGO_WYLLIE : PJ_ALGO_RULING_SET;
  p.bound[0] = n0;
  if (p.algo == PJ_ALGO_WYLLIE) {
    p.wy_rounds = ilog2((int)std::max<int64_t>(max_size, 1));
    return p;
  }
  p.chosen = chosen;
  if (n0 <= kMaxCutoff && n0 <= o.cutoff && chosen == 0) {
    p.small = true;
    return p;
  }
  int lv = 0;
  for (;;) {
    const int64_t b = p.bound[lv];
    if (lv > 0) {
      if (b <= o.cutoff) {
        p.base_kind = 1;
        break;
      }
      if (lv >= PJ_MAX_LEVELS || b * 4 > p.bound[lv - 1] * 3) {
        p.base_kind = 2;
        p.wide_rounds = ilog2((int)b);
        break;
      }
    }
    const int spacing = lv == 0 ? o.spacing : o.spacing_up;
    p.log2B[lv] = ilog2(std::max(2, spacing));
    const int64_t r = lv == 0 && chosen > 0 ? chosen
                                            : (b + (1ll << p.log2B[lv]) - 1) >> p.log2B[lv];
    int mw = o.max_walk;
    if (lv == 0) {
      // Pack (sublist id, offset) into 31 bits when the id space allows an
      // offset of at least 4 bits; the cut length then bounds the offset.
      p.packed = false;
      for (int kb = bits_for(mw); pack && kb >= 4; --kb) {
        const int mwk = std::min(mw, 1 << kb);
        const int64_t ids = r + L + b / mwk + 64;
        if (bits_for(ids) + kb <= 31) {
          p.packed = true;
          p.kbits = kb;
          mw = mwk;
          break;
        }
      }
      p.max_walk0 = mw;
    }
    p.cap[lv] = (int)(b / mw + 64);
    p.bound[lv + 1] = r + L + p.cap[lv];
    ++lv;
  }
  p.levels = lv;
  return p;
}

// Completes a plan made for level-0 spacing kLocalSpacing with the far
// alternative (see lr_walk): its packing and cut length.  The far sublist ids
// are fewer, so the offset may take more bits; the cut length may only grow,
// which keeps the planned cut-point capacity sufficient.
void add_far_spacing(Plan& p, int64_t n0, int64_t L, int far, int max_walk) {
  if (far <= 0 || p.levels < 1 || p.algo != PJ_ALGO_RULING_SET || p.chosen > 0) return;
  const int lg = ilog2(far);
  const int64_t r = (n0 + (1ll << lg) - 1) >> lg;
  if (!p.packed) {
    p.log2B_far = lg;
    p.max_walk_far = p.max_walk0;
    return;
  }
  for (int kb = bits_for(max_walk); kb >= 4; --kb) {
    const int mwk = std::min(max_walk, 1 << kb);
    if (mwk < p.max_walk0) break;
    if (bits_for(r + L + n0 / mwk + 64) + kb <= 31) {
      p.log2B_far = lg;
      p.kbits_far = kb;
      p.max_walk_far = mwk;
      return;
    }
  }
}

struct Buffers {
  LrCtl* ctl = nullptr;
  unsigned long long* lsum = nullptr;
  int32_t* ltails = nullptr;
  int32_t* lerr = nullptr;
  int64_t* off1 = nullptr;            // {0, n} for the single-list call
  int2* state[PJ_MAX_LEVELS + 1] = {};
  int2* link[PJ_MAX_LEVELS + 2] = {};  // link[l] = input of level l (l >= 1)
  int32_t* srank[PJ_MAX_LEVELS + 2] = {};
  int32_t* wide_lnk = nullptr;
  unsigned long long* wide_pl = nullptr;
  unsigned long long* wy_pair = nullptr;
  int32_t* chk = nullptr;
  int32_t* status_tmp = nullptr;
  int32_t* ssucc = nullptr;           // successors of caller-chosen splitters
  int32_t* sub_max = nullptr;         // stats: longest level-0 sublist
};

// Carve (or, with ws == nullptr, just count) the buffers a plan needs.
size_t carve(const Plan& p, int64_t L, bool single, bool validate, bool want_status,
             Workspace* ws, Buffers* b) {
  size_t bytes = 0;
  auto take = [&](auto*& ptr, size_t count) {
    using T = std::remove_pointer_t<std::remove_reference_t<decltype(ptr)>>;
    bytes += ws_bytes(count, sizeof(T));
    if (ws) ptr = ws->take<T>(count);
  };
  take(b->ctl, 1);
  take(b->lsum, (size_t)std::max<int64_t>(L, 1));
  take(b->ltails, (size_t)std::max<int64_t>(L, 1));
  take(b->lerr, (size_t)std::max<int64_t>(L, 1));
  if (single) take(b->off1, 2);
  if (validate) take(b->chk, (size_t)p.bound[0]);
  if (want_status) take(b->status_tmp, (size_t)std::max<int64_t>(L, 1));
  if (p.algo == PJ_ALGO_WYLLIE) {
    take(b->wy_pair, (size_t)p.bound[0]);
    return bytes;
  }
  if (p.small) return bytes;
  take(b->sub_max, 1);
  if (p.chosen > 0) take(b->ssucc, (size_t)p.chosen);
  for (int l = 0; l < p.levels; ++l) {
    if (!(l == 0 && p.packed)) take(b->state[l], (size_t)p.bound[l]);
    take(b->link[l + 1], (size_t)p.bound[l + 1]);
    take(b->srank[l + 1], (size_t)p.bound[l + 1]);
  }
  if (p.base_kind == 2) {
    take(b->wide_lnk, (size_t)p.bound[p.levels]);
    take(b->wide_pl, (size_t)p.bound[p.levels]);
  }
  return bytes;
}

}  // namespace

int list_rank_impl(const int32_t* succ, const int64_t* d_off, int64_t L, const int64_t* h_off,
                   int64_t n_single, int32_t* rank, const pj_opts* user, hipStream_t stream,
                   const int32_t* weight) {
  const bool single = d_off == nullptr;
  if (L < 0) return PJ_EINVAL;
  if (single) L = 1;
  if (L > INT32_MAX / 2) return PJ_EINVAL;
  pj_opts o = resolved_opts(user);
  if (o.spacing > 65536 || o.spacing_up > 65536) return PJ_EINVAL;
  if (user && user->stats) {
    *user->stats = pj_stats{};
    user->stats->status = PJ_OK;
  }

  // total nodes and the largest list, from the host's view of the offsets
  int64_t n0 = 0, max_size = 0;
  std::vector<int64_t> hbuf;
  if (single) {
    n0 = n_single;
    max_size = n0;
  } else {
    if (L == 0) return PJ_OK;
    const int64_t* ho = h_off;
    if (!ho) {
      hbuf.resize((size_t)L + 1);
      PJ_HIP(hipMemcpyAsync(hbuf.data(), d_off, sizeof(int64_t) * (L + 1),
                            hipMemcpyDeviceToHost, stream));
      PJ_HIP(hipStreamSynchronize(stream));
      ho = hbuf.data();
    }
    if (ho[0] != 0) return PJ_EINVAL;
    for (int64_t l = 0; l < L; ++l) {
      const int64_t s = ho[l + 1] - ho[l];
      if (s < 0) return PJ_EINVAL;
      max_size = std::max(max_size, s);
    }
    n0 = ho[L];
  }
  if (n0 < 0 || n0 >= INT32_MAX) return PJ_EINVAL;
  if (n0 > 0 && (!succ || !rank)) return PJ_EINVAL;
  PJ_TRY(check_alias(succ, rank, n0, o.validate != 0));
  if (weight) {
    // weighted ranks are exclusive prefix sums from the head by the ruling
    // set; the to-tail form and the full check (a permutation test) do not
    // apply
    if (o.algo == PJ_ALGO_WYLLIE || o.to_tail || o.validate) return PJ_EINVAL;
    const uintptr_t w0 = (uintptr_t)weight, r0 = (uintptr_t)rank;
    const uintptr_t bytes = (uintptr_t)n0 * sizeof(int32_t);
    if (n0 > 0 && w0 < r0 + bytes && r0 < w0 + bytes) return PJ_EINVAL;
  }
  const bool want_status = o.validate && !o.d_status;
  if (n0 == 0 && !o.d_status) return PJ_OK;
  if (o.level0_state != PJ_STATE_AUTO && o.level0_state != PJ_STATE_SEPARATE) return PJ_EINVAL;
  // caller-chosen level-0 splitters: one unweighted list, ruling set, the
  // packed state (the marks live in the successor copy)
  const int64_t chosen = o.d_splitters && n0 > 0 ? o.n_splitters : 0;
  if (o.d_splitters && n0 > 0 &&
      (!single || weight || o.algo == PJ_ALGO_WYLLIE || o.level0_state == PJ_STATE_SEPARATE ||
       o.n_splitters < 1 || o.n_splitters > n0))
    return PJ_EINVAL;

  int far_spacing = 0;
  {  // ruling-set parameters left at zero come from the tune cache, if tuned
    pj_opts raw;
    pj_opts_init(&raw);
    if (user) raw = *user;
    apply_tuned(raw, n0, L);
    far_spacing = level0_spacing(raw.spacing, n0, single, &o.spacing);
    o.spacing_up = raw.spacing_up > 0 ? raw.spacing_up : o.spacing_up;
    o.cutoff = raw.cutoff > 0 ? std::min(std::max(raw.cutoff, 64), 16384) : o.cutoff;
    o.max_walk = raw.max_walk > 0 ? std::max(raw.max_walk, 16) : o.max_walk;
    if (raw.block > 0) o.block = std::min(1024, (raw.block + 63) / 64 * 64);
  }
  Plan p = make_plan(n0, L, max_size, o,
                     weight == nullptr && o.level0_state != PJ_STATE_SEPARATE, chosen);
  if (chosen > 0 && !p.packed) return PJ_EINVAL;  // too many splitters for the packed state
  add_far_spacing(p, n0, L, far_spacing, o.max_walk);
  Buffers b;
  const size_t need = carve(p, L, single, o.validate != 0, want_status, nullptr, &b);
  Workspace ws;
  PJ_TRY(workspace_acquire(ws, need, &o, stream));
  carve(p, L, single, o.validate != 0, want_status, &ws, &b);
  const int64_t* off = single ? b.off1 : d_off;
  int32_t* status = o.d_status ? o.d_status : b.status_tmp;

  PhaseTimer tm;
  pj_stats* st = user ? user->stats : nullptr;
  PJ_TRY(tm.begin(st != nullptr, stream));

  const int n = (int)n0;
  const int Li = (int)L;
  const int blk = o.block;
  const int cus = device_info().cus;
  const int gcap = cus * 16;

  hipLaunchKernelGGL(lr_init, dim3(grid_for(std::max<int64_t>(L, 64), 256, 1024)), dim3(256), 0,
                     stream, b.ctl, n, b.lsum, b.ltails, b.lerr, Li, b.off1);
  PJ_HIP(hipGetLastError());
  tm.mark("init");

  bool check_total = false, check_tails = false;
  if (n0 > 0 && p.algo == PJ_ALGO_WYLLIE) {
    if (o.validate || o.d_status) {
      if (single)
        hipLaunchKernelGGL(lr_headfind_single<false>, dim3(grid_for(n / 4 + 1, 256, 1024)),
                           dim3(256), 0, stream, succ, n, nullptr, b.lsum, b.ltails, b.lerr,
                           nullptr);
      else
        hipLaunchKernelGGL(lr_headfind_batched<false>,
                           dim3(grid_for(n / (kHfChunk * 4) + 1, 256, gcap)), dim3(256), 0,
                           stream, succ, off, Li, n, nullptr, b.lsum, b.ltails, b.lerr);
      check_tails = true;
      tm.mark("headfind");
    }
    const int g = grid_for(n, blk, gcap);
    if (single)
      hipLaunchKernelGGL(wy_init<false>, dim3(g), dim3(blk), 0, stream, succ, off, Li, n,
                         b.wy_pair, b.lerr);
    else
      hipLaunchKernelGGL(wy_init<true>, dim3(g), dim3(blk), 0, stream, succ, off, Li, n,
                         b.wy_pair, b.lerr);
    tm.mark("wyllie_init");
    for (int it = 0; it < p.wy_rounds; ++it)
      hipLaunchKernelGGL(wy_jump, dim3(g), dim3(blk), 0, stream, b.wy_pair, n);
    tm.mark("wyllie_jump");
    if (single) {
      if (o.to_tail)
        hipLaunchKernelGGL((wy_final<false, true>), dim3(g), dim3(blk), 0, stream, b.wy_pair, off,
                           Li, n, rank, b.lerr);
      else
        hipLaunchKernelGGL((wy_final<false, false>), dim3(g), dim3(blk), 0, stream, b.wy_pair,
                           off, Li, n, rank, b.lerr);
    } else {
      if (o.to_tail)
        hipLaunchKernelGGL((wy_final<true, true>), dim3(g), dim3(blk), 0, stream, b.wy_pair, off,
                           Li, n, rank, b.lerr);
      else
        hipLaunchKernelGGL((wy_final<true, false>), dim3(g), dim3(blk), 0, stream, b.wy_pair,
                           off, Li, n, rank, b.lerr);
    }
    tm.mark("wyllie_final");
  } else if (n0 > 0 && p.small) {
    hipLaunchKernelGGL(lr_small, dim3(1), dim3(kBaseThreads), 0, stream, succ, weight, off, Li,
                       n, rank, o.to_tail, b.ltails, b.lerr);
    check_tails = true;
    tm.mark("small");
  } else if (n0 > 0) {
    // level 0 head find (and, in the packed form, the successor copy, which
    // in place is already there)
    int32_t* copy = p.packed ? rank : nullptr;
    const bool copy_succ = p.packed && (const void*)succ != (const void*)rank;
    if (single) {
      auto k = copy_succ ? lr_headfind_single<true> : lr_headfind_single<false>;
      hipLaunchKernelGGL(k, dim3(grid_for(n / 4 + 1, 256, 1024)), dim3(256), 0, stream, succ, n,
                         copy, b.lsum, b.ltails, b.lerr, &b.ctl->near);
    } else {
      auto k = copy_succ ? lr_headfind_batched<true> : lr_headfind_batched<false>;
      hipLaunchKernelGGL(k, dim3(grid_for(n / (kHfChunk * 4) + 1, 256, gcap)), dim3(256), 0,
                         stream, succ, off, Li, n, copy, b.lsum, b.ltails, b.lerr);
    }
    PJ_HIP(hipGetLastError());
    if (p.chosen > 0) {
      hipLaunchKernelGGL(lr_mark_splitters, dim3(grid_for(p.chosen, 256, gcap)), dim3(256), 0,
                         stream, copy, o.d_splitters, (int)p.chosen, n, b.ssucc, b.lerr);
      PJ_HIP(hipGetLastError());
    }
    tm.mark("headfind");
    check_total = weight == nullptr;
    if (weight && status)
      for (int lv = 0; lv < p.levels; ++lv)
        hipLaunchKernelGGL(lr_state_clear, dim3(grid_for(p.bound[lv], 256, gcap)), dim3(256), 0,
                           stream, b.state[lv], p.bound[lv]);
    check_tails = true;
    // walks, level by level
    for (int lv = 0; lv < p.levels; ++lv) {
      WalkArgs a{};
      a.succ0 = succ;
      a.weight0 = weight;
      a.link_in = b.link[lv];
      a.off = off;
      a.lsum = b.lsum;
      a.ltails = b.ltails;
      a.lerr = b.lerr;
      a.state = b.state[lv];
      a.work = copy;
      a.link_out = b.link[lv + 1];
      a.ctl = b.ctl;
      a.L = Li;
      a.level = lv;
      a.log2B = p.log2B[lv];
      a.log2B_far = lv == 0 && single ? p.log2B_far : 0;
      a.kbits_far = p.kbits_far;
      a.max_walk_far = p.max_walk_far;
      a.max_walk = lv == 0 ? p.max_walk0 : o.max_walk;
      a.cap = p.cap[lv];
      a.cap_prev = lv > 0 ? p.cap[lv - 1] : 0;
      a.kbits = p.kbits;
      a.seed = level_seed(o.seed, lv);
      void (*kfn)(WalkArgs);
      if (lv > 0) kfn = lr_walk<false, false, false>;
      else if (single) kfn = p.packed ? lr_walk<true, false, true> : lr_walk<true, false, false>;
      else kfn = p.packed ? lr_walk<true, true, true> : lr_walk<true, true, false>;
      const bool marked = lv == 0 && p.chosen > 0;
      const int64_t items =
          marked ? p.chosen + 1 : ((p.bound[lv] + (1ll << a.log2B) - 1) >> a.log2B) + L;
      // workgroup size o.block (tunable): it sets how many lanes share one
      // LDS work counter and contiguous range of splitters
      int g = marked ? persistent_grid((const void*)lr_walk_marked, blk, 0)
                     : persistent_grid((const void*)kfn, blk, 0);
      g = (int)std::min<int64_t>(g, (items + blk - 1) / blk);
      if (g < 1) g = 1;
      if (marked)
        hipLaunchKernelGGL(lr_walk_marked, dim3(g), dim3(blk), 0, stream, a, o.d_splitters,
                           (const int32_t*)b.ssucc, (int)p.chosen);
      else
        hipLaunchKernelGGL(kfn, dim3(g), dim3(blk), 0, stream, a);
      PJ_HIP(hipGetLastError());
      tm.mark(lv == 0 ? "walk0" : "walk_up");
    }
    // base ranking of the top level
    const int top = p.levels;
    const int cap_prev = p.cap[top - 1];
    if (p.base_kind == 1) {
      hipLaunchKernelGGL(lr_base_lds, dim3(1), dim3(kBaseThreads), 0, stream, b.link[top],
                         b.srank[top], b.ctl, top, Li, cap_prev);
    } else {
      const int g = grid_for(p.bound[top], 256, gcap);
      hipLaunchKernelGGL(wide_clear, dim3(g), dim3(256), 0, stream, b.wide_lnk, b.ctl, top, Li,
                         cap_prev);
      hipLaunchKernelGGL(wide_pred, dim3(g), dim3(256), 0, stream, b.link[top], b.wide_lnk, b.ctl,
                         top, Li, cap_prev);
      hipLaunchKernelGGL(wide_init, dim3(g), dim3(256), 0, stream, b.link[top], b.wide_lnk,
                         b.wide_pl, b.ctl, top, Li, cap_prev);
      for (int it = 0; it < p.wide_rounds; ++it)
        hipLaunchKernelGGL(wide_jump, dim3(g), dim3(256), 0, stream, b.wide_pl, b.ctl, top, Li,
                           cap_prev);
      hipLaunchKernelGGL(wide_final, dim3(g), dim3(256), 0, stream, b.wide_pl, b.srank[top],
                         b.ctl, top, Li, cap_prev);
    }
    PJ_HIP(hipGetLastError());
    tm.mark("base");
    // expand back down
    for (int lv = top - 1; lv >= 1; --lv) {
      const int g = grid_for(p.bound[lv], 256, gcap);
      hipLaunchKernelGGL(lr_expand, dim3(g), dim3(256), 0, stream, b.state[lv], b.srank[lv + 1],
                         b.srank[lv], b.ctl, lv, Li, p.cap[lv - 1], p.cap[lv]);
    }
    tm.mark("expand_up");
    const int g0 = grid_for(n, 256, gcap);
    void (*ex0)(const int2*, const int32_t*, int32_t*, const int64_t*, LrCtl*, int, int, int, int);
    if (single) {
      if (o.to_tail) ex0 = p.packed ? lr_expand0<false, true, true> : lr_expand0<false, true, false>;
      else ex0 = p.packed ? lr_expand0<false, false, true> : lr_expand0<false, false, false>;
    } else {
      if (o.to_tail) ex0 = p.packed ? lr_expand0<true, true, true> : lr_expand0<true, true, false>;
      else ex0 = p.packed ? lr_expand0<true, false, true> : lr_expand0<true, false, false>;
    }
    hipLaunchKernelGGL(ex0, dim3(g0), dim3(256), 0, stream, b.state[0], b.srank[1], rank, off,
                       b.ctl, Li, p.cap[0], p.kbits, single ? p.kbits_far : 0);
    PJ_HIP(hipGetLastError());
    tm.mark("expand0");
  }

  if (o.validate && n0 > 0) {
    const int g = grid_for(n, 256, gcap);
    hipLaunchKernelGGL(chk_clear, dim3(g), dim3(256), 0, stream, b.chk, n);
    if (single) {
      hipLaunchKernelGGL(chk_count<false>, dim3(g), dim3(256), 0, stream, succ, rank, off, Li, n,
                         o.to_tail, b.chk, b.lerr);
      hipLaunchKernelGGL(chk_perm<false>, dim3(g), dim3(256), 0, stream, b.chk, off, Li, n,
                         b.lerr);
    } else {
      hipLaunchKernelGGL(chk_count<true>, dim3(g), dim3(256), 0, stream, succ, rank, off, Li, n,
                         o.to_tail, b.chk, b.lerr);
      hipLaunchKernelGGL(chk_perm<true>, dim3(g), dim3(256), 0, stream, b.chk, off, Li, n,
                         b.lerr);
    }
    PJ_HIP(hipGetLastError());
    tm.mark("validate");
  }
  if (status) {
    hipLaunchKernelGGL(lr_status, dim3(grid_for(L, 256, 1024)), dim3(256), 0, stream,
                       p.algo == PJ_ALGO_RULING_SET && !p.small ? b.ctl : nullptr, b.lerr,
                       b.ltails, off, Li, n, check_total ? 1 : 0, check_tails ? 1 : 0, status);
    PJ_HIP(hipGetLastError());
  }

  int result = PJ_OK;
  if (want_status) {
    std::vector<int32_t> hs((size_t)L);
    PJ_HIP(hipMemcpyAsync(hs.data(), status, sizeof(int32_t) * L, hipMemcpyDeviceToHost, stream));
    PJ_HIP(hipStreamSynchronize(stream));
    for (int64_t l = 0; l < L; ++l)
      if (hs[l] != PJ_OK) {
        result = hs[l];
        break;
      }
  }
  if (st) {
    PJ_TRY(tm.finish(st));
    st->algo = p.algo;
    st->levels = p.levels;
    st->base_kind = p.small ? 0 : p.base_kind;
    int32_t hmax = 0;
    if (p.algo == PJ_ALGO_RULING_SET && !p.small && n0 > 0) {
      PJ_HIP(hipMemsetAsync(b.sub_max, 0, sizeof(int32_t), stream));
      hipLaunchKernelGGL(lr_sublist_max, dim3(grid_for(p.bound[1], 256, gcap)), dim3(256), 0,
                         stream, (const int2*)b.link[1], (const LrCtl*)b.ctl, Li, p.cap[0],
                         b.sub_max);
      PJ_HIP(hipGetLastError());
      PJ_HIP(hipMemcpyAsync(&hmax, b.sub_max, sizeof hmax, hipMemcpyDeviceToHost, stream));
    }
    LrCtl hc{};
    PJ_HIP(hipMemcpyAsync(&hc, b.ctl, sizeof hc, hipMemcpyDeviceToHost, stream));
    PJ_HIP(hipStreamSynchronize(stream));
    st->level_nodes[0] = n0;
    for (int l = 1; l <= p.levels && l <= PJ_MAX_LEVELS; ++l)
      st->level_nodes[l] = hc.lv[l - 1].r + L + std::min(hc.lv[l - 1].dyn, p.cap[l - 1]);
    if (p.levels > 0) {
      st->sublists0 = st->level_nodes[1];
      st->cuts0 = std::min(hc.lv[0].dyn, p.cap[0]);
      st->max_sublist0 = hmax;
    }
    if (p.algo == PJ_ALGO_WYLLIE) st->rounds = n0 > 0 ? p.wy_rounds : 0;
    st->status = result;
  }
  PJ_TRY(workspace_release(ws));
  return result;
}

// First-level splitter spacing when the caller leaves it at zero: about 2^20
// splitters, so the splitter ranks that the final scatter gathers (4 B each)
// stay near one XCD's 4 MiB L2, from 8 (short walks for small, latency-bound
// lists) up to 256 for one list (2^28 nodes: 14.5 ms at 256 against 15.9 at
// 64, measured; longer walks cost imbalance, a larger table costs L2
// misses) and up to 64 for a batch, whose many short lists end most walks
// early anyway.
int list_rank_default_spacing(int64_t n, bool single) {
  const int cap = single ? 256 : 64;
  int sp = 8;
  while (sp < cap && (n >> 20) > sp) sp *= 2;
  return sp;
}

// Level-0 spacing actually planned.  A caller's (or tuned) value is used as
// is.  Otherwise a single list of at least 2^22 nodes is planned with
// spacing kLocalSpacing and lets the walk switch to the size default on the
// device when its successors are not local (the returned far spacing);
// smaller lists and batches use the size default.
constexpr int kLocalSpacing = 8;
constexpr int64_t kAdaptiveMin = int64_t(1) << 22;

int level0_spacing(int requested, int64_t n0, bool single, int32_t* planned) {
  if (requested > 0) {
    *planned = requested;
    return 0;
  }
  const int dflt = list_rank_default_spacing(n0, single);
  if (single && n0 >= kAdaptiveMin && dflt != kLocalSpacing) {
    *planned = kLocalSpacing;
    return dflt;
  }
  *planned = dflt;
  return 0;
}

size_t list_rank_workspace(int64_t n0, int64_t L, const pj_opts* user, bool single,
                           bool weighted) {
  pj_opts raw;
  pj_opts_init(&raw);
  if (user) raw = *user;
  apply_tuned(raw, n0, L);
  (void)level0_spacing(raw.spacing, n0, single, &raw.spacing);
  pj_opts o = resolved_opts(&raw);
  const int64_t chosen = o.d_splitters && single && !weighted && n0 > 0
                             ? std::max<int64_t>(1, std::min(o.n_splitters, n0)) : 0;
  Plan p = make_plan(n0, L, n0, o, !weighted && o.level0_state != PJ_STATE_SEPARATE, chosen);
  Buffers b;
  return carve(p, L, single, o.validate != 0, o.validate && !o.d_status, nullptr, &b);
}

}  // namespace pj

extern "C" {

int pj_list_rank_ex(const int32_t* succ, int64_t n, int32_t* rank, const pj_opts* opts,
                    pj_stream_t stream) {
  if (n < 0) return PJ_EINVAL;
  return pj::list_rank_impl(succ, nullptr, 1, nullptr, n, rank, opts, (hipStream_t)stream);
}

int pj_list_rank(const int32_t* succ, int64_t n, int32_t* rank, pj_stream_t stream) {
  return pj_list_rank_ex(succ, n, rank, nullptr, stream);
}

int pj_list_rank_batched_ex(const int32_t* succ, const int64_t* offsets, int64_t L,
                            int32_t* rank, const pj_opts* opts, pj_stream_t stream) {
  if (!offsets || L < 0) return PJ_EINVAL;
  if (opts && opts->use_graph && !opts->stats && !(opts->validate && !opts->d_status) && L > 0) {
    std::vector<int64_t> hbuf;
    const int64_t* ho = opts->h_offsets;
    if (!ho) {
      hbuf.resize((size_t)L + 1);
      PJ_HIP(hipMemcpyAsync(hbuf.data(), offsets, sizeof(int64_t) * (L + 1),
                            hipMemcpyDeviceToHost, (hipStream_t)stream));
      PJ_HIP(hipStreamSynchronize((hipStream_t)stream));
      ho = hbuf.data();
    }
    if (ho[0] != 0 || ho[L] < 0 || ho[L] >= INT32_MAX) return PJ_EINVAL;
    for (int64_t l = 0; l < L; ++l)
      if (ho[l + 1] < ho[l]) return PJ_EINVAL;
    if (ho[L] > 0 && (!succ || !rank)) return PJ_EINVAL;
    PJ_TRY(pj::check_alias(succ, rank, ho[L], opts->validate != 0));
    return pj::graph_batched(succ, offsets, L, ho, rank, *opts, (hipStream_t)stream);
  }
  return pj::list_rank_impl(succ, offsets, L, opts ? opts->h_offsets : nullptr, 0, rank, opts,
                            (hipStream_t)stream);
}

int pj_list_rank_batched(const int32_t* succ, const int64_t* offsets, int64_t L, int32_t* rank,
                         pj_stream_t stream) {
  return pj_list_rank_batched_ex(succ, offsets, L, rank, nullptr, stream);
}

int pj_list_rank_weighted(const int32_t* succ, const int32_t* weight, int64_t n, int32_t* rank,
                          const pj_opts* opts, pj_stream_t stream) {
  if (n < 0 || (n > 0 && !weight)) return PJ_EINVAL;
  return pj::list_rank_impl(succ, nullptr, 1, nullptr, n, rank, opts, (hipStream_t)stream,
                            n > 0 ? weight : nullptr);
}

int pj_list_rank_weighted_batched(const int32_t* succ, const int32_t* weight,
                                  const int64_t* offsets, int64_t L, int32_t* rank,
                                  const pj_opts* opts, pj_stream_t stream) {
  if (!offsets || L < 0 || (L > 0 && !weight)) return PJ_EINVAL;
  return pj::list_rank_impl(succ, offsets, L, opts ? opts->h_offsets : nullptr, 0, rank, opts,
                            (hipStream_t)stream, weight);
}

size_t pj_list_rank_weighted_workspace_bytes(int64_t total_nodes, int64_t L,
                                             const pj_opts* opts) {
  if (total_nodes < 0 || L < 1) return 0;
  const size_t batched = pj::list_rank_workspace(total_nodes, L, opts, false, true);
  return L > 1 ? batched
               : std::max(batched, pj::list_rank_workspace(total_nodes, L, opts, true, true));
}

size_t pj_list_rank_workspace_bytes(int64_t total_nodes, int64_t L, const pj_opts* opts) {
  if (total_nodes < 0 || L < 1) return 0;
  // one list may go through either entry point: size for the larger layout
  const size_t batched = pj::list_rank_workspace(total_nodes, L, opts, false);
  return L > 1 ? batched
               : std::max(batched, pj::list_rank_workspace(total_nodes, L, opts, true));
}

}  // extern "C"
