// Connected components on gfx950: Shiloach-Vishkin hook and shortcut
// (Section 4, the paper's SV-GPU), then labels canonicalised to the smallest
// vertex id of each component.
//
// State: parent array D (held in the caller's label buffer), and two round
// stamps per vertex: NS[r] = s marks root r's tree as not a star in round s,
// Q[r] = s marks r as involved in a conditional hook in round s.  Stamps
// avoid clearing the arrays between rounds.
//
// Round s, one kernel per step, each kernel boundary a grid-wide barrier:
//   1a  shortcut          D[v] <- D[D[v]], repeated while it changes
//                         something (at most kCompressPasses passes)
//   1b  mark non-stars    if D[v] != D[D[v]]: NS[D[D[v]]] = s
//       (1a must be complete for every vertex first, hence two kernels)
//   2   conditional hook  edge (i,j), a = D[i]: if a is the root of a star and
//                         b = D[j] < a: D[a] = b, Q[b] = s (SV also
//                         stamps a, but a hooked root is never tested again)
//   3   stagnant hook     if a is the root of a star with Q[a] != s and
//                         b = D[j] != a: D[a] = b (the stagnant roots are
//                         found first by a vertex pass, as a bitmap)
//   4   shortcut          D[v] <- D[D[v]]
//   5   change flag       any non-star mark or hook sets w[s] (an OR by
//                         concurrent writes); the solve ends after the first
//                         round with w[s] == 0.
// Each pair is processed in both orientations by the thread that reads it.
// Before step 2 a compaction kernel replaces every pair by the pair of its
// ends' parents and drops it when the two agree (see sv_compact); steps 2
// and 3 read the survivors.  Round 1 starts from D = identity, skips 1a,
// and does steps 2 and 3 by sorting the input pairs by slice and hooking
// them (see sv_bucket and sv_hook_first).
// Concurrent writes to one root land in arbitrary order; every outcome is
// one the arbitrary-CRCW algorithm allows: step 2 only hooks star roots onto
// strictly smaller ids, step 3 only hooks stars that no step-2 hook touched,
// and two such stars are never adjacent, so no cycle can form.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "pj_internal.hpp"

namespace pj {
namespace {

struct CcCtl {
  int32_t err;
  int32_t rounds;
};

// Memory access discipline.  Within one kernel, other workgroups may write a
// word of D, NS or Q while it is read, and several may write the same word
// (two hooks of one root, many stamps of one root).  Loads are plain: a load
// may return a value from the start of the kernel or any later one, and every
// step below is correct under that (a stale D[a] == a only repeats a hook that
// arbitrary concurrent writes allow; a stale parent is still an ancestor).
// Stores of hooks and stamps are device-scope relaxed atomic stores, written
// through to the device-coherent level.  With plain stores, such writes from
// workgroups on different XCDs (each XCD has its own write-back L2) were seen
// to be lost now and then: a lost stamp lets a root that received a hook look
// stagnant and hook back (a cycle), and a lost hook makes a root a root again
// after the pairs that joined it were dropped, splitting a component.  The
// shortcut's store stays plain: each word has one writer, and losing it would
// only leave an older ancestor in place.
// `publish`, `load_coherent` and `raise_flag` (the shared device helpers)
// implement this discipline.

// The round-s kernels do nothing once an earlier round saw no change.
__device__ __forceinline__ bool converged(const int32_t* w, int s) { return s > 1 && w[s - 1] == 0; }

// Per-workgroup claim table in LDS (kClaim slots, cleared to -1 at kernel
// start): true the first time `key` is offered in this workgroup, and when
// its slot already holds another key.  Late in a solve thousands of pairs
// hook or stamp the same few roots; the claim cuts their write-through stores
// to about one per workgroup.  Which of several equal hooks lands is
// arbitrary anyway.
constexpr int kClaim = 1024;

__device__ __forceinline__ void claim_clear(int* tab) {
  for (int i = threadIdx.x; i < kClaim; i += blockDim.x) tab[i] = -1;
  __syncthreads();
}

__device__ __forceinline__ bool claim(int* tab, int key) {
  return atomicCAS(&tab[mix32((uint32_t)key) & (kClaim - 1)], -1, key) != key;
}

__global__ void sv_init(int32_t* __restrict__ D, int32_t* __restrict__ NS, int32_t* __restrict__ Q,
                        int n, int32_t* w, unsigned long long* mcount, int32_t* any,
                        int32_t* sc_flags, int wlen, int sc_len, CcCtl* ctl) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int v = tid; v < n; v += stride) {
    D[v] = v;
    NS[v] = 0;
    Q[v] = 0;
  }
  for (int i = tid; i < wlen; i += stride) {
    w[i] = 0;
    mcount[i] = 0ull;
    any[i] = 0;
  }
  for (int i = tid; i < sc_len; i += stride) sc_flags[i] = 0;
  if (tid == 0) {
    ctl->err = 0;
    ctl->rounds = 0;
  }
}

// Step 1a and step 4: D[v] <- D[D[v]].  Step 1a repeats the pass up to
// kCompressPasses times, each pass running only if the one before changed a
// parent (`prev` flag, raised through `changed`), so trees enter step 1b as
// stars wherever a few passes suffice: every root can then hook in step 2,
// and the number of trees falls far faster per round than with one pass.
// Extra shortcuts never change what a tree contains, only its depth.
constexpr int kCompressPasses = 8;

__global__ void __launch_bounds__(256) sv_shortcut(int32_t* __restrict__ D, int n,
                                                   const int32_t* w, int s,
                                                   int32_t* changed, const int32_t* prev) {
  if (converged(w, s) || (prev && *prev == 0)) return;
  const int stride = gridDim.x * blockDim.x;
  bool moved = false;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int p = D[v];
    const int gp = D[p];
    if (gp != p) {
      D[v] = gp;
      moved = true;
    }
  }
  if (changed) raise_flag(changed, moved);
}

// Step 1b.
__global__ void __launch_bounds__(256) sv_mark(const int32_t* __restrict__ D,
                                               int32_t* __restrict__ NS, int n, int32_t* w,
                                               int s, CcCtl* ctl) {
  if (converged(w, s)) return;
  __shared__ int tab[kClaim];
  claim_clear(tab);
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->rounds = s;
  const int stride = gridDim.x * blockDim.x;
  bool changed = false;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int p = D[v];
    const int gp = D[p];
    if (p != gp) {
      // most marks repeat the stamp of one root
      if (NS[gp] != s && claim(tab, gp)) publish(&NS[gp], s);
      changed = true;
    }
  }
  raise_flag(&w[s], changed);
}

// ------------------------------------------------ XCD-local pair layout
// The parent array of a large graph (16 MiB at 2^22 vertices) is four
// times one XCD's L2, so a gather or store at a random vertex misses that
// L2 most of the time, and round 1's 2^25 random hook stores dirty partial
// lines.  The vertices are therefore dealt into kSlices slices, one per XCD,
// by blocks of 2^sshift consecutive ids (slice_of), and round 1 first sorts
// every chunk of input pairs by the slice of the end it will hook
// (sv_bucket).  Workgroups
// are dispatched round-robin over the XCDs, so the workgroups of one XCD
// (blockIdx.x % kSlices) take the runs of one slice: round 1's hooks
// (sv_hook_first) then store into, and round 2's compaction gathers one end
// from, an eighth of D that stays in that XCD's L2.  Nothing depends on the
// mapping for correctness, only the hit rate.  Dealing blocks round-robin,
// not one contiguous id range per slice, keeps the slices equally loaded
// when pair ends are not uniform over the ids (the larger end of a uniform
// pair is not).  Blocks are 4 KiB of D (2^10 ids; fewer for small graphs,
// so that every slice holds at least 32 blocks): on the 2^22-vertex graph,
// measured, 2.61 ms per solve against 2.76 ms with 128-byte blocks and
// 2.98 ms with 64 KiB blocks.
constexpr int kSlices = 8;
constexpr int kSliceShiftMax = 10;
constexpr int kCompactPer = 8;
constexpr int kCompactWaves = 256 / kWave;
constexpr int kBucketChunk = 256 * kCompactPer;  // pairs per sorted chunk
constexpr int kSegStride = kSlices + 1;
constexpr int kGroupChunks = 8;                  // chunks per unit of work

__device__ __forceinline__ int slice_of(int v, int sshift) { return (v >> sshift) & (kSlices - 1); }

// Slice block size for n vertices: 2^10 ids, or fewer so that each slice
// gets at least 32 blocks (never below one 128-byte line).
inline int slice_shift(int64_t n) {
  int lg = 0;
  while ((int64_t(1) << lg) < n) ++lg;
  return std::max(5, std::min(kSliceShiftMax, lg - 8));
}

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int u = __shfl_up(v, o, kWave);
    if (lane >= o) v += u;
  }
  return v;
}

// Round 1, first pass.  Every pair is range-checked, self-loops are dropped,
// and each kept pair is oriented (a, b) with a > b (the hook D[a] = b of
// round 1) and written back inside its own chunk of kBucketChunk positions,
// sorted by slice_of(a).  seg[c * kSegStride + q] is where slice q's run
// starts inside chunk c, seg[c * kSegStride + kSlices] the chunk's kept
// pairs.  The order inside a run is the input order, wave by wave.
__global__ void __launch_bounds__(256) sv_bucket(const int32_t* __restrict__ src,
                                                 const int32_t* __restrict__ dst, int64_t m,
                                                 int n, int sshift, int2* __restrict__ pout,
                                                 int32_t* __restrict__ seg, int32_t* w,
                                                 CcCtl* ctl) {
  // (slice, item, wave) counts, slice-major, then their exclusive prefix
  __shared__ int cnt[kSlices * kCompactPer * kCompactWaves];
  __shared__ int wsum[kCompactWaves];
  static_assert(kSlices * kCompactPer * kCompactWaves == 256, "one count per thread");
  const int wave = threadIdx.x / kWave;
  const int lane = lane_id();
  const int64_t nchunks = (m + kBucketChunk - 1) / kBucketChunk;
  bool bad = false, any = false;
  for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const int64_t c0 = c * kBucketChunk;
    int a[kCompactPer], b[kCompactPer], q[kCompactPer], rk[kCompactPer];
#pragma unroll
    for (int t = 0; t < kCompactPer; ++t) {
      const int64_t e = c0 + t * 256 + threadIdx.x;
      a[t] = b[t] = 0;
      q[t] = -1;
      if (e < m) {
        const int u = src[e], v = dst[e];
        if ((unsigned)u >= (unsigned)n || (unsigned)v >= (unsigned)n) {
          bad = true;
        } else if (u != v) {
          a[t] = u > v ? u : v;
          b[t] = u > v ? v : u;
          q[t] = slice_of(a[t], sshift);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < kCompactPer; ++t) {
      rk[t] = 0;
#pragma unroll
      for (int k = 0; k < kSlices; ++k) {
        const uint64_t mk = __ballot(q[t] == k);
        if (q[t] == k) rk[t] = lanes_below(mk);
        if (lane == 0) cnt[(k * kCompactPer + t) * kCompactWaves + wave] = __popcll(mk);
      }
    }
    __syncthreads();
    const int mine = cnt[threadIdx.x];
    const int incl = wave_incl_scan(mine);
    if (lane == kWave - 1) wsum[wave] = incl;
    __syncthreads();
    int excl = incl - mine;
    for (int i = 0; i < wave; ++i) excl += wsum[i];
    cnt[threadIdx.x] = excl;  // each thread rewrites only the entry it read
    if (threadIdx.x % (kCompactPer * kCompactWaves) == 0)
      seg[c * kSegStride + threadIdx.x / (kCompactPer * kCompactWaves)] = excl;
    if (threadIdx.x == 255) seg[c * kSegStride + kSlices] = excl + mine;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kCompactPer; ++t)
      if (q[t] >= 0) {
        pout[c0 + cnt[(q[t] * kCompactPer + t) * kCompactWaves + wave] + rk[t]] =
            make_int2(a[t], b[t]);
        any = true;
      }
    __syncthreads();  // cnt and wsum are reused by the next chunk
  }
  if (__ballot(bad) && lane == 0) atomicOr(&ctl->err, kErrRange);
  raise_flag(&w[1], any);
}

// One unit of work of the slice-sorted pairs: slice q's runs in the
// kGroupChunks chunks of group g, as a flat range [0, pre[kGroupChunks]);
// flat item f lies in chunk j with pre[j] <= f < pre[j + 1], at position
// start[j] + f - pre[j].  Called by every thread; ends with a barrier.
__device__ __forceinline__ void load_unit(const int32_t* __restrict__ seg, int64_t nchunks,
                                          int64_t g, int q, int* pre, int64_t* start) {
  if (threadIdx.x < kGroupChunks) {
    const int64_t c = g * kGroupChunks + threadIdx.x;
    int len = 0;
    int64_t st = 0;
    if (c < nchunks) {
      const int lo = seg[c * kSegStride + q];
      len = seg[c * kSegStride + q + 1] - lo;
      st = c * kBucketChunk + lo;
    }
    start[threadIdx.x] = st;
    pre[threadIdx.x + 1] = len;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    pre[0] = 0;
    for (int j = 1; j <= kGroupChunks; ++j) pre[j] += pre[j - 1];
  }
  __syncthreads();
}

__device__ __forceinline__ int64_t unit_pos(const int* pre, const int64_t* start, int f) {
  int j = 0;
  while (pre[j + 1] <= f) ++j;  // f < pre[kGroupChunks], so j < kGroupChunks
  return start[j] + (f - pre[j]);
}

// Round 1, second pass: step 2 with every vertex the root of a star.  Each
// kept pair (a, b), a > b, hooks D[a] = b (concurrent writes to one a land
// in arbitrary order).  Every vertex with a pair is then hooked (the larger
// end of one) or hooked onto (the smaller end), so step 3 finds no stagnant
// root and the stamps of step 2 are never read: only the hooks are stored.
// The workgroups of slice q store only into slice q's lines.  Plain stores:
// D is not read in this kernel; an L2 writes back only the bytes stored, so
// whichever of the concurrent stores to D[a] lands last, D[a] is a smaller
// neighbour of a (the pointers form a forest of strictly decreasing ids),
// and the kernel boundary makes every store visible to all XCDs.  Even a
// store lost outright would only leave a a root for round 2 to hook, since
// every pair survives into round 2.
constexpr int kHookFirstPer = 12;

__global__ void __launch_bounds__(256) sv_hook_first(const int2* __restrict__ pairs,
                                                     const int32_t* __restrict__ seg,
                                                     int64_t nchunks, int32_t* __restrict__ D) {
  __shared__ int pre[kGroupChunks + 1];
  __shared__ int64_t start[kGroupChunks];
  const int q = blockIdx.x % kSlices;
  const int64_t ngroups = (nchunks + kGroupChunks - 1) / kGroupChunks;
  for (int64_t g = blockIdx.x / kSlices; g < ngroups; g += gridDim.x / kSlices) {
    load_unit(seg, nchunks, g, q, pre, start);
    const int total = pre[kGroupChunks];
    for (int f0 = 0; f0 < total; f0 += 256 * kHookFirstPer) {
      int2 p[kHookFirstPer];
#pragma unroll
      for (int t = 0; t < kHookFirstPer; ++t) {
        const int f = f0 + t * 256 + threadIdx.x;
        p[t] = f < total ? pairs[unit_pos(pre, start, f)] : make_int2(-1, 0);
      }
#pragma unroll
      for (int t = 0; t < kHookFirstPer; ++t)
        if (p[t].x >= 0) D[p[t].x] = p[t].y;
    }
    __syncthreads();  // pre and start are reused by the next unit
  }
}

// Pair compaction, a kernel of its own between steps 1b and 2 (rounds 2 and
// later).  A stored pair (x, y) stands for an input pair (i, j) with x in
// i's tree and y in j's tree; it is replaced by (D[x], D[y]).  Parents lie
// in the same trees, so the connectivity the pair carries is unchanged, and
// after round 2 the stored ends are roots or near-roots: a shrinking set of
// words that stays in cache, instead of gathers over the whole parent array
// every round.  Pairs whose two parents agree lie inside one tree for good
// (trees only merge) and are dropped.  The survivors are exactly the parents
// steps 2 and 3 need.  D is not written while this kernel runs: step 2 may
// hook one root twice (arbitrary winner), and a drop decided between two
// such writes could rest on a parent the second write replaces.  A
// workgroup reserves room for the survivors of each chunk of kCompactPer *
// 256 pairs with one atomic.
//
// kSorted (round 2) reads round 1's slice-sorted pairs unit by unit, the
// workgroups of slice q taking slice q's runs, so one of the two gathers
// stays in the XCD's L2; later rounds read the dense survivors.
//
// A workgroup also drops repeats within its chunk: contracted pairs pile up
// on the few roots that remain late in a solve (thousands of copies of one
// pair of roots), and a copy joins nothing the first does not.  Open
// addressing in LDS, pairs ordered (min, max); a pair that finds no free
// slot within kDedupProbes is kept.
constexpr int kDedupSlots = 4096;  // >= 2 * 256 * kCompactPer
constexpr int kDedupProbes = 8;
constexpr unsigned long long kDedupEmpty = ~0ull;

template <bool kSorted>
__global__ void __launch_bounds__(256) sv_compact(const int2* __restrict__ pin,
                                                  const unsigned long long* m_dev,
                                                  const int32_t* __restrict__ seg,
                                                  int64_t nchunks, int32_t* __restrict__ D,
                                                  int2* __restrict__ pout,
                                                  unsigned long long* m_out, int32_t* w,
                                                  int s) {
  if (converged(w, s)) return;
  __shared__ int cnt[kCompactPer][kCompactWaves];
  __shared__ unsigned long long chunk_base;
  __shared__ unsigned long long seen[kDedupSlots];
  __shared__ int pre[kGroupChunks + 1];
  __shared__ int64_t start[kGroupChunks];
  const int wave = threadIdx.x / kWave;
  const int64_t m = kSorted ? 0 : (int64_t)*m_dev;
  const int q = blockIdx.x % kSlices;
  const int64_t nunits = kSorted ? (nchunks + kGroupChunks - 1) / kGroupChunks
                                 : (m + kBucketChunk - 1) / kBucketChunk;
  const int64_t ustep = kSorted ? gridDim.x / kSlices : gridDim.x;
  for (int64_t u = kSorted ? blockIdx.x / kSlices : blockIdx.x; u < nunits; u += ustep) {
    int total;
    if (kSorted) {
      load_unit(seg, nchunks, u, q, pre, start);
      total = pre[kGroupChunks];
    } else {
      total = (int)min((int64_t)kBucketChunk, m - u * kBucketChunk);
    }
    for (int f0 = 0; f0 < total; f0 += kBucketChunk) {
      for (int i = threadIdx.x; i < kDedupSlots; i += 256) seen[i] = kDedupEmpty;
      __syncthreads();
      int du[kCompactPer], dv[kCompactPer];
      bool keep[kCompactPer];
#pragma unroll
      for (int t = 0; t < kCompactPer; ++t) {
        const int f = f0 + t * 256 + threadIdx.x;
        keep[t] = false;
        du[t] = dv[t] = 0;
        if (f < total) {
          const int2 p = pin[kSorted ? unit_pos(pre, start, f) : u * kBucketChunk + f];
          const int x = D[p.x], y = D[p.y];
          du[t] = x < y ? x : y;
          dv[t] = x < y ? y : x;
          keep[t] = x != y;
        }
      }
#pragma unroll
      for (int t = 0; t < kCompactPer; ++t) {
        if (!keep[t]) continue;
        const unsigned long long key =
            ((unsigned long long)(unsigned)du[t] << 32) | (unsigned)dv[t];
        unsigned h = mix32((unsigned)du[t] * 0x9E3779B1u ^ (unsigned)dv[t]);
        for (int pr = 0; pr < kDedupProbes; ++pr, ++h) {
          const unsigned long long old =
              atomicCAS(&seen[h & (kDedupSlots - 1)], kDedupEmpty, key);
          if (old == kDedupEmpty) break;  // first copy in this chunk
          if (old == key) {               // a repeat
            keep[t] = false;
            break;
          }
        }
      }
#pragma unroll
      for (int t = 0; t < kCompactPer; ++t) {
        const uint64_t bm = __ballot(keep[t]);
        if (lane_id() == 0) cnt[t][wave] = __popcll(bm);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        int acc = 0;
        for (int t = 0; t < kCompactPer; ++t)
          for (int k = 0; k < kCompactWaves; ++k) {
            const int c = cnt[t][k];
            cnt[t][k] = acc;
            acc += c;
          }
        chunk_base = acc ? atomicAdd(m_out, (unsigned long long)acc) : 0ull;
      }
      __syncthreads();
      const unsigned long long cb = chunk_base;
#pragma unroll
      for (int t = 0; t < kCompactPer; ++t) {
        const uint64_t bm = __ballot(keep[t]);
        if (keep[t]) pout[cb + cnt[t][wave] + lanes_below(bm)] = make_int2(du[t], dv[t]);
      }
      __syncthreads();
    }
  }
}
// Pair kernels take kPairsPer pairs per thread per iteration, issuing all
// their loads before using any, so that enough gathers are in flight.
constexpr int kPairsPer = 8;

// Step 2 over the surviving pairs: the parents the compaction read at the
// start of the step (rounds 2 and later; round 1 is done by the compaction).
__global__ void __launch_bounds__(256) sv_hook(const int2* __restrict__ pairs,
                                               const unsigned long long* m_dev,
                                               int32_t* __restrict__ D,
                                               const int32_t* __restrict__ NS,
                                               int32_t* __restrict__ Q, int32_t* w, int s) {
  if (converged(w, s)) return;
  __shared__ int hooked_a[kClaim];  // roots this workgroup has hooked
  __shared__ int stamped_b[kClaim];  // hook targets it has stamped
  claim_clear(hooked_a);
  claim_clear(stamped_b);
  const int64_t m = (int64_t)*m_dev;
  const int64_t chunk = 256 * kPairsPer;
  bool hooked = false;
  for (int64_t c0 = (int64_t)blockIdx.x * chunk; c0 < m; c0 += (int64_t)gridDim.x * chunk) {
    int a[kPairsPer], b[kPairsPer], da[kPairsPer];
#pragma unroll
    for (int t = 0; t < kPairsPer; ++t) {
      const int64_t e = c0 + t * 256 + threadIdx.x;
      const int2 c = e < m ? pairs[e] : make_int2(-1, -1);
      a[t] = c.x > c.y ? c.x : c.y;
      b[t] = c.x > c.y ? c.y : c.x;
    }
#pragma unroll
    for (int t = 0; t < kPairsPer; ++t) da[t] = a[t] >= 0 ? D[a[t]] : -1;
#pragma unroll
    for (int t = 0; t < kPairsPer; ++t) {
      // A thread that loses the claim acts as if it had seen a hooked already;
      // the winner re-reads D[a] at the coherent level first, since late in a
      // solve thousands of workgroups hook the same few roots.
      if (a[t] >= 0 && da[t] == a[t] && NS[a[t]] != s && claim(hooked_a, a[t]) &&
          load_coherent(&D[a[t]]) == a[t]) {
        // Q[a] is not stamped: a hooked root is no root any more, so it is
        // never tested for stagnation
        publish(&D[a[t]], b[t]);
        if (Q[b[t]] != s && claim(stamped_b, b[t]) && load_coherent(&Q[b[t]]) != s)
          publish(&Q[b[t]], s);
        hooked = true;
      }
    }
  }
  raise_flag(&w[s], hooked);
}

// Step 3, first pass: the stagnant roots (roots of stars that no step-2
// hook touched: D[r] == r, NS[r] != s, Q[r] != s) as a bitmap, one ballot per
// wave of 64 consecutive vertices; any[s] records whether there is one.  The
// pair pass then tests bits of a small array (n / 8 bytes, cache-resident)
// instead of gathering D, NS and Q for both ends of every pair.
__global__ void __launch_bounds__(256) sv_stagnant_roots(const int32_t* __restrict__ D,
                                                         const int32_t* __restrict__ NS,
                                                         const int32_t* __restrict__ Q, int n,
                                                         uint64_t* __restrict__ bits,
                                                         int32_t* any, const int32_t* w, int s) {
  if (converged(w, s)) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool found = false;
  // the block size is a multiple of 64, so each wave covers one bitmap word
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - lane_id(); base < n;
       base += stride) {
    const int64_t v = base + lane_id();
    bool st = false;
    if (v < n) st = D[v] == (int)v && NS[v] != s && Q[v] != s;
    const uint64_t word = __ballot(st);
    if (lane_id() == 0) bits[base >> 6] = word;
    found |= word != 0;
  }
  raise_flag(&any[s], found);
}

__device__ __forceinline__ bool bit_set(const uint64_t* bits, int v) {
  return (bits[v >> 6] >> (v & 63)) & 1ull;
}

// Step 3, pair pass, with the parents read before step 2: a stagnant root
// hooks onto the other end's parent.  Two stagnant stars are never adjacent
// (step 2 would have hooked one onto the other), so no cycle forms; a parent
// that step 2 has since hooked is still a node of the tree it joins.
__global__ void __launch_bounds__(256) sv_stagnant(const int2* __restrict__ pairs,
                                                   const unsigned long long* m_dev,
                                                   int32_t* __restrict__ D,
                                                   const uint64_t* __restrict__ bits,
                                                   const int32_t* any, int32_t* w, int s) {
  if (converged(w, s) || any[s] == 0) return;
  __shared__ int hooked_r[kClaim];
  claim_clear(hooked_r);
  const int64_t m = (int64_t)*m_dev;
  const int64_t chunk = 256 * kPairsPer;
  bool hooked = false;
  for (int64_t c0 = (int64_t)blockIdx.x * chunk; c0 < m; c0 += (int64_t)gridDim.x * chunk) {
    int2 c[kPairsPer];
    bool bx[kPairsPer], by[kPairsPer];
#pragma unroll
    for (int t = 0; t < kPairsPer; ++t) {
      const int64_t e = c0 + t * 256 + threadIdx.x;
      c[t] = e < m ? pairs[e] : make_int2(-1, -1);
    }
#pragma unroll
    for (int t = 0; t < kPairsPer; ++t) {
      bx[t] = c[t].x >= 0 && bit_set(bits, c[t].x);
      by[t] = c[t].y >= 0 && bit_set(bits, c[t].y);
    }
#pragma unroll
    for (int t = 0; t < kPairsPer; ++t) {
      if (bx[t]) {
        if (claim(hooked_r, c[t].x)) publish(&D[c[t].x], c[t].y);
        hooked = true;
      } else if (by[t]) {
        if (claim(hooked_r, c[t].y)) publish(&D[c[t].y], c[t].x);
        hooked = true;
      }
    }
  }
  raise_flag(&w[s], hooked);
}

// ------------------------------------------------------- canonicalisation
// After convergence every component is one star.  M[root] = smallest member
// (M starts as the identity), then label[v] = M[D[v]].  A workgroup folds the
// members of the root of its first vertex before touching M, so a giant
// component costs one atomic per workgroup, not one per vertex.
constexpr int kCanonPerThread = 8;

// The epilogue kernels take `skip`: when it points at a non-zero word (the
// change flag of the last round a captured graph holds, i.e. the solve has
// not converged yet), they do nothing and the host finishes the solve.
__device__ __forceinline__ bool skipped(const int32_t* skip) { return skip && *skip != 0; }

__global__ void canon_init(int32_t* __restrict__ M, int n, const int32_t* skip) {
  if (skipped(skip)) return;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) M[v] = v;
}

__global__ void __launch_bounds__(256) canon_min(const int32_t* __restrict__ D,
                                                 int32_t* __restrict__ M, int n,
                                                 const int32_t* skip) {
  if (skipped(skip)) return;
  __shared__ int lead;
  __shared__ int wmin[256 / kWave];
  const int per_block = 256 * kCanonPerThread;
  for (int64_t c0 = (int64_t)blockIdx.x * per_block; c0 < n; c0 += (int64_t)gridDim.x * per_block) {
    __syncthreads();
    if (threadIdx.x == 0) lead = D[c0];
    __syncthreads();
    const int leader = lead;
    int mymin = INT32_MAX;
#pragma unroll
    for (int t = 0; t < kCanonPerThread; ++t) {
      const int64_t v = c0 + t * 256 + threadIdx.x;
      if (v >= n) break;
      const int r = D[v];
      if ((int)v >= r) continue;  // M[r] starts at r: only smaller members matter
      if (r == leader) mymin = min(mymin, (int)v);
      else atomicMin(&M[r], (int)v);
    }
    mymin = wave_min(mymin);
    if (lane_id() == 0) wmin[threadIdx.x / kWave] = mymin;
    __syncthreads();
    if (threadIdx.x == 0) {
      int bm = INT32_MAX;
      for (int i = 0; i < 256 / kWave; ++i) bm = min(bm, wmin[i]);
      if (bm != INT32_MAX) atomicMin(&M[leader], bm);
    }
  }
}

// label[v] = M[D[v]]; `D` and `label` may be the same array.  In the batched
// form labels are turned back into local ids.
template <bool kBatched>
__global__ void __launch_bounds__(256) canon_label(int32_t* D, const int32_t* __restrict__ M,
                                                   int n, const int64_t* __restrict__ voff,
                                                   int G, const int32_t* skip) {
  if (skipped(skip)) return;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    int lab = M[D[v]];
    if (kBatched) lab -= (int)voff[find_instance(voff, G, v)];
    D[v] = lab;
  }
}

// Batched: rewrite local pairs as global vertex ids (graph g's vertices start
// at voff[g]).  A pair whose ends leave its graph is made out of range so the
// rounds skip it and report it.
__global__ void gerr_clear(int32_t* gerr, int G) {
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < G; g += gridDim.x * blockDim.x)
    gerr[g] = 0;
}

__global__ void __launch_bounds__(256) cc_globalise(const int32_t* __restrict__ src,
                                                    const int32_t* __restrict__ dst,
                                                    const int64_t* __restrict__ voff,
                                                    const int64_t* __restrict__ eoff, int G,
                                                    int64_t m, int32_t* __restrict__ gsrc,
                                                    int32_t* __restrict__ gdst,
                                                    int32_t* __restrict__ gerr) {
  // Each wave owns a contiguous run of chunks of kWave * kGlobPer pairs: one
  // search of the offset table per wave, then every lane follows the graph
  // boundaries forward.  A chunk's loads are all issued before use.
  constexpr int kGlobPer = 16;
  constexpr int64_t kChunk = kWave * kGlobPer;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int nwaves = (gridDim.x * blockDim.x) / kWave;
  const int lane = lane_id();
  const int64_t nchunks = (m + kChunk - 1) / kChunk;
  const int64_t per = (nchunks + nwaves - 1) / nwaves;
  const int64_t ci0 = (int64_t)wave * per;
  const int64_t ci1 = ci0 + per < nchunks ? ci0 + per : nchunks;
  if (ci0 >= ci1) return;
  int g = find_instance(eoff, G, ci0 * kChunk);
  int64_t gend = eoff[g + 1], base = voff[g], size = voff[g + 1] - base;
  for (int64_t ci = ci0; ci < ci1; ++ci) {
    int us[kGlobPer], vs[kGlobPer];
#pragma unroll
    for (int t = 0; t < kGlobPer; ++t) {
      const int64_t e = ci * kChunk + t * kWave + lane;
      us[t] = e < m ? src[e] : 0;
      vs[t] = e < m ? dst[e] : 0;
    }
    for (int t = 0; t < kGlobPer; ++t) {
      const int64_t e = ci * kChunk + t * kWave + lane;
      if (e >= m) break;
      while (e >= gend) {  // later graphs (empty ones skipped)
        ++g;
        gend = eoff[g + 1];
        base = voff[g];
        size = voff[g + 1] - base;
      }
      const bool ok = (unsigned)us[t] < (uint64_t)size && (unsigned)vs[t] < (uint64_t)size;
      gsrc[e] = ok ? (int)(base + us[t]) : -1;
      gdst[e] = ok ? (int)(base + vs[t]) : -1;
      if (!ok) publish(&gerr[g], 1);  // flags of other graphs share the line
    }
  }
}

// Out-of-range pairs are charged to their own graph when the batch records
// them per graph (gerr); non-convergence concerns the whole solve.
__global__ void cc_status(const CcCtl* ctl, const int32_t* w, int max_rounds, int G,
                          const int32_t* gerr, int32_t* status, const int32_t* skip) {
  if (skipped(skip)) return;
  const bool noconv = ctl->rounds >= max_rounds && w[max_rounds] != 0;
  const bool range = (ctl->err & kErrRange) != 0;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < G; g += gridDim.x * blockDim.x) {
    int st = PJ_OK;
    if (gerr ? gerr[g] != 0 : range) st = PJ_EINVAL;
    else if (noconv) st = PJ_ENOCONV;
    status[g] = st;
  }
}

inline int grid_for(int64_t n, int block, int cap) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// Shiloach and Vishkin bound the rounds by floor(log_{3/2} n) + 2; the guard
// allows four times that before reporting non-convergence.
inline int round_guard(int64_t n) {
  const double lg = n > 1 ? std::floor(std::log((double)n) / std::log(1.5)) : 0.0;
  return 4 * ((int)lg + 2);
}

struct CcBuffers {
  CcCtl* ctl = nullptr;
  int32_t* NS = nullptr;
  int32_t* Q = nullptr;
  int32_t* w = nullptr;
  unsigned long long* mcount = nullptr;  // surviving pairs after compaction, per round
  int32_t* stag_any = nullptr;           // a stagnant root exists, per round
  int32_t* sc_flags = nullptr;           // step 1a passes that changed D, per round
  uint64_t* stag_bits = nullptr;         // stagnant roots of the current round
  int32_t* gsrc = nullptr;
  int32_t* gdst = nullptr;
  int32_t* gerr = nullptr;               // batched: per-graph out-of-range flag
  int2* pairs[2] = {};                   // surviving parent pairs (ping-pong)
  int32_t* seg = nullptr;                // round 1: slice runs of each sorted chunk
  int32_t* status_tmp = nullptr;
};

size_t cc_carve(int64_t n, int64_t m, int64_t G, bool batched, bool want_status, int wlen,
                Workspace* ws, CcBuffers* b) {
  size_t bytes = 0;
  auto take = [&](auto*& ptr, size_t count) {
    using T = std::remove_pointer_t<std::remove_reference_t<decltype(ptr)>>;
    bytes += ws_bytes(count, sizeof(T));
    if (ws) ptr = ws->take<T>(count);
  };
  take(b->ctl, 1);
  take(b->NS, (size_t)std::max<int64_t>(n, 1));
  take(b->Q, (size_t)std::max<int64_t>(n, 1));
  take(b->w, (size_t)wlen);
  take(b->mcount, (size_t)wlen);
  take(b->stag_any, (size_t)wlen);
  take(b->sc_flags, (size_t)wlen * kCompressPasses);
  take(b->stag_bits, (size_t)std::max<int64_t>((n + 63) / 64, 1));
  const size_t mm = (size_t)std::max<int64_t>(m, 1);
  take(b->pairs[0], mm);
  take(b->pairs[1], mm);
  take(b->seg, (size_t)std::max<int64_t>((m + kBucketChunk - 1) / kBucketChunk, 1) * kSegStride);
  if (batched) {
    take(b->gsrc, (size_t)std::max<int64_t>(m, 1));
    take(b->gdst, (size_t)std::max<int64_t>(m, 1));
    take(b->gerr, (size_t)std::max<int64_t>(G, 1));
  }
  if (want_status) take(b->status_tmp, (size_t)std::max<int64_t>(G, 1));
  return bytes;
}

// One solve's launch state: the buffers, grid sizes and the arrays the rounds
// read.  The launch steps below only enqueue work; the eager call and the
// graph capture compose them differently.
struct CcRun {
  int64_t n = 0, m = 0, G = 1;
  bool batched = false;
  const int64_t* d_voff = nullptr;
  const int64_t* d_eoff = nullptr;
  const int32_t* src = nullptr;
  const int32_t* dst = nullptr;
  const int32_t* es = nullptr;  // pairs the rounds read (globalised in a batch)
  const int32_t* ed = nullptr;
  int32_t* D = nullptr;         // parent array, in the caller's label buffer
  int32_t* status = nullptr;
  int max_rounds = 0, wlen = 0;
  int ni = 0, gv = 1, gp = 1, gh = 1, gcap = 1;
  int gq = kSlices;        // grids over slice-sorted units: a multiple of kSlices
  int sshift = 5;          // slice block: 2^sshift ids
  int64_t nchunks = 0;     // sorted chunks of round 1
  CcBuffers b;
  hipStream_t stream = nullptr;
  PhaseTimer* tm = nullptr;
};

void cc_setup(CcRun& r, const int32_t* src, const int32_t* dst, int64_t n, int64_t m,
              const int64_t* d_voff, const int64_t* d_eoff, int64_t G, int32_t* label,
              hipStream_t stream) {
  r.src = src;
  r.dst = dst;
  r.n = n;
  r.m = m;
  r.G = G;
  r.batched = d_voff != nullptr;
  r.d_voff = d_voff;
  r.d_eoff = d_eoff;
  r.D = label;
  r.stream = stream;
  r.max_rounds = round_guard(n);
  r.wlen = r.max_rounds + 2;
  r.ni = (int)n;
  r.gcap = device_info().cus * 16;
  r.gv = grid_for(n, 256, r.gcap);
  r.gp = grid_for((m + kPairsPer - 1) / kPairsPer, 256, r.gcap);
  r.gh = grid_for((m + kCompactPer - 1) / kCompactPer, 256, r.gcap);
  r.nchunks = (m + kBucketChunk - 1) / kBucketChunk;
  r.sshift = slice_shift(n);
  const int64_t units = (r.nchunks + kGroupChunks - 1) / kGroupChunks;
  r.gq = (int)std::max<int64_t>(kSlices, std::min<int64_t>(units * kSlices,
                                                           r.gcap / kSlices * kSlices));
}

void mark(CcRun& r, const char* phase) {
  if (r.tm) r.tm->mark(phase);
}

// Batched pair rewrite and the state initialisation.
int cc_prologue(CcRun& r) {
  CcBuffers& b = r.b;
  r.es = r.src;
  r.ed = r.dst;
  if (r.batched) {
    hipLaunchKernelGGL(gerr_clear, dim3(grid_for(r.G, 256, 1024)), dim3(256), 0, r.stream, b.gerr,
                       (int)r.G);
    if (r.m > 0) {
      hipLaunchKernelGGL(cc_globalise, dim3(grid_for(r.m, 256, r.gcap)), dim3(256), 0, r.stream,
                         r.src, r.dst, r.d_voff, r.d_eoff, (int)r.G, r.m, b.gsrc, b.gdst, b.gerr);
      r.es = b.gsrc;
      r.ed = b.gdst;
    }
  }
  hipLaunchKernelGGL(sv_init, dim3(r.gv), dim3(256), 0, r.stream, r.D, b.NS, b.Q, r.ni, b.w,
                     b.mcount, b.stag_any, b.sc_flags, r.wlen, r.wlen * kCompressPasses, b.ctl);
  PJ_HIP(hipGetLastError());
  mark(r, "sv0_init");
  return PJ_OK;
}

// Round s: every kernel returns at once if an earlier round changed nothing.
int cc_round(CcRun& r, int s) {
  CcBuffers& b = r.b;
  hipStream_t stream = r.stream;
  int32_t* D = r.D;
  const int ni = r.ni;
  // D is the identity in round 1: no shortcut, and mark only records the round
  if (s > 1)
    for (int q = 0; q < kCompressPasses; ++q) {
      int32_t* f = b.sc_flags + (int64_t)s * kCompressPasses + q;
      hipLaunchKernelGGL(sv_shortcut, dim3(r.gv), dim3(256), 0, stream, D, ni,
                         (const int32_t*)b.w, s, f, q ? (const int32_t*)(f - 1) : nullptr);
    }
  mark(r, "sv1a_shortcut");
  hipLaunchKernelGGL(sv_mark, dim3(r.gv), dim3(256), 0, stream, D, b.NS, ni, b.w, s, b.ctl);
  mark(r, "sv1b_mark");
  if (r.m > 0) {
    // round 1 sorts the input pairs by slice and hooks them; round 2 compacts
    // the sorted pairs, later rounds the survivors of the last one
    int2* out = b.pairs[s & 1];
    if (s == 1) {
      hipLaunchKernelGGL(sv_bucket, dim3(r.gh), dim3(256), 0, stream, r.es, r.ed, r.m, ni,
                         r.sshift, out, b.seg, b.w, b.ctl);
      hipLaunchKernelGGL(sv_hook_first, dim3(r.gq), dim3(256), 0, stream, (const int2*)out,
                         (const int32_t*)b.seg, r.nchunks, D);
    } else if (s == 2) {
      hipLaunchKernelGGL(sv_compact<true>, dim3(r.gq), dim3(256), 0, stream,
                         (const int2*)b.pairs[1], (const unsigned long long*)nullptr,
                         (const int32_t*)b.seg, r.nchunks, D, out, b.mcount + s, b.w, s);
    } else {
      hipLaunchKernelGGL(sv_compact<false>, dim3(r.gh), dim3(256), 0, stream,
                         (const int2*)b.pairs[(s - 1) & 1], b.mcount + (s - 1),
                         (const int32_t*)nullptr, (int64_t)0, D, out, b.mcount + s, b.w, s);
    }
    mark(r, "compact");
    if (s > 1) {  // round 1's steps 2 and 3 are done by its compaction
      hipLaunchKernelGGL(sv_hook, dim3(r.gp), dim3(256), 0, stream, (const int2*)out,
                         b.mcount + s, D, b.NS, b.Q, b.w, s);
      mark(r, "sv2_hook");
      hipLaunchKernelGGL(sv_stagnant_roots, dim3(r.gv), dim3(256), 0, stream, (const int32_t*)D,
                         (const int32_t*)b.NS, (const int32_t*)b.Q, ni, b.stag_bits, b.stag_any,
                         b.w, s);
      hipLaunchKernelGGL(sv_stagnant, dim3(r.gp), dim3(256), 0, stream, (const int2*)out,
                         b.mcount + s, D, (const uint64_t*)b.stag_bits,
                         (const int32_t*)b.stag_any, b.w, s);
      mark(r, "sv3_stagnant");
    }
  }
  hipLaunchKernelGGL(sv_shortcut, dim3(r.gv), dim3(256), 0, stream, D, ni, (const int32_t*)b.w, s,
                     (int32_t*)nullptr, (const int32_t*)nullptr);
  mark(r, "sv4_shortcut");
  PJ_HIP(hipGetLastError());
  return PJ_OK;
}

// Rounds first_round.. with a host convergence check every rounds_per_check
// rounds, until a round changes nothing or the guard is reached.  Returns the
// rounds enqueued in all.
int cc_rounds_eager(CcRun& r, int first_round, int rounds_per_check, int* rounds_out) {
  PinnedWord pinned;
  int32_t* hflag = pinned.get();
  if (!hflag) return PJ_ENOMEM;
  int rounds = first_round - 1;
  bool done = r.n == 0 || rounds >= r.max_rounds;
  while (!done) {
    const int chunk = std::min(rounds_per_check, r.max_rounds - rounds);
    for (int c = 0; c < chunk; ++c) PJ_TRY(cc_round(r, ++rounds));
    PJ_HIP(hipMemcpyAsync(hflag, r.b.w + rounds, sizeof(int32_t), hipMemcpyDeviceToHost,
                          r.stream));
    PJ_HIP(hipStreamSynchronize(r.stream));
    mark(r, "flag_check");
    if (*hflag == 0 || rounds >= r.max_rounds) done = true;
  }
  *rounds_out = rounds;
  return PJ_OK;
}

// Canonical labels and the statuses.  skip: see `skipped`.
int cc_epilogue(CcRun& r, const int32_t* skip) {
  CcBuffers& b = r.b;
  if (r.n > 0) {
    hipLaunchKernelGGL(canon_init, dim3(r.gv), dim3(256), 0, r.stream, b.NS, r.ni, skip);
    hipLaunchKernelGGL(canon_min, dim3(grid_for(r.n, 256 * kCanonPerThread, r.gcap)), dim3(256),
                       0, r.stream, (const int32_t*)r.D, b.NS, r.ni, skip);
    if (r.batched)
      hipLaunchKernelGGL(canon_label<true>, dim3(r.gv), dim3(256), 0, r.stream, r.D,
                         (const int32_t*)b.NS, r.ni, r.d_voff, (int)r.G, skip);
    else
      hipLaunchKernelGGL(canon_label<false>, dim3(r.gv), dim3(256), 0, r.stream, r.D,
                         (const int32_t*)b.NS, r.ni, r.d_voff, (int)r.G, skip);
    PJ_HIP(hipGetLastError());
    mark(r, "canonicalise");
  }
  if (r.status && r.G > 0) {
    hipLaunchKernelGGL(cc_status, dim3(grid_for(r.G, 256, 1024)), dim3(256), 0, r.stream,
                       (const CcCtl*)b.ctl, (const int32_t*)b.w, r.max_rounds, (int)r.G,
                       r.batched ? (const int32_t*)b.gerr : nullptr, r.status, skip);
    PJ_HIP(hipGetLastError());
  }
  return PJ_OK;
}

int cc_check_args(const int32_t* src, const int32_t* dst, int64_t n, int64_t m, int64_t G,
                  int32_t* label) {
  if (n < 0 || m < 0 || G < 0 || n >= INT32_MAX || m >= (int64_t(1) << 40)) return PJ_EINVAL;
  if (n > 0 && !label) return PJ_EINVAL;
  if (m > 0 && (!src || !dst)) return PJ_EINVAL;
  if (m > 0 && ((const void*)label == (const void*)src || (const void*)label == (const void*)dst))
    return PJ_EINVAL;
  if (m > 0 && n == 0) return PJ_EINVAL;
  return PJ_OK;
}

int cc_impl(const int32_t* src, const int32_t* dst, int64_t n, int64_t m, const int64_t* d_voff,
            const int64_t* d_eoff, int64_t G, int32_t* label, const pj_opts* user,
            hipStream_t stream) {
  const bool batched = d_voff != nullptr;
  if (!batched) G = 1;
  PJ_TRY(cc_check_args(src, dst, n, m, G, label));
  pj_opts o = resolved_opts(user);
  pj_stats* st = user ? user->stats : nullptr;
  if (st) *st = pj_stats{};
  const bool want_status = o.validate && !o.d_status;
  if (n == 0 && !o.d_status) return PJ_OK;

  CcRun r;
  cc_setup(r, src, dst, n, m, d_voff, d_eoff, G, label, stream);
  const size_t need = cc_carve(n, m, G, batched, want_status, r.wlen, nullptr, &r.b);
  Workspace ws;
  PJ_TRY(workspace_acquire(ws, need, &o, stream));
  cc_carve(n, m, G, batched, want_status, r.wlen, &ws, &r.b);
  r.status = o.d_status ? o.d_status : r.b.status_tmp;

  PhaseTimer tm;
  PJ_TRY(tm.begin(st != nullptr, stream));
  r.tm = &tm;

  PJ_TRY(cc_prologue(r));
  int rounds = 0;
  PJ_TRY(cc_rounds_eager(r, 1, o.rounds_per_check, &rounds));
  PJ_TRY(cc_epilogue(r, nullptr));
  int result = PJ_OK;
  if (want_status && G > 0) {
    int32_t hs = 0;
    PJ_HIP(hipMemcpyAsync(&hs, r.status, sizeof hs, hipMemcpyDeviceToHost, stream));
    PJ_HIP(hipStreamSynchronize(stream));
    result = hs;
  }
  if (st) {
    PJ_TRY(tm.finish(st));
    st->algo = PJ_ALGO_SV;
    CcCtl hc{};
    PJ_HIP(hipMemcpyAsync(&hc, r.b.ctl, sizeof hc, hipMemcpyDeviceToHost, stream));
    PJ_HIP(hipStreamSynchronize(stream));
    st->rounds = hc.rounds;
    st->level_nodes[0] = n;
    st->status = result;
  }
  PJ_TRY(workspace_release(ws));
  return result;
}

// ------------------------------------------------------------ graph replay
// A components solve captured once into a hipGraph: the prologue, the first
// kGraphRounds rounds and the epilogue, which does nothing unless the solve
// converged within those rounds.  Each call launches the graph, reads the
// last captured round's change flag, and only if it is still raised finishes
// the remaining rounds and the epilogue eagerly on the same state.  Rounds
// after convergence return at once on the device.  The cache owns the
// workspace; the key holds every address and size the capture used.
constexpr int kGraphRounds = 8;

using CcGraphKey = std::array<int64_t, 14>;
struct CcGraphEntry {
  hipGraphExec_t exec = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  uint64_t last_used = 0;
};
std::mutex g_ccg_mu;
std::map<CcGraphKey, CcGraphEntry> g_ccg;
uint64_t g_ccg_clock = 0;
constexpr size_t kMaxCcGraphs = 8;
std::map<int, hipStream_t> g_ccg_capture;

void cc_graph_drop(CcGraphEntry& e) {
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (e.ws) (void)hipFree(e.ws);
  e = CcGraphEntry{};
}

int cc_graph(const int32_t* src, const int32_t* dst, int64_t n, int64_t m, const int64_t* d_voff,
             const int64_t* d_eoff, int64_t G, int32_t* label, const pj_opts& o,
             hipStream_t stream) {
  const bool batched = d_voff != nullptr;
  if (!batched) G = 1;
  PJ_TRY(cc_check_args(src, dst, n, m, G, label));
  const bool want_status = o.validate && !o.d_status;
  if (n == 0 && !o.d_status) return PJ_OK;
  int dev = 0;
  PJ_HIP(hipGetDevice(&dev));
  const CcGraphKey key{dev,
                       (int64_t)(uintptr_t)src,
                       (int64_t)(uintptr_t)dst,
                       (int64_t)(uintptr_t)d_voff,
                       (int64_t)(uintptr_t)d_eoff,
                       (int64_t)(uintptr_t)label,
                       (int64_t)(uintptr_t)o.d_status,
                       G,
                       n,
                       m,
                       want_status ? 1 : 0,
                       kGraphRounds,
                       0,
                       0};
  std::lock_guard<std::mutex> lk(g_ccg_mu);
  CcRun r;
  cc_setup(r, src, dst, n, m, d_voff, d_eoff, G, label, stream);
  auto it = g_ccg.find(key);
  CcGraphEntry fresh;
  CcGraphEntry* e = nullptr;
  if (it != g_ccg.end()) {
    e = &it->second;
  } else {
    if (g_ccg.size() >= kMaxCcGraphs) {  // evict the least recently used
      auto lru = g_ccg.begin();
      for (auto j = g_ccg.begin(); j != g_ccg.end(); ++j)
        if (j->second.last_used < lru->second.last_used) lru = j;
      cc_graph_drop(lru->second);
      g_ccg.erase(lru);
    }
    fresh.ws_bytes = std::max<size_t>(
        cc_carve(n, m, G, batched, want_status, r.wlen, nullptr, &r.b), 256);
    PJ_HIP(hipMalloc(&fresh.ws, fresh.ws_bytes));
    e = &fresh;
  }
  Workspace ws;
  ws.base = static_cast<char*>(e->ws);
  ws.size = e->ws_bytes;
  cc_carve(n, m, G, batched, want_status, r.wlen, &ws, &r.b);
  r.status = o.d_status ? o.d_status : r.b.status_tmp;
  const int32_t* last_flag = r.b.w + std::min(kGraphRounds, r.max_rounds);
  if (it == g_ccg.end()) {
    hipStream_t& cap = g_ccg_capture[dev];
    if (!cap && hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
      cc_graph_drop(fresh);
      return PJ_EHIP;
    }
    r.stream = cap;
    hipGraph_t graph = nullptr;
    hipError_t he = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    int rc = he == hipSuccess ? PJ_OK : PJ_EHIP;
    if (rc == PJ_OK) rc = cc_prologue(r);
    for (int s = 1; rc == PJ_OK && s <= std::min(kGraphRounds, r.max_rounds); ++s)
      rc = cc_round(r, s);
    if (rc == PJ_OK) rc = cc_epilogue(r, last_flag);
    if (he == hipSuccess) he = hipStreamEndCapture(cap, &graph);
    if (rc == PJ_OK && he == hipSuccess)
      he = hipGraphInstantiate(&fresh.exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (rc != PJ_OK || he != hipSuccess) {
      cc_graph_drop(fresh);
      if (rc != PJ_OK) return rc;
      set_last_hip_error(he, "graph capture of components", __FILE__, __LINE__);
      return PJ_EHIP;
    }
    e = &g_ccg.emplace(key, fresh).first->second;
    r.stream = stream;
  }
  e->last_used = ++g_ccg_clock;
  PJ_HIP(hipGraphLaunch(e->exec, stream));
  // one host check: did the captured rounds reach convergence?
  PinnedWord pinned;
  int32_t* hflag = pinned.get();
  if (!hflag) return PJ_ENOMEM;
  PJ_HIP(hipMemcpyAsync(hflag, last_flag, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  PJ_HIP(hipStreamSynchronize(stream));
  if (*hflag != 0) {  // finish eagerly from the next round
    int rounds = 0;
    const pj_opts ro = resolved_opts(&o);
    PJ_TRY(cc_rounds_eager(r, std::min(kGraphRounds, r.max_rounds) + 1, ro.rounds_per_check,
                           &rounds));
    PJ_TRY(cc_epilogue(r, nullptr));
  }
  int result = PJ_OK;
  if (want_status && G > 0) {
    int32_t hs = 0;
    PJ_HIP(hipMemcpyAsync(&hs, r.status, sizeof hs, hipMemcpyDeviceToHost, stream));
    PJ_HIP(hipStreamSynchronize(stream));
    result = hs;
  }
  return result;
}

}  // namespace

void cc_graph_cache_clear() {
  std::lock_guard<std::mutex> lk(g_ccg_mu);
  (void)hipDeviceSynchronize();
  for (auto& kv : g_ccg) cc_graph_drop(kv.second);
  g_ccg.clear();
}

size_t cc_workspace(int64_t n, int64_t m, int64_t G, const pj_opts* user, bool batched) {
  pj_opts o = resolved_opts(user);
  CcBuffers b;
  return cc_carve(n, m, G, batched, o.validate && !o.d_status, round_guard(n) + 2, nullptr, &b);
}

}  // namespace pj

extern "C" {

int pj_connected_components_ex(const int32_t* src, const int32_t* dst, int64_t n, int64_t m,
                               int32_t* label, const pj_opts* opts, pj_stream_t stream) {
  if (opts && opts->use_graph && !opts->stats)
    return pj::cc_graph(src, dst, n, m, nullptr, nullptr, 1, label, *opts, (hipStream_t)stream);
  return pj::cc_impl(src, dst, n, m, nullptr, nullptr, 1, label, opts, (hipStream_t)stream);
}

int pj_connected_components(const int32_t* src, const int32_t* dst, int64_t n, int64_t m,
                            int32_t* label, pj_stream_t stream) {
  return pj_connected_components_ex(src, dst, n, m, label, nullptr, stream);
}

int pj_connected_components_batched_ex(const int32_t* src, const int32_t* dst,
                                       const int64_t* vtx_off, const int64_t* edge_off,
                                       int64_t G, int32_t* label, const pj_opts* opts,
                                       pj_stream_t stream) {
  if (!vtx_off || !edge_off || G < 0) return PJ_EINVAL;
  if (G == 0) return PJ_OK;
  hipStream_t s = (hipStream_t)stream;
  int64_t n = 0, m = 0;
  const int64_t* hv = opts ? opts->h_offsets : nullptr;
  const int64_t* he = opts ? opts->h_edge_offsets : nullptr;
  if (hv && he) {
    n = hv[G];
    m = he[G];
  } else {
    int64_t tmp[2] = {0, 0};
    if (hipMemcpyAsync(&tmp[0], vtx_off + G, sizeof(int64_t), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipMemcpyAsync(&tmp[1], edge_off + G, sizeof(int64_t), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return PJ_EHIP;
    n = tmp[0];
    m = tmp[1];
  }
  if (opts && opts->use_graph && !opts->stats)
    return pj::cc_graph(src, dst, n, m, vtx_off, edge_off, G, label, *opts, s);
  return pj::cc_impl(src, dst, n, m, vtx_off, edge_off, G, label, opts, s);
}

int pj_connected_components_batched(const int32_t* src, const int32_t* dst,
                                    const int64_t* vtx_off, const int64_t* edge_off, int64_t G,
                                    int32_t* label, pj_stream_t stream) {
  return pj_connected_components_batched_ex(src, dst, vtx_off, edge_off, G, label, nullptr,
                                            stream);
}

size_t pj_cc_workspace_bytes(int64_t n, int64_t m, int64_t G, const pj_opts* opts) {
  if (n < 0 || m < 0 || G < 1) return 0;
  // one graph may go through either entry point: size for the larger layout
  const size_t batched = pj::cc_workspace(n, m, G, opts, true);
  return G > 1 ? batched : std::max(batched, pj::cc_workspace(n, m, G, opts, false));
}

}  // extern "C"
