// Evaluate (Alg. 2; Sec. IV-C): breadth-first walk of the policy tree from the root,
// computing g(c) = g(p) + c(p, c) for each child c of a vertex p of the current
// level.  Every g is one binary32 addition in root-to-leaf order, so the values are
// the left fold of the parent-edge costs along each root path, exactly as a serial
// FIFO traversal produces them (the order inside a level does not matter: each
// vertex is written once, from its parent's final value).  Vertices the walk does
// not reach get +inf.
//
// Data layout: the tree is given by parent[] / pcost[]; a child CSR
// (child_ptr[n+1], child[n]) is rebuilt from it on every Evaluate with a count,
// an exclusive scan and a scatter.  The scatter pops the counts back to zero, so
// the count array never needs clearing.
//
// Two evaluators compute the same values.  The default (k_eval_walk, below) needs
// one launch.  The level-synchronous one is kept as an independent check:
//
// The walk is level synchronous.  Tree levels near the root and near the leaves
// are small, the ones in between large (tens of thousands of vertices for a
// million-vertex tree), so three kernels share it:
//   head  : one 1024-thread workgroup walks the top levels while the frontier fits
//           (workgroup barriers between levels);
//   level : one launch per large level, a wide grid striding over the frontier;
//   tail  : one workgroup walks whatever remains, of any size.
// Frontier sizes live in lvl[k] on the device; a launch that finds its level empty
// does nothing, so the host only chooses how many level launches to enqueue (from
// the previous Evaluate's profile) and never waits on a frontier size.
#include "internal.h"

namespace pirrt {

namespace {

constexpr int kThreads = 256;
constexpr int kWgThreads = 1024;  // head / tail workgroup

inline unsigned blocks_for(int64_t n, int per_block = kThreads) {
  int64_t b = (n + per_block - 1) / per_block;
  return (unsigned)(b > 0 ? b : 1);
}

// Counter reads after atomics of the same kernel bypass the per-CU L1.
__device__ __forceinline__ int32_t load_counter(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The root is read from the problem state (not baked into a launch argument), so a
// captured loop body stays valid when a later Replan on the same graph changes it.
__global__ void __launch_bounds__(kThreads) k_eval_prep(int32_t n, const ProblemState* __restrict__ ps,
                                                       const int32_t* __restrict__ parent, float* __restrict__ g,
                                                       int32_t* __restrict__ child_cnt) {
  if (!ps->needs_eval) return;
  const int32_t root = ps->root;
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  if (v == root) {
    g[v] = 0.0f;
    return;
  }
  g[v] = pos_inf();
  int32_t p = parent[v];
  if (p >= 0) atomicAdd(&child_cnt[p], 1);
}

__global__ void __launch_bounds__(kThreads) k_eval_fill(int32_t n, const ProblemState* __restrict__ ps,
                                                       const int32_t* __restrict__ parent,
                                                       const int32_t* __restrict__ child_ptr,
                                                       int32_t* __restrict__ child_cnt, int32_t* __restrict__ child) {
  if (!ps->needs_eval) return;
  const int32_t root = ps->root;
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || v == root) return;
  int32_t p = parent[v];
  if (p >= 0) {
    int32_t k = atomicSub(&child_cnt[p], 1) - 1;
    child[child_ptr[p] + k] = (int32_t)v;
  }
}

// Expands one frontier vertex per active lane: writes its children's g and appends
// them to the next frontier (one atomic per wave).  Every lane of the wave calls it.
// kSameKernel: g[u] was written earlier in this same launch (head / tail
// workgroup), so it is read past the L1.
template <bool kSameKernel>
__device__ __forceinline__ void expand(int32_t u, const int32_t* __restrict__ child_ptr,
                                       const int32_t* __restrict__ child, const float* __restrict__ pcost,
                                       float* __restrict__ g, int32_t* __restrict__ next, int32_t* __restrict__ ncount) {
  int32_t a = 0, b = 0;
  if (u >= 0) {
    a = child_ptr[u];
    b = child_ptr[u + 1];
  }
  int slot = wave_reserve(ncount, b - a);
  if (b > a) {
    const float gu = kSameKernel ? __hip_atomic_load(&g[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : g[u];
    for (int32_t k = a; k < b; ++k) {
      int32_t c = child[k];
      g[c] = add_rn(gu, pcost[c]);
      next[slot + (k - a)] = c;
    }
  }
}

struct Bfs {
  const int32_t* child_ptr;
  const int32_t* child;
  const float* pcost;
  float* g;
  int32_t* fr0;
  int32_t* fr1;
  int32_t* lvl;  // lvl[k] = size of level k
  EvalInfo* info;
  const ProblemState* ps;  // the walk runs only when ps->needs_eval
};

__global__ void __launch_bounds__(kWgThreads) k_bfs_head(int32_t limit, Bfs B) {
  if (!B.ps->needs_eval) return;
  if (threadIdx.x == 0) {
    B.fr0[0] = B.ps->root;
    B.lvl[0] = 1;
    B.lvl[1] = 0;
    B.lvl[2] = 0;
    B.info->levels = 0;
    B.info->big_end = 0;
  }
  __syncthreads();
  int k = 0;
  for (;;) {
    const int32_t size = load_counter(&B.lvl[k]);
    if (size == 0 || size > limit) break;
    const int32_t* in = (k & 1) ? B.fr1 : B.fr0;
    int32_t* out = (k & 1) ? B.fr0 : B.fr1;
    for (int32_t base = 0; base < size; base += kWgThreads) {
      int32_t t = base + (int32_t)threadIdx.x;
      expand<true>(t < size ? load_counter(&in[t]) : -1, B.child_ptr, B.child, B.pcost, B.g, out, &B.lvl[k + 1]);
    }
    if (threadIdx.x == 0) B.lvl[k + 2] = 0;
    __syncthreads();
    ++k;
  }
  if (threadIdx.x == 0) {
    B.info->head_end = k;
    B.info->levels = k;
  }
}

// Level head_end + j.  lvl[k+1] was cleared by the launch of level k-1; this
// launch clears lvl[k+2] for the next one, also when its own level is empty.
__global__ void __launch_bounds__(kThreads) k_bfs_level(int32_t j, int32_t tail_limit, Bfs B) {
  if (!B.ps->needs_eval) return;
  const int32_t k = B.info->head_end + j;
  const int32_t size = B.lvl[k];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    B.lvl[k + 2] = 0;
    if (size > 0) atomicMax(&B.info->levels, k + 1);
    if (size > tail_limit) atomicMax(&B.info->big_end, k + 1);
  }
  if (size == 0) return;
  const int32_t* in = (k & 1) ? B.fr1 : B.fr0;
  int32_t* out = (k & 1) ? B.fr0 : B.fr1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < size; base += stride) {
    int64_t t = base + threadIdx.x;
    expand<false>(t < size ? in[t] : -1, B.child_ptr, B.child, B.pcost, B.g, out, &B.lvl[k + 1]);
  }
}

__global__ void __launch_bounds__(kWgThreads) k_bfs_tail(int32_t j0, int32_t tail_limit, Bfs B) {
  if (!B.ps->needs_eval) return;
  int k = B.info->head_end + j0;
  int levels = 0, big_end = 0;
  for (;;) {
    const int32_t size = load_counter(&B.lvl[k]);
    if (size == 0) break;
    levels = k + 1;
    if (size > tail_limit) big_end = k + 1;
    const int32_t* in = (k & 1) ? B.fr1 : B.fr0;
    int32_t* out = (k & 1) ? B.fr0 : B.fr1;
    for (int32_t base = 0; base < size; base += kWgThreads) {
      int32_t t = base + (int32_t)threadIdx.x;
      expand<true>(t < size ? load_counter(&in[t]) : -1, B.child_ptr, B.child, B.pcost, B.g, out, &B.lvl[k + 1]);
    }
    if (threadIdx.x == 0) B.lvl[k + 2] = 0;
    __syncthreads();
    ++k;
  }
  if (threadIdx.x == 0) {
    if (levels > B.info->levels) B.info->levels = levels;
    if (big_end > B.info->big_end) B.info->big_end = big_end;
  }
}

// ---------------------------------------------------------------------------
// Walk evaluation: one launch, no level barriers.
//
// Each vertex v walks up its parent chain until it meets a vertex whose value of
// this Evaluate is already known (a 64-bit word {epoch, g bits} stamped with the
// current epoch), the root (g = 0), or a vertex without parent that is not the
// root (the chain is detached: +inf).  It then folds the recorded path downward,
// g(x) = g(parent x) + pcost(x) one binary32 addition at a time -- exactly the
// additions, in exactly the order, of the breadth-first walk -- and stamps every
// vertex it computed.  Threads that meet each other's stamps stop early; stamps
// that are not yet visible only cost extra walking, never a wrong value, because
// any word carrying the current epoch holds the final value of its vertex.
//
// The path is kept in a ring of kRing slots per thread in LDS; a longer path folds
// its top kRing vertices, stamps them and walks again from v (which now stops
// there).  Single graphs keep each path vertex's edge cost beside it (32 KB per
// workgroup, 4 waves per SIMD; more waves in flight meet more ancestors not yet
// stamped, and the 1M-vertex walk gets slower with 6 or 8); batches keep the vertex
// only and read its cost again in the fold (16 KB, 8 waves per SIMD: their deep 2D
// and 3D trees are bound by the latency of long climbs).  A walk longer than n hops
// can only be a parent cycle away from the root; its vertices are unreachable and get
// +inf.
//
// kTrunc (single graphs): the truncated Evaluate.  A vertex is visited only when its
// parent is the root or a visited vertex with fl(g + h) < G0, G0 being the problem's
// threshold when the launch starts (g(goal) before this Evaluate).  The fold carries
// that rule down the path: a visited vertex gets its fresh g, and its stamp says
// whether its children are visited (kWalkNoChildren clear) or not; vertices below
// one whose children are not visited -- and detached or cyclic chains -- are stamped
// kWalkNoChildren and keep the g they had.  The stamps of this walk are what the
// next promising list reads.
constexpr int kWalkThreads = 256;
constexpr int kRing = 16;

// kCoherent: stamps are read and written at device scope (visible across XCDs
// within the launch); otherwise they are plain accesses (visible within the XCD
// and to later launches).
template <bool kCoherent>
__device__ __forceinline__ unsigned long long load_word(const unsigned long long* p) {
  if (kCoherent) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <bool kCoherent>
__device__ __forceinline__ void store_word(unsigned long long* p, unsigned long long w) {
  if (kCoherent)
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// kFinish (single graphs, the walk after an Improve): the walk takes the finish step.
// The counter copies accumulate over the Replan; every workgroup sums the parents
// switched so far and runs only if that moved past ps->changed_seen (set by the
// promising list at the start of the iteration, unchanged during this launch);
// workgroup 0 of the first part writes the totals, the convergence test and the cap to
// the problem state and the loop flags, which only later launches read.
template <bool kFinish>
__device__ __forceinline__ bool walk_finish(ProblemState* __restrict__ ps, LoopCtl* __restrict__ ctl,
                                            const IterCounters* __restrict__ ctr, int book) {
  if (!kFinish) return ctl->any_eval != 0;
  __shared__ int run_flag;
  if (threadIdx.x < kCounterSlots) {  // one wave
    const IterCounters& c = ctr[threadIdx.x];
    unsigned long long ch = (unsigned)c.changed, np = (unsigned)c.nP, nd = (unsigned)c.nD, ed = c.edges,
                       pe = (unsigned)c.pedges;
#pragma unroll
    for (int off = kCounterSlots / 2; off > 0; off >>= 1) {
      ch += __shfl_xor(ch, off, kCounterSlots);
      np += __shfl_xor(np, off, kCounterSlots);
      nd += __shfl_xor(nd, off, kCounterSlots);
      ed += __shfl_xor(ed, off, kCounterSlots);
      pe += __shfl_xor(pe, off, kCounterSlots);
    }
    if (threadIdx.x == 0) {
      run_flag = ch != ps->changed_seen;
      if (book && blockIdx.x == 0) {
        ProblemState& q = *ps;
        if (q.active) {
          q.iterations += 1;
          q.edges = ed;
          q.sum_P = np;
          q.sum_D = nd;
          q.mark_edges = pe;
          const bool switched = ch != q.changed_total;
          q.changed_total = ch;
          if (!switched) {  // no parent switched: fixed point (dJ = 0)
            q.active = 0;
            q.needs_eval = 0;
          } else {
            q.needs_eval = 1;
            if (q.iterations >= q.cap) {
              q.active = 0;
              q.status = 1;
            }
          }
        } else {
          q.needs_eval = 0;
        }
        ctl->any_active = q.active;
        ctl->npromising = 0;
        ctl->epoch = next_mark_epoch(ctl->epoch);
      }
    }
  }
  __syncthreads();
  return run_flag != 0;
}

template <bool kCountHops, bool kCoherent, bool kBatched, bool kTrunc, bool kFinish = false>
__global__ void __launch_bounds__(kWalkThreads) k_eval_walk(int32_t lo, int32_t hi, int32_t n,
                                                           const int32_t* __restrict__ prob,
                                                           ProblemState* __restrict__ ps,
                                                           LoopCtl* __restrict__ ctl,
                                                           const int32_t* __restrict__ parent,
                                                           const float* __restrict__ pcost, float* __restrict__ g,
                                                           unsigned long long* __restrict__ word,
                                                           unsigned long long* __restrict__ hops,
                                                           const int32_t* __restrict__ tiles,
                                                           const float* __restrict__ h,
                                                           const IterCounters* __restrict__ ctr, int book) {
  static_assert(!(kTrunc && kBatched), "the truncated Evaluate takes a single graph");
  __shared__ int32_t ring_v[kRing][kWalkThreads];
  constexpr bool kRingCost = !kBatched;  // the ring holds the edge costs too
  __shared__ float ring_c[kRingCost ? kRing : 1][kWalkThreads];
  static_assert(!(kFinish && kBatched), "batches keep their finish step");
  if (!walk_finish<kFinish>(ps, ctl, ctr, book)) return;  // no parent switched in this iteration
  const unsigned long long tag = (unsigned long long)ctl->eval_epoch << 32;
  const float G0 = kTrunc ? ps[0].thr : 0.0f;
  unsigned long long walked = 0;
  // a batch loops over the units of its active tiles; a single graph has one unit
  const int64_t units = kBatched ? tile_units(ctl, n, kWalkThreads) : 1;
  for (int64_t wu = kBatched ? blockIdx.x : 0; wu < units; wu += kBatched ? gridDim.x : 1) {
  const int64_t v = (kBatched ? tile_unit_slot(ctl, tiles, kWalkThreads, wu) : lo + (int64_t)blockIdx.x * blockDim.x) +
                    threadIdx.x;
  if (v >= hi) continue;
  if (!kFinish && !ps[kBatched ? prob[v] : 0].needs_eval) continue;
  for (;;) {
    int32_t u = (int32_t)v;
    int64_t k = 0;
    uint32_t top;  // g bits above the recorded path
    for (;;) {
      // the stamp, parent and parent-edge cost of u in one round trip
      const unsigned long long w = load_word<kCoherent>(&word[u]);
      const int32_t p = parent[u];
      const float c = pcost[u];
      if ((w & 0xffffffff00000000ull) == tag) {
        top = (uint32_t)w;
        break;
      }
      if (p == kRootMark) {  // a root: g = 0
        top = 0u;
        store_word<kCoherent>(&word[u], tag);
        g[u] = 0.0f;
        break;
      }
      ring_v[k % kRing][threadIdx.x] = u;
      if (kRingCost) ring_c[k % kRing][threadIdx.x] = c;
      ++k;
      if (p < 0 || k > n) {  // detached chain (or a cycle): unreachable
        top = kTrunc ? kWalkNoChildren : 0x7f800000u;
        break;
      }
      u = p;
    }
    walked += (unsigned long long)k;
    const int64_t stop = k > kRing ? k - kRing : 0;
    if (kTrunc) {
      // top: stamp bits of the vertex above the path (kWalkNoChildren or its g)
      uint32_t st = top;
      for (int64_t i = k - 1; i >= stop; --i) {
        const int32_t x = ring_v[i % kRing][threadIdx.x];
        if (!(st & kWalkNoChildren)) {  // x is visited: fresh g, then its own test
          const float acc = add_rn(__uint_as_float(st), kRingCost ? ring_c[i % kRing][threadIdx.x] : pcost[x]);
          g[x] = acc;
          st = __float_as_uint(acc) | (add_rn(acc, h ? h[x] : 0.0f) < G0 ? 0u : kWalkNoChildren);
        }
        store_word<kCoherent>(&word[x], tag | st);
      }
      if (stop == 0) break;
      continue;
    }
    float acc = __uint_as_float(top);
    for (int64_t i = k - 1; i >= stop; --i) {
      const int32_t x = ring_v[i % kRing][threadIdx.x];
      acc = add_rn(acc, kRingCost ? ring_c[i % kRing][threadIdx.x] : pcost[x]);
      store_word<kCoherent>(&word[x], tag | __float_as_uint(acc));
      g[x] = acc;
    }
    if (stop == 0) break;
  }
  }
  if (kCountHops) atomicAdd(hops, walked);
}

}  // namespace

void launch_eval_walk(const WalkArgs& a, hipStream_t s) {
  const int parts = a.prob ? 1 : (a.parts < 1 ? 1 : a.parts);
  const int64_t per = ((int64_t)a.n + parts - 1) / parts;
  for (int k = 0; k < parts; ++k) {
    const int32_t lo = (int32_t)(k * per < a.n ? k * per : a.n);
    const int32_t hi = (int32_t)((k + 1) * per < a.n ? (k + 1) * per : a.n);
    if (hi <= lo && k > 0) break;
    // batches launch whole tiles (the live ones are picked on the device)
    const int64_t units = (((int64_t)a.n + kTileSlots - 1) / kTileSlots) * (kTileSlots / kWalkThreads);
    const dim3 grid(a.prob ? (unsigned)(units < a.blocks ? (units > 0 ? units : 1) : a.blocks)
                           : blocks_for(hi - lo, kWalkThreads));
#define PIRRT_WALK1(H, C, B, T, F)                                                                          \
  hipLaunchKernelGGL((k_eval_walk<H, C, B, T, F>), grid, dim3(kWalkThreads), 0, s, lo, hi, a.n, a.prob, a.ps, \
                     a.ctl, a.parent, a.pcost, a.g, a.word, a.hops, a.tiles, a.h, a.ctr, k == 0 ? 1 : 0)
#define PIRRT_WALK(H, C, B)                                              \
  do {                                                                   \
    if (!B && a.finish) PIRRT_WALK1(H, C, false, false, true);           \
    else PIRRT_WALK1(H, C, B, false, false);                             \
  } while (0)
#define PIRRT_WALK_TRUNC(H, C)                                           \
  do {                                                                   \
    if (a.finish) PIRRT_WALK1(H, C, false, true, true);                  \
    else PIRRT_WALK1(H, C, false, true, false);                          \
  } while (0)
    const bool b = a.prob != nullptr;
    if (a.truncated && !b) {  // the host rejects the truncated Evaluate for batches
      if (a.hops) {
        if (a.coherent) PIRRT_WALK_TRUNC(true, true); else PIRRT_WALK_TRUNC(true, false);
      } else {
        if (a.coherent) PIRRT_WALK_TRUNC(false, true); else PIRRT_WALK_TRUNC(false, false);
      }
      continue;
    }
    if (a.hops) {
      if (a.coherent) { if (b) PIRRT_WALK(true, true, true); else PIRRT_WALK(true, true, false); }
      else { if (b) PIRRT_WALK(true, false, true); else PIRRT_WALK(true, false, false); }
    } else {
      if (a.coherent) { if (b) PIRRT_WALK(false, true, true); else PIRRT_WALK(false, true, false); }
      else { if (b) PIRRT_WALK(false, false, true); else PIRRT_WALK(false, false, false); }
    }
#undef PIRRT_WALK
#undef PIRRT_WALK_TRUNC
#undef PIRRT_WALK1
  }
}

void launch_evaluate(const EvalArgs& a, hipStream_t s) {
  const int32_t n = a.n;
  hipLaunchKernelGGL(k_eval_prep, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, a.ps, a.parent, a.g, a.child_cnt);
  scan_i32_to_i32(a.child_cnt, n, a.child_ptr, a.scan_scratch, s);
  hipLaunchKernelGGL(k_eval_fill, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, a.ps, a.parent, a.child_ptr,
                     a.child_cnt, a.child);
  Bfs B{a.child_ptr, a.child, a.pcost, a.g, a.fr0, a.fr1, a.lvl, a.info, a.ps};
  hipLaunchKernelGGL(k_bfs_head, dim3(1), dim3(kWgThreads), 0, s, (int32_t)kWgThreads, B);
  for (int32_t j = 0; j < a.mid_launches; ++j)
    hipLaunchKernelGGL(k_bfs_level, dim3(a.level_blocks), dim3(kThreads), 0, s, j, (int32_t)kWgThreads, B);
  hipLaunchKernelGGL(k_bfs_tail, dim3(1), dim3(kWgThreads), 0, s, a.mid_launches, (int32_t)kWgThreads, B);
}

}  // namespace pirrt
