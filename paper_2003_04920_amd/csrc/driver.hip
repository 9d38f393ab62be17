// Device side of the Replan loop (Alg. 2) for one or many problems: per-problem
// thresholds, the per-iteration bookkeeping of the convergence test, and the root
// marks.  The loop itself never waits on the host: each iteration is
//   mark -> domain list -> improve -> finish -> evaluate -> after-eval (thresholds)
// and a problem whose Improve switched no parent stops (its threshold becomes
// -inf, so the later kernels skip it), exactly when the serial loop would break.
#include "internal.h"

namespace pirrt {

namespace {

// Mark epochs are stored as their low byte: skip the values whose low byte is 0
// (the cleared stamp).

// Marks the roots, clears the counters and takes fresh epochs.  The threshold is set
// to g(goal) as stored before any Evaluate of this Replan (the truncated Evaluate's
// first walk reads it; the full one ignores it).
__global__ void k_replan_init(int32_t P, ProblemState* __restrict__ ps, int32_t* __restrict__ parent,
                              float* __restrict__ pcost, IterCounters* __restrict__ ctr, LoopCtl* __restrict__ ctl,
                              const float* __restrict__ g, int prune) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (int64_t)P * kCounterSlots) {
    IterCounters& c = ctr[t];
    c.changed = 0;
    c.nP = 0;
    c.nD = 0;
    c.pedges = 0;
    c.edges = 0ull;
  }
  if (t < P) {
    const int32_t r = ps[t].root;
    parent[r] = kRootMark;
    pcost[r] = 0.0f;
    ps[t].thr = prune ? g[ps[t].goal] : pos_inf();
  }
  if (t == 0) {
    ctl->epoch = next_mark_epoch(ctl->epoch);
    ctl->eval_epoch = next_epoch(ctl->eval_epoch);
    ctl->any_active = 1;
    ctl->any_eval = 1;
    ctl->ntiles = -1;
    ctl->ndomain = 0;
    ctl->npromising = 0;
    ctl->tiles_stale = 1;
  }
}

// A single graph's set-up in one launch, with no copies from the host: the previous
// roots (caller ids in droots[0..nold)) lose their mark, the new root gets it and is
// recorded in droots[0], and the problem state starts from the kernel arguments.
// Otherwise as k_replan_init.
__global__ void __launch_bounds__(kCounterSlots) k_replan_init_single(
    ProblemState* __restrict__ ps, int32_t root, int32_t goal, int32_t cap, int32_t root_id, int32_t nold,
    int32_t* __restrict__ droots, const int32_t* __restrict__ slot_of, int32_t* __restrict__ parent,
    float* __restrict__ pcost, IterCounters* __restrict__ ctr, LoopCtl* __restrict__ ctl, const float* __restrict__ g,
    int prune) {
  const int t = threadIdx.x;
  IterCounters& c = ctr[t];
  c.changed = 0;
  c.nP = 0;
  c.nD = 0;
  c.pedges = 0;
  c.edges = 0ull;
  if (t == 0) {
    for (int32_t i = 0; i < nold; ++i) {  // in order, before the new mark (a root may repeat)
      const int32_t s = slot_of[droots[i]];
      if (parent[s] == kRootMark) parent[s] = -1;
    }
    droots[0] = root_id;
    parent[root] = kRootMark;
    pcost[root] = 0.0f;
    ProblemState q = {};
    q.root = root;
    q.goal = goal;
    q.thr = prune ? g[goal] : pos_inf();
    q.active = 1;
    q.needs_eval = 1;
    q.cap = cap;
    ps[0] = q;
    ctl->epoch = next_mark_epoch(ctl->epoch);
    ctl->eval_epoch = next_epoch(ctl->eval_epoch);
    ctl->any_active = 1;
    ctl->any_eval = 1;
    ctl->ntiles = -1;
    ctl->ndomain = 0;
    ctl->npromising = 0;
  }
}

// One workgroup of kCounterSlots threads per problem: sums and clears the counter
// copies, then applies the convergence test and the iteration cap.  single: a single
// graph, whose loop has no after-eval step -- its promising list takes that step's
// place -- so the problem's state goes to the loop flags here.
__global__ void __launch_bounds__(kCounterSlots) k_finish(int32_t P, ProblemState* __restrict__ ps,
                                                          IterCounters* __restrict__ ctr, LoopCtl* __restrict__ ctl,
                                                          int single) {
  const int32_t i = blockIdx.x;
  const int t = threadIdx.x;
  IterCounters& c = ctr[(int64_t)i * kCounterSlots + t];
  unsigned long long ch = (unsigned)c.changed, np = (unsigned)c.nP, nd = (unsigned)c.nD, ed = c.edges,
                     pe = (unsigned)c.pedges;
  c.changed = 0;
  c.nP = 0;
  c.nD = 0;
  c.pedges = 0;
  c.edges = 0ull;
#pragma unroll
  for (int off = kCounterSlots / 2; off > 0; off >>= 1) {
    ch += __shfl_xor(ch, off, kCounterSlots);
    np += __shfl_xor(np, off, kCounterSlots);
    nd += __shfl_xor(nd, off, kCounterSlots);
    ed += __shfl_xor(ed, off, kCounterSlots);
    pe += __shfl_xor(pe, off, kCounterSlots);
  }
  if (t == 0) {
    ProblemState& s = ps[i];
    if (s.active) {
      s.iterations += 1;
      s.edges += ed;
      s.sum_P += np;
      s.sum_D += nd;
      s.changed_total += ch;
      s.mark_edges += pe;
      if (ch == 0) {  // no parent switched: fixed point (dJ = 0)
        s.active = 0;
        s.needs_eval = 0;
      } else {
        s.needs_eval = 1;
        if (s.iterations >= s.cap) {
          s.active = 0;
          s.status = 1;
        }
        atomicOr(&ctl->any_eval, 1);
      }
      if (!s.active) atomicOr(&ctl->tiles_stale, 1);
    } else {
      s.needs_eval = 0;
    }
    if (single) {
      ctl->any_active = s.active;
      ctl->npromising = 0;
    }
  }
  if (i == 0 && t == 0) ctl->epoch = next_mark_epoch(ctl->epoch);
}

// Runs after the Evaluate of an iteration (and after the first Evaluate of a
// Replan): a new evaluate epoch, whether any problem still iterates, and each
// problem's promising threshold G for the next iteration (Alg. 2's test against
// g(x_goal), +inf without pruning, -inf for a problem that has stopped).
// In a batch it also lists the tiles that overlap a problem still iterating (a tile
// spans at most a few problems: each holds thousands of slots), in tile order for the
// mark and the domain list and, for the Evaluate walk, by their rank inside their
// problem.
constexpr int kAfterEvalThreads = 1024;
constexpr int kAfterEvalWords = 8192;  // tile bitmap in LDS: up to 262,144 tiles (2^30 slots)
constexpr int kWordsPerThread = kAfterEvalWords / kAfterEvalThreads;
constexpr int kRanks = kAfterEvalThreads;  // tile ranks inside a problem kept apart (the rest share the last)

// Whether tile t0, the first tile of problem i, is also a tile of an earlier problem
// that still iterates (that problem lists it).
__device__ __forceinline__ bool listed_before(int32_t i, int64_t t0_slot, const int64_t* __restrict__ base,
                                              const ProblemState* __restrict__ ps) {
  for (int32_t q = i - 1; q >= 0 && base[q + 1] > t0_slot; --q)
    if (ps[q].active && base[q + 1] > base[q]) return true;
  return false;
}

__global__ void __launch_bounds__(kAfterEvalThreads) k_after_eval(int32_t P, ProblemState* __restrict__ ps,
                                                                 const float* __restrict__ g, int prune,
                                                                 LoopCtl* __restrict__ ctl, int32_t n,
                                                                 const int32_t* __restrict__ prob,
                                                                 const int64_t* __restrict__ base,
                                                                 int32_t* __restrict__ tiles, int32_t bitmap_tiles,
                                                                 int32_t* __restrict__ tiles_walk) {
  __shared__ int any, count, rebuild;
  __shared__ int rank_at[kRanks];
  __shared__ uint32_t bits[kAfterEvalWords];
  __shared__ int wsum[kAfterEvalThreads / kWave + 1];
  const int32_t T = prob ? (int32_t)(((int64_t)n + kTileSlots - 1) / kTileSlots) : 0;
  // a problem's slots are the range [base[p], base[p + 1]), so its tiles are a range
  // too: the active problems set their tiles' bits, and the list is read off the
  // bitmap in tile order
  const bool bitmap = T <= bitmap_tiles && T <= kAfterEvalWords * 32;
  // The lists stay as they are while no problem has stopped since they were built
  // (problems only ever stop, and listed tiles of a stopped problem cost work but
  // change no result).
  if (threadIdx.x == 0) {
    any = 0;
    rebuild = prob && (ctl->tiles_stale != 0 || ctl->ntiles < 0);
    count = rebuild ? 0 : ctl->ntiles;
  }
  for (int w = threadIdx.x; w < kAfterEvalWords; w += kAfterEvalThreads) bits[w] = 0u;
  __syncthreads();  // also: rebuild is set
  for (int32_t i = threadIdx.x; i < P; i += blockDim.x) {
    ProblemState& s = ps[i];
    const bool a = s.active != 0;
    if (a) any = 1;
    s.thr = a ? (prune ? g[s.goal] : pos_inf()) : -pos_inf();
    if (rebuild && bitmap && a && base[i + 1] > base[i]) {
      const int32_t t0 = (int32_t)(base[i] / kTileSlots), t1 = (int32_t)((base[i + 1] - 1) / kTileSlots);
      for (int32_t t = t0; t <= t1; ++t) atomicOr(&bits[t >> 5], 1u << (t & 31));
    }
  }
  __syncthreads();
  if (rebuild && bitmap) {
    // each thread takes kWordsPerThread consecutive words; a block scan places them
    const int w0 = threadIdx.x * kWordsPerThread;
    int c = 0;
#pragma unroll
    for (int k = 0; k < kWordsPerThread; ++k) c += __popc(bits[w0 + k]);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    int incl = c;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const int y = __shfl_up(incl, off, kWave);
      if (lane >= off) incl += y;
    }
    if (lane == kWave - 1) wsum[wid] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
      int t = 0;
      for (int w = 0; w < kAfterEvalThreads / kWave; ++w) {
        const int x = wsum[w];
        wsum[w] = t;
        t += x;
      }
      count = t;
    }
    __syncthreads();
    int pos = wsum[wid] + incl - c;
#pragma unroll
    for (int k = 0; k < kWordsPerThread; ++k)
      for (uint32_t m = bits[w0 + k]; m; m &= m - 1) tiles[pos++] = (w0 + k) * 32 + __ffs(m) - 1;
  } else if (rebuild) {
    // more tiles than the bitmap holds: test each tile's first and last problem
    for (int32_t t = threadIdx.x; t < T; t += blockDim.x) {
      const int64_t s0 = (int64_t)t * kTileSlots;
      const int64_t s1 = (s0 + kTileSlots < n ? s0 + kTileSlots : n) - 1;
      bool act = false;
      for (int32_t p = prob[s0]; p <= prob[s1]; ++p) act = act || ps[p].active != 0;
      if (act) tiles[atomicAdd(&count, 1)] = t;
    }
  }
  if (rebuild && tiles_walk) {
    // The same tiles for the Evaluate walk, ordered by their rank inside their problem:
    // every problem's first tiles, then every problem's second tiles, ...  Slots are
    // numbered breadth-first inside a problem, so the walk then reaches the shallow
    // parts of every tree before the deep ones, and climbs meet stamped ancestors
    // sooner.  A tile shared by two problems is listed by the first one that iterates.
    rank_at[threadIdx.x] = 0;
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      for (int32_t i = threadIdx.x; i < P; i += blockDim.x) {
        if (!ps[i].active || base[i + 1] <= base[i]) continue;
        const int32_t t0 = (int32_t)(base[i] / kTileSlots), t1 = (int32_t)((base[i + 1] - 1) / kTileSlots);
        const int32_t skip = base[i] % kTileSlots != 0 && listed_before(i, (int64_t)t0 * kTileSlots, base, ps);
        for (int32_t t = t0 + skip; t <= t1; ++t) {
          const int r = t - t0 < kRanks ? t - t0 : kRanks - 1;
          if (pass == 0)
            atomicAdd(&rank_at[r], 1);
          else
            tiles_walk[atomicAdd(&rank_at[r], 1)] = t;
        }
      }
      __syncthreads();
      if (pass == 0) {  // counts -> first position of each rank
        const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
        const int c = rank_at[threadIdx.x];
        int incl = c;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
          const int y = __shfl_up(incl, off, kWave);
          if (lane >= off) incl += y;
        }
        if (lane == kWave - 1) wsum[wid] = incl;
        __syncthreads();
        if (threadIdx.x == 0) {
          int t = 0;
          for (int w = 0; w < kAfterEvalThreads / kWave; ++w) {
            const int x = wsum[w];
            wsum[w] = t;
            t += x;
          }
        }
        __syncthreads();
        rank_at[threadIdx.x] = wsum[wid] + incl - c;
        __syncthreads();
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    ctl->any_active = any;
    ctl->any_eval = 0;
    ctl->ndomain = 0;
    ctl->npromising = 0;
    ctl->ntiles = prob ? count : -1;
    ctl->tiles_stale = 0;
    ctl->eval_epoch = next_epoch(ctl->eval_epoch);
  }
}

}  // namespace

void launch_replan_init(int32_t P, ProblemState* ps, int32_t* parent, float* pcost, IterCounters* ctr,
                        LoopCtl* ctl, const float* g, int prune, hipStream_t s) {
  const int64_t t = (int64_t)P * kCounterSlots;
  hipLaunchKernelGGL(k_replan_init, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, P, ps, parent, pcost, ctr,
                     ctl, g, prune);
}

void launch_replan_init_single(ProblemState* ps, int32_t root, int32_t goal, int32_t cap, int32_t root_id,
                               int32_t nold, int32_t* droots, const int32_t* slot_of, int32_t* parent, float* pcost,
                               IterCounters* ctr, LoopCtl* ctl, const float* g, int prune, hipStream_t s) {
  hipLaunchKernelGGL(k_replan_init_single, dim3(1), dim3(kCounterSlots), 0, s, ps, root, goal, cap, root_id, nold,
                     droots, slot_of, parent, pcost, ctr, ctl, g, prune);
}

void launch_finish(int32_t P, ProblemState* ps, IterCounters* ctr, LoopCtl* ctl, bool single, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(P), dim3(kCounterSlots), 0, s, P, ps, ctr, ctl, single ? 1 : 0);
}

void launch_after_eval(int32_t P, ProblemState* ps, const float* g, int prune, LoopCtl* ctl, int32_t n,
                       const int32_t* prob, const int64_t* base, int32_t* tiles, int32_t bitmap_tiles,
                       int32_t* tiles_walk, hipStream_t s) {
  hipLaunchKernelGGL(k_after_eval, dim3(1), dim3(kAfterEvalThreads), 0, s, P, ps, g, prune, ctl, n, prob, base,
                     tiles, bitmap_tiles, tiles_walk);
}

}  // namespace pirrt
