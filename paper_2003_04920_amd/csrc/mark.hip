// Promising set and Improve domain (Alg. 2; Sec. IV-B, IV-C).
//
// P = { v : g(v) + h(v) < G } with G = g(goal) of v's problem (or +inf without
// pruning; -inf for a problem that no longer iterates).  Every v of P and every
// neighbour of v is stamped with the iteration's epoch, which makes D = P u N(P)
// without a clearing pass; the domain list then compacts the stamped slots.  With
// the narrowed domain (StepArgs::lookahead) a neighbour w of a promising u is
// stamped only when fl(fl(g(u) + c(u, w)) + h(w)) < G.
//
// Stamps are one byte: the low byte of the mark epoch (never 0).  The host clears
// them before every Replan, and the domain compaction clears every stamp it reads in
// the iteration after which the low byte would wrap, so a stamp never survives 255
// epochs.
//
// Work split: one group of GW lanes per row, Q aligned quads of row entries per lane
// in flight.  kBatched: several problems share the arrays; prob[slot] names the
// problem of a slot.  Without it every slot belongs to problem 0.
#include "rowpass.h"

namespace pirrt {

namespace {

using rows::kThreads;
using rows::flush_counters;
using rows::grid_for;
using rows::batch_grid;

// Idx: uint32_t when every adjacency offset fits (32-bit offsets let the loads use a
// scalar base plus a 32-bit vector offset), int64_t otherwise.
//
// Rows are read in aligned quads of entries (16-byte loads of neighbour slots and of
// costs): quad k holds entries 4k .. 4k+3, and the entries of a quad that lie outside
// the row [a, b) are masked (their neighbour is replaced by slot 0 before any
// gather).  The adjacency arrays keep at least three entries of slack past the last
// one, so the last quad of the last row stays inside the allocation.
template <int GW, int Q, typename Idx, bool kBatched, bool kLook>
__global__ void __launch_bounds__(kThreads) k_mark(int32_t n, const int32_t* __restrict__ prob,
                                                  const ProblemState* __restrict__ ps,
                                                  const LoopCtl* __restrict__ ctl, const float* __restrict__ g,
                                                  const float* __restrict__ h, const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col, const float* __restrict__ cst,
                                                  uint8_t* __restrict__ stamp, IterCounters* __restrict__ ctr,
                                                  const int32_t* __restrict__ tiles) {
  if (ctl->any_active == 0) return;  // every problem has converged
  const uint8_t ep = (uint8_t)ctl->epoch;
  const int gl = threadIdx.x % GW;
  // a batch loops over the units of its active tiles; a single graph has one unit
  const int64_t units = kBatched ? tile_units(ctl, n, kThreads / GW) : 1;
  for (int64_t w = kBatched ? blockIdx.x : 0; w < units; w += kBatched ? gridDim.x : 1) {
  const int64_t vbase =
      kBatched ? tile_unit_slot(ctl, tiles, kThreads / GW, w) : (int64_t)blockIdx.x * (kThreads / GW);
  const int64_t v = vbase + threadIdx.x / GW;
  const int32_t x = v < n ? (int32_t)v : n - 1;
  const int p = kBatched ? prob[x] : 0;
  const float G = ps[p].thr;
  const float gx = g[x], hx = h ? h[x] : 0.0f;
  const Idx ra = (Idx)rp[x], rb = (Idx)rp[x + 1];
  const bool in = v < n && add_rn(gx, hx) < G;
  if (in) {
    if (gl == 0) stamp[x] = ep;
    const int4* col4 = reinterpret_cast<const int4*>(col);
    const float4* cst4 = reinterpret_cast<const float4*>(cst);
    const Idx qa = ra >> 2, qb = (rb + 3) >> 2;
    for (Idx k = qa + gl; k < qb; k += GW * Q) {
      int4 w[Q];
      float4 cw[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const Idx kk = k + q * GW < qb ? k + q * GW : qa;
        w[q] = col4[kk];
        if (kLook) cw[q] = cst4[kk];
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        if (k + q * GW >= qb) continue;
        const Idx j0 = (k + q * GW) * 4;
        const int32_t u[4] = {w[q].x, w[q].y, w[q].z, w[q].w};
        float c[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (kLook) {
          c[0] = cw[q].x;
          c[1] = cw[q].y;
          c[2] = cw[q].z;
          c[3] = cw[q].w;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (j0 + e >= ra && j0 + e < rb &&
              (!kLook || add_rn(add_rn(gx, c[e]), h ? h[u[e]] : 0.0f) < G))
            stamp[u[e]] = ep;
      }
    }
  }
  if (kBatched)
    rows::flush_counters_wave<true, false, false, false, true>(ctr, p, v < n && gl == 0, in ? 1 : 0, 0, 0ull, 0,
                                                               in ? (int)(rb - ra) : 0);
  else
    flush_counters(ctr, p, v < n && gl == 0, in ? 1 : 0, 0, 0ull, 0, in ? (int)(rb - ra) : 0);
  }
}

// Compacted Improve domain: the slots stamped with this iteration's epoch.  Each
// thread tests kListPer consecutive stamps (one 16-byte load), a workgroup scan
// places them, and one atomic per workgroup reserves the workgroup's chunk
// (ascending inside the chunk), which is staged in LDS and written out coalesced.
// When the next mark epoch wraps its low byte, every stamp is cleared here after being
// read.
constexpr int kListPer = 16;

// In a batch only the active tiles are scanned, and a slot of a problem that has
// stopped never enters the list (its stamps may be stale: tiles of stopped problems
// are not cleared at the wrap).
__global__ void __launch_bounds__(kThreads) k_domain_list(int32_t n, LoopCtl* __restrict__ ctl,
                                                         uint8_t* __restrict__ stamp, int32_t* __restrict__ dlist,
                                                         const int32_t* __restrict__ prob,
                                                         const ProblemState* __restrict__ ps,
                                                         const int32_t* __restrict__ tiles) {
  if (ctl->any_active == 0) return;  // every problem has converged
  const uint32_t epoch = ctl->epoch;
  const uint8_t ep = (uint8_t)epoch;
  const bool wrap = (epoch & 0xffu) == 0xffu;
  const int64_t units = prob ? tile_units(ctl, n, kThreads * kListPer) : 1;
  for (int64_t wu = prob ? blockIdx.x : 0; wu < units; wu += prob ? gridDim.x : 1) {
  const int64_t bbase =
      prob ? tile_unit_slot(ctl, tiles, kThreads * kListPer, wu) : (int64_t)blockIdx.x * kThreads * kListPer;
  const int64_t v0 = bbase + (int64_t)threadIdx.x * kListPer;
  uint32_t mask = 0;
  if (v0 + kListPer <= n) {
    uint4* p4 = reinterpret_cast<uint4*>(stamp + v0);
    const uint4 w = *p4;
    const uint32_t words[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (((words[q] >> (8 * b)) & 0xffu) == ep) mask |= 1u << (4 * q + b);
    if (wrap && (w.x | w.y | w.z | w.w) != 0u) *p4 = make_uint4(0u, 0u, 0u, 0u);
  } else {
    for (int i = 0; i < kListPer; ++i) {
      if (v0 + i >= n) break;
      const uint8_t sv = stamp[v0 + i];
      if (sv == ep) mask |= 1u << i;
      if (wrap && sv != 0) stamp[v0 + i] = 0;
    }
  }
  if (prob && mask) {
    // the thread's slots nearly always belong to one problem: one flag to read
    const int64_t last = v0 + kListPer <= n ? v0 + kListPer - 1 : n - 1;
    const int32_t pa = prob[v0], pb = prob[last];
    if (pa == pb) {
      if (!ps[pa].active) mask = 0;
    } else {
      for (uint32_t m = mask; m; m &= m - 1) {
        const int i = __ffs(m) - 1;
        if (!ps[prob[v0 + i]].active) mask &= ~(1u << i);
      }
    }
  }
  // workgroup exclusive scan of the per-thread counts
  __shared__ int wsum[kThreads / kWave];
  __shared__ int base, total;
  __shared__ int32_t staged[kThreads * kListPer];  // the unit's list, written out coalesced
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  __syncthreads();  // the previous unit's readers of wsum / base are done
  const int c = __popc(mask);
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
    for (int w = 0; w < kThreads / kWave; ++w) {
      const int x = wsum[w];
      wsum[w] = t;
      t += x;
    }
    base = t ? atomicAdd(&ctl->ndomain, t) : 0;
    total = t;
  }
  __syncthreads();
  int pos = wsum[wid] + incl - c;
  while (mask) {
    const int i = __ffs(mask) - 1;
    mask &= mask - 1;
    staged[pos++] = (int32_t)(v0 + i);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < total; j += kThreads) dlist[base + j] = staged[j];
  }
}

// Single graphs mark in two steps.  k_promising_list tests kListPer consecutive
// vertices per thread (16-byte loads of g and h), stamps the promising ones and lists
// them (one atomic per workgroup, the chunk staged in LDS and written out coalesced);
// k_mark_rows then stamps the neighbours of the
// listed vertices only, so the row work follows |P| rather than n.
// kTrunc: P is the set the last (truncated) walk queued: the vertices other than the
// root whose walk stamp lacks kWalkNoChildren (every vertex is stamped by each walk).
//
// It also takes the place of the after-eval step of a batch: every workgroup derives
// the threshold G from g(goal) of the last Evaluate (or +inf without pruning; the loop
// stops once the problem is inactive), and workgroup 0 publishes it with the loop
// flags for the kernels that follow and takes a fresh Evaluate epoch.
template <bool kTrunc>
__global__ void __launch_bounds__(kThreads) k_promising_list(int32_t n, ProblemState* __restrict__ ps,
                                                            LoopCtl* __restrict__ ctl, const float* __restrict__ g,
                                                            const float* __restrict__ h,
                                                            uint8_t* __restrict__ stamp, int32_t* __restrict__ plist,
                                                            IterCounters* __restrict__ ctr,
                                                            const unsigned long long* __restrict__ word, int prune,
                                                            const int64_t* __restrict__ rp) {
  const bool active = ps[0].active != 0;
  const float G = active ? (prune ? g[ps[0].goal] : pos_inf()) : -pos_inf();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ps[0].thr = G;
    ctl->any_active = active ? 1 : 0;
    ctl->any_eval = 0;
    ctl->ndomain = 0;
    ctl->ntiles = -1;
    ctl->eval_epoch = next_epoch(ctl->eval_epoch);
    ps[0].changed_seen = ps[0].changed_total;  // the walk after this Improve compares against it
  }
  if (!active) return;  // the problem has converged
  const uint8_t ep = (uint8_t)ctl->epoch;
  const int64_t v0 = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * kListPer;
  uint32_t mask = 0;
  if (kTrunc) {
    const int32_t root = ps[0].root;
    for (int i = 0; i < kListPer; ++i) {
      const int64_t v = v0 + i;
      if (v < n && v != root && !((uint32_t)word[v] & kWalkNoChildren)) mask |= 1u << i;
    }
  } else if (v0 + kListPer <= n) {
    const float4* g4 = reinterpret_cast<const float4*>(g + v0);
    const float4* h4 = reinterpret_cast<const float4*>(h ? h + v0 : g);
#pragma unroll
    for (int q = 0; q < kListPer / 4; ++q) {
      const float4 a = g4[q];
      const float4 b = h ? h4[q] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (add_rn(a.x, b.x) < G) mask |= 1u << (4 * q);
      if (add_rn(a.y, b.y) < G) mask |= 1u << (4 * q + 1);
      if (add_rn(a.z, b.z) < G) mask |= 1u << (4 * q + 2);
      if (add_rn(a.w, b.w) < G) mask |= 1u << (4 * q + 3);
    }
  } else {
    for (int i = 0; i < kListPer && v0 + i < n; ++i)
      if (add_rn(g[v0 + i], h ? h[v0 + i] : 0.0f) < G) mask |= 1u << i;
  }
  // the degrees of the listed rows (the rows the mark walks), for the counters: the
  // thread's kListPer + 1 row offsets in one batch of 16-byte loads
  int pe = 0;
  if (mask) {
    if (v0 + kListPer <= n) {
      const longlong2* r2 = reinterpret_cast<const longlong2*>(rp + v0);
      int64_t r[kListPer + 1];
#pragma unroll
      for (int q = 0; q < kListPer / 2; ++q) {
        const longlong2 t = r2[q];
        r[2 * q] = t.x;
        r[2 * q + 1] = t.y;
      }
      r[kListPer] = rp[v0 + kListPer];
#pragma unroll
      for (int i = 0; i < kListPer; ++i)
        if (mask & (1u << i)) pe += (int)(r[i + 1] - r[i]);
    } else {
      for (uint32_t m = mask; m; m &= m - 1) {
        const int64_t v = v0 + __ffs(m) - 1;
        pe += (int)(rp[v + 1] - rp[v]);
      }
    }
  }
  __shared__ int wsum[kThreads / kWave];
  __shared__ int wpe[kThreads / kWave];
  __shared__ int base, total;
  __shared__ int32_t staged[kThreads * kListPer];  // the workgroup's list, written out coalesced
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int c = __popc(mask);
  int incl = c;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int y = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += y;
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) pe += __shfl_xor(pe, off, kWave);
  if (lane == kWave - 1) wsum[wid] = incl;
  if (lane == 0) wpe[wid] = pe;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0, e = 0;
    for (int w = 0; w < kThreads / kWave; ++w) {
      const int x = wsum[w];
      wsum[w] = t;
      t += x;
      e += wpe[w];
    }
    base = t ? atomicAdd(&ctl->npromising, t) : 0;
    total = t;
    if (t) atomicAdd(&ctr[blockIdx.x % kCounterSlots].nP, t);
    if (e) atomicAdd(&ctr[blockIdx.x % kCounterSlots].pedges, e);
  }
  __syncthreads();
  int pos = wsum[wid] + incl - c;
  while (mask) {
    const int i = __ffs(mask) - 1;
    mask &= mask - 1;
    stamp[v0 + i] = ep;
    staged[pos++] = (int32_t)(v0 + i);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < total; j += kThreads) plist[base + j] = staged[j];
}


// Neighbour stamping of the listed promising vertices (single graphs).  The rows one
// workgroup takes are neighbours in the storage order, so they share most of their
// neighbours: the 32 rows of a 6D workgroup list each distinct neighbour about twice.
// Each pass writes every entry's slot id into a direct-mapped table in LDS (the last
// writer keeps a position), then stamps once per table position in use; an entry
// whose id lost its position is stamped directly.  Slot u sits at position
// (mix(u / 32) + u % 32) mod the table size, so the ids of one 128-byte line of stamps
// occupy neighbouring positions and their stores leave from neighbouring lanes, which
// lets the memory pipeline merge them: about half the L2 write requests of one store
// per entry.
constexpr int32_t kTabEmpty = -1;

__device__ __forceinline__ uint32_t tab_pos(int32_t u) {
  return (((uint32_t)u >> 5) * 0x9E3779B1u >> 16) + ((uint32_t)u & 31u);
}

// 64 table positions per row of the workgroup (a 6D row has ~54 entries).
template <int GW>
constexpr int tab_slots() { return (kThreads / GW) * 64; }

template <int GW, int Q, typename Idx, bool kLook>
__global__ void __launch_bounds__(kThreads) k_mark_rows(const ProblemState* __restrict__ ps,
                                                       const LoopCtl* __restrict__ ctl,
                                                       const int32_t* __restrict__ plist,
                                                       const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                       const float* __restrict__ cst, const float* __restrict__ g,
                                                       const float* __restrict__ h, uint8_t* __restrict__ stamp) {
  constexpr int kSlots = tab_slots<GW>();
  constexpr int kPer = kSlots / kThreads;
  __shared__ int32_t keys[kSlots];
  __shared__ uint32_t offer[kLook ? kSlots : 1];  // best offer (binary32 bits, >= 0) per position
  if (ctl->any_active == 0) return;
  const int64_t cnt = ctl->npromising;
  const uint8_t ep = (uint8_t)ctl->epoch;
  const int64_t step = (int64_t)gridDim.x * (kThreads / GW);  // one pass when the grid covers the list
  for (int64_t first = (int64_t)blockIdx.x * (kThreads / GW); first < cnt; first += step) {
  const int gl = threadIdx.x % GW;
  const int64_t gi = first + threadIdx.x / GW;
  const bool valid = gi < cnt;
  const int32_t x = plist[valid ? gi : cnt - 1];
  const Idx ra = valid ? (Idx)rp[x] : 0, rb = valid ? (Idx)rp[x + 1] : 0;
  const float gx = kLook ? g[x] : 0.0f, G = kLook ? ps[0].thr : 0.0f;
  const int4* col4 = reinterpret_cast<const int4*>(col);
  const float4* cst4 = reinterpret_cast<const float4*>(cst);
  const Idx qa = ra >> 2, qb = (rb + 3) >> 2;
  Idx k = qa + gl;
  for (;;) {
    for (int i = threadIdx.x; i < kSlots; i += kThreads) {
      keys[i] = kTabEmpty;
      if (kLook) offer[i] = 0x7f800000u;
    }
    if (!__syncthreads_or(k < qb)) break;  // also: the clears are done
    int32_t u[4 * Q];
    uint32_t ob[4 * Q];  // with kLook: the offer fl(g(x) + c) of x to each entry
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const Idx kk = k + q * GW < qb ? k + q * GW : qa;
      const int4 w = col4[kk];
      const Idx j0 = (k + q * GW) * 4;
      const bool live = k + q * GW < qb;
      const int32_t uu[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) u[4 * q + e] = live && j0 + e >= ra && j0 + e < rb ? uu[e] : -1;
      if (kLook) {
        const float4 cw = cst4[kk];
        ob[4 * q] = __float_as_uint(add_rn(gx, cw.x));
        ob[4 * q + 1] = __float_as_uint(add_rn(gx, cw.y));
        ob[4 * q + 2] = __float_as_uint(add_rn(gx, cw.z));
        ob[4 * q + 3] = __float_as_uint(add_rn(gx, cw.w));
      }
    }
#pragma unroll
    for (int i = 0; i < 4 * Q; ++i)
      if (u[i] >= 0) keys[tab_pos(u[i]) & (kSlots - 1)] = u[i];
    __syncthreads();
    // Entries whose id kept its position: with kLook the position keeps the smallest
    // offer (offers are >= 0, so their bits order as unsigned integers).  The others
    // are handled directly.  Rounding is monotone, so fl(min offer + h) < G holds
    // exactly when fl(offer + h) < G holds for some offer.
#pragma unroll
    for (int i = 0; i < 4 * Q; ++i) {
      if (u[i] < 0) continue;
      const uint32_t pos = tab_pos(u[i]) & (kSlots - 1);
      if (keys[pos] == u[i]) {
        if (kLook) atomicMin(&offer[pos], ob[i]);
      } else if (!kLook || add_rn(__uint_as_float(ob[i]), h ? h[u[i]] : 0.0f) < G) {
        stamp[u[i]] = ep;
      }
    }
    if (kLook) __syncthreads();  // the offers are complete
    {
      int32_t y[kPer];
      float hv[kPer];
#pragma unroll
      for (int j = 0; j < kPer; ++j) y[j] = keys[threadIdx.x + j * kThreads];
#pragma unroll
      for (int j = 0; j < kPer; ++j) hv[j] = kLook && h ? h[y[j] != kTabEmpty ? y[j] : 0] : 0.0f;
#pragma unroll
      for (int j = 0; j < kPer; ++j)
        if (y[j] != kTabEmpty &&
            (!kLook || add_rn(__uint_as_float(offer[kLook ? threadIdx.x + j * kThreads : 0]), hv[j]) < G))
          stamp[y[j]] = ep;
    }
    k += GW * Q;
    __syncthreads();  // every read of the table is done before it is cleared
  }
  }
}

// On large graphs the listed rows' grid covers half the vertices: a workgroup takes a
// second chunk of rows only while more than half the vertices are promising (the first
// iterations), and the launch carries half as many workgroups that find nothing to do.
// Measured on the 1M graph: 1% per Replan against a grid for all n (a quarter or an
// eighth: no better).  Graphs below kMarkRowsHalfGridMin vertices, where that was not
// measured, keep one chunk of rows per workgroup.
constexpr int kMarkRowsGridDiv = 2;
constexpr int32_t kMarkRowsHalfGridMin = 1 << 18;

template <int GW, int U, bool B>
void launch_mark_t(const StepArgs& a, hipStream_t s) {
  if (!B) {  // single graph: promising list, then the rows of the listed vertices
    const int64_t per_block = (int64_t)kThreads * kListPer;
    const dim3 pgrid((unsigned)((a.n + per_block - 1) / per_block));
    if (a.truncated)
      hipLaunchKernelGGL(k_promising_list<true>, pgrid, dim3(kThreads), 0, s, a.n, a.ps, a.ctl, a.g, a.h, a.stamp,
                         a.plist, a.ctr, a.word, a.prune, a.rp);
    else
      hipLaunchKernelGGL(k_promising_list<false>, pgrid, dim3(kThreads), 0, s, a.n, a.ps, a.ctl, a.g, a.h, a.stamp,
                         a.plist, a.ctr, a.word, a.prune, a.rp);
    const bool narrow = a.nnz < ((int64_t)1 << 32) - 64 * GW;
    const int div = a.n >= kMarkRowsHalfGridMin ? kMarkRowsGridDiv : 1;
    const dim3 rgrid = grid_for((a.n + div - 1) / div, GW);
#define PIRRT_MARK_ROWS(I, L)                                                                                   \
  hipLaunchKernelGGL((k_mark_rows<GW, U, I, L>), rgrid, dim3(kThreads), 0, s, a.ps, a.ctl, a.plist, a.rp, a.col, \
                     a.cst, a.g, a.h, a.stamp)
    if (narrow) {
      if (a.lookahead) PIRRT_MARK_ROWS(uint32_t, true); else PIRRT_MARK_ROWS(uint32_t, false);
    } else {
      if (a.lookahead) PIRRT_MARK_ROWS(int64_t, true); else PIRRT_MARK_ROWS(int64_t, false);
    }
#undef PIRRT_MARK_ROWS
    return;
  }
  const dim3 grid = batch_grid(a.n, kThreads / GW, a.blocks);
#define PIRRT_MARK(I, L)                                                                                         \
  hipLaunchKernelGGL((k_mark<GW, U, I, B, L>), grid, dim3(kThreads), 0, s, a.n, a.prob, a.ps, a.ctl, a.g, a.h, a.rp, \
                     a.col, a.cst, a.stamp, a.ctr, a.tiles)
  if (a.nnz < ((int64_t)1 << 32) - 64 * GW) {
    if (a.lookahead) PIRRT_MARK(uint32_t, true); else PIRRT_MARK(uint32_t, false);
  } else {
    if (a.lookahead) PIRRT_MARK(int64_t, true); else PIRRT_MARK(int64_t, false);
  }
#undef PIRRT_MARK
}

template <int GW, int U>
void launch_mark_b(const StepArgs& a, hipStream_t s) {
  if (a.prob) launch_mark_t<GW, U, true>(a, s); else launch_mark_t<GW, U, false>(a, s);
}

// Alg. 3's test |B'| > |B| after an Extend batch: how many of the caller ids
// [first, first + count) are promising under the stored policy, fl(g + h) < g(goal)
// (h indexed from `first`; NULL = 0).  One atomic per wave.
__global__ void __launch_bounds__(kThreads) k_count_promising(int64_t first, int64_t count, int32_t goal_slot,
                                                             const int32_t* __restrict__ slot_of,
                                                             const float* __restrict__ g,
                                                             const float* __restrict__ h,
                                                             unsigned long long* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool p = false;
  if (i < count) p = add_rn(g[slot_of[first + i]], h ? h[i] : 0.0f) < g[goal_slot];
  const unsigned long long b = __ballot(p);
  if ((threadIdx.x & (kWave - 1)) == 0 && b) atomicAdd(out, (unsigned long long)__popcll(b));
}

}  // namespace

void launch_count_promising(int64_t first, int64_t count, int32_t goal_slot, const int32_t* slot_of, const float* g,
                            const float* h, unsigned long long* out, hipStream_t s) {
  if (count > 0)
    hipLaunchKernelGGL(k_count_promising, dim3((unsigned)((count + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                       first, count, goal_slot, slot_of, g, h, out);
}

void launch_domain_list(const StepArgs& a, hipStream_t s) {
  const int64_t per_block = (int64_t)kThreads * kListPer;
  static_assert(kThreads * kListPer == kTileSlots, "one domain-list workgroup per tile");
  const dim3 grid = a.prob ? batch_grid(a.n, (int)per_block, a.blocks) : dim3((unsigned)((a.n + per_block - 1) / per_block));
  hipLaunchKernelGGL(k_domain_list, grid, dim3(kThreads), 0, s, a.n, a.ctl, a.stamp, a.dlist, a.prob, a.ps,
                     a.tiles);
}

// Variants: lanes per row x quads per lane in flight (GW x Q x 4 entries per pass).
void launch_mark(const StepArgs& a, int variant, hipStream_t s) {
  switch (variant) {
    case 0: launch_mark_b<16, 1>(a, s); break;
    case 1: launch_mark_b<8, 2>(a, s); break;
    case 2: launch_mark_b<4, 4>(a, s); break;
    default: launch_mark_b<8, 1>(a, s); break;
  }
}

}  // namespace pirrt
