// Promising set, Improve domain and Improve (Alg. 2; Sec. IV-B, IV-C).
//
// mark    : P = { v : g(v) + h(v) < G } with G = g(goal) of v's problem (or +inf
//           without pruning; -inf for a problem that no longer iterates).  Every v
//           of P and every neighbour of v is stamped with the iteration's epoch,
//           which makes D = P u N(P) without a clearing pass.
// improve : for every stamped v other than its problem's root, the lexicographic
//           minimum of (g(n) + c(n, v), n, c) over v's row, n being the caller's
//           vertex id (storage slots may be renumbered); the parent switches only
//           when that value is strictly below g(v).  g is only read (Jacobi step),
//           so all rows are independent.
//
// Work split: one group of GW lanes per vertex slot, Q aligned quads of row entries
// per lane in flight (GW x Q x 4 = 64 entries per pass over a row by default); the
// grid covers all slots.  Loads are issued unconditionally (quads past the end of
// the row re-read the first one and are masked): `vmcnt` is an in-order counter, so
// a load under a branch would make every later load wait for it.  The per-row
// minimum is a DPP butterfly.
//
// Stamps are one byte: the low byte of the mark epoch (never 0).  The host clears
// them before every Replan, and the domain compaction clears every stamp it reads in
// the iteration after which the low byte would wrap, so a stamp never survives 255
// epochs.  Improve runs over the compacted domain list, not over all slots.
//
// kBatched: several problems share the arrays; prob[slot] names the problem of a
// slot.  Without it every slot belongs to problem 0.
#include "internal.h"

namespace pirrt {

namespace {

constexpr int kThreads = 256;

// Adds the per-vertex counters of the workgroup into its problem's counter copy:
// one atomic per counter and workgroup when the workgroup lies in one problem,
// one per vertex otherwise.
__device__ __forceinline__ void flush_counters(IterCounters* ctr, int p, bool leader, int nP, int nD,
                                               unsigned long long edges, int changed) {
  __shared__ int block_p, mixed;
  __shared__ unsigned long long red[4];
  __syncthreads();  // a previous call of this workgroup may still read red
  if (threadIdx.x == 0) {
    block_p = p;
    mixed = 0;
    red[0] = red[1] = red[2] = red[3] = 0ull;
  }
  __syncthreads();
  if (leader && p != block_p) mixed = 1;
  __syncthreads();
  const int slot = blockIdx.x % kCounterSlots;
  if (mixed) {
    if (leader && (nP | nD | changed)) {
      IterCounters& C = ctr[(int64_t)p * kCounterSlots + slot];
      if (nP) atomicAdd(&C.nP, nP);
      if (nD) atomicAdd(&C.nD, nD);
      if (edges) atomicAdd(&C.edges, edges);
      if (changed) atomicAdd(&C.changed, changed);
    }
    return;
  }
  const int lane = threadIdx.x & (kWave - 1);
  unsigned long long a = leader ? (unsigned long long)nP : 0ull, b = leader ? (unsigned long long)nD : 0ull,
                     c = leader ? edges : 0ull, d = leader ? (unsigned long long)changed : 0ull;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, kWave);
    b += __shfl_xor(b, off, kWave);
    c += __shfl_xor(c, off, kWave);
    d += __shfl_xor(d, off, kWave);
  }
  if (lane == 0) {
    if (a) atomicAdd(&red[0], a);
    if (b) atomicAdd(&red[1], b);
    if (c) atomicAdd(&red[2], c);
    if (d) atomicAdd(&red[3], d);
  }
  __syncthreads();
  if (threadIdx.x < 4 && red[threadIdx.x]) {
    IterCounters& C = ctr[(int64_t)block_p * kCounterSlots + slot];
    const unsigned long long t = red[threadIdx.x];
    if (threadIdx.x == 0) atomicAdd(&C.nP, (int)t);
    if (threadIdx.x == 1) atomicAdd(&C.nD, (int)t);
    if (threadIdx.x == 2) atomicAdd(&C.edges, t);
    if (threadIdx.x == 3) atomicAdd(&C.changed, (int)t);
  }
}

// Idx: uint32_t when every adjacency offset fits (32-bit offsets let the loads use a
// scalar base plus a 32-bit vector offset), int64_t otherwise.
//
// Rows are read in aligned quads of entries (16-byte loads of neighbour slots and of
// costs): quad k holds entries 4k .. 4k+3, and the entries of a quad that lie outside
// the row [a, b) are masked (their neighbour is replaced by slot 0 before any
// gather).  The adjacency arrays keep at least three entries of slack past the last
// one, so the last quad of the last row stays inside the allocation.
template <int GW, int Q, typename Idx, bool kBatched>
__global__ void __launch_bounds__(kThreads) k_mark(int32_t n, const int32_t* __restrict__ prob,
                                                  const ProblemState* __restrict__ ps,
                                                  const LoopCtl* __restrict__ ctl, const float* __restrict__ g,
                                                  const float* __restrict__ h, const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col, uint8_t* __restrict__ stamp,
                                                  IterCounters* __restrict__ ctr, const int32_t* __restrict__ tiles) {
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
    const Idx qa = ra >> 2, qb = (rb + 3) >> 2;
    for (Idx k = qa + gl; k < qb; k += GW * Q) {
      int4 w[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) w[q] = col4[k + q * GW < qb ? k + q * GW : qa];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        if (k + q * GW >= qb) continue;
        const Idx j0 = (k + q * GW) * 4;
        const int32_t u[4] = {w[q].x, w[q].y, w[q].z, w[q].w};
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (j0 + e >= ra && j0 + e < rb) stamp[u[e]] = ep;
      }
    }
  }
  flush_counters(ctr, p, v < n && gl == 0, in ? 1 : 0, 0, 0ull, 0);
  }
}

// Compacted Improve domain: the slots stamped with this iteration's epoch.  Each
// thread tests kListPer consecutive stamps (one 16-byte load), a workgroup scan
// places them, and one atomic per workgroup reserves the workgroup's chunk
// (ascending inside the chunk).  When the next mark epoch wraps its low byte, every
// stamp is cleared here after being read.
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
  if (prob) {
    for (uint32_t m = mask; m; m &= m - 1) {
      const int i = __ffs(m) - 1;
      if (!ps[prob[v0 + i]].active) mask &= ~(1u << i);
    }
  }
  // workgroup exclusive scan of the per-thread counts
  __shared__ int wsum[kThreads / kWave];
  __shared__ int base;
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
  }
  __syncthreads();
  int pos = base + wsum[wid] + incl - c;
  while (mask) {
    const int i = __ffs(mask) - 1;
    mask &= mask - 1;
    dlist[pos++] = (int32_t)(v0 + i);
  }
  }
}

// Improve over the compacted domain: group i takes entry i of dlist; workgroups past
// the domain's end leave at once.
// Single graphs mark in two steps.  k_promising_list tests kListPer consecutive
// vertices per thread (16-byte loads of g and h), stamps the promising ones and lists
// them (one atomic per workgroup); k_mark_rows then stamps the neighbours of the
// listed vertices only, so the row work follows |P| rather than n.
__global__ void __launch_bounds__(kThreads) k_promising_list(int32_t n, const ProblemState* __restrict__ ps,
                                                            LoopCtl* __restrict__ ctl, const float* __restrict__ g,
                                                            const float* __restrict__ h,
                                                            uint8_t* __restrict__ stamp, int32_t* __restrict__ plist,
                                                            IterCounters* __restrict__ ctr) {
  if (ctl->any_active == 0) return;  // the problem has converged
  const uint8_t ep = (uint8_t)ctl->epoch;
  const float G = ps[0].thr;
  const int64_t v0 = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * kListPer;
  uint32_t mask = 0;
  if (v0 + kListPer <= n) {
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
  __shared__ int wsum[kThreads / kWave];
  __shared__ int base;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
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
    base = t ? atomicAdd(&ctl->npromising, t) : 0;
    if (t) atomicAdd(&ctr[blockIdx.x % kCounterSlots].nP, t);
  }
  __syncthreads();
  int pos = base + wsum[wid] + incl - c;
  while (mask) {
    const int i = __ffs(mask) - 1;
    mask &= mask - 1;
    stamp[v0 + i] = ep;
    plist[pos++] = (int32_t)(v0 + i);
  }
}


template <int GW, int Q, typename Idx, bool kBatched>
__global__ void __launch_bounds__(kThreads) k_improve(int32_t n, const int32_t* __restrict__ prob,
                                                     const ProblemState* __restrict__ ps,
                                                     const LoopCtl* __restrict__ ctl, const float* __restrict__ g,
                                                     const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                     const float* __restrict__ cst, const int32_t* __restrict__ dlist,
                                                     const int32_t* __restrict__ ext_of,
                                                     int32_t* __restrict__ parent, float* __restrict__ pcost,
                                                     IterCounters* __restrict__ ctr) {
  if (ctl->any_active == 0) return;  // every problem has converged
  const int64_t cnt = ctl->ndomain;
  // a batch strides over the domain with a fixed grid; a single graph's grid covers it
  const int64_t step = kBatched ? (int64_t)gridDim.x * (kThreads / GW) : cnt;
  for (int64_t first = (int64_t)blockIdx.x * (kThreads / GW); first < cnt; first += step) {
  const int lane = threadIdx.x & (kWave - 1);
  const int grp = lane / GW, gl = threadIdx.x % GW;
  const int64_t gi = first + threadIdx.x / GW;
  const bool valid = gi < cnt;
  const int32_t x = dlist[valid ? gi : cnt - 1];
  const int p = kBatched ? prob[x] : 0;
  const float gx = g[x];
  const Idx ra = (Idx)rp[x], rb = (Idx)rp[x + 1];
  const bool in = valid && x != ps[p].root;
  const Idx a = in ? ra : 0, b = in ? rb : 0;
  const int4* col4 = reinterpret_cast<const int4*>(col);
  const float4* cst4 = reinterpret_cast<const float4*>(cst);
  // lane-local minimum of (g(u) + c, caller id of u, c); bu = slot of u
  uint32_t bv = 0xffffffffu, bc = 0xffffffffu;
  int32_t bu = -1;
  const Idx qa = a >> 2, qb = (b + 3) >> 2;
  for (Idx k = qa + gl; k < qb; k += GW * Q) {
    int4 w[Q];
    float4 cw[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const Idx kk = k + q * GW < qb ? k + q * GW : qa;
      w[q] = col4[kk];
      cw[q] = cst4[kk];
    }
    int32_t u[4 * Q];
    float c[4 * Q];
    bool ok[4 * Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const Idx j0 = (k + q * GW) * 4;
      const bool live = k + q * GW < qb;
      const int32_t uu[4] = {w[q].x, w[q].y, w[q].z, w[q].w};
      const float cc[4] = {cw[q].x, cw[q].y, cw[q].z, cw[q].w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        ok[4 * q + e] = live && j0 + e >= a && j0 + e < b;
        u[4 * q + e] = ok[4 * q + e] ? uu[e] : 0;
        c[4 * q + e] = cc[e];
      }
    }
    float gu[4 * Q];
#pragma unroll
    for (int i = 0; i < 4 * Q; ++i) gu[i] = g[u[i]];
#pragma unroll
    for (int i = 0; i < 4 * Q; ++i) {
      if (!ok[i]) continue;
      const uint32_t vb = __float_as_uint(add_rn(gu[i], c[i])), cb = __float_as_uint(c[i]);
      if (vb >= 0x7f800000u) continue;  // +inf never improves anything
      if (vb < bv) {
        bv = vb;
        bu = u[i];
        bc = cb;
      } else if (vb == bv) {  // equal candidates within one lane: rare
        const int32_t e1 = ext_of[u[i]], e0 = ext_of[bu];
        if (e1 < e0 || (e1 == e0 && cb < bc)) {
          bu = u[i];
          bc = cb;
        }
      }
    }
  }
  // group minimum: value first; the caller id is fetched only for real ties
  const uint32_t mv = dpp_group_min_u32<GW>(bv);
  const bool tied = bu >= 0 && bv == mv;
  const unsigned long long tb = group_bits<GW>(__ballot(tied), grp);
  const bool multi = __popcll(tb) > 1;
  const uint32_t e = tied ? (multi ? (uint32_t)ext_of[bu] : 0u) : 0xffffffffu;
  const unsigned long long k2 = ((unsigned long long)e << 32) | (tied ? bc : 0xffffffffu);
  const unsigned long long m2 = dpp_group_min_u64<GW>(k2);
  const unsigned long long wb = group_bits<GW>(__ballot(tied && k2 == m2), grp);
  const int src = grp * GW + (wb ? __ffsll((long long)wb) - 1 : 0);
  const int32_t wu = __shfl(bu, src, kWave);
  const uint32_t wc = __shfl(bc, src, kWave);
  int changed = 0;
  if (in && gl == 0 && wb != 0 && __uint_as_float(mv) < gx) {
    parent[x] = wu;
    pcost[x] = __uint_as_float(wc);
    changed = 1;
  }
  flush_counters(ctr, p, valid && gl == 0, 0, in ? 1 : 0, in ? (unsigned long long)(b - a) : 0ull, changed);
  }
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

template <int GW, int Q, typename Idx>
__global__ void __launch_bounds__(kThreads) k_mark_rows(const LoopCtl* __restrict__ ctl,
                                                       const int32_t* __restrict__ plist,
                                                       const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                       uint8_t* __restrict__ stamp) {
  constexpr int kSlots = tab_slots<GW>();
  __shared__ int32_t keys[kSlots];
  if (ctl->any_active == 0) return;
  const int64_t cnt = ctl->npromising;
  const int64_t first = (int64_t)blockIdx.x * (kThreads / GW);
  if (first >= cnt) return;  // the whole workgroup
  const uint8_t ep = (uint8_t)ctl->epoch;
  const int gl = threadIdx.x % GW;
  const int64_t gi = first + threadIdx.x / GW;
  const bool valid = gi < cnt;
  const int32_t x = plist[valid ? gi : cnt - 1];
  const Idx ra = valid ? (Idx)rp[x] : 0, rb = valid ? (Idx)rp[x + 1] : 0;
  const int4* col4 = reinterpret_cast<const int4*>(col);
  const Idx qa = ra >> 2, qb = (rb + 3) >> 2;
  Idx k = qa + gl;
  for (;;) {
    for (int i = threadIdx.x; i < kSlots; i += kThreads) keys[i] = kTabEmpty;
    if (!__syncthreads_or(k < qb)) break;  // also: the clears are done
    int32_t u[4 * Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int4 w = col4[k + q * GW < qb ? k + q * GW : qa];
      const Idx j0 = (k + q * GW) * 4;
      const bool live = k + q * GW < qb;
      const int32_t uu[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) u[4 * q + e] = live && j0 + e >= ra && j0 + e < rb ? uu[e] : -1;
    }
#pragma unroll
    for (int i = 0; i < 4 * Q; ++i)
      if (u[i] >= 0) keys[tab_pos(u[i]) & (kSlots - 1)] = u[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4 * Q; ++i)
      if (u[i] >= 0 && keys[tab_pos(u[i]) & (kSlots - 1)] != u[i]) stamp[u[i]] = ep;
    for (int i = threadIdx.x; i < kSlots; i += kThreads) {
      const int32_t y = keys[i];
      if (y != kTabEmpty) stamp[y] = ep;
    }
    k += GW * Q;
    __syncthreads();  // every read of the table is done before it is cleared
  }
}

inline dim3 grid_for(int64_t n, int gw) {
  const int64_t b = ((int64_t)n * gw + kThreads - 1) / kThreads;
  return dim3((unsigned)(b > 0 ? b : 1));
}

// Batches use a fixed grid that strides over the live work.
inline dim3 batch_grid(int64_t n, int per_block) {
  const int64_t T = (n + kTileSlots - 1) / kTileSlots;
  const int64_t units = T * (kTileSlots / per_block);
  return dim3((unsigned)(units < kBatchBlocks ? (units > 0 ? units : 1) : kBatchBlocks));
}

template <int GW, int U, bool B>
void launch_mark_t(const StepArgs& a, hipStream_t s) {
  if (!B) {  // single graph: promising list, then the rows of the listed vertices
    const int64_t per_block = (int64_t)kThreads * kListPer;
    hipLaunchKernelGGL(k_promising_list, dim3((unsigned)((a.n + per_block - 1) / per_block)), dim3(kThreads), 0, s,
                       a.n, a.ps, a.ctl, a.g, a.h, a.stamp, a.plist, a.ctr);
    if (a.nnz < ((int64_t)1 << 32) - 64 * GW)
      hipLaunchKernelGGL((k_mark_rows<GW, U, uint32_t>), grid_for(a.n, GW), dim3(kThreads), 0, s, a.ctl, a.plist,
                         a.rp, a.col, a.stamp);
    else
      hipLaunchKernelGGL((k_mark_rows<GW, U, int64_t>), grid_for(a.n, GW), dim3(kThreads), 0, s, a.ctl, a.plist, a.rp,
                         a.col, a.stamp);
    return;
  }
  const dim3 grid = batch_grid(a.n, kThreads / GW);
  if (a.nnz < ((int64_t)1 << 32) - 64 * GW)
    hipLaunchKernelGGL((k_mark<GW, U, uint32_t, B>), grid, dim3(kThreads), 0, s, a.n, a.prob, a.ps, a.ctl, a.g, a.h,
                       a.rp, a.col, a.stamp, a.ctr, a.tiles);
  else
    hipLaunchKernelGGL((k_mark<GW, U, int64_t, B>), grid, dim3(kThreads), 0, s, a.n, a.prob, a.ps, a.ctl, a.g, a.h,
                       a.rp, a.col, a.stamp, a.ctr, a.tiles);
}

template <int GW, int U, bool B>
void launch_improve_t(const StepArgs& a, hipStream_t s) {
  const dim3 grid = B ? batch_grid(a.n, kThreads / GW) : grid_for(a.n, GW);
  if (a.nnz < ((int64_t)1 << 32) - 64 * GW)
    hipLaunchKernelGGL((k_improve<GW, U, uint32_t, B>), grid, dim3(kThreads), 0, s, a.n, a.prob, a.ps, a.ctl, a.g,
                       a.rp, a.col, a.cst, a.dlist, a.ext_of, a.parent, a.pcost, a.ctr);
  else
    hipLaunchKernelGGL((k_improve<GW, U, int64_t, B>), grid, dim3(kThreads), 0, s, a.n, a.prob, a.ps, a.ctl, a.g,
                       a.rp, a.col, a.cst, a.dlist, a.ext_of, a.parent, a.pcost, a.ctr);
}

template <int GW, int U>
void launch_mark_b(const StepArgs& a, hipStream_t s) {
  if (a.prob) launch_mark_t<GW, U, true>(a, s); else launch_mark_t<GW, U, false>(a, s);
}

template <int GW, int U>
void launch_improve_b(const StepArgs& a, hipStream_t s) {
  if (a.prob) launch_improve_t<GW, U, true>(a, s); else launch_improve_t<GW, U, false>(a, s);
}

}  // namespace

void launch_domain_list(const StepArgs& a, hipStream_t s) {
  const int64_t per_block = (int64_t)kThreads * kListPer;
  static_assert(kThreads * kListPer == kTileSlots, "one domain-list workgroup per tile");
  const dim3 grid = a.prob ? batch_grid(a.n, (int)per_block) : dim3((unsigned)((a.n + per_block - 1) / per_block));
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

void launch_improve(const StepArgs& a, int variant, hipStream_t s) {
  switch (variant) {
    case 0: launch_improve_b<16, 1>(a, s); break;
    case 1: launch_improve_b<8, 2>(a, s); break;
    case 2: launch_improve_b<4, 4>(a, s); break;
    default: launch_improve_b<8, 1>(a, s); break;
  }
}

}  // namespace pirrt
