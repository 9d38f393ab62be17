// Vertex storage order.
//
// The library keeps every per-vertex array and the adjacency in an internal
// order ("slots") and translates at the ABI: ext_of[slot] is the caller's vertex
// id, slot_of[id] its slot.  Results never depend on the order: every minimum
// breaks ties on the caller's ids, and Evaluate's sums do not depend on where a
// vertex is stored.
//
// Why: Improve gathers g of every neighbour of every domain vertex.  With ids in
// sampling order the neighbours of a vertex are scattered over the whole g array
// and nearly every 4-byte gather costs a cache line from the MALL or HBM.  After a
// breadth-first renumbering of the graph from x_init, neighbours sit a few BFS
// levels apart, so the rows of consecutive slots gather from a window of g that
// stays in the XCD's L2; the policy tree (close to a shortest-path tree) inherits
// the same locality, which helps Evaluate and the promising-set marks too.
//
// New vertices are appended after the existing slots; the whole graph is
// renumbered again when it has grown enough since the last renumbering.
#include "internal.h"

namespace pirrt {

namespace {

constexpr int kThreads = 256;

inline unsigned blocks_for(int64_t n, int per_block = kThreads) {
  int64_t b = (n + per_block - 1) / per_block;
  return (unsigned)(b > 0 ? b : 1);
}

__global__ void __launch_bounds__(kThreads) k_identity_ids(int64_t lo, int64_t hi, int32_t* __restrict__ ext_of,
                                                          int32_t* __restrict__ slot_of, int32_t* __restrict__ prob,
                                                          int32_t problem) {
  int64_t s = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= hi) return;
  ext_of[s] = (int32_t)s;
  slot_of[s] = (int32_t)s;
  if (prob) prob[s] = problem;
}

__global__ void __launch_bounds__(kThreads) k_fill_i32(int64_t lo, int64_t hi, int32_t value, int32_t* __restrict__ a) {
  int64_t s = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < hi) a[s] = value;
}

// prob[s] = the problem whose slot range [base[p], base[p + 1]) holds s.
__global__ void __launch_bounds__(kThreads) k_problem_map(int64_t n, int32_t P, const int64_t* __restrict__ base,
                                                         int32_t* __restrict__ prob) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  int32_t lo = 0, hi = P - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (base[mid] <= s) lo = mid; else hi = mid - 1;
  }
  prob[s] = lo;
}

// parent[slot_of[id]] = -1 for the given caller ids whose parent carries the root
// mark (the roots of an earlier Replan).
__global__ void __launch_bounds__(kThreads) k_unmark_roots(int32_t m, const int32_t* __restrict__ ids,
                                                          const int32_t* __restrict__ slot_of,
                                                          int32_t* __restrict__ parent) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int32_t s = slot_of[ids[i]];
  if (parent[s] == kRootMark) parent[s] = -1;
}

__global__ void __launch_bounds__(kThreads) k_translate(int64_t m, const int32_t* __restrict__ ids,
                                                       const int32_t* __restrict__ slot_of,
                                                       int32_t* __restrict__ out) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) out[j] = slot_of[ids[j]];
}

// Sources of the renumbering BFS: problem i starts at slot roots[i] and fills
// order[base_i ..] of its own slot range (problems occupy contiguous ranges).
__global__ void k_bfs_init(int32_t P, const int32_t* __restrict__ roots, const int64_t* __restrict__ base,
                           int32_t* __restrict__ order, int32_t* __restrict__ visited, int32_t* __restrict__ pcnt,
                           int32_t* __restrict__ frontier, int32_t* __restrict__ fcount) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *fcount = P;
  if (i >= P) return;
  const int32_t r = roots[i];
  order[base[i]] = r;
  visited[r] = 1;
  pcnt[i] = (int32_t)base[i] + 1;
  frontier[i] = r;
}

// One breadth-first level, in the order a sequential queue would produce: the
// vertices a level reaches are grouped by the frontier index of their first
// discoverer (the lowest frontier index among their neighbours), in frontier order.
// Children of one parent thus sit together and next to their parent's siblings'
// children, which keeps a vertex's neighbours in few cache lines of g.
//
// discover: every frontier vertex offers its index to each unvisited neighbour
//           (atomicMin on key); the first offer also lists the neighbour.  A
//           neighbour reached in this level is tagged `tag` (not 0), so later offers
//           of the same level still reach the minimum.
__global__ void __launch_bounds__(kThreads) k_bfs_discover(int32_t fsize, const int32_t* __restrict__ frontier,
                                                          int32_t tag, const int64_t* __restrict__ rp,
                                                          const int32_t* __restrict__ col,
                                                          int32_t* __restrict__ visited, int32_t* __restrict__ key,
                                                          int32_t* __restrict__ cand, int32_t* __restrict__ ccount) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= fsize) return;
  const int32_t u = frontier[t];
  for (int64_t j = rp[u]; j < rp[u + 1]; ++j) {
    const int32_t w = col[j];
    const int32_t st = visited[w];
    if (st != 0 && st != tag) continue;
    atomicMin(&key[w], (int32_t)t);
    if (st == 0 && atomicCAS(&visited[w], 0, tag) == 0) cand[atomicAdd(ccount, 1)] = w;
  }
}

// hist[key]++ over the reached vertices.
__global__ void __launch_bounds__(kThreads) k_bfs_hist(int32_t m, const int32_t* __restrict__ cand,
                                                      const int32_t* __restrict__ key, int32_t* __restrict__ hist) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) atomicAdd(&hist[key[cand[i]]], 1);
}

// next[off[key] + k]: the reached vertices grouped by discoverer (the order inside a
// group is arbitrary).
__global__ void __launch_bounds__(kThreads) k_bfs_scatter(int32_t m, const int32_t* __restrict__ cand,
                                                         const int32_t* __restrict__ key,
                                                         const int64_t* __restrict__ off,
                                                         int32_t* __restrict__ cursor, int32_t* __restrict__ next) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int32_t w = cand[i], t = key[w];
  next[off[t] + atomicAdd(&cursor[t], 1)] = w;
}

// The level is grouped by problem in problem order (frontiers are); pstart[p] = the
// first index of problem p in next.
__global__ void __launch_bounds__(kThreads) k_bfs_starts(int32_t m, const int32_t* __restrict__ next,
                                                        const int32_t* __restrict__ prob,
                                                        int32_t* __restrict__ pstart) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int32_t p = prob ? prob[next[i]] : 0;
  if (i == 0 || (prob ? prob[next[i - 1]] : 0) != p) pstart[p] = (int32_t)i;
}

// order positions: problem p's part of the level follows its earlier levels.
__global__ void __launch_bounds__(kThreads) k_bfs_place(int32_t m, const int32_t* __restrict__ next,
                                                       const int32_t* __restrict__ prob,
                                                       const int32_t* __restrict__ pstart,
                                                       const int32_t* __restrict__ pcnt, int32_t* __restrict__ order) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int32_t w = next[i];
  const int32_t p = prob ? prob[w] : 0;
  order[pcnt[p] + ((int32_t)i - pstart[p])] = w;
}

// pcnt[p] += size of problem p's part (written by the part's last element).
__global__ void __launch_bounds__(kThreads) k_bfs_advance(int32_t m, const int32_t* __restrict__ next,
                                                         const int32_t* __restrict__ prob,
                                                         const int32_t* __restrict__ pstart,
                                                         int32_t* __restrict__ pcnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int32_t p = prob ? prob[next[i]] : 0;
  if (i == m - 1 || (prob ? prob[next[i + 1]] : 0) != p) pcnt[p] += (int32_t)i - pstart[p] + 1;
}

// Clustered order (optional): a maximal independent set of "seeds" by Luby's rounds
// on hashed priorities, every other vertex joins its highest-priority neighbouring
// seed, and clusters follow their seed's breadth-first rank.  Vertices of one cluster
// are within one hop of a common seed, so a wave's rows share more lines of g.
__device__ __forceinline__ uint32_t mis_prio(uint32_t v) {  // a bijection of 32-bit values
  v ^= v >> 16;
  v *= 0x85ebca6bu;
  v ^= v >> 13;
  v *= 0xc2b2ae35u;
  v ^= v >> 16;
  return v;
}

// state: 0 undecided, 1 seed, 2 covered.  win[v] = 1 if v beats every undecided
// neighbour this round.
__global__ void __launch_bounds__(kThreads) k_mis_select(int32_t n, const int64_t* __restrict__ rp,
                                                        const int32_t* __restrict__ col,
                                                        const int32_t* __restrict__ state, int32_t* __restrict__ win) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int32_t w = 0;
  if (state[v] == 0) {
    w = 1;
    const uint32_t pv = mis_prio((uint32_t)v);
    for (int64_t j = rp[v]; j < rp[v + 1]; ++j) {
      const int32_t u = col[j];
      if (u != v && state[u] == 0 && mis_prio((uint32_t)u) > pv) {
        w = 0;
        break;
      }
    }
  }
  win[v] = w;
}

__global__ void __launch_bounds__(kThreads) k_mis_apply(int32_t n, const int64_t* __restrict__ rp,
                                                       const int32_t* __restrict__ col,
                                                       const int32_t* __restrict__ win, int32_t* __restrict__ state,
                                                       int32_t* __restrict__ undecided) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || state[v] != 0) return;
  if (win[v]) {
    state[v] = 1;
    return;
  }
  for (int64_t j = rp[v]; j < rp[v + 1]; ++j) {
    const int32_t u = col[j];
    if (win[u] || state[u] == 1) {  // old seeds are stable; this round's come through win
      state[v] = 2;
      return;
    }
  }
  atomicAdd(undecided, 1);
}

// key[v] = breadth-first rank of v's cluster seed; hist[key]++.
__global__ void __launch_bounds__(kThreads) k_mis_key(int32_t n, const int64_t* __restrict__ rp,
                                                     const int32_t* __restrict__ col,
                                                     const int32_t* __restrict__ state,
                                                     const int32_t* __restrict__ rank, int32_t* __restrict__ key,
                                                     int32_t* __restrict__ hist) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int32_t seed = (int32_t)v;
  if (state[v] != 1) {
    uint32_t best = 0;
    bool found = false;
    for (int64_t j = rp[v]; j < rp[v + 1]; ++j) {
      const int32_t u = col[j];
      if (state[u] != 1) continue;
      const uint32_t pu = mis_prio((uint32_t)u);
      if (!found || pu > best) {
        best = pu;
        seed = u;
        found = true;
      }
    }
  }
  const int32_t k = rank[seed];
  key[v] = k;
  atomicAdd(&hist[k], 1);
}

__global__ void __launch_bounds__(kThreads) k_mis_scatter(int32_t n, const int32_t* __restrict__ order,
                                                         const int32_t* __restrict__ key,
                                                         const int64_t* __restrict__ off,
                                                         int32_t* __restrict__ cursor, int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t v = order[i];  // breadth-first order: members keep roughly that order
  const int32_t k = key[v];
  out[off[k] + atomicAdd(&cursor[k], 1)] = v;
}

__global__ void __launch_bounds__(kThreads) k_rank_of(int32_t n, const int32_t* __restrict__ order,
                                                     int32_t* __restrict__ rank) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) rank[order[i]] = (int32_t)i;
}

// Vertices the BFS did not reach follow in their problem's range.
__global__ void __launch_bounds__(kThreads) k_append_unvisited(int32_t n, const int32_t* __restrict__ visited,
                                                              int32_t* __restrict__ order,
                                                              const int32_t* __restrict__ prob,
                                                              int32_t* __restrict__ pcnt) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n && visited[s] == 0) order[atomicAdd(&pcnt[prob ? prob[s] : 0], 1)] = (int32_t)s;
}

__global__ void __launch_bounds__(kThreads) k_invert(int32_t n, const int32_t* __restrict__ order,
                                                    int32_t* __restrict__ newslot, const int64_t* __restrict__ rp,
                                                    int32_t* __restrict__ deg) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int32_t o = order[k];
  newslot[o] = (int32_t)k;
  deg[k] = (int32_t)(rp[o + 1] - rp[o]);
}

// Row k of the new adjacency is old row order[k] with its neighbours renamed and
// sorted by their new slot (ties, i.e. parallel edges, keep their order), so the
// entries that Improve reads together gather g from nearby slots.  One wave per row:
// the row's keys go to LDS and every entry moves to its rank.  Rows longer than
// kSortCap keep their order.
constexpr int kSortCap = 512;

__global__ void __launch_bounds__(kThreads) k_permute_rows(int32_t n, const int32_t* __restrict__ order,
                                                          const int32_t* __restrict__ newslot,
                                                          const int64_t* __restrict__ rp,
                                                          const int32_t* __restrict__ col,
                                                          const float* __restrict__ cst,
                                                          const int64_t* __restrict__ rp_new,
                                                          int32_t* __restrict__ col_new, float* __restrict__ cst_new) {
  __shared__ int32_t skey[kThreads / kWave][kSortCap];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (k >= n) return;
  const int32_t o = order[k];
  const int64_t a = rp[o], b = rp[o + 1], dst = rp_new[k];
  const int64_t len = b - a;
  if (len > kSortCap) {
    for (int64_t j = a + lane; j < b; j += kWave) {
      col_new[dst + (j - a)] = newslot[col[j]];
      cst_new[dst + (j - a)] = cst[j];
    }
    return;
  }
  const int m = (int)len;
  for (int j = lane; j < m; j += kWave) skey[w][j] = newslot[col[a + j]];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  for (int j = lane; j < m; j += kWave) {
    const int32_t key = skey[w][j];
    int rank = 0;
    for (int i = 0; i < m; ++i) {
      const int32_t ki = skey[w][i];
      rank += (ki < key || (ki == key && i < j)) ? 1 : 0;
    }
    col_new[dst + rank] = key;
    cst_new[dst + rank] = cst[a + j];
  }
}

__global__ void __launch_bounds__(kThreads) k_permute_vertices(int32_t n, const int32_t* __restrict__ order,
                                                              const int32_t* __restrict__ newslot,
                                                              const float* __restrict__ g,
                                                              const int32_t* __restrict__ parent,
                                                              const float* __restrict__ pcost,
                                                              const int32_t* __restrict__ ext_of,
                                                              float* __restrict__ g2, int32_t* __restrict__ parent2,
                                                              float* __restrict__ pcost2, int32_t* __restrict__ ext2,
                                                              int32_t* __restrict__ slot_of) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int32_t o = order[k];
  g2[k] = g[o];
  const int32_t p = parent[o];
  parent2[k] = p >= 0 ? newslot[p] : p;  // -1 and the root mark stay
  pcost2[k] = pcost[o];
  const int32_t e = ext_of[o];
  ext2[k] = e;
  slot_of[e] = (int32_t)k;
}

__global__ void __launch_bounds__(kThreads) k_gather_by_slot(int32_t n, const int32_t* __restrict__ ext_of,
                                                            const float* __restrict__ src_ext,
                                                            float* __restrict__ dst_slot) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) dst_slot[s] = src_ext[ext_of[s]];
}

__global__ void __launch_bounds__(kThreads) k_policy_to_ext(int32_t n, const int32_t* __restrict__ slot_of,
                                                           const int32_t* __restrict__ ext_of,
                                                           const int32_t* __restrict__ prob,
                                                           const int64_t* __restrict__ base,
                                                           const float* __restrict__ g,
                                                           const int32_t* __restrict__ parent,
                                                           const float* __restrict__ pcost, float* __restrict__ g_ext,
                                                           int32_t* __restrict__ parent_ext,
                                                           float* __restrict__ pcost_ext) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int32_t s = slot_of[e];
  if (g_ext) g_ext[e] = g[s];
  if (parent_ext) {
    const int32_t p = parent[s];
    parent_ext[e] = p >= 0 ? (int32_t)(ext_of[p] - (prob ? base[prob[s]] : 0)) : -1;
  }
  if (pcost_ext) pcost_ext[e] = pcost[s];
}

__global__ void __launch_bounds__(kThreads) k_policy_from_ext(int32_t n, const int32_t* __restrict__ slot_of,
                                                             const int32_t* __restrict__ prob,
                                                             const int64_t* __restrict__ base,
                                                             const float* __restrict__ g_ext,
                                                             const int32_t* __restrict__ parent_ext,
                                                             const float* __restrict__ pcost_ext,
                                                             float* __restrict__ g, int32_t* __restrict__ parent,
                                                             float* __restrict__ pcost) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int32_t s = slot_of[e];
  g[s] = g_ext[e];
  const int32_t p = parent_ext[e];
  parent[s] = p >= 0 ? slot_of[p + (prob ? base[prob[s]] : 0)] : -1;
  pcost[s] = pcost_ext[e];
}

}  // namespace

void launch_identity_ids(int64_t lo, int64_t hi, int32_t* ext_of, int32_t* slot_of, hipStream_t s, int32_t* prob,
                         int32_t problem) {
  if (hi > lo)
    hipLaunchKernelGGL(k_identity_ids, dim3(blocks_for(hi - lo)), dim3(kThreads), 0, s, lo, hi, ext_of, slot_of, prob,
                       problem);
}

void launch_translate(int64_t m, const int32_t* ids, const int32_t* slot_of, int32_t* out, hipStream_t s) {
  if (m > 0) hipLaunchKernelGGL(k_translate, dim3(blocks_for(m)), dim3(kThreads), 0, s, m, ids, slot_of, out);
}

void launch_fill_i32(int64_t lo, int64_t hi, int32_t value, int32_t* a, hipStream_t s) {
  if (hi > lo) hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(hi - lo)), dim3(kThreads), 0, s, lo, hi, value, a);
}

void launch_problem_map(int64_t n, int32_t P, const int64_t* base, int32_t* prob, hipStream_t s) {
  if (n > 0 && P > 0) hipLaunchKernelGGL(k_problem_map, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, P, base, prob);
}

void launch_unmark_roots(int32_t m, const int32_t* ids, const int32_t* slot_of, int32_t* parent, hipStream_t s) {
  if (m > 0) hipLaunchKernelGGL(k_unmark_roots, dim3(blocks_for(m)), dim3(kThreads), 0, s, m, ids, slot_of, parent);
}

void launch_bfs_init(int32_t P, const int32_t* roots, const int64_t* base, int32_t* order, int32_t* visited,
                     int32_t* pcnt, int32_t* frontier, int32_t* fcount, hipStream_t s) {
  hipLaunchKernelGGL(k_bfs_init, dim3(blocks_for(P)), dim3(kThreads), 0, s, P, roots, base, order, visited, pcnt,
                     frontier, fcount);
}

void launch_bfs_discover(int32_t fsize, const int32_t* frontier, int32_t tag, const int64_t* rp, const int32_t* col,
                         int32_t* visited, int32_t* key, int32_t* cand, int32_t* ccount, hipStream_t s) {
  if (fsize > 0)
    hipLaunchKernelGGL(k_bfs_discover, dim3(blocks_for(fsize)), dim3(kThreads), 0, s, fsize, frontier, tag, rp, col,
                       visited, key, cand, ccount);
}

void launch_bfs_order_level(int32_t fsize, int32_t m, const int32_t* cand, const int32_t* key, int32_t* hist,
                            int64_t* off, int32_t* cursor, int32_t* next, const int32_t* prob, int32_t* pstart,
                            int32_t* pcnt, int32_t* order, void* scan_scratch, hipStream_t s) {
  if (m <= 0) return;
  hipMemsetAsync(hist, 0, sizeof(int32_t) * (size_t)fsize, s);
  hipMemsetAsync(cursor, 0, sizeof(int32_t) * (size_t)fsize, s);
  hipLaunchKernelGGL(k_bfs_hist, dim3(blocks_for(m)), dim3(kThreads), 0, s, m, cand, key, hist);
  scan_i32_to_i64(hist, fsize, off, scan_scratch, s);
  hipLaunchKernelGGL(k_bfs_scatter, dim3(blocks_for(m)), dim3(kThreads), 0, s, m, cand, key, off, cursor, next);
  hipLaunchKernelGGL(k_bfs_starts, dim3(blocks_for(m)), dim3(kThreads), 0, s, m, next, prob, pstart);
  hipLaunchKernelGGL(k_bfs_place, dim3(blocks_for(m)), dim3(kThreads), 0, s, m, next, prob, pstart, pcnt, order);
  hipLaunchKernelGGL(k_bfs_advance, dim3(blocks_for(m)), dim3(kThreads), 0, s, m, next, prob, pstart, pcnt);
}

void launch_mis_round(int32_t n, const int64_t* rp, const int32_t* col, int32_t* state, int32_t* win,
                      int32_t* undecided, hipStream_t s) {
  hipLaunchKernelGGL(k_mis_select, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, rp, col, state, win);
  hipLaunchKernelGGL(k_mis_apply, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, rp, col, win, state, undecided);
}

void launch_cluster_order(int32_t n, const int64_t* rp, const int32_t* col, const int32_t* state, const int32_t* order,
                          int32_t* rank, int32_t* key, int32_t* hist, int64_t* off, int32_t* cursor, int32_t* out,
                          void* scan_scratch, hipStream_t s) {
  hipLaunchKernelGGL(k_rank_of, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, order, rank);
  hipMemsetAsync(hist, 0, sizeof(int32_t) * (size_t)n, s);
  hipMemsetAsync(cursor, 0, sizeof(int32_t) * (size_t)n, s);
  hipLaunchKernelGGL(k_mis_key, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, rp, col, state, rank, key, hist);
  scan_i32_to_i64(hist, n, off, scan_scratch, s);
  hipLaunchKernelGGL(k_mis_scatter, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, order, key, off, cursor, out);
}

void launch_append_unvisited(int32_t n, const int32_t* visited, int32_t* order, const int32_t* prob, int32_t* pcnt,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_append_unvisited, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, visited, order, prob, pcnt);
}

void launch_permute(const PermuteArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_invert, dim3(blocks_for(a.n)), dim3(kThreads), 0, s, a.n, a.order, a.newslot, a.rp, a.deg);
  scan_i32_to_i64(a.deg, a.n, a.rp_new, a.scan_scratch, s);
  hipLaunchKernelGGL(k_permute_rows, dim3(blocks_for((int64_t)a.n * kWave)), dim3(kThreads), 0, s, a.n, a.order,
                     a.newslot, a.rp, a.col, a.cst, a.rp_new, a.col_new, a.cst_new);
  hipLaunchKernelGGL(k_permute_vertices, dim3(blocks_for(a.n)), dim3(kThreads), 0, s, a.n, a.order, a.newslot, a.g,
                     a.parent, a.pcost, a.ext_of, a.g2, a.parent2, a.pcost2, a.ext2, a.slot_of);
}

void launch_gather_by_slot(int32_t n, const int32_t* ext_of, const float* src_ext, float* dst_slot, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_by_slot, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, ext_of, src_ext, dst_slot);
}

void launch_policy_to_ext(int32_t n, const int32_t* slot_of, const int32_t* ext_of, const int32_t* prob,
                          const int64_t* base, const float* g, const int32_t* parent, const float* pcost,
                          float* g_ext, int32_t* parent_ext, float* pcost_ext, hipStream_t s) {
  hipLaunchKernelGGL(k_policy_to_ext, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, slot_of, ext_of, prob, base, g,
                     parent, pcost, g_ext, parent_ext, pcost_ext);
}

void launch_policy_from_ext(int32_t n, const int32_t* slot_of, const int32_t* prob, const int64_t* base,
                            const float* g_ext, const int32_t* parent_ext, const float* pcost_ext, float* g,
                            int32_t* parent, float* pcost, hipStream_t s) {
  hipLaunchKernelGGL(k_policy_from_ext, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, slot_of, prob, base, g_ext,
                     parent_ext, pcost_ext, g, parent, pcost);
}

}  // namespace pirrt
