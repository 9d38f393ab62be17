// Replan of one small graph in a single workgroup (Alg. 2; Sec. IV-B, IV-C).
//
// At a thousand vertices every kernel of the multi-kernel loop is a short launch, and
// a Replan costs about 35 µs per iteration, mostly in launches.  Here one workgroup
// of 1024 threads runs the whole loop, with the per-vertex state (g,
// parent, parent-edge cost, the evaluated flags, the domain marks and list) in LDS and the adjacency read from global memory, so an iteration costs a
// handful of barriers.  It computes what the multi-kernel loop computes, step for
// step:
//
//   Evaluate : g(v) = g(parent) + pcost(v), one binary32 addition each, from the root
//              down; vertices off the root's tree get +inf.  In rounds: each thread
//              walks from a vertex not yet evaluated up at most kHop parents; if it
//              reaches an evaluated vertex it evaluates the path downwards, if it
//              reaches a missing parent the path is off the tree; otherwise it
//              retries in the next round (after the paths above it are done).
//   mark     : P = { v : g(v) + h(v) < G }, G = g(goal) (or +inf without pruning);
//              D = P and every neighbour of P (with the narrowed domain, only the
//              neighbours w with fl(fl(g(u) + c) + h(w)) < G), minus the root.
//   Improve  : for v in D, the lexicographic minimum of (g(u) + c, caller id of u, c)
//              over v's row; the parent switches when that value is strictly below
//              g(v).  g is only read (Jacobi step).
//   loop     : stop after a pass with no switch; otherwise Evaluate, then stop with
//              the iteration cap.
//
// The counters (iterations, edges examined, |P| and |D| sums, switches) and the cap
// status go to the problem's state as the multi-kernel loop leaves them.
#include "internal.h"

namespace pirrt {

namespace {

constexpr int kSmallThreads = 1024;
constexpr int kHop = 8;      // parents one Evaluate walk climbs per round
constexpr int kRowChunk = 8;  // row entries loaded together

// Exclusive scan of one int per thread over the workgroup; *total gets the sum.
__device__ __forceinline__ int block_exclusive_sum(int x, int* wsum, int* total) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  int incl = x;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int y = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += y;
  }
  if (lane == kWave - 1) wsum[wid] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kSmallThreads / kWave; ++w) {
      const int v = wsum[w];
      wsum[w] = t;
      t += v;
    }
    wsum[kSmallThreads / kWave] = t;
  }
  __syncthreads();
  const int out = wsum[wid] + incl - x;
  *total = wsum[kSmallThreads / kWave];
  __syncthreads();  // wsum is reused by the next call
  return out;
}

template <bool kLook>
__global__ void __launch_bounds__(kSmallThreads) k_replan_small(int32_t n, const int64_t* __restrict__ rp,
                                                                const int32_t* __restrict__ col,
                                                                const float* __restrict__ cst,
                                                                const float* __restrict__ h,
                                                                const int32_t* __restrict__ ext_of, int prune,
                                                                ProblemState* __restrict__ ps,
                                                                int32_t* __restrict__ parent_io,
                                                                float* __restrict__ pcost_io, float* __restrict__ g_out) {
  __shared__ float g[kSmallMax];
  __shared__ int32_t par[kSmallMax];
  __shared__ float pc[kSmallMax];
  __shared__ int32_t fa[kSmallMax];  // the domain list
  __shared__ uint32_t done[kSmallMax];  // evaluated in the current Evaluate
  __shared__ uint8_t inP[kSmallMax];
  __shared__ uint8_t inD[kSmallMax];
  __shared__ int wsum[kSmallThreads / kWave + 1];
  __shared__ int red_chg;
  __shared__ unsigned long long red_edges;

  const int t = threadIdx.x;
  const int32_t root = ps[0].root, goal = ps[0].goal, cap = ps[0].cap;
  for (int v = t; v < n; v += kSmallThreads) {
    par[v] = v == root ? -1 : parent_io[v];
    pc[v] = v == root ? 0.0f : pcost_io[v];
  }
  __syncthreads();

  // Evaluate in rounds of bounded walks.  A vertex is published evaluated (release)
  // only after its g is written, and a walk reads the flag with acquire before g.
  auto evaluate = [&]() {
    for (int v = t; v < n; v += kSmallThreads) {
      g[v] = v == root ? 0.0f : __int_as_float(0x7f800000);
      done[v] = v == root ? 1u : 0u;
    }
    __syncthreads();
    // every round evaluates at least the vertices whose parent is evaluated, so n
    // rounds suffice unless the pointers hold a cycle, whose vertices stay +inf
    for (int round = 0;; ++round) {
      int pending = 0;
      for (int v = t; v < n; v += kSmallThreads) {
        if (__hip_atomic_load(&done[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) continue;
        int32_t path[kHop];
        path[0] = v;
        int k = 1;
        int32_t u = par[v];
        int state = 0;  // 0 climbing, 1 reached an evaluated vertex, 2 off the tree
#pragma unroll
        for (int s = 0; s < kHop; ++s) {
          if (state == 0) {
            if (u < 0) {
              state = 2;
            } else if (__hip_atomic_load(&done[u], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)) {
              state = 1;
            } else if (s + 1 < kHop) {
              path[s + 1] = u;
              k = s + 2;
              u = par[u];
            }
          }
        }
        if (state == 0) {
          pending = 1;  // longer than kHop: the next round, after the vertices above
          continue;
        }
        float acc = state == 1 ? g[u] : __int_as_float(0x7f800000);
#pragma unroll
        for (int i = kHop - 1; i >= 0; --i) {
          if (i < k) {
            const int32_t x = path[i];
            acc = __fadd_rn(acc, pc[x]);
            g[x] = acc;
            __hip_atomic_store(&done[x], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
          }
        }
      }
      if (!__syncthreads_or(pending) || round >= n) break;
    }
  };

  evaluate();
  int32_t iters = 0;
  unsigned long long edges_sum = 0, p_sum = 0, d_sum = 0, chg_sum = 0, pe_sum = 0;
  int32_t status = 0;
  for (;;) {
    const float G = prune ? g[goal] : __int_as_float(0x7f800000);
    // promising set
    int np = 0;
    for (int v = t; v < n; v += kSmallThreads) {
      const bool p = __fadd_rn(g[v], h ? h[v] : 0.0f) < G;
      inP[v] = p ? 1 : 0;
      inD[v] = p ? 1 : 0;
      np += p ? 1 : 0;
    }
    __syncthreads();
    // their neighbours
    int pe = 0;
    for (int u = t; u < n; u += kSmallThreads) {
      if (!inP[u]) continue;
      const float gu = g[u];
      const int64_t a = rp[u], b = rp[u + 1];
      pe += (int)(b - a);
      for (int64_t j0 = a; j0 < b; j0 += kRowChunk) {
        int32_t w[kRowChunk];
        float c[kRowChunk];
#pragma unroll
        for (int e = 0; e < kRowChunk; ++e) {  // loads first, all in flight together
          const int64_t j = j0 + e < b ? j0 + e : a;
          w[e] = col[j];
          c[e] = kLook ? cst[j] : 0.0f;
        }
#pragma unroll
        for (int e = 0; e < kRowChunk; ++e) {
          if (j0 + e >= b) continue;
          if (kLook && !(__fadd_rn(__fadd_rn(gu, c[e]), h ? h[w[e]] : 0.0f) < G)) continue;
          inD[w[e]] = 1;
        }
      }
    }
    __syncthreads();
    if (t == 0) inD[root] = 0;
    __syncthreads();
    // the domain list (a contiguous block of vertices per thread, ascending)
    int nd_local = 0;
    const int per = (n + kSmallThreads - 1) / kSmallThreads;
    const int lo = t * per, hi = lo + per < n ? lo + per : n;
    for (int v = lo; v < hi; ++v) nd_local += inD[v];
    int nd;
    int pos = block_exclusive_sum(nd_local, wsum, &nd);
    for (int v = lo; v < hi; ++v)
      if (inD[v]) fa[pos++] = v;
    int np_total;
    (void)block_exclusive_sum(np, wsum, &np_total);  // also a barrier after the list
    int pe_total;
    (void)block_exclusive_sum(pe, wsum, &pe_total);
    if (t == 0) {
      red_chg = 0;
      red_edges = 0ull;
    }
    __syncthreads();
    // Improve over the list: one thread per row
    int chg = 0;
    unsigned long long ex = 0;
    for (int i = t; i < nd; i += kSmallThreads) {
      const int32_t x = fa[i];
      const int64_t a = rp[x], b = rp[x + 1];
      ex += (unsigned long long)(b - a);
      uint32_t bv = 0xffffffffu, bc = 0xffffffffu;
      int32_t bu = -1;
      for (int64_t j0 = a; j0 < b; j0 += kRowChunk) {
        int32_t uu[kRowChunk];
        float cc[kRowChunk];
#pragma unroll
        for (int e = 0; e < kRowChunk; ++e) {  // loads first, all in flight together
          const int64_t j = j0 + e < b ? j0 + e : a;
          uu[e] = col[j];
          cc[e] = cst[j];
        }
#pragma unroll
        for (int e = 0; e < kRowChunk; ++e) {
          if (j0 + e >= b) continue;
          const int32_t u = uu[e];
          const float c = cc[e];
          const uint32_t vb = __float_as_uint(__fadd_rn(g[u], c)), cb = __float_as_uint(c);
          if (vb >= 0x7f800000u) continue;  // +inf never improves anything
          if (vb < bv) {
            bv = vb;
            bu = u;
            bc = cb;
          } else if (vb == bv) {
            const int32_t e1 = ext_of[u], e0 = ext_of[bu];
            if (e1 < e0 || (e1 == e0 && cb < bc)) {
              bu = u;
              bc = cb;
            }
          }
        }
      }
      if (bu >= 0 && __uint_as_float(bv) < g[x]) {
        par[x] = bu;
        pc[x] = __uint_as_float(bc);
        ++chg;
      }
    }
    if (chg) atomicAdd(&red_chg, chg);
    if (ex) atomicAdd(&red_edges, ex);
    __syncthreads();
    const int changed = red_chg;
    ++iters;
    edges_sum += red_edges;
    p_sum += (unsigned long long)np_total;
    d_sum += (unsigned long long)nd;
    chg_sum += (unsigned long long)changed;
    pe_sum += (unsigned long long)pe_total;
    __syncthreads();  // every thread has read red_* before the next pass clears them
    if (changed == 0) break;
    evaluate();
    if (iters >= cap) {
      status = 1;
      break;
    }
  }
  // results: the policy and g into global memory, the counters into the state
  for (int v = t; v < n; v += kSmallThreads) {
    g_out[v] = g[v];
    if (v != root) {
      parent_io[v] = par[v];
      pcost_io[v] = pc[v];
    }
  }
  if (t == 0) {
    ProblemState& q = ps[0];
    q.iterations = iters;
    q.status = status;
    q.active = 0;
    q.needs_eval = 0;
    q.edges = edges_sum;
    q.sum_P = p_sum;
    q.sum_D = d_sum;
    q.changed_total = chg_sum;
    q.mark_edges = pe_sum;
  }
}

}  // namespace

void launch_replan_small(int32_t n, const int64_t* rp, const int32_t* col, const float* cst, const float* h,
                         const int32_t* ext_of, bool prune, bool lookahead, ProblemState* ps, int32_t* parent,
                         float* pcost, float* g, hipStream_t s) {
  if (lookahead)
    hipLaunchKernelGGL(k_replan_small<true>, dim3(1), dim3(kSmallThreads), 0, s, n, rp, col, cst, h, ext_of,
                       prune ? 1 : 0, ps, parent, pcost, g);
  else
    hipLaunchKernelGGL(k_replan_small<false>, dim3(1), dim3(kSmallThreads), 0, s, n, rp, col, cst, h, ext_of,
                       prune ? 1 : 0, ps, parent, pcost, g);
}

}  // namespace pirrt
