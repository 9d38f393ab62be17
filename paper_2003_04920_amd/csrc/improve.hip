// Improve (Alg. 2; Sec. IV-B).
//
// For every slot of the compacted domain other than its problem's root: the
// lexicographic minimum of (g(n) + c(n, v), n, c) over v's row, n being the caller's
// vertex id (storage slots may be renumbered); the parent switches only when that
// value is strictly below g(v).  g is only read (Jacobi step), so all rows are
// independent.
//
// Work split: one group of GW lanes per domain entry, Q aligned quads of row entries
// per lane in flight (GW x Q x 4 = 64 entries per pass over a row by default).  Loads
// are issued unconditionally (quads past the end of the row re-read the first one
// and are masked): `vmcnt` is an in-order counter, so a load under a branch would
// make every later load wait for it.  The per-row minimum is a DPP butterfly.
//
// kBatched: several problems share the arrays; prob[slot] names the problem of a
// slot.  Without it every slot belongs to problem 0.
//
// kTrunc (truncated Evaluate, single graphs): g(v) may be stale, and the minimum may
// be v's own parent and cost below it; that leaves the policy as it is and is not
// counted as a switch.
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
//
// Improve runs over the compacted domain: group i takes entry i of dlist; workgroups
// past the domain's end leave at once.
template <int GW, int Q, typename Idx, bool kBatched, bool kTrunc>
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
  if (in && gl == 0 && wb != 0 && __uint_as_float(mv) < gx &&
      (!kTrunc || wu != parent[x] || wc != __float_as_uint(pcost[x]))) {
    parent[x] = wu;
    pcost[x] = __uint_as_float(wc);
    changed = 1;
  }
  if (kBatched)
    rows::flush_counters_wave<false, true, true, true, false>(ctr, p, valid && gl == 0, 0, in ? 1 : 0,
                                                              in ? (unsigned long long)(b - a) : 0ull, changed);
  else
    flush_counters(ctr, p, valid && gl == 0, 0, in ? 1 : 0, in ? (unsigned long long)(b - a) : 0ull, changed);
  }
}

template <int GW, int U, bool B, bool T>
void launch_improve_t(const StepArgs& a, hipStream_t s) {
  const dim3 grid = B ? batch_grid(a.n, kThreads / GW, a.blocks) : grid_for(a.n, GW);
  if (a.nnz < ((int64_t)1 << 32) - 64 * GW)
    hipLaunchKernelGGL((k_improve<GW, U, uint32_t, B, T>), grid, dim3(kThreads), 0, s, a.n, a.prob, a.ps, a.ctl, a.g,
                       a.rp, a.col, a.cst, a.dlist, a.ext_of, a.parent, a.pcost, a.ctr);
  else
    hipLaunchKernelGGL((k_improve<GW, U, int64_t, B, T>), grid, dim3(kThreads), 0, s, a.n, a.prob, a.ps, a.ctl, a.g,
                       a.rp, a.col, a.cst, a.dlist, a.ext_of, a.parent, a.pcost, a.ctr);
}

template <int GW, int U>
void launch_improve_b(const StepArgs& a, hipStream_t s) {
  if (a.prob)
    launch_improve_t<GW, U, true, false>(a, s);
  else if (a.truncated)
    launch_improve_t<GW, U, false, true>(a, s);
  else
    launch_improve_t<GW, U, false, false>(a, s);
}

}  // namespace

void launch_improve(const StepArgs& a, int variant, hipStream_t s) {
  switch (variant) {
    case 0: launch_improve_b<16, 1>(a, s); break;
    case 1: launch_improve_b<8, 2>(a, s); break;
    case 2: launch_improve_b<4, 4>(a, s); break;
    default: launch_improve_b<8, 1>(a, s); break;
  }
}

}  // namespace pirrt
