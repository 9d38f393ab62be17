// Promising set, Improve domain and Improve (Alg. 2; Sec. IV-B, IV-C).
//
// mark    : P = { v : g(v) + h(v) < G } with G = g(goal) (or +inf without
//           pruning).  Every v of P and every neighbour of v is stamped with the
//           iteration's epoch, which makes D = P u N(P) without a clearing pass.
// improve : for every stamped v other than the root, the lexicographic minimum of
//           (g(n) + c(n, v), n, c) over v's row, n being the caller's vertex id
//           (storage slots may be renumbered); the parent switches only when
//           that value is strictly below g(v).  g is only read (Jacobi step), so
//           all rows are independent.
//
// Both kernels give each wave 64 consecutive vertex ids.  A ballot over the 64
// lanes yields the members (of P, resp. D) of the chunk; their rows are then
// streamed by groups of GW lanes (64 / GW rows at a time, U entries per lane in
// flight), so short rows do not leave most of a wave idle.  Rows of consecutive
// members are contiguous in the CSR, which keeps the streaming coalesced.
#include "internal.h"

namespace pirrt {

namespace {

constexpr int kThreads = 256;
constexpr int kWavesPerBlock = kThreads / kWave;

__device__ __forceinline__ unsigned long long lanes_below(int lane) {
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

template <int GW, int U>
__global__ void __launch_bounds__(kThreads) k_mark(int32_t n, int32_t goal, int prune, const float* __restrict__ g,
                                                  const float* __restrict__ h, const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col, uint32_t* __restrict__ stamp,
                                                  uint32_t epoch, IterCounters* __restrict__ ctr) {
  __shared__ int32_t members[kWavesPerBlock][kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const float G = prune ? g[goal] : pos_inf();
  const int64_t v = ((int64_t)blockIdx.x * kWavesPerBlock + wid) * kWave + lane;
  bool in = false;
  if (v < n) {
    const float f = add_rn(g[v], h ? h[v] : 0.0f);
    in = f < G;
  }
  const unsigned long long mask = __ballot(in);
  const int cnt = __popcll(mask);
  if (in) {
    stamp[v] = epoch;
    members[wid][__popcll(mask & lanes_below(lane))] = (int32_t)v;
  }
  __syncthreads();
  constexpr int R = kWave / GW;
  const int grp = lane / GW, gl = lane % GW;
  for (int r = 0; r < cnt; r += R) {
    const int idx = r + grp;
    if (idx < cnt) {
      const int32_t u = members[wid][idx];
      const int64_t a = rp[u], b = rp[u + 1];  // (mark: rows of P only)
      for (int64_t j = a + gl; j < b; j += GW * U) {
        // every load is issued unconditionally (clamped to an entry of the row) so
        // the U loads of a lane are in flight together
        int32_t w[U];
#pragma unroll
        for (int q = 0; q < U; ++q) w[q] = col[j + q * GW < b ? j + q * GW : a];
#pragma unroll
        for (int q = 0; q < U; ++q)
          if (j + q * GW < b) stamp[w[q]] = epoch;
      }
    }
  }
  if (lane == 0 && cnt > 0) atomicAdd(&ctr->nP, cnt);
}

template <int GW, int U>
__global__ void __launch_bounds__(kThreads) k_improve(int32_t n, int32_t root, const float* __restrict__ g,
                                                     const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                     const float* __restrict__ cst, const uint32_t* __restrict__ stamp,
                                                     uint32_t epoch, const int32_t* __restrict__ ext_of,
                                                     int32_t* __restrict__ parent, float* __restrict__ pcost,
                                                     IterCounters* __restrict__ ctr) {
  __shared__ int32_t members[kWavesPerBlock][kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int64_t v = ((int64_t)blockIdx.x * kWavesPerBlock + wid) * kWave + lane;
  const bool in = v < n && v != root && stamp[v] == epoch;
  const unsigned long long mask = __ballot(in);
  const int cnt = __popcll(mask);
  if (in) members[wid][__popcll(mask & lanes_below(lane))] = (int32_t)v;
  __syncthreads();
  constexpr int R = kWave / GW;
  const int grp = lane / GW, gl = lane % GW;
  unsigned long long edges = 0;
  int changed = 0;
  for (int r = 0; r < cnt; r += R) {
    const int idx = r + grp;
    const bool act = idx < cnt;
    const int32_t x = members[wid][act ? idx : 0];
    const int64_t ra = rp[x], rb = rp[x + 1];
    const int64_t a = act ? ra : 0, b = act ? rb : 0;
    // lane-local minimum of (g(u) + c, caller id of u, c); bu = slot of u
    uint32_t bv = 0xffffffffu, bc = 0xffffffffu;
    int32_t bu = -1;
    for (int64_t j = a + gl; j < b; j += GW * U) {
      // loads are unconditional (entries past the row end re-read entry a and are
      // masked below): one wait for the U entries, one for their U gathers
      int32_t u[U];
      float c[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int64_t jj = j + q * GW < b ? j + q * GW : a;
        u[q] = col[jj];
        c[q] = cst[jj];
      }
      float gu[U];
#pragma unroll
      for (int q = 0; q < U; ++q) gu[q] = g[u[q]];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        if (j + q * GW >= b) continue;
        const uint32_t vb = __float_as_uint(add_rn(gu[q], c[q])), cb = __float_as_uint(c[q]);
        if (vb >= 0x7f800000u) continue;  // +inf never improves anything
        if (vb < bv) {
          bv = vb;
          bu = u[q];
          bc = cb;
        } else if (vb == bv) {  // equal candidates within one lane: rare
          const int32_t e1 = ext_of[u[q]], e0 = ext_of[bu];
          if (e1 < e0 || (e1 == e0 && cb < bc)) {
            bu = u[q];
            bc = cb;
          }
        }
      }
    }
    // group minimum: value first; the caller id is fetched only for real ties
    const uint32_t mv = group_min_u32<GW>(bv);
    const bool tied = bu >= 0 && bv == mv;
    const unsigned long long tb = group_bits<GW>(__ballot(tied), grp);
    const bool multi = __popcll(tb) > 1;
    const uint32_t e = tied ? (multi ? (uint32_t)ext_of[bu] : 0u) : 0xffffffffu;
    const unsigned long long k2 = ((unsigned long long)e << 32) | (tied ? bc : 0xffffffffu);
    const unsigned long long m2 = group_min_u64<GW>(k2);
    const unsigned long long wb = group_bits<GW>(__ballot(tied && k2 == m2), grp);
    const int src = grp * GW + (wb ? __ffsll((long long)wb) - 1 : 0);
    const int32_t wu = __shfl(bu, src, kWave);
    const uint32_t wc = __shfl(bc, src, kWave);
    if (act && gl == 0) {
      edges += (unsigned long long)(b - a);
      if (wb != 0 && __uint_as_float(mv) < g[x]) {
        parent[x] = wu;
        pcost[x] = __uint_as_float(wc);
        ++changed;
      }
    }
  }
  // one atomic per wave for each counter
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    edges += __shfl_xor(edges, off, kWave);
    changed += __shfl_xor(changed, off, kWave);
  }
  if (lane == 0) {
    if (cnt > 0) {
      atomicAdd(&ctr->nD, cnt);
      atomicAdd(&ctr->edges, edges);
    }
    if (changed > 0) atomicAdd(&ctr->changed, changed);
  }
}

template <int GW, int U>
void launch_mark_t(const StepArgs& a, hipStream_t s) {
  const int64_t chunks = ((int64_t)a.n + kWave - 1) / kWave;
  const unsigned blocks = (unsigned)((chunks + kWavesPerBlock - 1) / kWavesPerBlock);
  hipLaunchKernelGGL((k_mark<GW, U>), dim3(blocks > 0 ? blocks : 1), dim3(kThreads), 0, s, a.n, a.goal, a.prune, a.g,
                     a.h, a.rp, a.col, a.stamp, a.epoch, a.ctr);
}

template <int GW, int U>
void launch_improve_t(const StepArgs& a, hipStream_t s) {
  const int64_t chunks = ((int64_t)a.n + kWave - 1) / kWave;
  const unsigned blocks = (unsigned)((chunks + kWavesPerBlock - 1) / kWavesPerBlock);
  hipLaunchKernelGGL((k_improve<GW, U>), dim3(blocks > 0 ? blocks : 1), dim3(kThreads), 0, s, a.n, a.root, a.g,
                     a.rp, a.col, a.cst, a.stamp, a.epoch, a.ext_of, a.parent, a.pcost, a.ctr);
}

}  // namespace

// Row-mapping variants: group width (lanes per row) x entries per lane in flight.
void launch_mark(const StepArgs& a, int variant, hipStream_t s) {
  switch (variant) {
    case 0: launch_mark_t<16, 4>(a, s); break;
    case 1: launch_mark_t<32, 2>(a, s); break;
    case 2: launch_mark_t<64, 1>(a, s); break;
    default: launch_mark_t<8, 8>(a, s); break;
  }
}

void launch_improve(const StepArgs& a, int variant, hipStream_t s) {
  switch (variant) {
    case 0: launch_improve_t<16, 4>(a, s); break;
    case 1: launch_improve_t<32, 2>(a, s); break;
    case 2: launch_improve_t<64, 1>(a, s); break;
    default: launch_improve_t<8, 8>(a, s); break;
  }
}

}  // namespace pirrt
