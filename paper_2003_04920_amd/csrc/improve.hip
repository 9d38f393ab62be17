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
// Work split: a group of GW lanes per vertex, U row entries per lane in flight
// (GW x U = 64 entries per pass over a row).  Two grid shapes share one body:
//   kStatic      one group per vertex, the grid covers all slots (a wave whose
//                vertices are all outside the set leaves after one round trip and
//                frees its slot for the next);
//   persistent   about one residency of workgroups striding over the slots,
//                either round-robin or XCD-aware (the hardware hands workgroup b
//                to XCD b % 8; XCD x then strides over the x-th eighth of the
//                slots only, keeping its gathers in its own L2).
// Loads are issued unconditionally (row positions past the end re-read the first
// entry and are masked), so a lane's U loads are in flight together; the per-row
// minimum is a DPP butterfly.
#include "internal.h"

namespace pirrt {

namespace {

constexpr int kThreads = 256;
constexpr int kXcds = 8;

// This workgroup's share of the slots [0, n): range of its XCD, first group base
// and stride (in vertices).  The grid is a multiple of kXcds.
struct Span {
  int64_t hi, base, stride;
};

enum Grid { kStatic = 0, kRoundRobin = 1, kXcdAware = 2 };

template <int GW, int kGrid>
__device__ __forceinline__ Span work_span(int64_t n) {
  constexpr int64_t gpb = kThreads / GW;  // vertices per workgroup pass
  Span s;
  if (kGrid == kXcdAware) {
    const int64_t xcd = blockIdx.x % kXcds, local = blockIdx.x / kXcds, bpx = gridDim.x / kXcds;
    const int64_t per = (n + kXcds - 1) / kXcds;
    const int64_t lo = xcd * per < n ? xcd * per : n;
    s.hi = lo + per < n ? lo + per : n;
    s.base = lo + local * gpb;
    s.stride = bpx * gpb;
  } else {
    s.hi = n;
    s.base = (int64_t)blockIdx.x * gpb;
    s.stride = kGrid == kStatic ? n + 1 : (int64_t)gridDim.x * gpb;  // static: one pass
  }
  return s;
}

// Adds the workgroup's counters (one global atomic per counter and workgroup).
__device__ __forceinline__ void flush_counters(IterCounters* ctr, unsigned long long* red, int nP, int nD,
                                               unsigned long long edges, int changed) {
  const int lane = threadIdx.x & (kWave - 1);
  unsigned long long a = (unsigned long long)nP, b = (unsigned long long)nD, c = edges,
                     d = (unsigned long long)changed;
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
    IterCounters& C = ctr[blockIdx.x % kCounterSlots];
    const unsigned long long t = red[threadIdx.x];
    if (threadIdx.x == 0) atomicAdd(&C.nP, (int)t);
    if (threadIdx.x == 1) atomicAdd(&C.nD, (int)t);
    if (threadIdx.x == 2) atomicAdd(&C.edges, t);
    if (threadIdx.x == 3) atomicAdd(&C.changed, (int)t);
  }
}

template <int GW, int U, int kGrid>
__global__ void __launch_bounds__(kThreads) k_mark(int32_t n, int32_t goal, int prune, const float* __restrict__ g,
                                                  const float* __restrict__ h, const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col, uint32_t* __restrict__ stamp,
                                                  uint32_t epoch, IterCounters* __restrict__ ctr) {
  __shared__ unsigned long long red[4];
  if (threadIdx.x < 4) red[threadIdx.x] = 0ull;
  __syncthreads();
  const int gib = threadIdx.x / GW, gl = threadIdx.x % GW;
  const float G = prune ? g[goal] : pos_inf();
  const Span sp = work_span<GW, kGrid>(n);
  int nP = 0;
  for (int64_t v0 = sp.base; v0 < sp.hi; v0 += sp.stride) {
    const int64_t v = v0 + gib;
    const bool valid = v < sp.hi;
    const int32_t x = (int32_t)(valid ? v : v0);
    const float gx = g[x], hx = h ? h[x] : 0.0f;
    const int64_t ra = rp[x], rb = rp[x + 1];
    const bool in = valid && add_rn(gx, hx) < G;
    if (__ballot(in) == 0) continue;
    if (in) {
      if (gl == 0) {
        stamp[x] = epoch;
        ++nP;
      }
      for (int64_t j = ra + gl; j < rb; j += GW * U) {
        int32_t w[U];
#pragma unroll
        for (int q = 0; q < U; ++q) w[q] = col[j + q * GW < rb ? j + q * GW : ra];
#pragma unroll
        for (int q = 0; q < U; ++q)
          if (j + q * GW < rb) stamp[w[q]] = epoch;
      }
    }
  }
  flush_counters(ctr, red, nP, 0, 0ull, 0);
}

template <int GW, int U, int kGrid>
__global__ void __launch_bounds__(kThreads) k_improve(int32_t n, int32_t root, const float* __restrict__ g,
                                                     const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                     const float* __restrict__ cst, const uint32_t* __restrict__ stamp,
                                                     uint32_t epoch, const int32_t* __restrict__ ext_of,
                                                     int32_t* __restrict__ parent, float* __restrict__ pcost,
                                                     IterCounters* __restrict__ ctr) {
  __shared__ unsigned long long red[4];
  if (threadIdx.x < 4) red[threadIdx.x] = 0ull;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int grp = lane / GW, gib = threadIdx.x / GW, gl = threadIdx.x % GW;
  const Span sp = work_span<GW, kGrid>(n);
  int nD = 0, changed = 0;
  unsigned long long edges = 0;
  for (int64_t v0 = sp.base; v0 < sp.hi; v0 += sp.stride) {
    const int64_t v = v0 + gib;
    const bool valid = v < sp.hi;
    const int32_t x = (int32_t)(valid ? v : v0);
    const uint32_t sx = stamp[x];
    const float gx = g[x];
    const int64_t ra = rp[x], rb = rp[x + 1];
    const bool in = valid && x != root && sx == epoch;
    if (__ballot(in) == 0) continue;
    const int64_t a = in ? ra : 0, b = in ? rb : 0;
    // lane-local minimum of (g(u) + c, caller id of u, c); bu = slot of u
    uint32_t bv = 0xffffffffu, bc = 0xffffffffu;
    int32_t bu = -1;
    for (int64_t j = a + gl; j < b; j += GW * U) {
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
    if (in && gl == 0) {
      ++nD;
      edges += (unsigned long long)(b - a);
      if (wb != 0 && __uint_as_float(mv) < gx) {
        parent[x] = wu;
        pcost[x] = __uint_as_float(wc);
        ++changed;
      }
    }
  }
  flush_counters(ctr, red, 0, nD, edges, changed);
}

inline unsigned grid_for(int64_t n, int gw, int kGrid, int max_blocks) {
  int64_t b = ((int64_t)n * gw + kThreads - 1) / kThreads;
  if (kGrid != kStatic && b > max_blocks) b = max_blocks;
  b = (b + kXcds - 1) / kXcds * kXcds;
  return (unsigned)(b > 0 ? b : kXcds);
}

template <int GW, int U, int kGrid>
void launch_mark_t(const StepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_mark<GW, U, kGrid>), dim3(grid_for(a.n, GW, kGrid, a.max_blocks)), dim3(kThreads), 0, s,
                     a.n, a.goal, a.prune, a.g, a.h, a.rp, a.col, a.stamp, a.epoch, a.ctr);
}

template <int GW, int U, int kGrid>
void launch_improve_t(const StepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_improve<GW, U, kGrid>), dim3(grid_for(a.n, GW, kGrid, a.max_blocks)), dim3(kThreads), 0, s,
                     a.n, a.root, a.g, a.rp, a.col, a.cst, a.stamp, a.epoch, a.ext_of, a.parent, a.pcost, a.ctr);
}

}  // namespace

// Variants: lanes per row x entries per lane in flight, and grid shape.
void launch_mark(const StepArgs& a, int variant, hipStream_t s) {
  switch (variant) {
    case 0: launch_mark_t<16, 4, kStatic>(a, s); break;
    case 1: launch_mark_t<8, 8, kStatic>(a, s); break;
    case 2: launch_mark_t<16, 4, kRoundRobin>(a, s); break;
    case 3: launch_mark_t<16, 4, kXcdAware>(a, s); break;
    case 4: launch_mark_t<4, 16, kStatic>(a, s); break;
    default: launch_mark_t<32, 2, kStatic>(a, s); break;
  }
}

void launch_improve(const StepArgs& a, int variant, hipStream_t s) {
  switch (variant) {
    case 0: launch_improve_t<16, 4, kStatic>(a, s); break;
    case 1: launch_improve_t<8, 8, kStatic>(a, s); break;
    case 2: launch_improve_t<16, 4, kRoundRobin>(a, s); break;
    case 3: launch_improve_t<16, 4, kXcdAware>(a, s); break;
    case 4: launch_improve_t<4, 16, kStatic>(a, s); break;
    default: launch_improve_t<32, 2, kStatic>(a, s); break;
  }
}

}  // namespace pirrt
