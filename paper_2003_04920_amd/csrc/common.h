// Shared device-side definitions of the gfx950 Replan library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pirrt {

constexpr int kWave = 64;  // CDNA wavefront width

// Parent value that marks a Replan root inside the library (callers see -1).
constexpr int32_t kRootMark = -2;

// Per-iteration counters of one problem, written by the mark / improve kernels.
// Each problem has kCounterSlots copies (workgroup b adds into copy
// b % kCounterSlots) so that the atomics do not pile onto one address; the finish
// kernel sums and clears them.
constexpr int kCounterSlots = 64;
struct IterCounters {
  int32_t changed;           // parents switched by Improve
  int32_t nP;                // |promising set|
  int32_t nD;                // |Improve domain|
  int32_t pedges;            // sum of the degrees over the promising set (the rows marked)
  unsigned long long edges;  // sum of the degrees over the Improve domain
};

// Replan state of one problem (a graph, or one graph of a batch) on the device.
struct ProblemState {
  int32_t root;        // slot of x_init
  int32_t goal;        // slot of x_goal
  float thr;           // promising threshold G of the current iteration (-inf: idle)
  int32_t active;      // still iterating
  int32_t needs_eval;  // Evaluate after the current Improve
  int32_t iterations;  // Improve passes so far
  int32_t status;      // 0 running / converged, 1 iteration cap reached
  int32_t cap;         // iteration cap
  unsigned long long edges, sum_P, sum_D, changed_total;
  unsigned long long mark_edges;  // sum over iterations of the promising rows' degrees
  // Single graphs with the walk Evaluate: changed_total when the current iteration began
  // (the walk that follows Improve compares the counters against it).
  unsigned long long changed_seen;
};

// Device-side loop control shared by the kernels of one Replan.
struct LoopCtl {
  uint32_t epoch;       // stamp of the current promising-set / domain marks
  uint32_t eval_epoch;  // stamp of the current Evaluate
  int32_t any_active;   // some problem runs this iteration (set by the thresholds)
  int32_t any_eval;     // some problem needs an Evaluate after this iteration
  int32_t ndomain;      // entries of the compacted Improve domain of this iteration
  int32_t ntiles;       // batches: entries of the active tile list; -1 = every tile
  int32_t npromising;   // single graphs: entries of the compacted promising set
  int32_t tiles_stale;  // batches: a problem stopped since the tile lists were built
};

// Truncated Evaluate: the low word of a vertex's walk stamp carries this bit when the
// walk does not visit its children (the vertex was not reached, or failed the
// promising test); g bits are >= 0, so their sign bit is free.
constexpr uint32_t kWalkNoChildren = 0x80000000u;

// Batches run their per-slot kernels over tiles of kTileSlots consecutive slots;
// after each Evaluate the tiles that overlap a problem still iterating are listed
// (LoopCtl::ntiles, -1 = all tiles in slot order).
constexpr int kTileSlots = 4096;

// Work units of a batch: every active tile is cut into kTileSlots / per_unit units
// of per_unit consecutive slots.  Kernels loop over the units with a grid stride.
__device__ __forceinline__ int64_t tile_units(const LoopCtl* ctl, int32_t n, int per_unit) {
  const int32_t nt = ctl->ntiles;
  const int64_t T = nt < 0 ? ((int64_t)n + kTileSlots - 1) / kTileSlots : nt;
  return T * (kTileSlots / per_unit);
}

__device__ __forceinline__ int64_t tile_unit_slot(const LoopCtl* ctl, const int32_t* tiles, int per_unit,
                                                  int64_t w) {
  const int64_t upt = kTileSlots / per_unit;
  const int64_t ti = w / upt;
  const int64_t t = ctl->ntiles < 0 ? ti : tiles[ti];
  return t * kTileSlots + (w % upt) * per_unit;
}

// Workgroups of a batch kernel's grid-stride launch.
constexpr int kBatchBlocks = 2048;

// Bookkeeping of one Evaluate (breadth-first walk of the policy tree).
struct EvalInfo {
  int32_t head_end;  // first level the single-workgroup head kernel left to others
  int32_t levels;    // number of non-empty levels (tree depth + 1)
  int32_t big_end;   // 1 + last level whose frontier exceeded the tail threshold
  int32_t pad;
};

__device__ __forceinline__ float pos_inf() { return __int_as_float(0x7f800000); }

// Next mark epoch: its low byte (the stamp value) is never 0, so a cleared stamp never
// matches.
__device__ __forceinline__ uint32_t next_mark_epoch(uint32_t e) { return ((e + 1) & 0xffu) == 0 ? e + 2 : e + 1; }

// Next Evaluate epoch (0 is never used, so a cleared stamp word never matches).
__device__ __forceinline__ uint32_t next_epoch(uint32_t e) { return e + 1 == 0 ? 1u : e + 1; }

// Binary32 addition with round-to-nearest-even, never contracted.
__device__ __forceinline__ float add_rn(float a, float b) { return __fadd_rn(a, b); }

// Exclusive prefix sum of x over the 64 lanes of the wave; *total gets the sum.
__device__ __forceinline__ int wave_exclusive_sum(int x, int* total) {
  const int lane = threadIdx.x & (kWave - 1);
  int v = x;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    int y = __shfl_up(v, off, kWave);
    if (lane >= off) v += y;
  }
  *total = __shfl(v, kWave - 1, kWave);
  return v - x;
}

// Reserves `count` slots of a global counter for each lane, one atomic per wave.
// Returns the first slot of the calling lane.
__device__ __forceinline__ int wave_reserve(int* counter, int count) {
  int total;
  int off = wave_exclusive_sum(count, &total);
  int base = 0;
  const int lane = threadIdx.x & (kWave - 1);
  if (lane == 0 && total > 0) base = atomicAdd(counter, total);
  base = __shfl(base, 0, kWave);
  return base + off;
}

// Cross-lane moves through DPP (a VALU operand modifier, no LDS round trip).
// Controls: quad_perm(1,0,3,2) = 0xB1, quad_perm(2,3,0,1) = 0x4E,
// row_half_mirror = 0x141, row_mirror = 0x140.  All lanes must be active.
template <int ctrl>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, ctrl, 0xf, 0xf, false);
}

// Minimum over groups of `width` (2, 4, 8 or 16) consecutive lanes with DPP;
// wider groups continue with lane shuffles.  Every lane ends with its group's
// minimum.
template <int width>
__device__ __forceinline__ uint32_t dpp_group_min_u32(uint32_t x) {
  uint32_t y;
  if (width >= 2) { y = dpp_u32<0xB1>(x); x = y < x ? y : x; }
  if (width >= 4) { y = dpp_u32<0x4E>(x); x = y < x ? y : x; }
  if (width >= 8) { y = dpp_u32<0x141>(x); x = y < x ? y : x; }
  if (width >= 16) { y = dpp_u32<0x140>(x); x = y < x ? y : x; }
#pragma unroll
  for (int off = 16; off < width; off <<= 1) {
    y = __shfl_xor(x, off, kWave);
    x = y < x ? y : x;
  }
  return x;
}

template <int width>
__device__ __forceinline__ unsigned long long dpp_group_min_u64(unsigned long long x) {
  uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32), ylo, yhi;
#define PIRRT_DPP_MIN64(ctrl)                                            \
  ylo = dpp_u32<ctrl>(lo);                                               \
  yhi = dpp_u32<ctrl>(hi);                                               \
  if (yhi < hi || (yhi == hi && ylo < lo)) { hi = yhi; lo = ylo; }
  if (width >= 2) { PIRRT_DPP_MIN64(0xB1) }
  if (width >= 4) { PIRRT_DPP_MIN64(0x4E) }
  if (width >= 8) { PIRRT_DPP_MIN64(0x141) }
  if (width >= 16) { PIRRT_DPP_MIN64(0x140) }
#undef PIRRT_DPP_MIN64
#pragma unroll
  for (int off = 16; off < width; off <<= 1) {
    ylo = __shfl_xor(lo, off, kWave);
    yhi = __shfl_xor(hi, off, kWave);
    if (yhi < hi || (yhi == hi && ylo < lo)) { hi = yhi; lo = ylo; }
  }
  return ((unsigned long long)hi << 32) | lo;
}

// Minimum over groups of `width` consecutive lanes (width a power of two <= 64);
// every lane of the group ends with the group minimum.
template <int width>
__device__ __forceinline__ uint32_t group_min_u32(uint32_t x) {
#pragma unroll
  for (int off = width / 2; off > 0; off >>= 1) {
    uint32_t y = __shfl_xor(x, off, kWave);
    x = y < x ? y : x;
  }
  return x;
}

template <int width>
__device__ __forceinline__ unsigned long long group_min_u64(unsigned long long x) {
#pragma unroll
  for (int off = width / 2; off > 0; off >>= 1) {
    uint32_t lo = __shfl_xor((uint32_t)x, off, kWave);
    uint32_t hi = __shfl_xor((uint32_t)(x >> 32), off, kWave);
    unsigned long long y = ((unsigned long long)hi << 32) | lo;
    x = y < x ? y : x;
  }
  return x;
}

// Bits [grp*width, grp*width + width) of a wave-wide ballot, as the low bits.
template <int width>
__device__ __forceinline__ unsigned long long group_bits(unsigned long long ballot, int grp) {
  return width == 64 ? ballot : (ballot >> (grp * width)) & ((1ull << width) - 1ull);
}

}  // namespace pirrt
