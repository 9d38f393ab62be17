// Shared device-side definitions of the gfx950 Replan library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pirrt {

constexpr int kWave = 64;  // CDNA wavefront width

// Per-iteration counters written by the mark / improve kernels.
struct IterCounters {
  int32_t changed;           // parents switched by Improve
  int32_t nP;                // |promising set|
  int32_t nD;                // |Improve domain|
  int32_t pad;
  unsigned long long edges;  // sum of the degrees over the Improve domain
};

// Bookkeeping of one Evaluate (breadth-first walk of the policy tree).
struct EvalInfo {
  int32_t head_end;  // first level the single-workgroup head kernel left to others
  int32_t levels;    // number of non-empty levels (tree depth + 1)
  int32_t big_end;   // 1 + last level whose frontier exceeded the tail threshold
  int32_t pad;
};

__device__ __forceinline__ float pos_inf() { return __int_as_float(0x7f800000); }

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
