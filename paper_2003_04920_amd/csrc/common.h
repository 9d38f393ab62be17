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

// Lexicographic (key, cost) minimum, key = (binary32 bits of the candidate << 32 |
// neighbour id).  All candidates are >= +0, so the bit patterns order like the
// values; +inf stays above every finite candidate.
struct Cand {
  unsigned long long key;
  uint32_t cbits;
};

__device__ __forceinline__ void cand_min(Cand& a, unsigned long long k, uint32_t c) {
  if (k < a.key || (k == a.key && c < a.cbits)) {
    a.key = k;
    a.cbits = c;
  }
}

// Butterfly minimum over groups of `width` consecutive lanes (width a power of
// two <= 64); every lane of the group ends with the group minimum.
template <int width>
__device__ __forceinline__ Cand group_min(Cand a) {
#pragma unroll
  for (int off = width / 2; off > 0; off >>= 1) {
    uint32_t lo = (uint32_t)a.key, hi = (uint32_t)(a.key >> 32);
    uint32_t olo = __shfl_xor(lo, off, kWave);
    uint32_t ohi = __shfl_xor(hi, off, kWave);
    uint32_t oc = __shfl_xor(a.cbits, off, kWave);
    cand_min(a, ((unsigned long long)ohi << 32) | olo, oc);
  }
  return a;
}

}  // namespace pirrt
