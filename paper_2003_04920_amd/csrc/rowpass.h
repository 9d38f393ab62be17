// Device helpers shared by the row passes of mark.hip and improve.hip.
#pragma once

#include "internal.h"

namespace pirrt {
namespace rows {

constexpr int kThreads = 256;

// Adds the per-vertex counters of the workgroup into its problem's counter copy:
// one atomic per counter and workgroup when the workgroup lies in one problem,
// one per vertex otherwise.
__device__ __forceinline__ void flush_counters(IterCounters* ctr, int p, bool leader, int nP, int nD,
                                               unsigned long long edges, int changed, int pedges = 0) {
  __shared__ int block_p, mixed;
  __shared__ unsigned long long red[5];
  __syncthreads();  // a previous call of this workgroup may still read red
  if (threadIdx.x == 0) {
    block_p = p;
    mixed = 0;
    red[0] = red[1] = red[2] = red[3] = red[4] = 0ull;
  }
  __syncthreads();
  if (leader && p != block_p) mixed = 1;
  __syncthreads();
  const int slot = blockIdx.x % kCounterSlots;
  if (mixed) {
    if (leader && (nP | nD | changed | pedges)) {
      IterCounters& C = ctr[(int64_t)p * kCounterSlots + slot];
      if (nP) atomicAdd(&C.nP, nP);
      if (nD) atomicAdd(&C.nD, nD);
      if (edges) atomicAdd(&C.edges, edges);
      if (changed) atomicAdd(&C.changed, changed);
      if (pedges) atomicAdd(&C.pedges, pedges);
    }
    return;
  }
  const int lane = threadIdx.x & (kWave - 1);
  unsigned long long a = leader ? (unsigned long long)nP : 0ull, b = leader ? (unsigned long long)nD : 0ull,
                     c = leader ? edges : 0ull, d = leader ? (unsigned long long)changed : 0ull,
                     e = leader ? (unsigned long long)pedges : 0ull;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, kWave);
    b += __shfl_xor(b, off, kWave);
    c += __shfl_xor(c, off, kWave);
    d += __shfl_xor(d, off, kWave);
    e += __shfl_xor(e, off, kWave);
  }
  if (lane == 0) {
    if (a) atomicAdd(&red[0], a);
    if (b) atomicAdd(&red[1], b);
    if (c) atomicAdd(&red[2], c);
    if (d) atomicAdd(&red[3], d);
    if (e) atomicAdd(&red[4], e);
  }
  __syncthreads();
  if (threadIdx.x < 5 && red[threadIdx.x]) {
    IterCounters& C = ctr[(int64_t)block_p * kCounterSlots + slot];
    const unsigned long long t = red[threadIdx.x];
    if (threadIdx.x == 0) atomicAdd(&C.nP, (int)t);
    if (threadIdx.x == 1) atomicAdd(&C.nD, (int)t);
    if (threadIdx.x == 2) atomicAdd(&C.edges, t);
    if (threadIdx.x == 3) atomicAdd(&C.changed, (int)t);
    if (threadIdx.x == 4) atomicAdd(&C.pedges, (int)t);
  }
}

// The same sums per wave, without the workgroup's barriers (the grid-stride loops of
// a batch call it once per work unit): when every leader lane of the wave lies in one
// problem, lane 0 adds the wave's sums, one atomic per counter; otherwise each leader
// adds its own.  Counters that a caller never sets are left out at compile time.
template <bool kP, bool kD, bool kE, bool kC, bool kPE>
__device__ __forceinline__ void flush_counters_wave(IterCounters* ctr, int p, bool leader, int nP, int nD,
                                                    unsigned long long edges, int changed, int pedges = 0) {
  const unsigned long long lm = __ballot(leader);
  if (lm == 0ull) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int p0 = __shfl(p, __ffsll((long long)lm) - 1, kWave);
  const int slot = (int)((blockIdx.x * (kThreads / kWave) + threadIdx.x / kWave) % kCounterSlots);
  if (__ballot(leader && p != p0) != 0ull) {  // the wave straddles problems
    if (leader) {
      IterCounters& C = ctr[(int64_t)p * kCounterSlots + slot];
      if (kP && nP) atomicAdd(&C.nP, nP);
      if (kD && nD) atomicAdd(&C.nD, nD);
      if (kE && edges) atomicAdd(&C.edges, edges);
      if (kC && changed) atomicAdd(&C.changed, changed);
      if (kPE && pedges) atomicAdd(&C.pedges, pedges);
    }
    return;
  }
  int a = kP && leader ? nP : 0, b = kD && leader ? nD : 0, d = kC && leader ? changed : 0,
      e = kPE && leader ? pedges : 0;
  unsigned long long c = kE && leader ? edges : 0ull;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    if (kP) a += __shfl_xor(a, off, kWave);
    if (kD) b += __shfl_xor(b, off, kWave);
    if (kE) c += __shfl_xor(c, off, kWave);
    if (kC) d += __shfl_xor(d, off, kWave);
    if (kPE) e += __shfl_xor(e, off, kWave);
  }
  if (lane == 0) {
    IterCounters& C = ctr[(int64_t)p0 * kCounterSlots + slot];
    if (kP && a) atomicAdd(&C.nP, a);
    if (kD && b) atomicAdd(&C.nD, b);
    if (kE && c) atomicAdd(&C.edges, c);
    if (kC && d) atomicAdd(&C.changed, d);
    if (kPE && e) atomicAdd(&C.pedges, e);
  }
}

inline dim3 grid_for(int64_t n, int gw) {
  const int64_t b = ((int64_t)n * gw + kThreads - 1) / kThreads;
  return dim3((unsigned)(b > 0 ? b : 1));
}

// Batches use a fixed grid of `blocks` workgroups (at most one per work unit) that
// strides over the live work.
inline dim3 batch_grid(int64_t n, int per_block, int blocks) {
  const int64_t T = (n + kTileSlots - 1) / kTileSlots;
  const int64_t units = T * (kTileSlots / per_block);
  return dim3((unsigned)(units < blocks ? (units > 0 ? units : 1) : blocks));
}

}  // namespace rows
}  // namespace pirrt
