// Exclusive prefix sums (reduce-then-scan, 2048 items per 256-thread workgroup).
// Used to turn per-vertex counts into CSR offsets: out[0..n], out[n] = total.
#include "internal.h"

namespace pirrt {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    T y = __shfl_up(v, off, kWave);
    if (lane >= off) v += y;
  }
  return v;
}

// Exclusive scan of one value per thread across the workgroup; *total = sum.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T x, T* total) {
  __shared__ T wsum[kScanThreads / kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  T incl = wave_incl_scan(x);
  if (lane == kWave - 1) wsum[wid] = incl;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / kWave; ++w) {
    T s = wsum[w];
    if (w < wid) before += s;
    all += s;
  }
  __syncthreads();
  *total = all;
  return before + incl - x;
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const TI* __restrict__ in, int64_t n,
                                                             TO* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  TO s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) s += (TO)in[base + k];
  TO total;
  block_excl_scan<TO>(s, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const TI* __restrict__ in, int64_t n,
                                                            const TO* __restrict__ offsets,
                                                            TO* __restrict__ out) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  TO v[kScanItems];
  TO s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? (TO)in[base + k] : (TO)0;
    s += v[k];
  }
  TO total;
  TO run = block_excl_scan<TO>(s, &total) + (offsets ? offsets[blockIdx.x] : (TO)0);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
    if (base + k == n - 1) out[n] = run;
  }
}

template <typename T>
__global__ void k_zero_one(T* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

}  // namespace

size_t scan_scratch_bytes(int64_t n) {
  size_t bytes = 0;
  while (n > kScanTile) {
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    bytes += sizeof(int64_t) * (size_t)(2 * nb + 2);
    n = nb;
  }
  return bytes + 256;
}

template <typename TI, typename TO>
static void scan_rec(const TI* in, int64_t n, TO* out, char* scratch, hipStream_t s) {
  if (n <= 0) {
    hipLaunchKernelGGL(k_zero_one<TO>, dim3(1), dim3(1), 0, s, out);
    return;
  }
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 1) {
    hipLaunchKernelGGL((k_scan_apply<TI, TO>), dim3(1), dim3(kScanThreads), 0, s, in, n,
                       (const TO*)nullptr, out);
    return;
  }
  TO* sums = (TO*)scratch;
  TO* offs = sums + nb;
  char* rest = (char*)(offs + nb + 1);
  hipLaunchKernelGGL((k_scan_reduce<TI, TO>), dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, sums);
  scan_rec<TO, TO>(sums, nb, offs, rest, s);
  hipLaunchKernelGGL((k_scan_apply<TI, TO>), dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n,
                     (const TO*)offs, out);
}

void scan_i32_to_i64(const int32_t* in, int64_t n, int64_t* out, void* scratch, hipStream_t s) {
  scan_rec<int32_t, int64_t>(in, n, out, (char*)scratch, s);
}

void scan_i32_to_i32(const int32_t* in, int64_t n, int32_t* out, void* scratch, hipStream_t s) {
  scan_rec<int32_t, int32_t>(in, n, out, (char*)scratch, s);
}

}  // namespace pirrt
