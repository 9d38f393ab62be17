// Graph store: appending a batch of vertices to the symmetric CSR adjacency, and
// Extend's insertion-time policy for the new vertices (Sec. III local relaxation;
// Sec. IV-A cached edge costs).
//
// The adjacency is one CSR over all vertex slots: int64 row offsets and, per entry,
// an int32 neighbour slot and a binary32 cost in two parallel arrays.  A batch
// arrives as forward rows (each new vertex lists its lower-index neighbours),
// translated to slots before it gets here.  Appending rebuilds the CSR into a spare
// buffer in one streaming pass: every row keeps its old entries, a new vertex's
// row starts with its forward entries, and each forward edge (v, u) is mirrored
// into u's row.  Entry order inside a row is not fixed (mirrors are placed with
// atomics); nothing downstream depends on it because every minimum is taken on
// (value, neighbour, cost).
#include "internal.h"

namespace pirrt {

namespace {

constexpr int kThreads = 256;

inline unsigned blocks_for(int64_t n, int per_block = kThreads) {
  int64_t b = (n + per_block - 1) / per_block;
  return (unsigned)(b > 0 ? b : 1);
}

// Error bits raised by validation.
enum { kErrRowPtr = 1, kErrCol = 2, kErrCost = 4 };

// The per-row kernels of an insert give each row a group of kRowGW lanes, so a batch
// of a thousand rows spreads over the chip instead of looping in a thousand threads.
constexpr int kRowGW = 8;

__global__ void __launch_bounds__(kThreads) k_validate_rows(int32_t n_new, int64_t n_old, int64_t lo_bound,
                                                           const int64_t* __restrict__ rp,
                                                           const int32_t* __restrict__ col,
                                                           const float* __restrict__ cost, int64_t nnz_arg,
                                                           const int64_t* __restrict__ nnz_dev,
                                                           int* __restrict__ err) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t / kRowGW;
  const int gl = (int)(t % kRowGW);
  if (i >= n_new) return;
  const int64_t nnz = nnz_dev ? *nnz_dev : nnz_arg;
  if (nnz < 0 || nnz > ((int64_t)1 << 40)) {
    atomicOr(err, kErrRowPtr);
    return;
  }
  int64_t a = rp[i], b = rp[i + 1];
  int bad = 0;
  if (i == 0 && a != 0) bad |= kErrRowPtr;
  if (a < 0 || b < a || b > nnz) {
    atomicOr(err, bad | kErrRowPtr);
    return;
  }
  const int64_t self = n_old + i;
  for (int64_t j = a + gl; j < b; j += kRowGW) {
    int32_t c = col[j];
    uint32_t w = __float_as_uint(cost[j]);
    if ((int64_t)c < lo_bound || (int64_t)c >= self) bad |= kErrCol;
    // finite, >= 0 and sign bit clear (rejects NaN, inf, negatives and -0.0)
    if ((w >> 31) != 0 || (w & 0x7f800000u) == 0x7f800000u) bad |= kErrCost;
  }
  if (bad) atomicOr(err, bad);
}

// add[v] += forward length of new vertex v; add[u] += 1 per mirrored entry.
__global__ void __launch_bounds__(kThreads) k_count_new(int32_t n_new, int64_t n_old,
                                                       const int64_t* __restrict__ brp,
                                                       const int32_t* __restrict__ bcol,
                                                       int32_t* __restrict__ add) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t / kRowGW;
  const int gl = (int)(t % kRowGW);
  if (i >= n_new) return;
  int64_t a = brp[i], b = brp[i + 1];
  if (gl == 0 && b > a) atomicAdd(&add[n_old + i], (int)(b - a));
  for (int64_t j = a + gl; j < b; j += kRowGW) atomicAdd(&add[bcol[j]], 1);
}

// deg[v] = old degree + added entries (counted in cnt, which is cleared here); add[v]
// becomes the fill cursor of v's row (old degree + forward length, mirrors go after
// it).
__global__ void __launch_bounds__(kThreads) k_degrees(int64_t n1, int64_t n_old,
                                                     const int64_t* __restrict__ rp_old,
                                                     const int64_t* __restrict__ brp, int32_t* __restrict__ cnt,
                                                     int32_t* __restrict__ add, int32_t* __restrict__ deg) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n1) return;
  int32_t old = v < n_old ? (int32_t)(rp_old[v + 1] - rp_old[v]) : 0;
  int32_t fwd = v >= n_old ? (int32_t)(brp[v - n_old + 1] - brp[v - n_old]) : 0;
  const int32_t c = cnt[v];
  cnt[v] = 0;
  deg[v] = old + c;
  add[v] = old + fwd;
}

// Copies every old row to its new offset: one wave per row, lanes striding.
__global__ void __launch_bounds__(kThreads) k_copy_rows(int64_t n_old, const int64_t* __restrict__ rp_old,
                                                       const int32_t* __restrict__ col_old,
                                                       const float* __restrict__ cst_old,
                                                       const int64_t* __restrict__ rp_new,
                                                       int32_t* __restrict__ col_new, float* __restrict__ cst_new) {
  const int lane = threadIdx.x & (kWave - 1);
  int64_t v = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (v >= n_old) return;
  int64_t a = rp_old[v], b = rp_old[v + 1], dst = rp_new[v];
  for (int64_t j = a + lane; j < b; j += kWave) {
    col_new[dst + (j - a)] = col_old[j];
    cst_new[dst + (j - a)] = cst_old[j];
  }
}

// Forward entries of each new row, and their mirrors into the lower endpoint.
__global__ void __launch_bounds__(kThreads) k_scatter_new(int32_t n_new, int64_t n_old,
                                                         const int64_t* __restrict__ brp,
                                                         const int32_t* __restrict__ bcol,
                                                         const float* __restrict__ bcost,
                                                         const int64_t* __restrict__ rp_new,
                                                         int32_t* __restrict__ cursor,
                                                         int32_t* __restrict__ col_new,
                                                         float* __restrict__ cst_new) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t / kRowGW;
  const int gl = (int)(t % kRowGW);
  if (i >= n_new) return;
  const int32_t v = (int32_t)(n_old + i);
  int64_t a = brp[i], b = brp[i + 1], dst = rp_new[v];
  for (int64_t j = a + gl; j < b; j += kRowGW) {
    int32_t u = bcol[j];
    float c = bcost[j];
    col_new[dst + (j - a)] = u;
    cst_new[dst + (j - a)] = c;
    int64_t pos = rp_new[u] + atomicAdd(&cursor[u], 1);
    col_new[pos] = v;
    cst_new[pos] = c;
  }
}

// pending[i] = number of same-batch lower neighbours of new vertex n_old + i; the
// ones with none start the first dependency level.  Every lane of the grid reaches the
// wave-wide reservation.
__global__ void __launch_bounds__(kThreads) k_pending(int32_t n_new, int64_t n_old,
                                                     const int64_t* __restrict__ brp,
                                                     const int32_t* __restrict__ bcol,
                                                     int32_t* __restrict__ pending,
                                                     int32_t* __restrict__ frontier, int32_t* __restrict__ fcount) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t / kRowGW;
  const int gl = (int)(t % kRowGW);
  int cnt = 0;
  if (i < n_new)
    for (int64_t j = brp[i] + gl; j < brp[i + 1]; j += kRowGW) cnt += (bcol[j] >= n_old);
#pragma unroll
  for (int off = kRowGW / 2; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, kWave);
  const bool ready = i < n_new && gl == 0 && cnt == 0;
  if (i < n_new && gl == 0) pending[i] = cnt;
  int slot = wave_reserve(fcount, ready);
  if (ready) frontier[slot] = (int32_t)(n_old + i);
}

// Extend's local relaxation of new vertices whose lower neighbours are all final, one
// group of kInsGW lanes per vertex (every lane of the wave calls it; a group with
// valid = false takes no part): the minimum over (g(u) + c, u, c) of the vertex's
// forward row, u the caller's id (bcol) and g read at the storage slot (bslot), the
// row's entries spread over the lanes and the lexicographic minimum taken with DPP.
// kSameLaunch: g of same-batch neighbours was written earlier in this launch by
// another wave of the workgroup, so it is read past the L1.  Then the vertex releases
// its same-batch higher neighbours (the mirror part of its row, also spread over the
// lanes); those whose last pending lower neighbour it was go through push().
constexpr int kInsGW = 8;

template <bool kSameLaunch, class Push>
__device__ __forceinline__ void insert_group(bool valid, int32_t v, int64_t n_old, int32_t insert_root,
                                             const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol,
                                             const int32_t* __restrict__ bslot, const float* __restrict__ bcost,
                                             const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                             float* __restrict__ g, int32_t* __restrict__ parent,
                                             float* __restrict__ pcost, int32_t* __restrict__ pending, Push push) {
  const int gl = threadIdx.x % kInsGW;
  const int64_t i = valid ? v - n_old : 0;
  const int64_t a = valid ? brp[i] : 0, b = valid ? brp[i + 1] : 0;
  const bool relax = valid && v != insert_root;
  uint32_t bv = 0xffffffffu, bc = 0xffffffffu, be = 0xffffffffu;
  int32_t bs = -1;
  if (relax) {
    for (int64_t j = a + gl; j < b; j += kInsGW) {
      const uint32_t u = (uint32_t)bcol[j];
      const float c = bcost[j];
      const int32_t su = bslot[j];
      const float gu = kSameLaunch && su >= n_old ? __hip_atomic_load(&g[su], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                                  : g[su];
      const uint32_t vb = __float_as_uint(add_rn(gu, c)), cb = __float_as_uint(c);
      if (vb < bv || (vb == bv && (u < be || (u == be && cb < bc)))) {
        bv = vb;
        be = u;
        bc = cb;
        bs = su;
      }
    }
  }
  // (value, id) first, then the cost among the lanes that hold that pair
  const unsigned long long k = ((unsigned long long)bv << 32) | be;
  const unsigned long long km = dpp_group_min_u64<kInsGW>(k);
  const uint32_t cm = dpp_group_min_u32<kInsGW>(k == km ? bc : 0xffffffffu);
  const int grp = (threadIdx.x & (kWave - 1)) / kInsGW;
  const unsigned long long wb = group_bits<kInsGW>(__ballot(k == km && bc == cm), grp);
  const int32_t ws = __shfl(bs, grp * kInsGW + (wb ? __ffsll((long long)wb) - 1 : 0), kWave);
  if (valid && gl == 0) {
    if (!relax) {  // x_init of the graph (or of a new problem of a batch)
      g[v] = 0.0f;
      parent[v] = -1;
      pcost[v] = 0.0f;
    } else if (ws >= 0 && (uint32_t)(km >> 32) < 0x7f800000u) {
      g[v] = __uint_as_float((uint32_t)(km >> 32));
      parent[v] = ws;
      pcost[v] = __uint_as_float(cm);
    } else {
      g[v] = pos_inf();
      parent[v] = -1;
      pcost[v] = 0.0f;
    }
  }
  // release the same-batch higher neighbours (the mirror part of v's row)
  if (valid) {
    for (int64_t j = rp[v] + (b - a) + gl; j < rp[v + 1]; j += kInsGW) {
      const int32_t w = col[j];
      if (atomicSub(&pending[w - n_old], 1) == 1) push(w);
    }
  }
}

// One dependency level of the insertion-time policy: every vertex of the frontier
// has all its lower neighbours final, so its local relaxation is final too.  New
// vertices occupy slots equal to their ids.
__global__ void __launch_bounds__(kThreads) k_insert_level(const int32_t* __restrict__ fsize_dev,
                                                          int32_t* __restrict__ done,
                                                          const int32_t* __restrict__ frontier,
                                                          int64_t n_old, int32_t insert_root,
                                                          const int64_t* __restrict__ brp,
                                                          const int32_t* __restrict__ bcol,
                                                          const int32_t* __restrict__ bslot,
                                                          const float* __restrict__ bcost,
                                                          const int64_t* __restrict__ rp,
                                                          const int32_t* __restrict__ col, float* __restrict__ g,
                                                          int32_t* __restrict__ parent, float* __restrict__ pcost,
                                                          int32_t* __restrict__ pending,
                                                          int32_t* __restrict__ next, int32_t* __restrict__ ncount) {
  const int32_t fsize = *fsize_dev;  // this level's frontier (the grid covers the whole batch)
  const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kInsGW;
  if (blockIdx.x == 0 && threadIdx.x == 0 && fsize > 0) atomicAdd(done, fsize);
  if ((int64_t)blockIdx.x * (blockDim.x / kInsGW) >= fsize) return;  // the whole workgroup
  const bool valid = t < fsize;
  insert_group<false>(valid, valid ? frontier[t] : 0, n_old, insert_root, brp, bcol, bslot, bcost, rp, col, g,
                      parent, pcost, pending, [&](int32_t w) { next[atomicAdd(ncount, 1)] = w; });
}

// Every dependency level of a small batch in one workgroup, with a workgroup barrier
// between levels (the frontiers alternate between f0 and f1, their sizes in LDS): a
// batch of a few thousand vertices needs a dozen levels, each far too small for a
// launch of its own.  fsize0 (device) is the first frontier, already in f0.  Writes the
// number of vertices placed to *done.
constexpr int kBlockThreads = 1024;

__global__ void __launch_bounds__(kBlockThreads) k_insert_block(const int32_t* __restrict__ fsize0,
                                                               int32_t* __restrict__ done,
                                                               int32_t* __restrict__ f0, int32_t* __restrict__ f1,
                                                               int64_t n_old, int32_t n_new, int32_t insert_root,
                                                               const int64_t* __restrict__ brp,
                                                               const int32_t* __restrict__ bcol,
                                                               const int32_t* __restrict__ bslot,
                                                               const float* __restrict__ bcost,
                                                               const int64_t* __restrict__ rp,
                                                               const int32_t* __restrict__ col, float* __restrict__ g,
                                                               int32_t* __restrict__ parent, float* __restrict__ pcost,
                                                               int32_t* __restrict__ pending) {
  constexpr int kGroups = kBlockThreads / kInsGW;
  __shared__ int32_t size_cur, size_next;
  if (threadIdx.x == 0) {
    size_cur = *fsize0;
    size_next = 0;
  }
  __syncthreads();
  int32_t placed = 0;  // thread 0's running total
  int32_t* cur = f0;
  int32_t* nxt = f1;
  for (int32_t level = 0; level <= n_new; ++level) {
    const int32_t size = size_cur;  // the same for every thread of the workgroup
    if (size == 0) break;
    placed += size;
    for (int32_t base = 0; base < size; base += kGroups) {
      const int32_t t = base + (int32_t)(threadIdx.x / kInsGW);
      const bool valid = t < size;
      const int32_t v = valid ? __hip_atomic_load(&cur[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
      insert_group<true>(valid, v, n_old, insert_root, brp, bcol, bslot, bcost, rp, col, g, parent, pcost, pending,
                         [&](int32_t w) {
                           __hip_atomic_store(&nxt[atomicAdd(&size_next, 1)], w, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                         });
    }
    __threadfence_block();
    __syncthreads();
    if (threadIdx.x == 0) {
      size_cur = size_next;
      size_next = 0;
    }
    __syncthreads();
    int32_t* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  if (threadIdx.x == 0) *done = placed;
}

}  // namespace

void launch_validate_rows(int32_t n_new, int64_t n_old, int64_t lo_bound, const int64_t* rp, const int32_t* col,
                          const float* cost, int64_t nnz, int* err, hipStream_t s, const int64_t* nnz_dev) {
  hipLaunchKernelGGL(k_validate_rows, dim3(blocks_for((int64_t)n_new * kRowGW)), dim3(kThreads), 0, s, n_new, n_old, lo_bound, rp,
                     col, cost, nnz, nnz_dev, err);
}

void launch_rebuild(int32_t n_new, int64_t n_old, const int64_t* brp, const int32_t* bcol, const float* bcost,
                    const int64_t* rp_old, const int32_t* col_old, const float* cst_old, int64_t* rp_new,
                    int32_t* col_new, float* cst_new, int32_t* add, int32_t* add0, int32_t* deg, void* scan_scratch,
                    hipStream_t s) {
  const int64_t n1 = n_old + n_new;
  if (n_new > 0)
    hipLaunchKernelGGL(k_count_new, dim3(blocks_for((int64_t)n_new * kRowGW)), dim3(kThreads), 0, s, n_new, n_old, brp, bcol, add0);
  hipLaunchKernelGGL(k_degrees, dim3(blocks_for(n1)), dim3(kThreads), 0, s, n1, n_old, rp_old, brp, add0, add, deg);
  scan_i32_to_i64(deg, n1, rp_new, scan_scratch, s);
  if (n_old > 0)
    hipLaunchKernelGGL(k_copy_rows, dim3(blocks_for(n_old * kWave)), dim3(kThreads), 0, s, n_old, rp_old,
                       col_old, cst_old, rp_new, col_new, cst_new);
  if (n_new > 0)
    hipLaunchKernelGGL(k_scatter_new, dim3(blocks_for((int64_t)n_new * kRowGW)), dim3(kThreads), 0, s, n_new, n_old, brp, bcol,
                       bcost, rp_new, add, col_new, cst_new);
}

namespace {

// Degrees of the vertices of an appended block (no entry touches an older row).
__global__ void __launch_bounds__(kThreads) k_degrees_append(int32_t n_new, int64_t n_old,
                                                            const int64_t* __restrict__ brp,
                                                            int32_t* __restrict__ add, int32_t* __restrict__ deg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_new) return;
  deg[i] = add[n_old + i];
  add[n_old + i] = (int32_t)(brp[i + 1] - brp[i]);
}

__global__ void __launch_bounds__(kThreads) k_offset_rows(int32_t n_new, int64_t n_old, int64_t base,
                                                         const int64_t* __restrict__ tmp, int64_t* __restrict__ rp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= n_new) rp[n_old + i] = base + tmp[i];
}

}  // namespace

void launch_append(int32_t n_new, int64_t n_old, int64_t nnz_old, const int64_t* brp, const int32_t* bcol,
                   const float* bcost, int64_t* rp, int32_t* col, float* cst, int32_t* add, int32_t* deg,
                   int64_t* tmp, void* scan_scratch, hipStream_t s) {
  hipMemsetAsync(add + n_old, 0, sizeof(int32_t) * (size_t)n_new, s);
  hipLaunchKernelGGL(k_count_new, dim3(blocks_for((int64_t)n_new * kRowGW)), dim3(kThreads), 0, s, n_new, n_old, brp, bcol, add);
  hipLaunchKernelGGL(k_degrees_append, dim3(blocks_for(n_new)), dim3(kThreads), 0, s, n_new, n_old, brp, add, deg);
  scan_i32_to_i64(deg, n_new, tmp, scan_scratch, s);
  hipLaunchKernelGGL(k_offset_rows, dim3(blocks_for((int64_t)n_new + 1)), dim3(kThreads), 0, s, n_new, n_old, nnz_old,
                     tmp, rp);
  hipLaunchKernelGGL(k_scatter_new, dim3(blocks_for((int64_t)n_new * kRowGW)), dim3(kThreads), 0, s, n_new, n_old, brp, bcol, bcost,
                     rp, add, col, cst);
}

void launch_pending(int32_t n_new, int64_t n_old, const int64_t* brp, const int32_t* bcol, int32_t* pending,
                    int32_t* frontier, int32_t* fcount, hipStream_t s) {
  hipLaunchKernelGGL(k_pending, dim3(blocks_for((int64_t)n_new * kRowGW)), dim3(kThreads), 0, s, n_new, n_old, brp, bcol, pending,
                     frontier, fcount);
}

void launch_insert_block(const int32_t* fsize0, int32_t* done, int32_t* f0, int32_t* f1, int64_t n_old, int32_t n_new,
                         int32_t insert_root, const int64_t* brp, const int32_t* bcol, const int32_t* bslot,
                         const float* bcost, const int64_t* rp, const int32_t* col, float* g, int32_t* parent,
                         float* pcost, int32_t* pending, hipStream_t s) {
  hipLaunchKernelGGL(k_insert_block, dim3(1), dim3(kBlockThreads), 0, s, fsize0, done, f0, f1, n_old, n_new,
                     insert_root, brp, bcol, bslot, bcost, rp, col, g, parent, pcost, pending);
}

void launch_insert_level(int32_t max_size, const int32_t* fsize, int32_t* done, const int32_t* frontier,
                         int64_t n_old, int32_t insert_root, const int64_t* brp, const int32_t* bcol,
                         const int32_t* bslot, const float* bcost, const int64_t* rp, const int32_t* col, float* g,
                         int32_t* parent, float* pcost, int32_t* pending, int32_t* next, int32_t* ncount,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_insert_level, dim3(blocks_for((int64_t)max_size * kInsGW)), dim3(kThreads), 0, s, fsize, done,
                     frontier, n_old,
                     insert_root, brp, bcol, bslot, bcost, rp, col, g, parent, pcost, pending, next, ncount);
}

// Growing problems of a batch.  The new vertices of all blocks are appended after
// every existing slot ("append ids" n_old, n_old + 1, ... in block order) and keep
// those ids until k_reid gives every vertex its final caller id.

// Block of row r: the last block whose first row is <= r (blocks are non-empty and
// in row order).
__device__ __forceinline__ int32_t block_of_row(int32_t nblk, const BatchBlock* __restrict__ blk, int64_t r) {
  int32_t lo = 0, hi = nblk - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (blk[mid].row_begin <= r) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Local neighbour ids -> the ids the insertion uses: an existing vertex its current
// caller id (its problem's old base + local id), a vertex of the same block its
// append id.  Local ids outside [0, own local id) raise kErrCol and are left as they
// are (the call fails before anything reads them).
__global__ void __launch_bounds__(kThreads) k_batch_rows(int32_t total, int32_t nblk,
                                                        const BatchBlock* __restrict__ blk,
                                                        const int64_t* __restrict__ brp, int32_t* __restrict__ bcol,
                                                        int* __restrict__ err) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= total) return;
  const BatchBlock b = blk[block_of_row(nblk, blk, r)];
  const int64_t own = (int64_t)b.n_old + (r - b.row_begin);
  int bad = 0;
  for (int64_t j = brp[r]; j < brp[r + 1]; ++j) {
    const int32_t c = bcol[j];
    if (c < 0 || (int64_t)c >= own) {
      bad = kErrCol;
      continue;
    }
    bcol[j] = c < b.n_old ? (int32_t)(b.base_old + c) : (int32_t)(b.app_base + (c - b.n_old));
  }
  if (bad) atomicOr(err, bad);
}

// prob of the appended slots [n_old, n_old + total).
__global__ void __launch_bounds__(kThreads) k_block_problems(int64_t n_old, int32_t total, int32_t nblk,
                                                            const BatchBlock* __restrict__ blk,
                                                            int32_t* __restrict__ prob) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= total) return;
  prob[n_old + r] = blk[block_of_row(nblk, blk, r)].problem;
}

// Final caller ids after the growth: problem p's vertices take [pbase_new[p],
// pbase_new[p + 1]) in local order (old vertices keep their local ids, the block's
// vertices follow them), so every comparison of ids inside a problem is unchanged.
__global__ void __launch_bounds__(kThreads) k_reid(int64_t n1, int64_t n_old, int32_t nblk,
                                                  const BatchBlock* __restrict__ blk,
                                                  const int64_t* __restrict__ pbase_old,
                                                  const int64_t* __restrict__ pbase_new,
                                                  const int32_t* __restrict__ prob, int32_t* __restrict__ ext_of,
                                                  int32_t* __restrict__ slot_of) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n1) return;
  const int32_t e = ext_of[s];
  int64_t e1;
  if (e < n_old) {
    const int32_t p = prob[s];
    e1 = pbase_new[p] + (e - pbase_old[p]);
  } else {
    const BatchBlock b = blk[block_of_row(nblk, blk, e - n_old)];
    e1 = pbase_new[b.problem] + b.n_old + (e - b.app_base);
  }
  ext_of[s] = (int32_t)e1;
  slot_of[e1] = (int32_t)s;
}

__global__ void __launch_bounds__(kThreads) k_offset_ids(int64_t m, int32_t offset, int32_t* __restrict__ ids) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) ids[j] += offset;
}

void launch_batch_rows(int32_t total, int32_t nblk, const BatchBlock* blk, const int64_t* brp, int32_t* bcol, int* err,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_batch_rows, dim3(blocks_for(total)), dim3(kThreads), 0, s, total, nblk, blk, brp, bcol, err);
}

void launch_block_problems(int64_t n_old, int32_t total, int32_t nblk, const BatchBlock* blk, int32_t* prob,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_block_problems, dim3(blocks_for(total)), dim3(kThreads), 0, s, n_old, total, nblk, blk, prob);
}

void launch_reid(int64_t n1, int64_t n_old, int32_t nblk, const BatchBlock* blk, const int64_t* pbase_old,
                 const int64_t* pbase_new, const int32_t* prob, int32_t* ext_of, int32_t* slot_of, hipStream_t s) {
  hipLaunchKernelGGL(k_reid, dim3(blocks_for(n1)), dim3(kThreads), 0, s, n1, n_old, nblk, blk, pbase_old, pbase_new,
                     prob, ext_of, slot_of);
}

void launch_offset_ids(int64_t m, int32_t offset, int32_t* ids, hipStream_t s) {
  if (m > 0 && offset != 0)
    hipLaunchKernelGGL(k_offset_ids, dim3(blocks_for(m)), dim3(kThreads), 0, s, m, offset, ids);
}

}  // namespace pirrt
