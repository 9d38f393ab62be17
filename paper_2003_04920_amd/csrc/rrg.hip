// Exploration support on the device: grows the random geometric graph that Replan
// works on (Sec. III, Extend; Alg. 3 with batches of S samples).
//
//   sample  : Philox4x32-10 counter-based draws (Salmon et al., SC'11), candidate k
//             of stream s under seed q -> coordinates (w_i >> 8) * 2^-24; obstacle
//             rejection (closed sets); free candidates kept in order of k.
//   connect : for every new vertex v, every earlier u with 0 < |x_u - x_v|^2 <= r^2
//             (binary64, axes summed in order) whose closed segment meets no
//             obstacle (sphere: clamped closest point; box: slab intersection),
//             cost = binary32 rounding of the binary64 length; rows ascending in u,
//             handed to pirrt_insert_batch / pirrt_batch_add_problem on the device.
//   heuristic: binary32 rounding of the binary64 distance to the goal.
//
// The radius search is brute force over all earlier vertices: a workgroup owns 256
// consecutive new vertices (one per thread) and streams the earlier points through
// LDS in tiles every thread reads by broadcast.  It runs twice (count, then write
// candidates in ascending u); the segment tests then run once per candidate and a
// scan compacts the survivors into rows.
#include <string.h>

#include <cmath>
#include <string>
#include <vector>

#include "internal.h"
#include "pirrt.h"

using namespace pirrt;

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 256;
constexpr int kMaxDim = 8;

struct ObsView {
  int32_t n;
  const int32_t* kind;
  const double* centre;
  const double* size;
};

__device__ __forceinline__ void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                                       uint32_t out[4]) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

template <int D>
__device__ __forceinline__ bool point_blocked(const double* x, const ObsView& ob) {
  for (int o = 0; o < ob.n; ++o) {
    const double* c = ob.centre + (int64_t)o * D;
    const double* s = ob.size + (int64_t)o * D;
    if (ob.kind[o] == 0) {
      double d2 = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const double e = x[k] - c[k];
        d2 = __dadd_rn(d2, __dmul_rn(e, e));
      }
      if (d2 <= __dmul_rn(s[0], s[0])) return true;
    } else {
      bool inside = true;
#pragma unroll
      for (int k = 0; k < D; ++k)
        if (fabs(x[k] - c[k]) > s[k]) inside = false;
      if (inside) return true;
    }
  }
  return false;
}

template <int D>
__device__ __forceinline__ bool hits_sphere(const double* a, const double* b, const double* c, double rad) {
  double ee = 0.0, ce = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double e = b[k] - a[k];
    ee = __dadd_rn(ee, __dmul_rn(e, e));
    ce = __dadd_rn(ce, __dmul_rn(c[k] - a[k], e));
  }
  double t = ee > 0.0 ? __ddiv_rn(ce, ee) : 0.0;
  if (t < 0.0) t = 0.0;
  if (t > 1.0) t = 1.0;
  double q2 = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double q = __dadd_rn(a[k], __dmul_rn(t, b[k] - a[k])) - c[k];
    q2 = __dadd_rn(q2, __dmul_rn(q, q));
  }
  return q2 <= __dmul_rn(rad, rad);
}

template <int D>
__device__ __forceinline__ bool hits_box(const double* a, const double* b, const double* c, const double* half) {
  double lo_t = 0.0, hi_t = 1.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double lo = c[k] - half[k], hi = c[k] + half[k];
    const double e = b[k] - a[k];
    if (e == 0.0) {
      if (a[k] < lo || a[k] > hi) return false;
      continue;
    }
    double t_lo = __ddiv_rn(lo - a[k], e), t_hi = __ddiv_rn(hi - a[k], e);
    if (t_lo > t_hi) {
      const double s = t_lo;
      t_lo = t_hi;
      t_hi = s;
    }
    if (t_lo > lo_t) lo_t = t_lo;
    if (t_hi < hi_t) hi_t = t_hi;
    if (lo_t > hi_t) return false;
  }
  return true;
}

template <int D>
__device__ __forceinline__ bool segment_blocked(const double* a, const double* b, const ObsView& ob) {
  for (int o = 0; o < ob.n; ++o) {
    const double* c = ob.centre + (int64_t)o * D;
    const double* s = ob.size + (int64_t)o * D;
    const bool hit = ob.kind[o] == 0 ? hits_sphere<D>(a, b, c, s[0]) : hits_box<D>(a, b, c, s);
    if (hit) return true;
  }
  return false;
}

template <int D>
__device__ __forceinline__ double dist2(const double* a, const double* b) {
  double d2 = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double e = a[k] - b[k];
    d2 = __dadd_rn(d2, __dmul_rn(e, e));
  }
  return d2;
}

// Candidates k0 .. k0 + T - 1: coordinates into cbuf, free flag into flag.
template <int D>
__global__ void __launch_bounds__(kThreads) k_candidates(int64_t T, uint64_t k0, uint64_t seed, uint32_t stream,
                                                         ObsView ob, double* __restrict__ cbuf,
                                                         int32_t* __restrict__ flag) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= T) return;
  const uint64_t k = k0 + (uint64_t)t;
  uint32_t w[8];
  philox((uint32_t)k, (uint32_t)(k >> 32), stream, 0u, (uint32_t)seed, (uint32_t)(seed >> 32), w);
  if (D > 4) philox((uint32_t)k, (uint32_t)(k >> 32), stream, 1u, (uint32_t)seed, (uint32_t)(seed >> 32), w + 4);
  double x[D];
#pragma unroll
  for (int i = 0; i < D; ++i) x[i] = (double)(w[i] >> 8) * (1.0 / 16777216.0);
#pragma unroll
  for (int i = 0; i < D; ++i) cbuf[t * D + i] = x[i];
  flag[t] = point_blocked<D>(x, ob) ? 0 : 1;
}

// Appends the free candidates whose rank (pos) is below `need`; records one past
// the candidate of rank need - 1 in *last.
template <int D>
__global__ void __launch_bounds__(kThreads) k_take(int64_t T, int64_t need, const double* __restrict__ cbuf,
                                                   const int32_t* __restrict__ flag, const int64_t* __restrict__ pos,
                                                   double* __restrict__ pts, int64_t* __restrict__ last) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= T || !flag[t]) return;
  const int64_t p = pos[t];
  if (p >= need) return;
#pragma unroll
  for (int i = 0; i < D; ++i) pts[p * D + i] = cbuf[t * D + i];
  if (p == need - 1) *last = t + 1;
}

// Radius search over a grid of (256 new vertices) x (kChunk earlier points).
// Pass 1 (WRITE = false): cc[row * nch + chunk] = candidates of that row in that
// chunk.  Pass 2 (WRITE = true): their ids, ascending, from off[row * nch + chunk]
// (the exclusive scan of cc in row-major order, so every row stays ascending in u).
constexpr int64_t kChunk = 8192;

template <int D, bool WRITE>
__global__ void __launch_bounds__(kThreads) k_radius(int64_t n_old, int64_t n, const double* __restrict__ pts,
                                                     double r2, int32_t nch, int32_t* __restrict__ cc,
                                                     const int64_t* __restrict__ off, int32_t* __restrict__ cand_u,
                                                     int32_t* __restrict__ cand_v) {
  __shared__ double tile[kTile * D];
  const int64_t vb = n_old + (int64_t)blockIdx.x * kThreads;
  const int64_t v = vb + threadIdx.x;
  const bool live = v < n;
  double xv[D];
#pragma unroll
  for (int k = 0; k < D; ++k) xv[k] = live ? pts[v * D + k] : 0.0;
  const int64_t vmax = (vb + kThreads < n ? vb + kThreads : n);  // u < vmax covers every thread
  const int64_t c0 = (int64_t)blockIdx.y * kChunk;
  const int64_t c1 = (c0 + kChunk < vmax ? c0 + kChunk : vmax);
  const int64_t slot = (v - n_old) * nch + blockIdx.y;
  int32_t c = 0;
  int64_t out = WRITE && live ? off[slot] : 0;
  for (int64_t u0 = c0; u0 < c1; u0 += kTile) {
    const int64_t m = (c1 - u0 < kTile ? c1 - u0 : kTile);
    __syncthreads();
    for (int64_t i = threadIdx.x; i < m * D; i += kThreads) tile[i] = pts[u0 * D + i];
    __syncthreads();
    if (live) {
      const int64_t lim = (v - u0 < m ? v - u0 : m);
      for (int64_t i = 0; i < lim; ++i) {
        const double d2 = dist2<D>(tile + i * D, xv);
        if (d2 <= r2 && d2 > 0.0) {
          if (WRITE) {
            cand_u[out] = (int32_t)(u0 + i);
            cand_v[out] = (int32_t)v;
            ++out;
          } else {
            ++c;
          }
        }
      }
    }
  }
  if (!WRITE && live) cc[slot] = c;
}

// Segment test and cost of every candidate edge.
template <int D>
__global__ void __launch_bounds__(kThreads) k_collide(int64_t m, const double* __restrict__ pts, ObsView ob,
                                                      const int32_t* __restrict__ cand_u,
                                                      const int32_t* __restrict__ cand_v, int32_t* __restrict__ keep,
                                                      float* __restrict__ ccost) {
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (j >= m) return;
  double a[D], b[D];
  const int64_t u = cand_u[j], v = cand_v[j];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    a[k] = pts[u * D + k];
    b[k] = pts[v * D + k];
  }
  const bool blocked = segment_blocked<D>(a, b, ob);
  keep[j] = blocked ? 0 : 1;
  ccost[j] = __double2float_rn(__dsqrt_rn(dist2<D>(a, b)));
}

// Survivors into rows: row_ptr[i] = kpos[cptr[i]], col / cost at kpos[j].
__global__ void __launch_bounds__(kThreads) k_compact(int64_t m, const int32_t* __restrict__ keep,
                                                      const int64_t* __restrict__ kpos,
                                                      const int32_t* __restrict__ cand_u,
                                                      const float* __restrict__ ccost, int32_t* __restrict__ col,
                                                      float* __restrict__ cost) {
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (j >= m || !keep[j]) return;
  col[kpos[j]] = cand_u[j];
  cost[kpos[j]] = ccost[j];
}

__global__ void __launch_bounds__(kThreads) k_row_ptr(int64_t rows, int32_t nch, const int64_t* __restrict__ off,
                                                      const int64_t* __restrict__ kpos, int64_t* __restrict__ rp) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i <= rows) rp[i] = kpos[off[i * nch]];
}

template <int D>
__global__ void __launch_bounds__(kThreads) k_heuristic(int64_t n, const double* __restrict__ pts,
                                                        const double* __restrict__ goal, float* __restrict__ h) {
  const int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (v >= n) return;
  double x[D], gx[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    x[k] = pts[v * D + k];
    gx[k] = goal[k];
  }
  h[v] = __double2float_rn(__dsqrt_rn(dist2<D>(x, gx)));
}

// Features of candidate samples: coordinates (as binary32), then the encoding.
template <int D>
__global__ void __launch_bounds__(kThreads) k_features(int32_t m, const double* __restrict__ pts,
                                                       const float* __restrict__ enc, int32_t in_dim,
                                                       float* __restrict__ feat) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= (int64_t)m * in_dim) return;
  const int64_t r = i / in_dim, k = i % in_dim;
  feat[i] = k < D ? (float)pts[r * D + k] : enc[k - D];
}

// The c best of m logits (m <= kSelMax): one workgroup sorts 64-bit keys {logit in
// a sign-ordered encoding, complement of the index} in LDS with a bitonic network
// (descending: highest logit first, the earlier candidate first among equal
// logits), flags the first c, then lists the flagged indices in ascending order.
constexpr int kSelThreads = 1024;
constexpr int kSelMax = 8192;

__global__ void __launch_bounds__(kSelThreads) k_select_top(int32_t m, int32_t c, const float* __restrict__ logits,
                                                            int32_t* __restrict__ flag, int32_t* __restrict__ sel) {
  __shared__ unsigned long long key[kSelMax];
  __shared__ int32_t part[kSelThreads];
  int N = 1;
  while (N < m) N <<= 1;
  for (int i = threadIdx.x; i < N; i += kSelThreads) {
    unsigned long long kk = 0ull;  // padding sorts last
    if (i < m) {
      uint32_t u = __float_as_uint(logits[i]);
      u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
      kk = ((unsigned long long)u << 32) | (unsigned long long)(~(uint32_t)i);
      flag[i] = 0;
    }
    key[i] = kk;
  }
  __syncthreads();
  for (int k = 2; k <= N; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < N; i += kSelThreads) {
        const int l = i ^ j;
        if (l > i) {
          const unsigned long long a = key[i], b = key[l];
          if (((i & k) == 0) ? (a < b) : (a > b)) {
            key[i] = b;
            key[l] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < c; i += kSelThreads) flag[~(uint32_t)key[i]] = 1;
  __syncthreads();
  const int chunk = (m + kSelThreads - 1) / kSelThreads;
  const int lo = threadIdx.x * chunk, hi = lo + chunk < m ? lo + chunk : m;
  int cnt = 0;
  for (int i = lo; i < hi; ++i) cnt += flag[i];
  part[threadIdx.x] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kSelThreads; ++w) {
      const int x = part[w];
      part[w] = t;
      t += x;
    }
  }
  __syncthreads();
  int pos = part[threadIdx.x];
  for (int i = lo; i < hi; ++i)
    if (flag[i]) sel[pos++] = i;
}

template <int D>
__global__ void __launch_bounds__(kThreads) k_gather_points(int32_t c, const int32_t* __restrict__ sel,
                                                            const double* __restrict__ cand, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= (int64_t)c * D) return;
  const int64_t j = i / D, k = i % D;
  dst[i] = cand[(int64_t)sel[j] * D + k];
}

__global__ void k_check_points(int64_t m, const double* __restrict__ x, int* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < m && !isfinite(x[i])) atomicOr(bad, 1);
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads > 0 ? (n + kThreads - 1) / kThreads : 1); }

}  // namespace

struct pirrt_rrg {
  int device = 0;
  hipStream_t stream = nullptr;
  int d = 0;
  int32_t nobs = 0;
  int32_t* okind = nullptr;
  double* ocentre = nullptr;
  double* osize = nullptr;
  double* pts = nullptr;
  int64_t n = 0, cap = 0;
  // scratch (grown on demand)
  double* cbuf = nullptr;
  int32_t* flag = nullptr;
  int64_t* pos = nullptr;
  int64_t cand_cap_s = 0;  // sampler candidates
  int32_t* cnt = nullptr;
  int64_t* cptr = nullptr;
  int64_t rows_cap = 0;
  int64_t rp_cap = 0;
  int32_t* cand_u = nullptr;
  int32_t* cand_v = nullptr;
  int32_t* keep = nullptr;
  int64_t* kpos = nullptr;
  float* ccost = nullptr;
  int64_t cand_cap = 0;
  int64_t* rp = nullptr;
  int32_t* col = nullptr;
  float* cost = nullptr;
  float* hbuf = nullptr;
  int64_t hcap = 0;
  // learned sampler scratch (at most kSelMax candidates)
  double* lpts = nullptr;
  float* lfeat = nullptr;
  float* llogit = nullptr;
  float* lenc = nullptr;
  int32_t* lflag = nullptr;
  int32_t* lsel = nullptr;
  void* scan = nullptr;
  size_t scan_bytes = 0;
  int64_t* dword = nullptr;
  int32_t* dflag = nullptr;
  int64_t* host = nullptr;  // pinned, 4 words
  bool poisoned = false;
  std::string err;
};

namespace {

thread_local std::string g_rrg_create_error;

int rfail(pirrt_rrg* R, int code, const std::string& m) {
  R->err = m;
  return code;
}

int rdev(pirrt_rrg* R, hipError_t e, const char* what) {
  R->poisoned = true;
  R->err = std::string("HIP error in ") + what + ": " + hipGetErrorString(e);
  return PIRRT_EDEVICE;
}

#define RHIP(R, expr)                                  \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return rdev(R, e_, #expr);   \
  } while (0)

template <class T>
bool ralloc(T** p, int64_t count) {
  *p = nullptr;
  if (count <= 0) count = 1;
  if (hipMalloc((void**)p, sizeof(T) * (size_t)count) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return false;
  }
  return true;
}

template <class T>
void rfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

int rguard(pirrt_rrg* R) {
  if (!R) return PIRRT_EINVAL;
  if (R->poisoned) return PIRRT_EDEVICE;
  hipError_t e = hipSetDevice(R->device);
  if (e != hipSuccess) return rdev(R, e, "hipSetDevice");
  return PIRRT_OK;
}

// Grows a device array, keeping `keep` leading elements.
template <class T>
int grow(pirrt_rrg* R, T** p, int64_t* cap, int64_t need, int64_t keep) {
  if (need <= *cap) return PIRRT_OK;
  int64_t c = *cap + *cap / 2;
  if (c < need) c = need;
  T* q = nullptr;
  if (!ralloc(&q, c)) return rfail(R, PIRRT_ENOMEM, "device allocation failed");
  if (keep > 0) RHIP(R, hipMemcpyAsync(q, *p, sizeof(T) * (size_t)keep, hipMemcpyDeviceToDevice, R->stream));
  RHIP(R, hipStreamSynchronize(R->stream));
  rfree(*p);
  *p = q;
  *cap = c;
  return PIRRT_OK;
}

int ensure_scan(pirrt_rrg* R, int64_t n) {
  const size_t need = scan_scratch_bytes(n);
  if (need <= R->scan_bytes) return PIRRT_OK;
  void* p = nullptr;
  if (hipMalloc(&p, need) != hipSuccess) {
    (void)hipGetLastError();
    return rfail(R, PIRRT_ENOMEM, "device allocation of scan scratch failed");
  }
  if (R->scan) (void)hipFree(R->scan);
  R->scan = p;
  R->scan_bytes = need;
  return PIRRT_OK;
}

ObsView obs_view(const pirrt_rrg* R) { return ObsView{R->nobs, R->okind, R->ocentre, R->osize}; }

template <int D>
void launch_candidates(pirrt_rrg* R, int64_t T, uint64_t k0, uint64_t seed, uint32_t stream) {
  hipLaunchKernelGGL(k_candidates<D>, dim3(blocks(T)), dim3(kThreads), 0, R->stream, T, k0, seed, stream,
                     obs_view(R), R->cbuf, R->flag);
}

template <int D>
void launch_take(pirrt_rrg* R, int64_t T, int64_t need, double* dst) {
  hipLaunchKernelGGL(k_take<D>, dim3(blocks(T)), dim3(kThreads), 0, R->stream, T, need, R->cbuf, R->flag, R->pos, dst,
                     R->dword);
}

template <int D>
void launch_radius(pirrt_rrg* R, int64_t n_old, double r2, int32_t nch, bool write) {
  const int64_t rows = R->n - n_old;
  const dim3 grid(blocks(rows), (unsigned)nch);
  if (write)
    hipLaunchKernelGGL((k_radius<D, true>), grid, dim3(kThreads), 0, R->stream, n_old, R->n, R->pts, r2, nch, R->cnt,
                       R->cptr, R->cand_u, R->cand_v);
  else
    hipLaunchKernelGGL((k_radius<D, false>), grid, dim3(kThreads), 0, R->stream, n_old, R->n, R->pts, r2, nch,
                       R->cnt, R->cptr, R->cand_u, R->cand_v);
}

template <int D>
void launch_collide(pirrt_rrg* R, int64_t m) {
  hipLaunchKernelGGL(k_collide<D>, dim3(blocks(m)), dim3(kThreads), 0, R->stream, m, R->pts, obs_view(R), R->cand_u,
                     R->cand_v, R->keep, R->ccost);
}

template <int D>
void launch_heuristic(pirrt_rrg* R, const double* goal, float* h) {
  hipLaunchKernelGGL(k_heuristic<D>, dim3(blocks(R->n)), dim3(kThreads), 0, R->stream, R->n, R->pts, goal, h);
}

#define PIRRT_BY_DIM(d, call)      \
  switch (d) {                     \
    case 1: call(1); break;        \
    case 2: call(2); break;        \
    case 3: call(3); break;        \
    case 4: call(4); break;        \
    case 5: call(5); break;        \
    case 6: call(6); break;        \
    case 7: call(7); break;        \
    default: call(8); break;       \
  }

// Forward rows of points [n_old, n) in R->rp / col / cost; *nnz their entries.
int build_rows(pirrt_rrg* R, int64_t n_old, double radius, int64_t* nnz) {
  const int64_t rows = R->n - n_old;
  hipStream_t s = R->stream;
  int rc;
  *nnz = 0;
  // per-(row, chunk) counts and their scan: cnt / cptr hold rows * nch (+1) entries
  const int32_t nch = (int32_t)((R->n + kChunk - 1) / kChunk);
  const int64_t cells = rows * nch;
  if (cells + 1 > R->rows_cap) {
    rfree(R->cnt);
    rfree(R->cptr);
    R->rows_cap = 0;
    const int64_t c = cells + 1 + (cells + 1) / 2;
    if (!ralloc(&R->cnt, c) || !ralloc(&R->cptr, c))
      return rfail(R, PIRRT_ENOMEM, "device allocation of row offsets failed");
    R->rows_cap = c;
  }
  if (rows + 1 > R->rp_cap) {
    rfree(R->rp);
    R->rp_cap = 0;
    if (!ralloc(&R->rp, rows + 1 + (rows + 1) / 2)) return rfail(R, PIRRT_ENOMEM, "device allocation of rows failed");
    R->rp_cap = rows + 1 + (rows + 1) / 2;
  }
  if (rows == 0) {
    RHIP(R, hipMemsetAsync(R->rp, 0, sizeof(int64_t), s));
    RHIP(R, hipStreamSynchronize(s));
    return PIRRT_OK;
  }
  if ((rc = ensure_scan(R, cells + 1))) return rc;
  const double r2 = radius * radius;
#define RAD_COUNT(D) launch_radius<D>(R, n_old, r2, nch, false)
  PIRRT_BY_DIM(R->d, RAD_COUNT);
#undef RAD_COUNT
  RHIP(R, hipGetLastError());
  scan_i32_to_i64(R->cnt, cells, R->cptr, R->scan, s);
  RHIP(R, hipGetLastError());
  RHIP(R, hipMemcpyAsync(R->host, R->cptr + cells, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  RHIP(R, hipStreamSynchronize(s));
  const int64_t m = R->host[0];
  if (m > ((int64_t)1 << 40)) return rdev(R, hipErrorUnknown, "candidate count out of range");
  if (m + 1 > R->cand_cap) {
    rfree(R->cand_u); rfree(R->cand_v); rfree(R->keep); rfree(R->kpos); rfree(R->ccost); rfree(R->col); rfree(R->cost);
    R->cand_cap = 0;
    const int64_t c = (m + 1) + (m + 1) / 4 + 1024;
    if (!ralloc(&R->cand_u, c) || !ralloc(&R->cand_v, c) || !ralloc(&R->keep, c) || !ralloc(&R->kpos, c + 1) ||
        !ralloc(&R->ccost, c) || !ralloc(&R->col, c) || !ralloc(&R->cost, c))
      return rfail(R, PIRRT_ENOMEM, "device allocation of candidate edges failed");
    R->cand_cap = c;
  }
  if ((rc = ensure_scan(R, m + 1))) return rc;
  if (m > 0) {
#define RAD_WRITE(D) launch_radius<D>(R, n_old, r2, nch, true)
    PIRRT_BY_DIM(R->d, RAD_WRITE);
#undef RAD_WRITE
    RHIP(R, hipGetLastError());
#define COLLIDE(D) launch_collide<D>(R, m)
    PIRRT_BY_DIM(R->d, COLLIDE);
#undef COLLIDE
    RHIP(R, hipGetLastError());
  }
  scan_i32_to_i64(R->keep, m, R->kpos, R->scan, s);
  RHIP(R, hipGetLastError());
  if (m > 0) {
    hipLaunchKernelGGL(k_compact, dim3(blocks(m)), dim3(kThreads), 0, s, m, R->keep, R->kpos, R->cand_u, R->ccost,
                       R->col, R->cost);
    RHIP(R, hipGetLastError());
  }
  hipLaunchKernelGGL(k_row_ptr, dim3(blocks(rows + 1)), dim3(kThreads), 0, s, rows, nch, R->cptr, R->kpos, R->rp);
  RHIP(R, hipGetLastError());
  RHIP(R, hipMemcpyAsync(R->host, R->kpos + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  RHIP(R, hipStreamSynchronize(s));
  *nnz = R->host[0];
  return PIRRT_OK;
}

// `count` free candidates of (seed, stream) from *counter on, in counter order, into
// dst (device, count * d doubles); *counter ends one past the last one taken.
int draw_free(pirrt_rrg* R, uint64_t seed, uint32_t stream_id, uint64_t* counter, int64_t count, double* dst) {
  const int d = R->d;
  int rc;
  uint64_t k = *counter;
  int64_t need = count, got_all = 0, tried = 0;
  while (need > 0) {
    const int64_t T = need + need / 2 + 4096;
    if (T > R->cand_cap_s) {
      rfree(R->cbuf); rfree(R->flag); rfree(R->pos);
      R->cand_cap_s = 0;
      if (!ralloc(&R->cbuf, T * d) || !ralloc(&R->flag, T) || !ralloc(&R->pos, T + 1))
        return rfail(R, PIRRT_ENOMEM, "device allocation of sampler candidates failed");
      R->cand_cap_s = T;
    }
    if ((rc = ensure_scan(R, T + 1))) return rc;
#define CANDS(D) launch_candidates<D>(R, T, k, seed, stream_id)
    PIRRT_BY_DIM(d, CANDS);
#undef CANDS
    RHIP(R, hipGetLastError());
    scan_i32_to_i64(R->flag, T, R->pos, R->scan, R->stream);
    RHIP(R, hipGetLastError());
    RHIP(R, hipMemsetAsync(R->dword, 0, sizeof(int64_t), R->stream));
    double* out = dst + got_all * d;
#define TAKE(D) launch_take<D>(R, T, need, out)
    PIRRT_BY_DIM(d, TAKE);
#undef TAKE
    RHIP(R, hipGetLastError());
    RHIP(R, hipMemcpyAsync(R->host, R->pos + T, sizeof(int64_t), hipMemcpyDeviceToHost, R->stream));
    RHIP(R, hipMemcpyAsync(R->host + 1, R->dword, sizeof(int64_t), hipMemcpyDeviceToHost, R->stream));
    RHIP(R, hipStreamSynchronize(R->stream));
    const int64_t got = R->host[0];
    if (got >= need) {
      k += (uint64_t)R->host[1];
      got_all += need;
      need = 0;
    } else {
      k += (uint64_t)T;
      got_all += got;
      need -= got;
    }
    tried += T;
    if (need > 0 && tried > count * 4096 + (1 << 24))
      return rfail(R, PIRRT_EINVAL, "the free space is too small: no free sample found");
  }
  *counter = k;
  return PIRRT_OK;
}

void release(pirrt_rrg* R) {
  rfree(R->okind); rfree(R->ocentre); rfree(R->osize); rfree(R->pts); rfree(R->cbuf); rfree(R->flag); rfree(R->pos);
  rfree(R->cnt); rfree(R->cptr); rfree(R->cand_u); rfree(R->cand_v); rfree(R->keep); rfree(R->kpos); rfree(R->ccost);
  rfree(R->rp); rfree(R->col); rfree(R->cost); rfree(R->hbuf); rfree(R->dword); rfree(R->dflag);
  rfree(R->lpts); rfree(R->lfeat); rfree(R->llogit); rfree(R->lenc); rfree(R->lflag); rfree(R->lsel);
  if (R->scan) (void)hipFree(R->scan);
  R->scan = nullptr;
  if (R->host) (void)hipHostFree(R->host);
  R->host = nullptr;
}

}  // namespace

extern "C" {

int pirrt_rrg_create(pirrt_rrg** out, const pirrt_rrg_config* cfg) {
  if (!out || !cfg) return PIRRT_EINVAL;
  *out = nullptr;
  if (cfg->d < 1 || cfg->d > kMaxDim || cfg->n_obstacles < 0 || cfg->point_capacity < 0) {
    g_rrg_create_error = "d outside 1..8 or negative count";
    return PIRRT_EINVAL;
  }
  const int d = cfg->d, m = cfg->n_obstacles;
  if (m > 0 && (!cfg->kind || !cfg->centre || !cfg->size)) {
    g_rrg_create_error = "obstacle arrays are NULL";
    return PIRRT_EINVAL;
  }
  for (int o = 0; o < m; ++o) {
    if (cfg->kind[o] != 0 && cfg->kind[o] != 1) {
      g_rrg_create_error = "obstacle kind must be 0 (sphere) or 1 (box)";
      return PIRRT_EINVAL;
    }
    for (int k = 0; k < d; ++k) {
      const double c = cfg->centre[(int64_t)o * d + k], s = cfg->size[(int64_t)o * d + k];
      if (!std::isfinite(c) || !std::isfinite(s) || ((cfg->kind[o] == 1 || k == 0) && s < 0.0)) {
        g_rrg_create_error = "obstacle centre or size not finite, or negative size";
        return PIRRT_EINVAL;
      }
    }
  }
  pirrt_rrg* R = new (std::nothrow) pirrt_rrg();
  if (!R) return PIRRT_ENOMEM;
  int dev = cfg->device;
  if (dev < 0 && hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    delete R;
    g_rrg_create_error = "no HIP device";
    return PIRRT_EDEVICE;
  }
  if (hipSetDevice(dev) != hipSuccess) {
    (void)hipGetLastError();
    delete R;
    g_rrg_create_error = "hipSetDevice failed";
    return PIRRT_EDEVICE;
  }
  R->device = dev;
  R->stream = (hipStream_t)cfg->hip_stream;
  R->d = d;
  R->nobs = m;
  bool ok = ralloc(&R->okind, m) && ralloc(&R->ocentre, (int64_t)m * d) && ralloc(&R->osize, (int64_t)m * d) &&
            ralloc(&R->dword, 1) && ralloc(&R->dflag, 1);
  if (ok && hipHostMalloc((void**)&R->host, 4 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    R->host = nullptr;
    ok = false;
  }
  if (ok && m > 0)
    ok = hipMemcpy(R->okind, cfg->kind, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(R->ocentre, cfg->centre, sizeof(double) * (size_t)m * d, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(R->osize, cfg->size, sizeof(double) * (size_t)m * d, hipMemcpyHostToDevice) == hipSuccess;
  if (ok && cfg->point_capacity > 0) ok = grow(R, &R->pts, &R->cap, cfg->point_capacity * d, 0) == PIRRT_OK;
  if (!ok) {
    (void)hipGetLastError();
    release(R);
    delete R;
    g_rrg_create_error = "device allocation failed at create";
    return PIRRT_ENOMEM;
  }
  *out = R;
  return PIRRT_OK;
}

int pirrt_rrg_destroy(pirrt_rrg* R) {
  if (!R) return PIRRT_OK;
  (void)hipSetDevice(R->device);
  if (!R->poisoned) (void)hipStreamSynchronize(R->stream);
  release(R);
  delete R;
  return PIRRT_OK;
}

int64_t pirrt_rrg_num_points(const pirrt_rrg* R) { return R ? R->n : -1; }

const char* pirrt_rrg_last_error(const pirrt_rrg* R) { return R ? R->err.c_str() : g_rrg_create_error.c_str(); }

int pirrt_rrg_add_points(pirrt_rrg* R, int32_t count, const double* pts, int mem_kind) {
  int rc = rguard(R);
  if (rc) return rc;
  if (mem_kind != PIRRT_MEM_HOST && mem_kind != PIRRT_MEM_DEVICE) return rfail(R, PIRRT_EINVAL, "bad mem_kind");
  if (count < 0) return rfail(R, PIRRT_EINVAL, "count < 0");
  if (count == 0) return PIRRT_OK;
  if (!pts) return rfail(R, PIRRT_EINVAL, "pts is NULL");
  if (R->n + count > (int64_t)INT32_MAX - 1) return rfail(R, PIRRT_EINVAL, "point ids beyond INT32_MAX");
  const int64_t m = (int64_t)count * R->d;
  if (mem_kind == PIRRT_MEM_HOST) {
    for (int64_t i = 0; i < m; ++i)
      if (!std::isfinite(pts[i])) return rfail(R, PIRRT_EINVAL, "point coordinate not finite");
  }
  if ((rc = grow(R, &R->pts, &R->cap, (R->n + count) * R->d, R->n * R->d))) return rc;
  RHIP(R, hipMemcpyAsync(R->pts + R->n * R->d, pts, sizeof(double) * (size_t)m,
                         mem_kind == PIRRT_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, R->stream));
  if (mem_kind == PIRRT_MEM_DEVICE) {
    RHIP(R, hipMemsetAsync(R->dflag, 0, sizeof(int32_t), R->stream));
    hipLaunchKernelGGL(k_check_points, dim3(blocks(m)), dim3(kThreads), 0, R->stream, m, R->pts + R->n * R->d,
                       R->dflag);
    RHIP(R, hipGetLastError());
    RHIP(R, hipMemcpyAsync(R->host, R->dflag, sizeof(int32_t), hipMemcpyDeviceToHost, R->stream));
  }
  RHIP(R, hipStreamSynchronize(R->stream));
  if (mem_kind == PIRRT_MEM_DEVICE && *(int32_t*)R->host) return rfail(R, PIRRT_EINVAL, "point coordinate not finite");
  R->n += count;
  return PIRRT_OK;
}

int pirrt_rrg_sample(pirrt_rrg* R, uint64_t seed, uint32_t stream_id, uint64_t* counter, int32_t count) {
  int rc = rguard(R);
  if (rc) return rc;
  if (!counter) return rfail(R, PIRRT_EINVAL, "counter is NULL");
  if (count < 0) return rfail(R, PIRRT_EINVAL, "count < 0");
  if (R->n + count > (int64_t)INT32_MAX - 1) return rfail(R, PIRRT_EINVAL, "point ids beyond INT32_MAX");
  if (count == 0) return PIRRT_OK;
  if ((rc = grow(R, &R->pts, &R->cap, (R->n + count) * R->d, R->n * R->d))) return rc;
  if ((rc = draw_free(R, seed, stream_id, counter, count, R->pts + R->n * R->d))) return rc;
  R->n += count;
  return PIRRT_OK;
}

int pirrt_rrg_sample_learned(pirrt_rrg* R, pirrt_mlp* net, const float* enc, int32_t enc_len, uint64_t seed,
                             uint32_t stream_id, uint64_t* counter, int32_t n_candidates, int32_t count) {
  int rc = rguard(R);
  if (rc) return rc;
  if (!net || !counter) return rfail(R, PIRRT_EINVAL, "net or counter is NULL");
  if (n_candidates < 1 || n_candidates > kSelMax) return rfail(R, PIRRT_EINVAL, "n_candidates outside 1..8192");
  if (count < 0 || count > n_candidates) return rfail(R, PIRRT_EINVAL, "count outside 0..n_candidates");
  if (enc_len < 0 || (enc_len > 0 && !enc)) return rfail(R, PIRRT_EINVAL, "bad encoding");
  const int d = R->d;
  const int32_t in_dim = d + enc_len;
  if (pirrt_mlp_in_dim(net) != in_dim) return rfail(R, PIRRT_EINVAL, "d + enc_len differs from the network's in_dim");
  if (R->n + count > (int64_t)INT32_MAX - 1) return rfail(R, PIRRT_EINVAL, "point ids beyond INT32_MAX");
  if (count == 0) return PIRRT_OK;
  if (!R->lpts) {
    if (!ralloc(&R->lpts, (int64_t)kSelMax * kMaxDim) || !ralloc(&R->lfeat, (int64_t)kSelMax * 288) ||
        !ralloc(&R->llogit, kSelMax) || !ralloc(&R->lenc, 288) || !ralloc(&R->lflag, kSelMax) ||
        !ralloc(&R->lsel, kSelMax))
      return rfail(R, PIRRT_ENOMEM, "device allocation of the learned sampler failed");
  }
  if ((rc = grow(R, &R->pts, &R->cap, (R->n + count) * d, R->n * d))) return rc;
  uint64_t k = *counter;
  if ((rc = draw_free(R, seed, stream_id, &k, n_candidates, R->lpts))) return rc;
  hipStream_t s = R->stream;
  if (enc_len > 0)
    RHIP(R, hipMemcpyAsync(R->lenc, enc, sizeof(float) * (size_t)enc_len, hipMemcpyHostToDevice, s));
#define FEAT(D)                                                                                               \
  hipLaunchKernelGGL(k_features<D>, dim3(blocks((int64_t)n_candidates * in_dim)), dim3(kThreads), 0, s, n_candidates, \
                     R->lpts, R->lenc, in_dim, R->lfeat)
  PIRRT_BY_DIM(d, FEAT);
#undef FEAT
  RHIP(R, hipGetLastError());
  RHIP(R, hipStreamSynchronize(s));
  rc = pirrt_mlp_forward(net, n_candidates, R->lfeat, R->llogit, PIRRT_MEM_DEVICE);
  if (rc) return rfail(R, rc, std::string("pirrt_mlp_forward: ") + pirrt_mlp_last_error(net));
  hipLaunchKernelGGL(k_select_top, dim3(1), dim3(kSelThreads), 0, s, n_candidates, count, R->llogit, R->lflag,
                     R->lsel);
  RHIP(R, hipGetLastError());
  double* dst = R->pts + R->n * d;
#define GATHER(D)                                                                                                \
  hipLaunchKernelGGL(k_gather_points<D>, dim3(blocks((int64_t)count * D)), dim3(kThreads), 0, s, count, R->lsel, \
                     R->lpts, dst)
  PIRRT_BY_DIM(d, GATHER);
#undef GATHER
  RHIP(R, hipGetLastError());
  RHIP(R, hipStreamSynchronize(s));
  R->n += count;
  *counter = k;
  return PIRRT_OK;
}

int pirrt_rrg_get_points(pirrt_rrg* R, int64_t first, int64_t count, double* out, int mem_kind) {
  int rc = rguard(R);
  if (rc) return rc;
  if (mem_kind != PIRRT_MEM_HOST && mem_kind != PIRRT_MEM_DEVICE) return rfail(R, PIRRT_EINVAL, "bad mem_kind");
  if (first < 0 || count < 0 || first + count > R->n) return rfail(R, PIRRT_EINVAL, "range outside the points");
  if (count == 0) return PIRRT_OK;
  if (!out) return rfail(R, PIRRT_EINVAL, "out is NULL");
  RHIP(R, hipMemcpyAsync(out, R->pts + first * R->d, sizeof(double) * (size_t)(count * R->d),
                         mem_kind == PIRRT_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, R->stream));
  RHIP(R, hipStreamSynchronize(R->stream));
  return PIRRT_OK;
}

int pirrt_rrg_rows(pirrt_rrg* R, int64_t n_old, double radius, int64_t* row_ptr, int32_t* col, float* cost,
                   int64_t capacity, int64_t* nnz, int mem_kind) {
  int rc = rguard(R);
  if (rc) return rc;
  if (mem_kind != PIRRT_MEM_HOST && mem_kind != PIRRT_MEM_DEVICE) return rfail(R, PIRRT_EINVAL, "bad mem_kind");
  if (n_old < 0 || n_old > R->n) return rfail(R, PIRRT_EINVAL, "n_old outside 0..n");
  if (!(radius > 0.0) || !std::isfinite(radius)) return rfail(R, PIRRT_EINVAL, "radius must be finite and > 0");
  if (!nnz || !row_ptr) return rfail(R, PIRRT_EINVAL, "nnz or row_ptr is NULL");
  int64_t m = 0;
  if ((rc = build_rows(R, n_old, radius, &m))) return rc;
  *nnz = m;
  if (m > capacity) return rfail(R, PIRRT_EINVAL, "capacity below the entry count (returned in *nnz)");
  const hipMemcpyKind kind = mem_kind == PIRRT_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  RHIP(R, hipMemcpyAsync(row_ptr, R->rp, sizeof(int64_t) * (size_t)(R->n - n_old + 1), kind, R->stream));
  if (m > 0 && col) RHIP(R, hipMemcpyAsync(col, R->col, sizeof(int32_t) * (size_t)m, kind, R->stream));
  if (m > 0 && cost) RHIP(R, hipMemcpyAsync(cost, R->cost, sizeof(float) * (size_t)m, kind, R->stream));
  RHIP(R, hipStreamSynchronize(R->stream));
  return PIRRT_OK;
}

int pirrt_rrg_connect(pirrt_rrg* R, int64_t n_old, double radius, pirrt_graph* g) {
  int rc = rguard(R);
  if (rc) return rc;
  if (!g) return rfail(R, PIRRT_EINVAL, "graph is NULL");
  if (pirrt_num_vertices(g) != n_old || n_old > R->n) return rfail(R, PIRRT_EINVAL, "the graph must hold points [0, n_old)");
  if (!(radius > 0.0) || !std::isfinite(radius)) return rfail(R, PIRRT_EINVAL, "radius must be finite and > 0");
  if (n_old == R->n) return PIRRT_OK;
  int64_t m = 0;
  if ((rc = build_rows(R, n_old, radius, &m))) return rc;
  rc = pirrt_insert_batch(g, (int32_t)(R->n - n_old), R->rp, R->col, R->cost, PIRRT_MEM_DEVICE);
  if (rc) return rfail(R, rc, std::string("pirrt_insert_batch: ") + pirrt_last_error(g));
  return PIRRT_OK;
}

int pirrt_rrg_connect_problem(pirrt_rrg* R, double radius, pirrt_batch* b, int32_t* index) {
  int rc = rguard(R);
  if (rc) return rc;
  if (!b) return rfail(R, PIRRT_EINVAL, "batch is NULL");
  if (R->n < 1) return rfail(R, PIRRT_EINVAL, "no points");
  if (!(radius > 0.0) || !std::isfinite(radius)) return rfail(R, PIRRT_EINVAL, "radius must be finite and > 0");
  int64_t m = 0;
  if ((rc = build_rows(R, 0, radius, &m))) return rc;
  rc = pirrt_batch_add_problem(b, (int32_t)R->n, R->rp, R->col, R->cost, PIRRT_MEM_DEVICE, index);
  if (rc) return rfail(R, rc, std::string("pirrt_batch_add_problem: ") + pirrt_batch_last_error(b));
  return PIRRT_OK;
}

int pirrt_rrg_heuristic(pirrt_rrg* R, int64_t goal, float* h_out, int mem_kind) {
  int rc = rguard(R);
  if (rc) return rc;
  if (mem_kind != PIRRT_MEM_HOST && mem_kind != PIRRT_MEM_DEVICE) return rfail(R, PIRRT_EINVAL, "bad mem_kind");
  if (goal < 0 || goal >= R->n) return rfail(R, PIRRT_EINVAL, "goal outside the points");
  if (!h_out) return rfail(R, PIRRT_EINVAL, "h_out is NULL");
  float* dst = h_out;
  if (mem_kind == PIRRT_MEM_HOST) {
    if ((rc = grow(R, &R->hbuf, &R->hcap, R->n, 0))) return rc;
    dst = R->hbuf;
  }
  const double* gp = R->pts + goal * R->d;
#define HEUR(D) launch_heuristic<D>(R, gp, dst)
  PIRRT_BY_DIM(R->d, HEUR);
#undef HEUR
  RHIP(R, hipGetLastError());
  if (mem_kind == PIRRT_MEM_HOST)
    RHIP(R, hipMemcpyAsync(h_out, R->hbuf, sizeof(float) * (size_t)R->n, hipMemcpyDeviceToHost, R->stream));
  RHIP(R, hipStreamSynchronize(R->stream));
  return PIRRT_OK;
}

}  // extern "C"
