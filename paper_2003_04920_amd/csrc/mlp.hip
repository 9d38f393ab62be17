// The learned sampling proposal's network on the device: features (sample
// coordinates + obstacle encoding, zero-padded to K = 288) -> 256 -> 256 -> 1 logit,
// ReLU hidden layers, bfloat16 operands with binary32 accumulation on MFMA, binary32
// master parameters, BCE-with-logits loss, Adam (Kingma and Ba, 2015).
//
// Rounding points (the contract the oracle states): X = bf16(f); A1 = bf16(relu(Z1));
// A2 = bf16(relu(Z2)); weights used by products are bf16 copies of the binary32
// masters; dZ2 = bf16(dz w3^T * [Z2 > 0]); dZ1 = bf16(dZ2 W2^T * [Z1 > 0]).
//
// Every matrix product is one MFMA kernel: a workgroup of four waves owns a 64 x 64
// output tile, each wave a 32 x 32 block accumulated by v_mfma_f32_32x32x16_bf16 over
// K in steps of 16.  Operands are read through strides, so the transposed products of
// the backward pass (A1^T dZ2, X^T dZ1, dZ2 W2^T) need no transposed copies; a
// contiguous K run is fetched with one 16-byte load per lane.
#include <string.h>

#include <cmath>
#include <mutex>
#include <string>

#include "internal.h"
#include "pirrt.h"

using namespace pirrt;

static __device__ __align__(256) uint16_t scratch[(PIRRT_MLP_NOALLOC_MAX_BATCH) * (288 + 2 * 256)];

namespace {

constexpr int kIn = 288;      // padded input width (a multiple of 16)
constexpr int kHidden = 256;  // hidden width
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + (int64_t)kIn * kHidden;
constexpr int64_t kOffW2 = kOffB1 + kHidden;
constexpr int64_t kOffB2 = kOffW2 + (int64_t)kHidden * kHidden;
constexpr int64_t kOffW3 = kOffB2 + kHidden;
constexpr int64_t kOffB3 = kOffW3 + kHidden;
constexpr int64_t kNumParams = kOffB3 + 1;
constexpr int kThreads = 256;

// Scratch of pirrt_mlp_forward_noalloc: the staged bf16 features X [kNoAllocRows x kIn]
// followed by the bf16 activations A1 and A2 [kNoAllocRows x kHidden each], 12.5 MiB.
// Each GPU the library runs on holds its own copy until the process ends.  Host code
// never passes this name to a kernel: it uses the device address that
// hipGetSymbolAddress returns for the current GPU (noalloc_scratch below).
constexpr int32_t kNoAllocRows = PIRRT_MLP_NOALLOC_MAX_BATCH;  // a multiple of 64
constexpr int64_t kScratchX = 0;
constexpr int64_t kScratchA1 = kScratchX + (int64_t)kNoAllocRows * kIn;
constexpr int64_t kScratchA2 = kScratchA1 + (int64_t)kNoAllocRows * kHidden;
constexpr int64_t kScratchElems = kScratchA2 + (int64_t)kNoAllocRows * kHidden;
static_assert(kNoAllocRows % 64 == 0, "rows are padded to 64");
static_assert(sizeof(scratch) == sizeof(uint16_t) * (size_t)kScratchElems, "scratch layout");
static_assert((kScratchA1 * 2) % 256 == 0 && (kScratchA2 * 2) % 256 == 0, "each part stays 256-byte aligned");

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (no NaN reaches here)
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

enum Epi { kEpiFwd = 0, kEpiMaskBf16 = 1, kEpiF32 = 2 };

struct GemmArgs {
  int32_t M, N, K;
  const uint16_t* A;  // element (m, k) at A[m * sam + k * sak]
  int64_t sam, sak;
  const uint16_t* B;  // element (k, n) at B[k * sbk + n * sbn]
  int64_t sbk, sbn;
  const float* bias;  // kEpiFwd: per column
  const float* zref;  // kEpiMaskBf16: fp32 [M x N] whose sign gates the output
  float* zout;        // kEpiFwd: fp32 pre-activation [M x N] (nullable); kEpiF32: output
  uint16_t* bout;     // kEpiFwd / kEpiMaskBf16: bf16 output [M x N]
  int64_t kchunk;     // split K: workgroup z sums k in [z * kchunk, (z + 1) * kchunk) and
                      // kEpiF32 writes its partial product to zout + z * M * N
};

template <bool kAContig>
__device__ __forceinline__ bf16x8 load_a(const GemmArgs& g, int64_t m, int64_t k) {
  if (kAContig) {
    const uint4 w = *reinterpret_cast<const uint4*>(g.A + m * g.sam + k);
    return __builtin_bit_cast(bf16x8, w);
  }
  uint16_t t[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) t[i] = g.A[m * g.sam + (k + i) * g.sak];
  return __builtin_bit_cast(bf16x8, t);
}

template <bool kBContig>
__device__ __forceinline__ bf16x8 load_b(const GemmArgs& g, int64_t k, int64_t n) {
  if (kBContig) {
    const uint4 w = *reinterpret_cast<const uint4*>(g.B + n * g.sbn + k);
    return __builtin_bit_cast(bf16x8, w);
  }
  uint16_t t[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) t[i] = g.B[(k + i) * g.sbk + n * g.sbn];
  return __builtin_bit_cast(bf16x8, t);
}

// One 32 x 32 output block per wave.  Lane l supplies A row l % 32 and B column
// l % 32 with the 8 consecutive K entries starting at 8 * (l / 32); accumulator
// register r of lane l holds row 8 * (r / 4) + 4 * (l / 32) + r % 4, column l % 32.
template <bool kAContig, bool kBContig, int kEpi>
__global__ void __launch_bounds__(kThreads) k_gemm(GemmArgs g) {
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int64_t m0 = (int64_t)blockIdx.y * 64 + (wave >> 1) * 32;
  const int64_t n0 = (int64_t)blockIdx.x * 64 + (wave & 1) * 32;
  if (m0 >= g.M || n0 >= g.N) return;  // whole wave outside (M, N are multiples of 32)
  const int64_t am = m0 + (lane & 31), bn = n0 + (lane & 31);
  const int kq = (lane >> 5) * 8;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  const int64_t k0 = (int64_t)blockIdx.z * g.kchunk;
  const int64_t k1 = k0 + g.kchunk < g.K ? k0 + g.kchunk : g.K;
  for (int64_t k = k0; k < k1; k += 16) {
    const bf16x8 a = load_a<kAContig>(g, am, k + kq);
    const bf16x8 b = load_b<kBContig>(g, k + kq, bn);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  const int64_t col = n0 + (lane & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t row = m0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    const int64_t o = row * g.N + col;
    if (kEpi == kEpiFwd) {
      const float v = acc[r] + g.bias[col];
      if (g.zout) g.zout[o] = v;
      g.bout[o] = to_bf16(v > 0.0f ? v : 0.0f);
    } else if (kEpi == kEpiMaskBf16) {
      g.bout[o] = to_bf16(g.zref[o] > 0.0f ? acc[r] : 0.0f);
    } else {
      g.zout[(int64_t)blockIdx.z * g.M * g.N + o] = acc[r];
    }
  }
}

// X = bf16(features), zero-padded to kIn columns and Bp rows.
__global__ void k_features(int32_t B, int32_t Bp, int32_t in_dim, const float* __restrict__ x,
                           uint16_t* __restrict__ X) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)Bp * kIn) return;
  const int64_t b = i / kIn, k = i % kIn;
  X[i] = (b < B && k < in_dim) ? to_bf16(x[b * in_dim + k]) : (uint16_t)0;
}

// z = A2 w3 + b3 per row (one thread per row, k ascending); with labels also
// dz = (sigmoid(z) - y) / B and the workgroup's loss sum (rows in order) in lpart.
// Without labels only rows b < B of z are written (z may be the caller's logits).
__global__ void __launch_bounds__(kThreads) k_layer3(int32_t B, int32_t Bp, const uint16_t* __restrict__ A2,
                                                     const uint16_t* __restrict__ w3b, const float* __restrict__ P,
                                                     const float* __restrict__ y, float* __restrict__ z,
                                                     float* __restrict__ dz, float* __restrict__ lpart) {
  __shared__ float wl[kHidden];
  __shared__ float red[kThreads];
  for (int k = threadIdx.x; k < kHidden; k += kThreads) wl[k] = from_bf16(w3b[k]);
  __syncthreads();
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.0f;
  if (b < Bp) {
    const uint4* row = reinterpret_cast<const uint4*>(A2 + b * kHidden);
    float s = 0.0f;
    for (int q = 0; q < kHidden / 8; ++q) {
      const uint4 w = row[q];
      const uint32_t h[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        s += __uint_as_float(h[e] << 16) * wl[8 * q + 2 * e];
        s += __uint_as_float(h[e] & 0xffff0000u) * wl[8 * q + 2 * e + 1];
      }
    }
    const float zb = s + P[kOffB3];
    if (y || b < B) z[b] = zb;  // a forward pass writes the B logits only
    if (y) {
      if (b < B) {
        const float yb = y[b];
        dz[b] = (1.0f / (1.0f + expf(-zb)) - yb) / (float)B;
        l = (fmaxf(zb, 0.0f) - zb * yb + log1pf(expf(-fabsf(zb)))) / (float)B;
      } else {
        dz[b] = 0.0f;
      }
    }
  }
  if (!y) return;
  red[threadIdx.x] = l;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int i = 0; i < kThreads; ++i) t += red[i];
    lpart[blockIdx.x] = t;
  }
}

// dZ2 = bf16(dz w3^T * [Z2 > 0])
__global__ void k_dz2(int32_t Bp, const float* __restrict__ dz, const uint16_t* __restrict__ w3b,
                      const float* __restrict__ Z2, uint16_t* __restrict__ dZ2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)Bp * kHidden) return;
  const int64_t b = i / kHidden, k = i % kHidden;
  dZ2[i] = to_bf16(Z2[i] > 0.0f ? dz[b] * from_bf16(w3b[k]) : 0.0f);
}

// out[n] = sum over rows of a bf16 [rows x N] matrix (one thread per column).
// Column sums over the batch in two fixed-order stages (the same bits on every run):
// workgroup (c, j) sums rows [j * rows_per, (j + 1) * rows_per) of 64 columns, four
// row phases per column then the phases in order, into part[j][col]; k_sum_parts then
// adds the kColParts partials of each column in order.  Column N (when `ones`) is the
// all-ones column, and `w` (nullable) weights the rows: sum_b w[b] M[b][col].
constexpr int kColParts = 64;
constexpr int kSplitK = 32;  // K splits of the weight-gradient products

__global__ void __launch_bounds__(kThreads) k_colsum_part(int32_t rows, int32_t rows_per, int32_t N, bool ones,
                                                         const uint16_t* __restrict__ M,
                                                         const float* __restrict__ w, float* __restrict__ part) {
  __shared__ float red[4][64];
  const int c = threadIdx.x & 63, ph = threadIdx.x >> 6;
  const int col = blockIdx.x * 64 + c;
  const int ncol = N + (ones ? 1 : 0);
  const int64_t r0 = (int64_t)blockIdx.y * rows_per;
  const int64_t r1 = r0 + rows_per < rows ? r0 + rows_per : rows;
  float s = 0.0f;
  if (col < ncol) {
    for (int64_t r = r0 + ph; r < r1; r += 4) {
      const float x = col < N ? from_bf16(M[r * N + col]) : 1.0f;
      s += w ? x * w[r] : x;
    }
  }
  red[ph][c] = s;
  __syncthreads();
  if (ph == 0 && col < ncol) part[(int64_t)blockIdx.y * ncol + col] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

// out[i] = sum over z < parts of part[z * count + i], in order of z (four outputs per
// thread, eight partials in flight).
__global__ void k_sum_parts(int64_t count, int32_t parts, const float* __restrict__ part, float* __restrict__ out) {
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i0 >= count) return;
  const int nv = count - i0 < 4 ? (int)(count - i0) : 4;
  float s[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  int32_t z = 0;
  for (; z + 8 <= parts; z += 8) {
    float v[8][4];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int j = 0; j < 4; ++j) v[u][j] = j < nv ? part[(int64_t)(z + u) * count + i0 + j] : 0.0f;
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int j = 0; j < 4; ++j) s[j] += v[u][j];
  }
  for (; z < parts; ++z)
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j] += j < nv ? part[(int64_t)z * count + i0 + j] : 0.0f;
  for (int j = 0; j < nv; ++j) out[i0 + j] = s[j];
}

__global__ void k_adam(int64_t np, float* __restrict__ P, const float* __restrict__ G, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const float g = G[i];
  const float mi = b1 * m[i] + (1.0f - b1) * g;
  const float vi = b2 * v[i] + (1.0f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// bf16 copies of the weights: W2b row-major (the backward product dZ2 W2^T reads its
// rows contiguously), W1t / W2t transposed (the forward products read their columns
// contiguously).
__global__ void k_refresh(const float* __restrict__ P, uint16_t* __restrict__ W1t, uint16_t* __restrict__ W2b,
                          uint16_t* __restrict__ W2t, uint16_t* __restrict__ w3b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)kIn * kHidden) {
    const int64_t k = i / kHidden, n = i % kHidden;
    W1t[n * kIn + k] = to_bf16(P[kOffW1 + i]);
  }
  if (i < (int64_t)kHidden * kHidden) {
    const int64_t k = i / kHidden, n = i % kHidden;
    const uint16_t b = to_bf16(P[kOffW2 + i]);
    W2b[i] = b;
    W2t[n * kHidden + k] = b;
  }
  if (i < kHidden) w3b[i] = to_bf16(P[kOffW3 + i]);
}

inline unsigned nblocks(int64_t n, int per = kThreads) { return (unsigned)((n + per - 1) / per > 0 ? (n + per - 1) / per : 1); }

}  // namespace

struct pirrt_mlp {
  int device = 0;
  hipStream_t stream = nullptr;
  int32_t in_dim = 0, max_batch = 0, bcap = 0;
  float lr = 1e-3f, beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  int64_t t = 0;
  float* P = nullptr;
  float* G = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  uint16_t* W1t = nullptr;  // bf16 W1 transposed [kHidden x kIn]
  uint16_t* W2b = nullptr;  // bf16 W2 [kHidden x kHidden]
  uint16_t* W2t = nullptr;  // bf16 W2 transposed
  uint16_t* w3b = nullptr;
  float* xin = nullptr;   // staging of host features
  float* yin = nullptr;
  uint16_t* X = nullptr;
  float* Z1 = nullptr;
  uint16_t* A1 = nullptr;
  float* Z2 = nullptr;
  uint16_t* A2 = nullptr;
  float* z = nullptr;
  float* dz = nullptr;
  uint16_t* dZ2 = nullptr;
  uint16_t* dZ1 = nullptr;
  float* dloss = nullptr;
  float* part = nullptr;   // partial sums of the split reductions
  float* hloss = nullptr;  // pinned
  bool poisoned = false;
  std::string err;
};

namespace {

thread_local std::string g_mlp_create_error;

int mfail(pirrt_mlp* N, int code, const std::string& m) {
  N->err = m;
  return code;
}

int mdev(pirrt_mlp* N, hipError_t e, const char* what) {
  N->poisoned = true;
  N->err = std::string("HIP error in ") + what + ": " + hipGetErrorString(e);
  return PIRRT_EDEVICE;
}

#define MHIP(N, expr)                                 \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return mdev(N, e_, #expr);  \
  } while (0)

template <class T>
bool malloc_dev(T** p, int64_t count) {
  *p = nullptr;
  if (hipMalloc((void**)p, sizeof(T) * (size_t)(count > 0 ? count : 1)) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return false;
  }
  return true;
}

template <class T>
void free_dev(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

void release(pirrt_mlp* N) {
  free_dev(N->P); free_dev(N->G); free_dev(N->m); free_dev(N->v); free_dev(N->W1t); free_dev(N->W2b);
  free_dev(N->W2t);
  free_dev(N->w3b); free_dev(N->xin); free_dev(N->yin); free_dev(N->X); free_dev(N->Z1); free_dev(N->A1);
  free_dev(N->Z2); free_dev(N->A2); free_dev(N->z); free_dev(N->dz); free_dev(N->dZ2); free_dev(N->dZ1);
  free_dev(N->dloss);
  free_dev(N->part);
  if (N->hloss) (void)hipHostFree(N->hloss);
  N->hloss = nullptr;
}

int mguard(pirrt_mlp* N) {
  if (!N) return PIRRT_EINVAL;
  if (N->poisoned) return PIRRT_EDEVICE;
  hipError_t e = hipSetDevice(N->device);
  if (e != hipSuccess) return mdev(N, e, "hipSetDevice");
  return PIRRT_OK;
}

void launch_gemm(const GemmArgs& g, bool a_contig, bool b_contig, int epi, hipStream_t s, int splits = 1) {
  const dim3 grid((unsigned)((g.N + 63) / 64), (unsigned)((g.M + 63) / 64), (unsigned)splits);
#define GEMM(AC, BC, E) hipLaunchKernelGGL((k_gemm<AC, BC, E>), grid, dim3(kThreads), 0, s, g)
  if (epi == kEpiFwd) {
    if (a_contig && b_contig) GEMM(true, true, kEpiFwd); else GEMM(true, false, kEpiFwd);
  } else if (epi == kEpiMaskBf16) {
    GEMM(true, true, kEpiMaskBf16);
  } else {
    if (a_contig) GEMM(true, false, kEpiF32); else GEMM(false, false, kEpiF32);
  }
#undef GEMM
}

// Deterministic column sums of a bf16 [rows x cols] matrix (see k_colsum_part) into out.
void launch_colsum(pirrt_mlp* N, int32_t rows, int32_t cols, bool ones, const uint16_t* M, const float* w,
                   float* out) {
  const int32_t ncol = cols + (ones ? 1 : 0);
  const int32_t per = (rows + kColParts - 1) / kColParts;
  hipLaunchKernelGGL(k_colsum_part, dim3((unsigned)((ncol + 63) / 64), kColParts), dim3(kThreads), 0, N->stream, rows,
                     per, cols, ones, M, w, N->part);
  hipLaunchKernelGGL(k_sum_parts, dim3(nblocks((ncol + 3) / 4)), dim3(kThreads), 0, N->stream, (int64_t)ncol,
                     kColParts, N->part, out);
}

// A weight gradient (M x N, K = the batch): the K range is split over kSplitK
// workgroup layers (an output tile alone would leave most of the chip idle), the
// partial products go to N->part and are added in split order.
void launch_weight_grad(pirrt_mlp* N, GemmArgs g, float* out) {
  const int64_t kc = ((g.K + kSplitK - 1) / kSplitK + 15) / 16 * 16;
  const int splits = (int)((g.K + kc - 1) / kc);
  g.kchunk = kc;
  g.zout = N->part;
  launch_gemm(g, false, false, kEpiF32, N->stream, splits);
  hipLaunchKernelGGL(k_sum_parts, dim3(nblocks(((int64_t)g.M * g.N + 3) / 4)), dim3(kThreads), 0, N->stream,
                     (int64_t)g.M * g.N, splits, N->part, out);
}

// Features into X (padded rows and columns are zero); B rows, Bp = B rounded up to 64.
int stage_inputs(pirrt_mlp* N, int32_t B, int32_t Bp, const float* x, const float* y, int mem_kind,
                 const float** yd) {
  hipStream_t s = N->stream;
  const float* xd = x;
  *yd = y;
  if (mem_kind == PIRRT_MEM_HOST) {
    MHIP(N, hipMemcpyAsync(N->xin, x, sizeof(float) * (size_t)B * N->in_dim, hipMemcpyHostToDevice, s));
    xd = N->xin;
    if (y) {
      MHIP(N, hipMemcpyAsync(N->yin, y, sizeof(float) * (size_t)B, hipMemcpyHostToDevice, s));
      *yd = N->yin;
    }
  }
  hipLaunchKernelGGL(k_features, dim3(nblocks((int64_t)Bp * kIn)), dim3(kThreads), 0, s, B, Bp, N->in_dim, xd, N->X);
  MHIP(N, hipGetLastError());
  return PIRRT_OK;
}

// X [Bp x kIn] -> A1 -> A2 ([Bp x kHidden] each, bf16); keep_z also stores the fp32
// pre-activations in the handle's Z1 / Z2 for the backward pass.
void enqueue_forward(pirrt_mlp* N, int32_t Bp, bool keep_z, const uint16_t* X, uint16_t* A1, uint16_t* A2) {
  hipStream_t s = N->stream;
  // element (k, n) of W1 is W1t[n * kIn + k]: contiguous in k
  GemmArgs g1{Bp, kHidden, kIn, X, kIn, 1, N->W1t, 1, kIn, N->P + kOffB1, nullptr, keep_z ? N->Z1 : nullptr,
              A1, kIn};
  launch_gemm(g1, true, true, kEpiFwd, s);
  GemmArgs g2{Bp, kHidden, kHidden, A1, kHidden, 1, N->W2t, 1, kHidden, N->P + kOffB2, nullptr,
              keep_z ? N->Z2 : nullptr, A2, kHidden};
  launch_gemm(g2, true, true, kEpiFwd, s);
}

// Forward + loss + gradients into N->G (the loss lands in N->dloss).
int enqueue_gradients(pirrt_mlp* N, int32_t B, int32_t Bp, const float* yd) {
  hipStream_t s = N->stream;
  enqueue_forward(N, Bp, true, N->X, N->A1, N->A2);
  const unsigned nb3 = nblocks(Bp);
  hipLaunchKernelGGL(k_layer3, dim3(nb3), dim3(kThreads), 0, s, B, Bp, N->A2, N->w3b, N->P, yd, N->z, N->dz,
                     N->part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kThreads), 0, s, (int64_t)1, (int32_t)nb3, N->part, N->dloss);
  // gw3 = A2^T dz and gb3 = sum dz: the weighted column sums of [A2 | 1]
  launch_colsum(N, Bp, kHidden, true, N->A2, N->dz, N->G + kOffW3);
  hipLaunchKernelGGL(k_dz2, dim3(nblocks((int64_t)Bp * kHidden)), dim3(kThreads), 0, s, Bp, N->dz, N->w3b, N->Z2,
                     N->dZ2);
  launch_colsum(N, Bp, kHidden, false, N->dZ2, nullptr, N->G + kOffB2);
  // gW2[i][j] = sum_b A1[b][i] dZ2[b][j]
  GemmArgs gw2{kHidden, kHidden, Bp, N->A1, 1, kHidden, N->dZ2, kHidden, 1, nullptr, nullptr, nullptr, nullptr, 0};
  launch_weight_grad(N, gw2, N->G + kOffW2);
  // dZ1 = bf16(dZ2 W2^T * [Z1 > 0]): element (k = j, n = i) of W2^T is W2b[i][j]
  GemmArgs gd1{Bp, kHidden, kHidden, N->dZ2, kHidden, 1, N->W2b, 1, kHidden, nullptr, N->Z1, nullptr, N->dZ1, kHidden};
  launch_gemm(gd1, true, true, kEpiMaskBf16, s);
  launch_colsum(N, Bp, kHidden, false, N->dZ1, nullptr, N->G + kOffB1);
  // gW1[i][j] = sum_b X[b][i] dZ1[b][j]
  GemmArgs gw1{kIn, kHidden, Bp, N->X, 1, kIn, N->dZ1, kHidden, 1, nullptr, nullptr, nullptr, nullptr, 0};
  launch_weight_grad(N, gw1, N->G + kOffW1);
  MHIP(N, hipGetLastError());
  return PIRRT_OK;
}

int check_batch(pirrt_mlp* N, int32_t B, const float* x, int mem_kind) {
  if (mem_kind != PIRRT_MEM_HOST && mem_kind != PIRRT_MEM_DEVICE) return mfail(N, PIRRT_EINVAL, "bad mem_kind");
  if (B < 1 || B > N->max_batch) return mfail(N, PIRRT_EINVAL, "batch size outside 1..max_batch");
  if (!x) return mfail(N, PIRRT_EINVAL, "x is NULL");
  return PIRRT_OK;
}

inline int32_t padded(int32_t B) { return (B + 63) / 64 * 64; }

// Device address of `scratch` on each GPU, looked up once per device with that device
// current (at pirrt_mlp_create, or at the first no-allocation call on the device).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint16_t* g_scratch_dev[kMaxDevices] = {};

// dev must be the current device.  Returns nullptr when the lookup fails.
uint16_t* noalloc_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_dev[dev] = static_cast<uint16_t*>(p);
  }
  return g_scratch_dev[dev];
}

}  // namespace

extern "C" {

int64_t pirrt_mlp_num_params(void) { return kNumParams; }

int32_t pirrt_mlp_in_dim(const pirrt_mlp* N) { return N ? N->in_dim : -1; }

int pirrt_mlp_create(pirrt_mlp** out, const pirrt_mlp_config* cfg) {
  if (!out || !cfg) return PIRRT_EINVAL;
  *out = nullptr;
  if (cfg->in_dim < 1 || cfg->in_dim > kIn || cfg->max_batch < 1 || cfg->max_batch > (1 << 24) ||
      !(cfg->lr > 0.0f) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) || !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) ||
      !(cfg->eps > 0.0f)) {
    g_mlp_create_error = "in_dim outside 1..288, max_batch outside 1..2^24, or bad Adam constants";
    return PIRRT_EINVAL;
  }
  pirrt_mlp* N = new (std::nothrow) pirrt_mlp();
  if (!N) return PIRRT_ENOMEM;
  int dev = cfg->device;
  if ((dev < 0 && hipGetDevice(&dev) != hipSuccess) || hipSetDevice(dev) != hipSuccess) {
    (void)hipGetLastError();
    delete N;
    g_mlp_create_error = "no HIP device";
    return PIRRT_EDEVICE;
  }
  N->device = dev;
  (void)noalloc_scratch(dev);  // set-up of the no-allocation forward on this device
  N->stream = (hipStream_t)cfg->hip_stream;
  N->in_dim = cfg->in_dim;
  N->max_batch = cfg->max_batch;
  N->bcap = padded(cfg->max_batch);
  N->lr = cfg->lr;
  N->beta1 = cfg->beta1;
  N->beta2 = cfg->beta2;
  N->eps = cfg->eps;
  const int64_t bc = N->bcap;
  bool ok = malloc_dev(&N->P, kNumParams) && malloc_dev(&N->G, kNumParams) && malloc_dev(&N->m, kNumParams) &&
            malloc_dev(&N->v, kNumParams) && malloc_dev(&N->W1t, (int64_t)kIn * kHidden) &&
            malloc_dev(&N->W2b, (int64_t)kHidden * kHidden) && malloc_dev(&N->W2t, (int64_t)kHidden * kHidden) &&
            malloc_dev(&N->w3b, kHidden) &&
            malloc_dev(&N->xin, (int64_t)N->max_batch * N->in_dim) && malloc_dev(&N->yin, N->max_batch) &&
            malloc_dev(&N->X, bc * kIn) && malloc_dev(&N->Z1, bc * kHidden) && malloc_dev(&N->A1, bc * kHidden) &&
            malloc_dev(&N->Z2, bc * kHidden) && malloc_dev(&N->A2, bc * kHidden) && malloc_dev(&N->z, bc) &&
            malloc_dev(&N->dz, bc) && malloc_dev(&N->dZ2, bc * kHidden) && malloc_dev(&N->dZ1, bc * kHidden) &&
            malloc_dev(&N->dloss, 1) &&
            malloc_dev(&N->part, std::max<int64_t>((int64_t)kSplitK * kIn * kHidden, (int64_t)kColParts * (kHidden + 1)));
  if (ok && hipHostMalloc((void**)&N->hloss, sizeof(float), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    N->hloss = nullptr;
    ok = false;
  }
  if (ok)
    ok = hipMemset(N->P, 0, sizeof(float) * kNumParams) == hipSuccess &&
         hipMemset(N->m, 0, sizeof(float) * kNumParams) == hipSuccess &&
         hipMemset(N->v, 0, sizeof(float) * kNumParams) == hipSuccess &&
         hipMemset(N->W1t, 0, sizeof(uint16_t) * kIn * kHidden) == hipSuccess &&
         hipMemset(N->W2b, 0, sizeof(uint16_t) * kHidden * kHidden) == hipSuccess &&
         hipMemset(N->W2t, 0, sizeof(uint16_t) * kHidden * kHidden) == hipSuccess &&
         hipMemset(N->w3b, 0, sizeof(uint16_t) * kHidden) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    release(N);
    delete N;
    g_mlp_create_error = "device allocation failed at create";
    return PIRRT_ENOMEM;
  }
  *out = N;
  return PIRRT_OK;
}

int pirrt_mlp_destroy(pirrt_mlp* N) {
  if (!N) return PIRRT_OK;
  (void)hipSetDevice(N->device);
  if (!N->poisoned) (void)hipStreamSynchronize(N->stream);
  release(N);
  delete N;
  return PIRRT_OK;
}

const char* pirrt_mlp_last_error(const pirrt_mlp* N) { return N ? N->err.c_str() : g_mlp_create_error.c_str(); }

int pirrt_mlp_set_params(pirrt_mlp* N, const float* params, int mem_kind) {
  int rc = mguard(N);
  if (rc) return rc;
  if (mem_kind != PIRRT_MEM_HOST && mem_kind != PIRRT_MEM_DEVICE) return mfail(N, PIRRT_EINVAL, "bad mem_kind");
  if (!params) return mfail(N, PIRRT_EINVAL, "params is NULL");
  if (mem_kind == PIRRT_MEM_HOST)
    for (int64_t i = 0; i < kNumParams; ++i)
      if (!std::isfinite(params[i])) return mfail(N, PIRRT_EINVAL, "parameter not finite");
  hipStream_t s = N->stream;
  MHIP(N, hipMemcpyAsync(N->P, params, sizeof(float) * kNumParams,
                         mem_kind == PIRRT_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
  MHIP(N, hipMemsetAsync(N->m, 0, sizeof(float) * kNumParams, s));
  MHIP(N, hipMemsetAsync(N->v, 0, sizeof(float) * kNumParams, s));
  hipLaunchKernelGGL(k_refresh, dim3(nblocks((int64_t)kIn * kHidden)), dim3(kThreads), 0, s, N->P, N->W1t, N->W2b,
                     N->W2t, N->w3b);
  MHIP(N, hipGetLastError());
  MHIP(N, hipStreamSynchronize(s));
  N->t = 0;
  return PIRRT_OK;
}

int pirrt_mlp_get_params(pirrt_mlp* N, float* params, int mem_kind) {
  int rc = mguard(N);
  if (rc) return rc;
  if (mem_kind != PIRRT_MEM_HOST && mem_kind != PIRRT_MEM_DEVICE) return mfail(N, PIRRT_EINVAL, "bad mem_kind");
  if (!params) return mfail(N, PIRRT_EINVAL, "params is NULL");
  MHIP(N, hipMemcpyAsync(params, N->P, sizeof(float) * kNumParams,
                         mem_kind == PIRRT_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, N->stream));
  MHIP(N, hipStreamSynchronize(N->stream));
  return PIRRT_OK;
}

int pirrt_mlp_forward(pirrt_mlp* N, int32_t B, const float* x, float* logits, int mem_kind) {
  int rc = mguard(N);
  if (rc) return rc;
  if ((rc = check_batch(N, B, x, mem_kind))) return rc;
  if (!logits) return mfail(N, PIRRT_EINVAL, "logits is NULL");
  const int32_t Bp = padded(B);
  const float* yd = nullptr;
  if ((rc = stage_inputs(N, B, Bp, x, nullptr, mem_kind, &yd))) return rc;
  enqueue_forward(N, Bp, false, N->X, N->A1, N->A2);
  hipLaunchKernelGGL(k_layer3, dim3(nblocks(Bp)), dim3(kThreads), 0, N->stream, B, Bp, N->A2, N->w3b, N->P, nullptr,
                     N->z, nullptr, nullptr);
  MHIP(N, hipGetLastError());
  MHIP(N, hipMemcpyAsync(logits, N->z, sizeof(float) * (size_t)B,
                         mem_kind == PIRRT_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, N->stream));
  MHIP(N, hipStreamSynchronize(N->stream));
  return PIRRT_OK;
}

int pirrt_mlp_forward_noalloc(pirrt_mlp* N, int32_t B, const float* x, float* logits) {
  int rc = mguard(N);
  if (rc) return rc;
  if (B < 1 || B > kNoAllocRows) return mfail(N, PIRRT_EINVAL, "batch size outside 1..PIRRT_MLP_NOALLOC_MAX_BATCH");
  if (!x || !logits) return mfail(N, PIRRT_EINVAL, "x or logits is NULL");
  uint16_t* base = noalloc_scratch(N->device);
  if (!base) return mfail(N, PIRRT_EDEVICE, "device address of the no-allocation scratch not available");
  const int32_t Bp = padded(B);
  hipStream_t s = N->stream;
  uint16_t* X = base + kScratchX;
  uint16_t* A1 = base + kScratchA1;
  uint16_t* A2 = base + kScratchA2;
  hipLaunchKernelGGL(k_features, dim3(nblocks((int64_t)Bp * kIn)), dim3(kThreads), 0, s, B, Bp, N->in_dim, x, X);
  enqueue_forward(N, Bp, false, X, A1, A2);
  hipLaunchKernelGGL(k_layer3, dim3(nblocks(Bp)), dim3(kThreads), 0, s, B, Bp, A2, N->w3b, N->P, nullptr, logits,
                     nullptr, nullptr);
  MHIP(N, hipGetLastError());
  return PIRRT_OK;
}

int pirrt_mlp_gradients(pirrt_mlp* N, int32_t B, const float* x, const float* y, float* grads, float* loss,
                        int mem_kind) {
  int rc = mguard(N);
  if (rc) return rc;
  if ((rc = check_batch(N, B, x, mem_kind))) return rc;
  if (!y) return mfail(N, PIRRT_EINVAL, "y is NULL");
  const int32_t Bp = padded(B);
  const float* yd = nullptr;
  if ((rc = stage_inputs(N, B, Bp, x, y, mem_kind, &yd))) return rc;
  if ((rc = enqueue_gradients(N, B, Bp, yd))) return rc;
  if (grads)
    MHIP(N, hipMemcpyAsync(grads, N->G, sizeof(float) * kNumParams,
                           mem_kind == PIRRT_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, N->stream));
  MHIP(N, hipMemcpyAsync(N->hloss, N->dloss, sizeof(float), hipMemcpyDeviceToHost, N->stream));
  MHIP(N, hipStreamSynchronize(N->stream));
  if (loss) *loss = *N->hloss;
  return PIRRT_OK;
}

int pirrt_mlp_train_step(pirrt_mlp* N, int32_t B, const float* x, const float* y, float* loss, int mem_kind) {
  int rc = mguard(N);
  if (rc) return rc;
  if ((rc = check_batch(N, B, x, mem_kind))) return rc;
  if (!y) return mfail(N, PIRRT_EINVAL, "y is NULL");
  const int32_t Bp = padded(B);
  const float* yd = nullptr;
  if ((rc = stage_inputs(N, B, Bp, x, y, mem_kind, &yd))) return rc;
  if ((rc = enqueue_gradients(N, B, Bp, yd))) return rc;
  N->t += 1;
  const float c1 = 1.0f - powf(N->beta1, (float)N->t), c2 = 1.0f - powf(N->beta2, (float)N->t);
  hipLaunchKernelGGL(k_adam, dim3(nblocks(kNumParams)), dim3(kThreads), 0, N->stream, kNumParams, N->P, N->G, N->m,
                     N->v, N->lr, N->beta1, N->beta2, N->eps, c1, c2);
  hipLaunchKernelGGL(k_refresh, dim3(nblocks((int64_t)kIn * kHidden)), dim3(kThreads), 0, N->stream, N->P, N->W1t,
                     N->W2b, N->W2t, N->w3b);
  MHIP(N, hipGetLastError());
  MHIP(N, hipMemcpyAsync(N->hloss, N->dloss, sizeof(float), hipMemcpyDeviceToHost, N->stream));
  MHIP(N, hipStreamSynchronize(N->stream));
  if (loss) *loss = *N->hloss;
  return PIRRT_OK;
}

}  // extern "C"
