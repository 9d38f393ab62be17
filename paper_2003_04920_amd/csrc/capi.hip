// Host runtime and C ABI (declared in include/pirrt.h): graph storage on the device,
// batch insertion, and the Replan driver of Alg. 2.
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"
#include "pirrt.h"

using namespace pirrt;

namespace {

constexpr int64_t kMinVertexCap = 1024;
constexpr int64_t kMinEdgeCap = 4096;

// Pinned host block read back once per Replan iteration.
struct HostBlock {
  IterCounters ctr[kCounterSlots];
  unsigned long long hops;
  EvalInfo info;
  int32_t flag;
  int32_t count[2];
  int64_t word;
};

// Validation kernels for device-resident inputs of replan / set_policy.
__global__ void k_check_h(int32_t n, const float* __restrict__ h, int* __restrict__ bad) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && !(h[v] >= 0.0f)) atomicOr(bad, 1);
}

__global__ void k_check_policy(int32_t n, const int32_t* __restrict__ parent, const float* __restrict__ pcost,
                               int* __restrict__ bad) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int32_t p = parent[v];
  uint32_t w = __float_as_uint(pcost[v]);
  if (p < -1 || p >= n || p == v) atomicOr(bad, 1);
  if ((w >> 31) != 0 || (w & 0x7f800000u) == 0x7f800000u) atomicOr(bad, 2);
}

inline unsigned grid_for(int64_t n, int per = 256) {
  int64_t b = (n + per - 1) / per;
  return (unsigned)(b > 0 ? b : 1);
}

thread_local std::string g_create_error;

}  // namespace

struct pirrt_graph {
  int device = 0;
  hipStream_t stream = nullptr;
  int32_t max_iters = 0;
  int64_t n = 0, nnz = 0;
  int64_t vcap = 0, ecap = 0, ecap2 = 0;
  // adjacency (current and spare for the rebuild)
  int64_t* rp = nullptr;
  int32_t* col = nullptr;
  float* cst = nullptr;
  int64_t* rp2 = nullptr;
  int32_t* col2 = nullptr;
  float* cst2 = nullptr;
  // policy (SoA: g, parent, parent-edge cost)
  float* g = nullptr;
  int32_t* parent = nullptr;
  float* pcost = nullptr;
  // snapshot
  float* sg = nullptr;
  int32_t* sparent = nullptr;
  float* spcost = nullptr;
  int64_t snap_n = -1, snap_cap = 0;
  // Evaluate scratch
  int32_t* child_cnt = nullptr;
  int32_t* child_ptr = nullptr;
  int32_t* child = nullptr;
  int32_t* fr0 = nullptr;
  int32_t* fr1 = nullptr;
  int32_t* lvl = nullptr;
  // promising / domain marks
  uint32_t* stamp = nullptr;
  uint32_t epoch = 0;
  // Evaluate stamps {epoch, g bits}
  unsigned long long* word = nullptr;
  uint32_t eval_epoch = 0;
  bool eval_levels = false;  // level-synchronous Evaluate instead of the walk
  int walk_parts = 1;        // walk launches over consecutive slot ranges
  bool walk_coherent = true; // device-scope stamp accesses
  // storage order: ext_of[slot] = caller id, slot_of[id] = slot (host mirror hslot)
  int32_t* ext_of = nullptr;
  int32_t* slot_of = nullptr;
  std::vector<int32_t> hslot;
  int64_t reorder_n = 0;       // vertex count at the last renumbering
  double reorder_growth = 1.25;  // renumber when n grows by this factor (0 = never)
  // insertion / renumbering / translation scratch
  int32_t* add = nullptr;
  int32_t* deg = nullptr;
  int32_t* pending = nullptr;
  float* hbuf = nullptr;
  float* g2 = nullptr;
  int32_t* parent2 = nullptr;
  float* pcost2 = nullptr;
  int32_t* ext2 = nullptr;
  // batch staging
  int64_t* brp = nullptr;
  int32_t* bcol = nullptr;
  int32_t* bslot = nullptr;
  float* bcost = nullptr;
  int64_t brows_cap = 0, bnnz_cap = 0;
  void* scan_scratch = nullptr;
  size_t scan_bytes = 0;
  // small device block and its pinned mirror
  IterCounters* ctr = nullptr;
  EvalInfo* info = nullptr;
  int32_t* dflag = nullptr;
  int32_t* dcount = nullptr;
  unsigned long long* dhops = nullptr;
  bool trace = false;  // per-iteration counters to stderr
  HostBlock* host = nullptr;
  hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  // tuning
  int32_t mid_hint = 64;
  int32_t max_blocks = 2048;  // persistent grids: CUs x 8 workgroups of 256 threads
  int row_variant = 0;
  bool poisoned = false;
  std::string err;
};

namespace {

int fail(pirrt_graph* G, int code, const std::string& msg) {
  G->err = msg;
  return code;
}

int fail_device(pirrt_graph* G, hipError_t e, const char* what) {
  G->poisoned = true;
  G->err = std::string("HIP error in ") + what + ": " + hipGetErrorString(e);
  return PIRRT_EDEVICE;
}

#define HIP_OR_FAIL(G, expr)                          \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return fail_device(G, e_, #expr); \
  } while (0)

template <class T>
bool dalloc(T** p, int64_t count) {
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
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

int guard(pirrt_graph* G) {
  if (!G) return PIRRT_EINVAL;
  if (G->poisoned) return PIRRT_EDEVICE;
  hipError_t e = hipSetDevice(G->device);
  if (e != hipSuccess) return fail_device(G, e, "hipSetDevice");
  return PIRRT_OK;
}

hipMemcpyKind in_kind(int mem_kind) { return mem_kind == PIRRT_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice; }
hipMemcpyKind out_kind(int mem_kind) { return mem_kind == PIRRT_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost; }

int ensure_scan(pirrt_graph* G, int64_t n) {
  size_t need = scan_scratch_bytes(n);
  if (need <= G->scan_bytes) return PIRRT_OK;
  void* p = nullptr;
  if (hipMalloc(&p, need) != hipSuccess) {
    (void)hipGetLastError();
    return fail(G, PIRRT_ENOMEM, "device allocation of scan scratch failed");
  }
  if (G->scan_scratch) (void)hipFree(G->scan_scratch);
  G->scan_scratch = p;
  G->scan_bytes = need;
  return PIRRT_OK;
}

void free_vertex_arrays(pirrt_graph* G) {
  dfree(G->rp); dfree(G->rp2); dfree(G->g); dfree(G->parent); dfree(G->pcost); dfree(G->child_cnt);
  dfree(G->child_ptr); dfree(G->child); dfree(G->fr0); dfree(G->fr1); dfree(G->lvl); dfree(G->stamp);
  dfree(G->add); dfree(G->deg); dfree(G->pending); dfree(G->hbuf); dfree(G->ext_of); dfree(G->slot_of);
  dfree(G->g2); dfree(G->parent2); dfree(G->pcost2); dfree(G->ext2); dfree(G->word);
}

void forget_vertex_arrays(pirrt_graph* T) {
  T->rp = T->rp2 = nullptr;
  T->g = T->pcost = T->hbuf = T->g2 = T->pcost2 = nullptr;
  T->parent = T->child_cnt = T->child_ptr = T->child = T->fr0 = T->fr1 = T->lvl = nullptr;
  T->add = T->deg = T->pending = T->ext_of = T->slot_of = T->parent2 = T->ext2 = nullptr;
  T->stamp = nullptr;
  T->word = nullptr;
}

// Grows every per-vertex array to hold `need` vertices, keeping g / parent / pcost
// and the row offsets.  On failure nothing changes.
int ensure_vcap(pirrt_graph* G, int64_t need) {
  if (need <= G->vcap) return PIRRT_OK;
  int64_t cap = G->vcap + G->vcap / 2;
  if (cap < need) cap = need;
  if (cap < kMinVertexCap) cap = kMinVertexCap;
  pirrt_graph T;  // holds the new arrays until all allocations succeeded
  bool ok = dalloc(&T.rp, cap + 1) && dalloc(&T.rp2, cap + 1) && dalloc(&T.g, cap) && dalloc(&T.parent, cap) &&
            dalloc(&T.pcost, cap) && dalloc(&T.child_cnt, cap) && dalloc(&T.child_ptr, cap + 1) &&
            dalloc(&T.child, cap) && dalloc(&T.fr0, cap) && dalloc(&T.fr1, cap) &&
            dalloc(&T.lvl, cap + kMaxMidLaunches + 8) && dalloc(&T.stamp, cap) && dalloc(&T.add, cap) &&
            dalloc(&T.deg, cap) && dalloc(&T.pending, cap) && dalloc(&T.hbuf, cap) && dalloc(&T.ext_of, cap) &&
            dalloc(&T.slot_of, cap) && dalloc(&T.g2, cap) && dalloc(&T.parent2, cap) && dalloc(&T.pcost2, cap) &&
            dalloc(&T.ext2, cap) && dalloc(&T.word, cap);
  if (!ok) {
    free_vertex_arrays(&T);
    return fail(G, PIRRT_ENOMEM, "device allocation for vertex storage failed");
  }
  hipStream_t s = G->stream;
  HIP_OR_FAIL(G, hipMemsetAsync(T.child_cnt, 0, sizeof(int32_t) * (size_t)cap, s));
  HIP_OR_FAIL(G, hipMemsetAsync(T.stamp, 0, sizeof(uint32_t) * (size_t)cap, s));
  HIP_OR_FAIL(G, hipMemsetAsync(T.word, 0, sizeof(unsigned long long) * (size_t)cap, s));
  HIP_OR_FAIL(G, hipMemsetAsync(T.rp, 0, sizeof(int64_t) * (size_t)(cap + 1), s));
  if (G->n > 0) {
    HIP_OR_FAIL(G, hipMemcpyAsync(T.rp, G->rp, sizeof(int64_t) * (size_t)(G->n + 1), hipMemcpyDeviceToDevice, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(T.g, G->g, sizeof(float) * (size_t)G->n, hipMemcpyDeviceToDevice, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(T.parent, G->parent, sizeof(int32_t) * (size_t)G->n, hipMemcpyDeviceToDevice, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(T.pcost, G->pcost, sizeof(float) * (size_t)G->n, hipMemcpyDeviceToDevice, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(T.ext_of, G->ext_of, sizeof(int32_t) * (size_t)G->n, hipMemcpyDeviceToDevice, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(T.slot_of, G->slot_of, sizeof(int32_t) * (size_t)G->n, hipMemcpyDeviceToDevice, s));
  }
  HIP_OR_FAIL(G, hipStreamSynchronize(s));
  free_vertex_arrays(G);
  G->rp = T.rp; G->rp2 = T.rp2; G->g = T.g; G->parent = T.parent; G->pcost = T.pcost;
  G->child_cnt = T.child_cnt; G->child_ptr = T.child_ptr; G->child = T.child; G->fr0 = T.fr0; G->fr1 = T.fr1;
  G->lvl = T.lvl; G->stamp = T.stamp; G->add = T.add; G->deg = T.deg; G->pending = T.pending; G->hbuf = T.hbuf;
  G->ext_of = T.ext_of; G->slot_of = T.slot_of; G->g2 = T.g2; G->parent2 = T.parent2; G->pcost2 = T.pcost2;
  G->ext2 = T.ext2;
  G->word = T.word;
  forget_vertex_arrays(&T);
  G->vcap = cap;
  G->epoch = 0;
  G->eval_epoch = 0;
  return ensure_scan(G, cap + 1);
}

// Spare adjacency arrays able to hold `need` entries.
int ensure_spare(pirrt_graph* G, int64_t need) {
  if (need <= G->ecap2) return PIRRT_OK;
  int64_t cap = G->ecap2 + G->ecap2 / 2;
  if (cap < need) cap = need;
  if (cap < kMinEdgeCap) cap = kMinEdgeCap;
  int32_t* c = nullptr;
  float* w = nullptr;
  if (!dalloc(&c, cap) || !dalloc(&w, cap)) {
    dfree(c);
    dfree(w);
    return fail(G, PIRRT_ENOMEM, "device allocation for adjacency failed");
  }
  dfree(G->col2);
  dfree(G->cst2);
  G->col2 = c;
  G->cst2 = w;
  G->ecap2 = cap;
  return PIRRT_OK;
}

int ensure_staging(pirrt_graph* G, int64_t rows, int64_t nnz) {
  if (rows + 1 > G->brows_cap) {
    int64_t* p = nullptr;
    int64_t cap = rows + 1 > 1024 ? rows + 1 : 1024;
    if (!dalloc(&p, cap)) return fail(G, PIRRT_ENOMEM, "device allocation for batch staging failed");
    dfree(G->brp);
    G->brp = p;
    G->brows_cap = cap;
  }
  if (nnz > G->bnnz_cap) {
    int32_t* c = nullptr;
    int32_t* t = nullptr;
    float* w = nullptr;
    int64_t cap = nnz > 4096 ? nnz : 4096;
    if (!dalloc(&c, cap) || !dalloc(&t, cap) || !dalloc(&w, cap)) {
      dfree(c);
      dfree(t);
      dfree(w);
      return fail(G, PIRRT_ENOMEM, "device allocation for batch staging failed");
    }
    dfree(G->bcol);
    dfree(G->bslot);
    dfree(G->bcost);
    G->bcol = c;
    G->bslot = t;
    G->bcost = w;
    G->bnnz_cap = cap;
  }
  return PIRRT_OK;
}

void release_all(pirrt_graph* G) {
  free_vertex_arrays(G);
  dfree(G->col); dfree(G->cst); dfree(G->col2); dfree(G->cst2);
  dfree(G->sg); dfree(G->sparent); dfree(G->spcost);
  dfree(G->brp); dfree(G->bcol); dfree(G->bslot); dfree(G->bcost);
  dfree(G->ctr); dfree(G->info); dfree(G->dflag); dfree(G->dcount); dfree(G->dhops);
  if (G->scan_scratch) (void)hipFree(G->scan_scratch);
  G->scan_scratch = nullptr;
  if (G->host) (void)hipHostFree(G->host);
  G->host = nullptr;
  for (auto& e : G->ev)
    if (e) {
      (void)hipEventDestroy(e);
      e = nullptr;
    }
}

// Reads one device flag word back (synchronising the stream).
int read_flag(pirrt_graph* G, int32_t* out) {
  HIP_OR_FAIL(G, hipMemcpyAsync(&G->host->flag, G->dflag, sizeof(int32_t), hipMemcpyDeviceToHost, G->stream));
  HIP_OR_FAIL(G, hipStreamSynchronize(G->stream));
  *out = G->host->flag;
  return PIRRT_OK;
}

double elapsed_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.0f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
    (void)hipGetLastError();
    return 0.0;
  }
  return (double)ms;
}

// Copies the policy out in caller order (device outputs are written directly;
// host outputs go through device staging).
int policy_out(pirrt_graph* G, float* g_out, int32_t* parent_out, float* pcost_out, int mem_kind) {
  const int32_t n = (int32_t)G->n;
  hipStream_t s = G->stream;
  if (n == 0) return PIRRT_OK;
  const bool dev = mem_kind == PIRRT_MEM_DEVICE;
  float* gd = g_out ? (dev ? g_out : G->g2) : nullptr;
  int32_t* pd = parent_out ? (dev ? parent_out : G->parent2) : nullptr;
  float* cd = pcost_out ? (dev ? pcost_out : G->pcost2) : nullptr;
  launch_policy_to_ext(n, G->slot_of, G->ext_of, G->g, G->parent, G->pcost, gd, pd, cd, s);
  HIP_OR_FAIL(G, hipGetLastError());
  if (!dev) {
    if (g_out) HIP_OR_FAIL(G, hipMemcpyAsync(g_out, G->g2, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost, s));
    if (parent_out)
      HIP_OR_FAIL(G, hipMemcpyAsync(parent_out, G->parent2, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
    if (pcost_out)
      HIP_OR_FAIL(G, hipMemcpyAsync(pcost_out, G->pcost2, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost, s));
  }
  return PIRRT_OK;
}

// Renumbers the storage slots in breadth-first order of the graph from x_init
// (vertex 0); vertices it cannot reach follow in their current order.
int renumber(pirrt_graph* G) {
  const int32_t n = (int32_t)G->n;
  hipStream_t s = G->stream;
  int rc;
  if ((rc = ensure_spare(G, G->nnz))) return rc;
  int32_t* visited = G->pending;
  int32_t* order = G->fr0;
  HIP_OR_FAIL(G, hipMemsetAsync(visited, 0, sizeof(int32_t) * (size_t)n, s));
  launch_bfs_init(G->hslot[0], order, visited, &G->dcount[0], s);
  int32_t lo = 0, hi = 1;
  while (hi > lo) {
    launch_graph_bfs_level(lo, hi, order, G->rp, G->col, visited, &G->dcount[0], s);
    HIP_OR_FAIL(G, hipGetLastError());
    HIP_OR_FAIL(G, hipMemcpyAsync(&G->host->count[0], &G->dcount[0], sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(G, hipStreamSynchronize(s));
    lo = hi;
    hi = G->host->count[0];
    if (hi > n) return fail_device(G, hipErrorUnknown, "renumbering visited too many vertices");
  }
  launch_append_unvisited(n, visited, order, &G->dcount[0], s);
  HIP_OR_FAIL(G, hipMemcpyAsync(&G->host->count[0], &G->dcount[0], sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(G, hipStreamSynchronize(s));
  if (G->host->count[0] != n) return fail_device(G, hipErrorUnknown, "renumbering lost vertices");
  PermuteArgs a;
  a.n = n;
  a.order = order;
  a.newslot = G->fr1;
  a.deg = G->deg;
  a.rp = G->rp;
  a.col = G->col;
  a.cst = G->cst;
  a.rp_new = G->rp2;
  a.col_new = G->col2;
  a.cst_new = G->cst2;
  a.g = G->g;
  a.parent = G->parent;
  a.pcost = G->pcost;
  a.ext_of = G->ext_of;
  a.g2 = G->g2;
  a.parent2 = G->parent2;
  a.pcost2 = G->pcost2;
  a.ext2 = G->ext2;
  a.slot_of = G->slot_of;
  a.scan_scratch = G->scan_scratch;
  launch_permute(a, s);
  HIP_OR_FAIL(G, hipGetLastError());
  std::swap(G->rp, G->rp2);
  std::swap(G->col, G->col2);
  std::swap(G->cst, G->cst2);
  std::swap(G->ecap, G->ecap2);
  std::swap(G->g, G->g2);
  std::swap(G->parent, G->parent2);
  std::swap(G->pcost, G->pcost2);
  std::swap(G->ext_of, G->ext2);
  G->hslot.resize((size_t)n);
  HIP_OR_FAIL(G, hipMemcpyAsync(G->hslot.data(), G->slot_of, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(G, hipStreamSynchronize(s));
  G->reorder_n = n;
  G->snap_n = -1;  // a snapshot in the old order is no longer valid
  return PIRRT_OK;
}

}  // namespace

extern "C" {

int pirrt_config_init(pirrt_config* cfg) {
  if (!cfg) return PIRRT_EINVAL;
  memset(cfg, 0, sizeof(*cfg));
  cfg->device = -1;
  return PIRRT_OK;
}

int pirrt_graph_create(pirrt_graph** out, const pirrt_config* cfg) {
  if (!out) return PIRRT_EINVAL;
  *out = nullptr;
  pirrt_config c;
  pirrt_config_init(&c);
  if (cfg) c = *cfg;
  if (c.vertex_capacity < 0 || c.edge_capacity < 0 || c.max_iters < 0) {
    g_create_error = "negative capacity or iteration cap";
    return PIRRT_EINVAL;
  }
  pirrt_graph* G = new (std::nothrow) pirrt_graph();
  if (!G) return PIRRT_ENOMEM;
  int dev = c.device;
  if (dev < 0) {
    if (hipGetDevice(&dev) != hipSuccess) {
      (void)hipGetLastError();
      delete G;
      g_create_error = "no HIP device";
      return PIRRT_EDEVICE;
    }
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || dev >= ndev) {
    (void)hipGetLastError();
    delete G;
    g_create_error = "HIP device not available";
    return PIRRT_EDEVICE;
  }
  G->device = dev;
  G->stream = (hipStream_t)c.hip_stream;
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      G->max_blocks = cus * 8;
    else
      (void)hipGetLastError();
  }
  G->max_iters = c.max_iters;
  if (hipSetDevice(dev) != hipSuccess) {
    (void)hipGetLastError();
    delete G;
    g_create_error = "hipSetDevice failed";
    return PIRRT_EDEVICE;
  }
  bool ok = dalloc(&G->ctr, kCounterSlots) && dalloc(&G->dhops, 1) && dalloc(&G->info, 1) && dalloc(&G->dflag, 1) && dalloc(&G->dcount, 2);
  if (ok && hipHostMalloc((void**)&G->host, sizeof(HostBlock), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    G->host = nullptr;
    ok = false;
  }
  for (auto& e : G->ev)
    if (ok && hipEventCreate(&e) != hipSuccess) {
      (void)hipGetLastError();
      e = nullptr;
      ok = false;
    }
  int rc = PIRRT_OK;
  if (ok && c.vertex_capacity > 0) rc = ensure_vcap(G, c.vertex_capacity);
  if (ok && rc == PIRRT_OK && c.edge_capacity > 0) {
    rc = ensure_spare(G, c.edge_capacity);
    if (rc == PIRRT_OK) {
      std::swap(G->col, G->col2);
      std::swap(G->cst, G->cst2);
      std::swap(G->ecap, G->ecap2);
      rc = ensure_spare(G, c.edge_capacity);
    }
  }
  if (!ok || rc != PIRRT_OK) {
    g_create_error = ok ? G->err : "device allocation failed at create";
    release_all(G);
    delete G;
    return ok ? rc : PIRRT_ENOMEM;
  }
  if (ensure_vcap(G, kMinVertexCap) != PIRRT_OK) {
    g_create_error = G->err;
    release_all(G);
    delete G;
    return PIRRT_ENOMEM;
  }
  // the row offsets of the empty graph
  if (hipMemsetAsync(G->rp, 0, sizeof(int64_t), G->stream) != hipSuccess ||
      hipStreamSynchronize(G->stream) != hipSuccess) {
    (void)hipGetLastError();
    g_create_error = "initialising the graph failed";
    release_all(G);
    delete G;
    return PIRRT_EDEVICE;
  }
  const char* growth = getenv("PIRRT_REORDER_GROWTH");
  if (growth) G->reorder_growth = atof(growth);
  const char* tr = getenv("PIRRT_TRACE");
  G->trace = tr && atoi(tr) > 0;
  const char* ev = getenv("PIRRT_EVALUATE");
  if (ev && strcmp(ev, "levels") == 0) G->eval_levels = true;
  const char* wp = getenv("PIRRT_WALK_PARTS");
  if (wp && atoi(wp) >= 1) G->walk_parts = atoi(wp);
  const char* wc = getenv("PIRRT_WALK_COHERENT");
  if (wc) G->walk_coherent = atoi(wc) != 0;
  const char* variant = getenv("PIRRT_ROW_VARIANT");
  if (variant) {
    int v = atoi(variant);
    if (v >= 0 && v < kRowVariants) G->row_variant = v;
  }
  const char* blocks = getenv("PIRRT_MAX_BLOCKS");
  if (blocks && atoi(blocks) >= 8) G->max_blocks = atoi(blocks);
  *out = G;
  return PIRRT_OK;
}

int pirrt_graph_destroy(pirrt_graph* G) {
  if (!G) return PIRRT_OK;
  (void)hipSetDevice(G->device);
  if (!G->poisoned) (void)hipStreamSynchronize(G->stream);
  release_all(G);
  delete G;
  return PIRRT_OK;
}

int64_t pirrt_num_vertices(const pirrt_graph* G) { return G ? G->n : -1; }
int64_t pirrt_num_edges(const pirrt_graph* G) { return G ? G->nnz : -1; }

const char* pirrt_last_error(const pirrt_graph* G) {
  if (!G) return g_create_error.c_str();
  return G->err.c_str();
}

const char* pirrt_strerror(int code) {
  switch (code) {
    case PIRRT_OK: return "success";
    case PIRRT_EINVAL: return "invalid argument";
    case PIRRT_ENOMEM: return "out of memory";
    case PIRRT_EDEVICE: return "device error";
    case PIRRT_ENOTCONVERGED: return "iteration cap reached before the fixed point";
    default: return "unknown error";
  }
}

int pirrt_insert_batch(pirrt_graph* G, int32_t n_new, const int64_t* row_ptr, const int32_t* col, const float* cost,
                       int mem_kind) {
  int rc = guard(G);
  if (rc) return rc;
  if (mem_kind != PIRRT_MEM_HOST && mem_kind != PIRRT_MEM_DEVICE) return fail(G, PIRRT_EINVAL, "bad mem_kind");
  if (n_new < 0) return fail(G, PIRRT_EINVAL, "n_new < 0");
  if (n_new == 0) return PIRRT_OK;
  if (!row_ptr) return fail(G, PIRRT_EINVAL, "row_ptr is NULL");
  if (G->n + (int64_t)n_new > (int64_t)INT32_MAX - 1) return fail(G, PIRRT_EINVAL, "vertex ids beyond INT32_MAX");
  hipStream_t s = G->stream;
  int64_t nnz_b = 0;
  if (mem_kind == PIRRT_MEM_HOST) {
    nnz_b = row_ptr[n_new];
  } else {
    HIP_OR_FAIL(G, hipMemcpyAsync(&G->host->word, row_ptr + n_new, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(G, hipStreamSynchronize(s));
    nnz_b = G->host->word;
  }
  if (nnz_b < 0 || nnz_b > ((int64_t)1 << 40)) return fail(G, PIRRT_EINVAL, "row_ptr[n_new] out of range");
  if (nnz_b > 0 && (!col || !cost)) return fail(G, PIRRT_EINVAL, "col or cost is NULL");
  if ((rc = ensure_staging(G, n_new, nnz_b))) return rc;
  HIP_OR_FAIL(G, hipMemcpyAsync(G->brp, row_ptr, sizeof(int64_t) * (size_t)(n_new + 1), in_kind(mem_kind), s));
  if (nnz_b > 0) {
    HIP_OR_FAIL(G, hipMemcpyAsync(G->bcol, col, sizeof(int32_t) * (size_t)nnz_b, in_kind(mem_kind), s));
    HIP_OR_FAIL(G, hipMemcpyAsync(G->bcost, cost, sizeof(float) * (size_t)nnz_b, in_kind(mem_kind), s));
  }
  HIP_OR_FAIL(G, hipMemsetAsync(G->dflag, 0, sizeof(int32_t), s));
  launch_validate_rows(n_new, G->n, G->brp, G->bcol, G->bcost, nnz_b, G->dflag, s);
  HIP_OR_FAIL(G, hipGetLastError());
  int32_t bad = 0;
  if ((rc = read_flag(G, &bad))) return rc;
  if (bad) {
    std::string m = "invalid batch:";
    if (bad & 1) m += " row_ptr not 0-based / non-decreasing / bounded;";
    if (bad & 2) m += " col outside [0, own id);";
    if (bad & 4) m += " cost not finite, negative or -0.0;";
    return fail(G, PIRRT_EINVAL, m);
  }
  const int64_t n_old = G->n, n1 = G->n + n_new;
  if ((rc = ensure_vcap(G, n1))) return rc;
  if ((rc = ensure_spare(G, G->nnz + 2 * nnz_b))) return rc;
  // new vertices take the slots after the existing ones; neighbours to slots
  launch_identity_ids(n_old, n1, G->ext_of, G->slot_of, s);
  launch_translate(nnz_b, G->bcol, G->slot_of, G->bslot, s);
  // adjacency rebuild into the spare arrays, then swap
  launch_rebuild(n_new, n_old, G->brp, G->bslot, G->bcost, G->rp, G->col, G->cst, G->rp2, G->col2, G->cst2, G->add,
                 G->deg, G->scan_scratch, s);
  HIP_OR_FAIL(G, hipGetLastError());
  std::swap(G->rp, G->rp2);
  std::swap(G->col, G->col2);
  std::swap(G->cst, G->cst2);
  std::swap(G->ecap, G->ecap2);
  G->n = n1;
  G->nnz += 2 * nnz_b;
  G->hslot.resize((size_t)n1);
  for (int64_t v = n_old; v < n1; ++v) G->hslot[(size_t)v] = (int32_t)v;
  // insertion-time policy, one dependency level at a time
  HIP_OR_FAIL(G, hipMemsetAsync(G->dcount, 0, 2 * sizeof(int32_t), s));
  launch_pending(n_new, n_old, G->brp, G->bcol, G->pending, G->fr0, &G->dcount[0], s);
  HIP_OR_FAIL(G, hipGetLastError());
  int64_t done = 0;
  for (int level = 0;; ++level) {
    const int cur = level & 1, nxt = cur ^ 1;
    HIP_OR_FAIL(G, hipMemcpyAsync(&G->host->count[cur], &G->dcount[cur], sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(G, hipStreamSynchronize(s));
    const int32_t size = G->host->count[cur];
    if (size == 0) break;
    done += size;
    if (done > n_new) return fail_device(G, hipErrorUnknown, "insertion levels exceed the batch");
    HIP_OR_FAIL(G, hipMemsetAsync(&G->dcount[nxt], 0, sizeof(int32_t), s));
    launch_insert_level(size, cur ? G->fr1 : G->fr0, n_old, G->brp, G->bcol, G->bslot, G->bcost, G->rp, G->col,
                        G->g, G->parent, G->pcost, G->pending, nxt ? G->fr1 : G->fr0, &G->dcount[nxt], s);
    HIP_OR_FAIL(G, hipGetLastError());
  }
  if (done != n_new) return fail_device(G, hipErrorUnknown, "insertion levels did not cover the batch");
  if (G->reorder_growth > 0.0 && (double)n1 >= G->reorder_growth * (double)G->reorder_n) {
    if ((rc = renumber(G))) return rc;
  }
  return PIRRT_OK;
}

int pirrt_replan(pirrt_graph* G, int32_t root, int32_t goal, const float* h, uint32_t flags, float* g_out,
                 int32_t* parent_out, int mem_kind, pirrt_stats* stats) {
  int rc = guard(G);
  if (rc) return rc;
  auto t_start = std::chrono::steady_clock::now();
  if (mem_kind != PIRRT_MEM_HOST && mem_kind != PIRRT_MEM_DEVICE) return fail(G, PIRRT_EINVAL, "bad mem_kind");
  if (G->n <= 0) return fail(G, PIRRT_EINVAL, "empty graph");
  if (root < 0 || root >= G->n || goal < 0 || goal >= G->n) return fail(G, PIRRT_EINVAL, "root or goal out of range");
  const int32_t n = (int32_t)G->n;
  hipStream_t s = G->stream;
  const int32_t rslot = G->hslot[(size_t)root], gslot = G->hslot[(size_t)goal];
  const float* hdev = nullptr;
  if (h) {
    const float* hsrc = h;
    if (mem_kind == PIRRT_MEM_HOST) {
      for (int32_t v = 0; v < n; ++v)
        if (!(h[v] >= 0.0f)) return fail(G, PIRRT_EINVAL, "h has a NaN or negative entry");
      HIP_OR_FAIL(G, hipMemcpyAsync(G->g2, h, sizeof(float) * (size_t)n, hipMemcpyHostToDevice, s));
      hsrc = G->g2;
    } else {
      HIP_OR_FAIL(G, hipMemsetAsync(G->dflag, 0, sizeof(int32_t), s));
      hipLaunchKernelGGL(k_check_h, dim3(grid_for(n)), dim3(256), 0, s, n, h, G->dflag);
      HIP_OR_FAIL(G, hipGetLastError());
      int32_t bad = 0;
      if ((rc = read_flag(G, &bad))) return rc;
      if (bad) return fail(G, PIRRT_EINVAL, "h has a NaN or negative entry");
    }
    launch_gather_by_slot(n, G->ext_of, hsrc, G->hbuf, s);
    HIP_OR_FAIL(G, hipGetLastError());
    hdev = G->hbuf;
  }
  const bool timing = (flags & PIRRT_TIMING) != 0;
  const int64_t cap = G->max_iters > 0 ? G->max_iters : 4 * (int64_t)n + 8;
  pirrt_stats st;
  memset(&st, 0, sizeof(st));

  EvalArgs ea;
  ea.n = n;
  ea.root = rslot;
  ea.parent = G->parent;
  ea.pcost = G->pcost;
  ea.g = G->g;
  ea.child_cnt = G->child_cnt;
  ea.child_ptr = G->child_ptr;
  ea.child = G->child;
  ea.fr0 = G->fr0;
  ea.fr1 = G->fr1;
  ea.lvl = G->lvl;
  ea.info = G->info;
  ea.ctr = G->ctr;
  ea.scan_scratch = G->scan_scratch;
  int64_t lb = (int64_t)n / 2048;
  ea.level_blocks = (int32_t)(lb < 16 ? 16 : (lb > 1024 ? 1024 : lb));

  StepArgs sa;
  sa.n = n;
  sa.root = rslot;
  sa.goal = gslot;
  sa.prune = (flags & PIRRT_NO_PRUNE) ? 0 : 1;
  sa.g = G->g;
  sa.h = hdev;
  sa.rp = G->rp;
  sa.col = G->col;
  sa.cst = G->cst;
  sa.stamp = G->stamp;
  sa.ext_of = G->ext_of;
  sa.parent = G->parent;
  sa.pcost = G->pcost;
  sa.ctr = G->ctr;
  sa.max_blocks = G->max_blocks;

  auto evaluate = [&]() -> int {
    int32_t mid = G->mid_hint;
    if (mid < 0) mid = 0;
    if (mid > kMaxMidLaunches) mid = kMaxMidLaunches;
    if (mid > n) mid = n;
    ea.mid_launches = mid;
    if (timing) HIP_OR_FAIL(G, hipEventRecord(G->ev[0], s));
    if (G->eval_levels) {
      launch_evaluate(ea, s);
    } else {
      if (++G->eval_epoch == 0) {
        HIP_OR_FAIL(G, hipMemsetAsync(G->word, 0, sizeof(unsigned long long) * (size_t)G->vcap, s));
        G->eval_epoch = 1;
      }
      if (G->trace) HIP_OR_FAIL(G, hipMemsetAsync(G->dhops, 0, sizeof(unsigned long long), s));
      launch_eval_walk(n, rslot, G->eval_epoch, G->parent, G->pcost, G->g, G->word, G->ctr,
                       G->trace ? G->dhops : nullptr, G->walk_parts, G->walk_coherent, s);
    }
    HIP_OR_FAIL(G, hipGetLastError());
    if (timing) HIP_OR_FAIL(G, hipEventRecord(G->ev[1], s));
    st.evaluate_calls += 1;
    return PIRRT_OK;
  };

  // the root has no parent (Alg. 2 walks the policy tree from x_init)
  HIP_OR_FAIL(G, hipMemsetAsync(G->parent + rslot, 0xff, sizeof(int32_t), s));
  HIP_OR_FAIL(G, hipMemsetAsync(G->pcost + rslot, 0, sizeof(float), s));
  if ((rc = evaluate())) return rc;
  bool pending_eval_time = timing;
  for (;;) {
    if (++G->epoch == 0) {
      HIP_OR_FAIL(G, hipMemsetAsync(G->stamp, 0, sizeof(uint32_t) * (size_t)G->vcap, s));
      G->epoch = 1;
    }
    sa.epoch = G->epoch;
    if (timing) HIP_OR_FAIL(G, hipEventRecord(G->ev[2], s));
    launch_mark(sa, G->row_variant, s);
    HIP_OR_FAIL(G, hipGetLastError());
    if (timing) HIP_OR_FAIL(G, hipEventRecord(G->ev[3], s));
    launch_improve(sa, G->row_variant, s);
    HIP_OR_FAIL(G, hipGetLastError());
    if (timing) HIP_OR_FAIL(G, hipEventRecord(G->ev[4], s));
    HIP_OR_FAIL(G, hipMemcpyAsync(G->host->ctr, G->ctr, sizeof(IterCounters) * kCounterSlots, hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(&G->host->info, G->info, sizeof(EvalInfo), hipMemcpyDeviceToHost, s));
    if (G->trace)
      HIP_OR_FAIL(G, hipMemcpyAsync(&G->host->hops, G->dhops, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(G, hipStreamSynchronize(s));
    if (timing) {
      if (pending_eval_time) st.ms_evaluate += elapsed_ms(G->ev[0], G->ev[1]);
      pending_eval_time = false;
      st.ms_mark += elapsed_ms(G->ev[2], G->ev[3]);
      st.ms_improve += elapsed_ms(G->ev[3], G->ev[4]);
      st.mark_launches += 1;
      st.improve_launches += 1;
    }
    IterCounters c{};
    for (int k = 0; k < kCounterSlots; ++k) {
      c.changed += G->host->ctr[k].changed;
      c.nP += G->host->ctr[k].nP;
      c.nD += G->host->ctr[k].nD;
      c.edges += G->host->ctr[k].edges;
    }
    const EvalInfo info = G->host->info;
    st.iterations += 1;
    st.edges_examined += (int64_t)c.edges;
    st.sum_P += c.nP;
    st.sum_D += c.nD;
    st.changed_total += c.changed;
    if (G->trace)
      fprintf(stderr, "pirrt iter %d: |P| %d |D| %d edges %llu changed %d walk hops %llu\n", st.iterations, c.nP,
              c.nD, (unsigned long long)c.edges, c.changed, G->eval_levels ? 0ull : G->host->hops);
    st.eval_levels = info.levels;
    // wide level launches for the next walk: the large levels seen this time, plus slack
    int32_t need = info.big_end - info.head_end;
    G->mid_hint = (need > 0 ? need : 0) + 2;
    if (c.changed == 0) break;
    if ((rc = evaluate())) return rc;
    pending_eval_time = timing;
    if (st.iterations >= cap) {
      rc = PIRRT_ENOTCONVERGED;
      break;
    }
  }
  if ((rc == PIRRT_OK || rc == PIRRT_ENOTCONVERGED) && (g_out || parent_out)) {
    const int keep = rc;
    if ((rc = policy_out(G, g_out, parent_out, nullptr, mem_kind))) return rc;
    rc = keep;
  }
  HIP_OR_FAIL(G, hipStreamSynchronize(s));
  if (timing && pending_eval_time) st.ms_evaluate += elapsed_ms(G->ev[0], G->ev[1]);
  st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  if (stats) *stats = st;
  if (rc == PIRRT_ENOTCONVERGED) return fail(G, rc, "iteration cap reached");
  return PIRRT_OK;
}

int pirrt_get_policy(pirrt_graph* G, float* g_out, int32_t* parent_out, float* pcost_out, int mem_kind) {
  int rc = guard(G);
  if (rc) return rc;
  if (mem_kind != PIRRT_MEM_HOST && mem_kind != PIRRT_MEM_DEVICE) return fail(G, PIRRT_EINVAL, "bad mem_kind");
  if ((rc = policy_out(G, g_out, parent_out, pcost_out, mem_kind))) return rc;
  HIP_OR_FAIL(G, hipStreamSynchronize(G->stream));
  return PIRRT_OK;
}

int pirrt_set_policy(pirrt_graph* G, const float* g_in, const int32_t* parent_in, const float* pcost_in,
                     int mem_kind) {
  int rc = guard(G);
  if (rc) return rc;
  if (mem_kind != PIRRT_MEM_HOST && mem_kind != PIRRT_MEM_DEVICE) return fail(G, PIRRT_EINVAL, "bad mem_kind");
  if (!g_in || !parent_in || !pcost_in) return fail(G, PIRRT_EINVAL, "NULL policy array");
  const int32_t n = (int32_t)G->n;
  if (n == 0) return PIRRT_OK;
  hipStream_t s = G->stream;
  if (mem_kind == PIRRT_MEM_HOST) {
    for (int32_t v = 0; v < n; ++v) {
      uint32_t w;
      memcpy(&w, &pcost_in[v], 4);
      if (parent_in[v] < -1 || parent_in[v] >= n || parent_in[v] == v) return fail(G, PIRRT_EINVAL, "bad parent");
      if ((w >> 31) != 0 || (w & 0x7f800000u) == 0x7f800000u) return fail(G, PIRRT_EINVAL, "bad pcost");
    }
  } else {
    HIP_OR_FAIL(G, hipMemsetAsync(G->dflag, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(k_check_policy, dim3(grid_for(n)), dim3(256), 0, s, n, parent_in, pcost_in, G->dflag);
    HIP_OR_FAIL(G, hipGetLastError());
    int32_t bad = 0;
    if ((rc = read_flag(G, &bad))) return rc;
    if (bad) return fail(G, PIRRT_EINVAL, "bad parent or pcost");
  }
  const float* gs = g_in;
  const int32_t* ps = parent_in;
  const float* cs = pcost_in;
  if (mem_kind == PIRRT_MEM_HOST) {
    HIP_OR_FAIL(G, hipMemcpyAsync(G->g2, g_in, sizeof(float) * (size_t)n, hipMemcpyHostToDevice, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(G->parent2, parent_in, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(G->pcost2, pcost_in, sizeof(float) * (size_t)n, hipMemcpyHostToDevice, s));
    gs = G->g2;
    ps = G->parent2;
    cs = G->pcost2;
  }
  launch_policy_from_ext(n, G->slot_of, gs, ps, cs, G->g, G->parent, G->pcost, s);
  HIP_OR_FAIL(G, hipGetLastError());
  HIP_OR_FAIL(G, hipStreamSynchronize(s));
  return PIRRT_OK;
}

int pirrt_snapshot_save(pirrt_graph* G) {
  int rc = guard(G);
  if (rc) return rc;
  const int64_t n = G->n;
  if (n > G->snap_cap) {
    float* a = nullptr;
    int32_t* b = nullptr;
    float* c = nullptr;
    if (!dalloc(&a, n) || !dalloc(&b, n) || !dalloc(&c, n)) {
      dfree(a);
      dfree(b);
      dfree(c);
      return fail(G, PIRRT_ENOMEM, "device allocation for the snapshot failed");
    }
    dfree(G->sg);
    dfree(G->sparent);
    dfree(G->spcost);
    G->sg = a;
    G->sparent = b;
    G->spcost = c;
    G->snap_cap = n;
  }
  hipStream_t s = G->stream;
  if (n > 0) {
    HIP_OR_FAIL(G, hipMemcpyAsync(G->sg, G->g, sizeof(float) * (size_t)n, hipMemcpyDeviceToDevice, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(G->sparent, G->parent, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(G->spcost, G->pcost, sizeof(float) * (size_t)n, hipMemcpyDeviceToDevice, s));
  }
  HIP_OR_FAIL(G, hipStreamSynchronize(s));
  G->snap_n = n;
  return PIRRT_OK;
}

int pirrt_snapshot_restore(pirrt_graph* G) {
  int rc = guard(G);
  if (rc) return rc;
  if (G->snap_n < 0 || G->snap_n != G->n) return fail(G, PIRRT_EINVAL, "no snapshot for this vertex count");
  const int64_t n = G->n;
  hipStream_t s = G->stream;
  if (n > 0) {
    HIP_OR_FAIL(G, hipMemcpyAsync(G->g, G->sg, sizeof(float) * (size_t)n, hipMemcpyDeviceToDevice, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(G->parent, G->sparent, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(G->pcost, G->spcost, sizeof(float) * (size_t)n, hipMemcpyDeviceToDevice, s));
  }
  HIP_OR_FAIL(G, hipStreamSynchronize(s));
  return PIRRT_OK;
}

int pirrt_get_adjacency(pirrt_graph* G, int64_t* ptr, int32_t* nbr, float* cost, int mem_kind) {
  int rc = guard(G);
  if (rc) return rc;
  if (mem_kind != PIRRT_MEM_HOST && mem_kind != PIRRT_MEM_DEVICE) return fail(G, PIRRT_EINVAL, "bad mem_kind");
  hipStream_t s = G->stream;
  const size_t n = (size_t)G->n, m = (size_t)G->nnz;
  // translated on the host: rows in caller order, neighbours as caller ids
  std::vector<int64_t> rp(n + 1), out_ptr(n + 1);
  std::vector<int32_t> col(m), ext(n), out_col(m);
  std::vector<float> cst(m), out_cst(m);
  HIP_OR_FAIL(G, hipMemcpyAsync(rp.data(), G->rp, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, s));
  if (m) {
    HIP_OR_FAIL(G, hipMemcpyAsync(col.data(), G->col, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(cst.data(), G->cst, sizeof(float) * m, hipMemcpyDeviceToHost, s));
  }
  if (n) HIP_OR_FAIL(G, hipMemcpyAsync(ext.data(), G->ext_of, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(G, hipStreamSynchronize(s));
  out_ptr[0] = 0;
  for (size_t e = 0; e < n; ++e) {
    const size_t sl = (size_t)G->hslot[e];
    int64_t k = out_ptr[e];
    for (int64_t j = rp[sl]; j < rp[sl + 1]; ++j, ++k) {
      out_col[(size_t)k] = ext[(size_t)col[(size_t)j]];
      out_cst[(size_t)k] = cst[(size_t)j];
    }
    out_ptr[e + 1] = k;
  }
  const hipMemcpyKind kind = mem_kind == PIRRT_MEM_DEVICE ? hipMemcpyHostToDevice : hipMemcpyHostToHost;
  if (ptr) HIP_OR_FAIL(G, hipMemcpy(ptr, out_ptr.data(), sizeof(int64_t) * (n + 1), kind));
  if (m && nbr) HIP_OR_FAIL(G, hipMemcpy(nbr, out_col.data(), sizeof(int32_t) * m, kind));
  if (m && cost) HIP_OR_FAIL(G, hipMemcpy(cost, out_cst.data(), sizeof(float) * m, kind));
  return PIRRT_OK;
}

}  // extern "C"
