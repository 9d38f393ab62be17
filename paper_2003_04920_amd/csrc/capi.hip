// Host runtime and C ABI (declared in include/pirrt.h): graph storage on the device,
// batch insertion, and the Replan driver of Alg. 2 for one graph or for a batch of
// independent graphs ("problems") stored side by side.
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
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
constexpr int kGraphIterCounts = 4;  // captured loop bodies of 1, 2, 4 and 8 iterations
constexpr int64_t kAdjSlack = 4;     // entries past the end of the adjacency arrays (quad loads)

// Pinned host block for small read-backs.
struct HostBlock {
  LoopCtl ctl;
  unsigned long long hops;
  int32_t flag;
  int32_t count[3];
  int64_t word;
};

// Validation kernels for device-resident inputs of replan / set_policy.
__global__ void k_check_h(int32_t n, const float* __restrict__ h, int* __restrict__ bad) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && !(h[v] >= 0.0f)) atomicOr(bad, 1);
}

// parent ids are local to the problem [base, base + len) of each vertex.
__global__ void k_check_policy(int32_t n, const int32_t* __restrict__ parent, const float* __restrict__ pcost,
                               const int32_t* __restrict__ prob, const int64_t* __restrict__ base,
                               int* __restrict__ bad) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int64_t b = prob ? base[prob[v]] : 0, len = prob ? base[prob[v] + 1] - b : n;
  int32_t p = parent[v];
  uint32_t w = __float_as_uint(pcost[v]);
  if (p < -1 || p >= len || p == v - b) atomicOr(bad, 1);
  if ((w >> 31) != 0 || (w & 0x7f800000u) == 0x7f800000u) atomicOr(bad, 2);
}

inline unsigned grid_for(int64_t n, int per = 256) {
  int64_t b = (n + per - 1) / per;
  return (unsigned)(b > 0 ? b : 1);
}

thread_local std::string g_create_error;

// Identity of a captured loop body: every pointer and size baked into its nodes.
struct LoopKey {
  const void* ptrs[17];
  int64_t n, nnz;
  int32_t P, prune, variant, walk_parts, walk_coherent, eval_levels, has_h, iters, mid, lookahead, truncated, blocks;
  int32_t bitmap_tiles, walk_rank;
  bool operator==(const LoopKey& o) const { return memcmp(this, &o, sizeof(LoopKey)) == 0; }
};

}  // namespace

// Device memory source of a handle: the caller's allocator callbacks (called with the
// handle's device current) or hipMalloc / hipFree.
struct DevAlloc {
  void* (*alloc)(size_t bytes, void* ctx) = nullptr;
  void (*free)(void* ptr, void* ctx) = nullptr;
  void* ctx = nullptr;
};

struct pirrt_graph {
  DevAlloc A;
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream used only to capture loop bodies
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
  // Evaluate scratch (the level-synchronous evaluator; the child arrays double as
  // renumbering scratch)
  int32_t* child_cnt = nullptr;
  int32_t* child_ptr = nullptr;
  int32_t* child = nullptr;
  int32_t* fr0 = nullptr;
  int32_t* fr1 = nullptr;
  int32_t* lvl = nullptr;
  // promising / domain marks and Evaluate stamps {epoch, g bits}
  uint8_t* stamp = nullptr;
  int32_t* dlist = nullptr;  // compacted Improve domain
  int32_t* tiles = nullptr;  // batches: active tile list
  unsigned long long* word = nullptr;
  bool eval_levels = false;   // level-synchronous Evaluate instead of the walk
  int walk_parts = 1;         // walk launches over consecutive slot ranges
  // Evaluate stamps at workgroup scope by default: a stale stamp only makes a walk climb
  // further (every path gives the same bits), and L1-cached stamp reads beat device-scope
  // ones (6D 100k per-batch Replans: 23% faster); the autotuner tries both.
  bool walk_coherent = false;
  // Single graphs up to this many vertices replan on the host (PIRRT_HOST_MAX; 0 = never)
  int64_t host_max = 512;
  uint64_t adj_version = 0;  // bumped whenever the adjacency or the slot order changes
  // host copies of the slot-ordered adjacency and ids for the host Replan
  uint64_t hm_version = ~0ull;
  std::vector<int64_t> hm_rp;
  std::vector<int32_t> hm_col, hm_ext;
  std::vector<float> hm_cst;
  // storage order: ext_of[slot] = caller id, slot_of[id] = slot (host mirror hslot)
  int32_t* ext_of = nullptr;
  int32_t* slot_of = nullptr;
  std::vector<int32_t> hslot;
  int64_t reorder_n = 0;          // vertex count at the last renumbering
  double reorder_growth = 1.25;   // renumber when n grows by this factor (0 = never)
  // ... and, below this many vertices, only when the batch itself brings that growth
  // (a graph built in one or a few large inserts): a small graph growing in many small
  // batches replans as fast in insertion order, and each renumbering costs more than it
  // saves there (PIRRT_REORDER_MIN)
  int64_t reorder_min = 131072;
  bool clustered_order = true;    // seed clusters on top of the breadth-first order
  bool renumber_pending = false;  // batch problems added since the last renumbering
  // problems: problem i holds caller ids [pbase[i], pbase[i+1]) and the same slots
  bool batched = false;
  std::vector<int64_t> pbase{0, 0};
  int32_t* prob = nullptr;  // problem of each slot (used by batches only)
  int64_t* dbase = nullptr;  // device copy of pbase
  char* dgrow = nullptr;     // growing problems: block table and the new bases
  int64_t dgrow_cap = 0;     // bytes
  int64_t dbase_cap = 0;
  // per-problem Replan state
  ProblemState* ps = nullptr;
  ProblemState* hps = nullptr;  // pinned mirror
  IterCounters* ctr = nullptr;
  LoopCtl* ctl = nullptr;
  int32_t* pscratch = nullptr;  // per-problem ints (renumbering counters)
  int32_t* pstart = nullptr;    // per-problem ints (renumbering level starts)
  int32_t* droots = nullptr;    // caller ids of the slots that carry root marks
  int32_t nroots = 0;
  std::vector<int32_t> hroots;       // host copy of droots
  std::vector<int32_t> snap_roots;   // the root marks held by the snapshot
  int64_t pcap = 0;
  // insertion / renumbering / translation scratch
  int32_t* add = nullptr;
  int32_t* add0 = nullptr;  // per-slot counts of an insert's new entries (zero between inserts)
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
  EvalInfo* info = nullptr;
  int32_t* dflag = nullptr;
  int32_t* dcount = nullptr;
  unsigned long long* dhops = nullptr;
  bool trace = false;  // per-iteration counters to stderr (direct loop only)
  HostBlock* host = nullptr;
  hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  // captured loop bodies
  bool use_graph = true;
  hipGraphExec_t loop_exec[kGraphIterCounts] = {nullptr, nullptr, nullptr, nullptr};
  LoopKey loop_key[kGraphIterCounts];
  int32_t last_iterations = 0;  // iterations of the previous Replan (loop planning)
  // tuning
  int32_t mid_hint = 64;
  int row_variant = 1;  // 8 lanes x 2 quads per row; the autotuner tries the others
  int batch_blocks = kBatchBlocks;  // batches: workgroups per grid-stride launch (autotuned)
  int cus = 256;                     // compute units of the device
  int32_t bitmap_tiles = INT32_MAX;  // batches: tile lists from the bitmap up to this many tiles
  bool walk_rank = true;  // batches: the walk takes the active tiles by their rank inside their problem
  bool lookahead = false;  // narrowed Improve domain for the current call (PIRRT_LOOKAHEAD)
  bool truncated = false;  // truncated Evaluate for the current call (PIRRT_TRUNCATED)
  LoopKey prev_key;          // loop arguments of the previous Replan (graphs when they repeat)
  bool have_prev_key = false;
  bool small_graphs = true;  // single-workgroup Replan up to kSmallMax vertices (PIRRT_SMALL=0: off)
  // Host-side fault hook (PIRRT_FAULT_INJECT at create): "launch" makes the next
  // Replan fail as if a kernel launch had returned a HIP error (no device work is
  // involved; the handle is poisoned like after a real one), "alloc" makes the next
  // growth of the vertex storage fail as if the device allocation had.
  bool fault_launch = false;
  bool fault_alloc = false;
  bool poisoned = false;
  std::string err;
};

struct pirrt_batch {
  pirrt_graph* G;
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

#define HIP_OR_FAIL(G, expr)                                \
  do {                                                      \
    hipError_t e_ = (expr);                                 \
    if (e_ != hipSuccess) return fail_device(G, e_, #expr); \
  } while (0)

void* raw_alloc(const DevAlloc& A, size_t bytes) {
  if (A.alloc) return A.alloc(bytes, A.ctx);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void raw_free(const DevAlloc& A, void* p) {
  if (!p) return;
  if (A.free)
    A.free(p, A.ctx);
  else
    (void)hipFree(p);
}

template <class T>
bool dalloc(const DevAlloc& A, T** p, int64_t count) {
  if (count <= 0) count = 1;
  *p = static_cast<T*>(raw_alloc(A, sizeof(T) * (size_t)count));
  return *p != nullptr;
}

template <class T>
void dfree(const DevAlloc& A, T*& p) {
  raw_free(A, p);
  p = nullptr;
}

int guard(pirrt_graph* G) {
  if (!G) return PIRRT_EINVAL;
  if (G->poisoned) return PIRRT_EDEVICE;
  hipError_t e = hipSetDevice(G->device);
  if (e != hipSuccess) return fail_device(G, e, "hipSetDevice");
  return PIRRT_OK;
}

hipMemcpyKind in_kind(int mem_kind) {
  return mem_kind == PIRRT_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
}

int ensure_scan(pirrt_graph* G, int64_t n) {
  size_t need = scan_scratch_bytes(n);
  if (need <= G->scan_bytes) return PIRRT_OK;
  void* p = raw_alloc(G->A, need);
  if (!p) return fail(G, PIRRT_ENOMEM, "device allocation of scan scratch failed");
  raw_free(G->A, G->scan_scratch);
  G->scan_scratch = p;
  G->scan_bytes = need;
  return PIRRT_OK;
}

void drop_loops(pirrt_graph* G) {
  for (int k = 0; k < kGraphIterCounts; ++k)
    if (G->loop_exec[k]) {
      (void)hipGraphExecDestroy(G->loop_exec[k]);
      G->loop_exec[k] = nullptr;
    }
}

void free_vertex_arrays(pirrt_graph* G) {
  dfree(G->A, G->rp); dfree(G->A, G->rp2); dfree(G->A, G->g); dfree(G->A, G->parent); dfree(G->A, G->pcost); dfree(G->A, G->child_cnt);
  dfree(G->A, G->child_ptr); dfree(G->A, G->child); dfree(G->A, G->fr0); dfree(G->A, G->fr1); dfree(G->A, G->lvl); dfree(G->A, G->stamp);
  dfree(G->A, G->add); dfree(G->A, G->deg); dfree(G->A, G->pending); dfree(G->A, G->hbuf); dfree(G->A, G->ext_of); dfree(G->A, G->slot_of);
  dfree(G->A, G->g2); dfree(G->A, G->parent2); dfree(G->A, G->pcost2); dfree(G->A, G->ext2); dfree(G->A, G->word); dfree(G->A, G->prob);
  dfree(G->A, G->dlist); dfree(G->A, G->tiles); dfree(G->A, G->add0);
}

void forget_vertex_arrays(pirrt_graph* T) {
  T->rp = T->rp2 = nullptr;
  T->g = T->pcost = T->hbuf = T->g2 = T->pcost2 = nullptr;
  T->parent = T->child_cnt = T->child_ptr = T->child = T->fr0 = T->fr1 = T->lvl = nullptr;
  T->add = T->deg = T->pending = T->ext_of = T->slot_of = T->parent2 = T->ext2 = T->prob = nullptr;
  T->stamp = nullptr;
  T->dlist = nullptr;
  T->tiles = nullptr;
  T->add0 = nullptr;
  T->word = nullptr;
}

// Grows every per-vertex array to hold `need` vertices, keeping the policy, the
// row offsets, the id maps and the problem map.  On failure nothing changes.
int ensure_vcap(pirrt_graph* G, int64_t need) {
  if (need <= G->vcap) return PIRRT_OK;
  if (G->fault_alloc) {  // injected failure, once
    G->fault_alloc = false;
    return fail(G, PIRRT_ENOMEM, "device allocation for vertex storage failed (injected by PIRRT_FAULT_INJECT)");
  }
  int64_t cap = G->vcap + G->vcap / 2;
  if (cap < need) cap = need;
  if (cap < kMinVertexCap) cap = kMinVertexCap;
  pirrt_graph T;  // holds the new arrays until all allocations succeeded
  T.A = G->A;
  bool ok = dalloc(G->A, &T.rp, cap + 1) && dalloc(G->A, &T.rp2, cap + 1) && dalloc(G->A, &T.g, cap) && dalloc(G->A, &T.parent, cap) &&
            dalloc(G->A, &T.pcost, cap) && dalloc(G->A, &T.child_cnt, cap) && dalloc(G->A, &T.child_ptr, cap + 1) &&
            dalloc(G->A, &T.child, cap) && dalloc(G->A, &T.fr0, cap) && dalloc(G->A, &T.fr1, cap) &&
            dalloc(G->A, &T.lvl, cap + kMaxMidLaunches + 8) && dalloc(G->A, &T.stamp, cap) && dalloc(G->A, &T.add, cap) &&
            dalloc(G->A, &T.deg, cap) && dalloc(G->A, &T.pending, cap) && dalloc(G->A, &T.hbuf, cap) && dalloc(G->A, &T.ext_of, cap) &&
            dalloc(G->A, &T.slot_of, cap) && dalloc(G->A, &T.g2, cap) && dalloc(G->A, &T.parent2, cap) && dalloc(G->A, &T.pcost2, cap) &&
            dalloc(G->A, &T.ext2, cap) && dalloc(G->A, &T.word, cap) && dalloc(G->A, &T.prob, cap) && dalloc(G->A, &T.dlist, cap) &&
            dalloc(G->A, &T.tiles, 2 * (cap / kTileSlots + 2)) && dalloc(G->A, &T.add0, cap);
  if (!ok) {
    free_vertex_arrays(&T);
    return fail(G, PIRRT_ENOMEM, "device allocation for vertex storage failed");
  }
  hipStream_t s = G->stream;
  HIP_OR_FAIL(G, hipMemsetAsync(T.child_cnt, 0, sizeof(int32_t) * (size_t)cap, s));
  HIP_OR_FAIL(G, hipMemsetAsync(T.stamp, 0, (size_t)cap, s));
  HIP_OR_FAIL(G, hipMemsetAsync(T.add0, 0, sizeof(int32_t) * (size_t)cap, s));
  HIP_OR_FAIL(G, hipMemsetAsync(T.word, 0, sizeof(unsigned long long) * (size_t)cap, s));
  HIP_OR_FAIL(G, hipMemsetAsync(T.rp, 0, sizeof(int64_t) * (size_t)(cap + 1), s));
  if (G->n > 0) {
    const size_t n = (size_t)G->n;
    HIP_OR_FAIL(G, hipMemcpyAsync(T.rp, G->rp, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(T.g, G->g, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(T.parent, G->parent, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(T.pcost, G->pcost, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(T.ext_of, G->ext_of, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(T.slot_of, G->slot_of, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(T.prob, G->prob, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
  }
  HIP_OR_FAIL(G, hipStreamSynchronize(s));
  free_vertex_arrays(G);
  G->rp = T.rp; G->rp2 = T.rp2; G->g = T.g; G->parent = T.parent; G->pcost = T.pcost;
  G->child_cnt = T.child_cnt; G->child_ptr = T.child_ptr; G->child = T.child; G->fr0 = T.fr0; G->fr1 = T.fr1;
  G->lvl = T.lvl; G->stamp = T.stamp; G->add = T.add; G->deg = T.deg; G->pending = T.pending; G->hbuf = T.hbuf;
  G->ext_of = T.ext_of; G->slot_of = T.slot_of; G->g2 = T.g2; G->parent2 = T.parent2; G->pcost2 = T.pcost2;
  G->ext2 = T.ext2; G->word = T.word; G->prob = T.prob; G->dlist = T.dlist; G->tiles = T.tiles; G->add0 = T.add0;
  forget_vertex_arrays(&T);
  G->vcap = cap;
  drop_loops(G);
  return ensure_scan(G, cap + 1);
}

// Per-problem state for `need` problems.
int ensure_pcap(pirrt_graph* G, int64_t need) {
  if (need <= G->pcap) return PIRRT_OK;
  int64_t cap = G->pcap * 2 > need ? G->pcap * 2 : need;
  if (cap < 16) cap = 16;
  ProblemState* ps = nullptr;
  IterCounters* ctr = nullptr;
  int32_t* scr = nullptr;
  int32_t* roots = nullptr;
  ProblemState* hps = nullptr;
  int32_t* pst = nullptr;
  bool ok = dalloc(G->A, &ps, cap) && dalloc(G->A, &ctr, cap * kCounterSlots) && dalloc(G->A, &scr, cap) && dalloc(G->A, &roots, cap) &&
            dalloc(G->A, &pst, cap);
  if (ok && hipHostMalloc((void**)&hps, sizeof(ProblemState) * (size_t)cap, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    hps = nullptr;
    ok = false;
  }
  if (!ok) {
    dfree(G->A, ps); dfree(G->A, ctr); dfree(G->A, scr); dfree(G->A, roots); dfree(G->A, pst);
    return fail(G, PIRRT_ENOMEM, "allocation of per-problem state failed");
  }
  if (G->nroots > 0)
    HIP_OR_FAIL(G, hipMemcpy(roots, G->droots, sizeof(int32_t) * (size_t)G->nroots, hipMemcpyDeviceToDevice));
  dfree(G->A, G->ps); dfree(G->A, G->ctr); dfree(G->A, G->pscratch); dfree(G->A, G->droots); dfree(G->A, G->pstart);
  if (G->hps) (void)hipHostFree(G->hps);
  G->ps = ps; G->ctr = ctr; G->pscratch = scr; G->droots = roots; G->hps = hps; G->pstart = pst;
  G->pcap = cap;
  drop_loops(G);
  return PIRRT_OK;
}

int upload_bases(pirrt_graph* G) {
  const int64_t m = (int64_t)G->pbase.size();
  if (m > G->dbase_cap) {
    int64_t* p = nullptr;
    int64_t cap = m * 2 > 64 ? m * 2 : 64;
    if (!dalloc(G->A, &p, cap)) return fail(G, PIRRT_ENOMEM, "allocation of problem table failed");
    dfree(G->A, G->dbase);
    G->dbase = p;
    G->dbase_cap = cap;
    drop_loops(G);
  }
  HIP_OR_FAIL(G, hipMemcpyAsync(G->dbase, G->pbase.data(), sizeof(int64_t) * (size_t)m, hipMemcpyHostToDevice,
                                G->stream));
  HIP_OR_FAIL(G, hipStreamSynchronize(G->stream));
  return PIRRT_OK;
}

// Spare adjacency arrays able to hold `need` entries.
int ensure_spare(pirrt_graph* G, int64_t need) {
  if (need <= G->ecap2) return PIRRT_OK;
  int64_t cap = G->ecap2 + G->ecap2 / 2;
  if (cap < need) cap = need;
  if (cap < kMinEdgeCap) cap = kMinEdgeCap;
  int32_t* c = nullptr;
  float* w = nullptr;
  if (!dalloc(G->A, &c, cap + kAdjSlack) || !dalloc(G->A, &w, cap + kAdjSlack)) {
    dfree(G->A, c);
    dfree(G->A, w);
    return fail(G, PIRRT_ENOMEM, "device allocation for adjacency failed");
  }
  dfree(G->A, G->col2);
  dfree(G->A, G->cst2);
  G->col2 = c;
  G->cst2 = w;
  G->ecap2 = cap;
  return PIRRT_OK;
}

// Room for `need` entries in the current adjacency arrays (keeping the entries).
int ensure_adjacency(pirrt_graph* G, int64_t need) {
  if (need <= G->ecap) return PIRRT_OK;
  int64_t cap = G->ecap + G->ecap / 2;
  if (cap < need) cap = need;
  if (cap < kMinEdgeCap) cap = kMinEdgeCap;
  int32_t* c = nullptr;
  float* w = nullptr;
  if (!dalloc(G->A, &c, cap + kAdjSlack) || !dalloc(G->A, &w, cap + kAdjSlack)) {
    dfree(G->A, c);
    dfree(G->A, w);
    return fail(G, PIRRT_ENOMEM, "device allocation for adjacency failed");
  }
  if (G->nnz > 0) {
    HIP_OR_FAIL(G, hipMemcpyAsync(c, G->col, sizeof(int32_t) * (size_t)G->nnz, hipMemcpyDeviceToDevice, G->stream));
    HIP_OR_FAIL(G, hipMemcpyAsync(w, G->cst, sizeof(float) * (size_t)G->nnz, hipMemcpyDeviceToDevice, G->stream));
  }
  HIP_OR_FAIL(G, hipStreamSynchronize(G->stream));
  dfree(G->A, G->col);
  dfree(G->A, G->cst);
  G->col = c;
  G->cst = w;
  G->ecap = cap;
  drop_loops(G);
  return PIRRT_OK;
}

int ensure_staging(pirrt_graph* G, int64_t rows, int64_t nnz) {
  if (rows + 1 > G->brows_cap) {
    int64_t* p = nullptr;
    int64_t cap = rows + 1 > 1024 ? rows + 1 : 1024;
    if (!dalloc(G->A, &p, cap)) return fail(G, PIRRT_ENOMEM, "device allocation for batch staging failed");
    dfree(G->A, G->brp);
    G->brp = p;
    G->brows_cap = cap;
  }
  if (nnz > G->bnnz_cap) {
    int32_t* c = nullptr;
    int32_t* t = nullptr;
    float* w = nullptr;
    int64_t cap = nnz > 4096 ? nnz : 4096;
    if (!dalloc(G->A, &c, cap) || !dalloc(G->A, &t, cap) || !dalloc(G->A, &w, cap)) {
      dfree(G->A, c);
      dfree(G->A, t);
      dfree(G->A, w);
      return fail(G, PIRRT_ENOMEM, "device allocation for batch staging failed");
    }
    dfree(G->A, G->bcol);
    dfree(G->A, G->bslot);
    dfree(G->A, G->bcost);
    G->bcol = c;
    G->bslot = t;
    G->bcost = w;
    G->bnnz_cap = cap;
  }
  return PIRRT_OK;
}

void release_all(pirrt_graph* G) {
  drop_loops(G);
  free_vertex_arrays(G);
  dfree(G->A, G->col); dfree(G->A, G->cst); dfree(G->A, G->col2); dfree(G->A, G->cst2);
  dfree(G->A, G->sg); dfree(G->A, G->sparent); dfree(G->A, G->spcost);
  dfree(G->A, G->brp); dfree(G->A, G->bcol); dfree(G->A, G->bslot); dfree(G->A, G->bcost);
  dfree(G->A, G->info); dfree(G->A, G->dflag); dfree(G->A, G->dcount); dfree(G->A, G->dhops);
  dfree(G->A, G->ps); dfree(G->A, G->ctr); dfree(G->A, G->ctl); dfree(G->A, G->pscratch); dfree(G->A, G->droots); dfree(G->A, G->dbase);
  dfree(G->A, G->pstart); dfree(G->A, G->dgrow);
  if (G->hps) (void)hipHostFree(G->hps);
  G->hps = nullptr;
  raw_free(G->A, G->scan_scratch);
  G->scan_scratch = nullptr;
  if (G->host) (void)hipHostFree(G->host);
  G->host = nullptr;
  for (auto& e : G->ev)
    if (e) {
      (void)hipEventDestroy(e);
      e = nullptr;
    }
  if (G->cap_stream) (void)hipStreamDestroy(G->cap_stream);
  G->cap_stream = nullptr;
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

int32_t* problem_map(pirrt_graph* G) { return G->batched ? G->prob : nullptr; }
const int64_t* base_map(pirrt_graph* G) { return G->batched ? G->dbase : nullptr; }
// The second half of the tile array: the walk's order of the active tiles.
int32_t* walk_tiles(pirrt_graph* G) {
  return G->batched && G->walk_rank ? G->tiles + (G->vcap / kTileSlots + 2) : nullptr;
}

// Copies the policy out in caller order (device outputs are written directly;
// host outputs go through device staging).  In a batch, parents are local ids.
int policy_out(pirrt_graph* G, float* g_out, int32_t* parent_out, float* pcost_out, int mem_kind) {
  const int32_t n = (int32_t)G->n;
  hipStream_t s = G->stream;
  if (n == 0) return PIRRT_OK;
  const bool dev = mem_kind == PIRRT_MEM_DEVICE;
  float* gd = g_out ? (dev ? g_out : G->g2) : nullptr;
  int32_t* pd = parent_out ? (dev ? parent_out : G->parent2) : nullptr;
  float* cd = pcost_out ? (dev ? pcost_out : G->pcost2) : nullptr;
  launch_policy_to_ext(n, G->slot_of, G->ext_of, problem_map(G), base_map(G), G->g, G->parent, G->pcost, gd, pd,
                       cd, s);
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

// Renumbers the storage slots in breadth-first order of the graph, each problem
// inside its own slot range from its x_init (its first vertex); vertices the BFS
// cannot reach follow in their current order.
int renumber(pirrt_graph* G) {
  const int32_t n = (int32_t)G->n;
  const int32_t P = (int32_t)G->pbase.size() - 1;
  hipStream_t s = G->stream;
  int rc;
  if (n == 0) return PIRRT_OK;
  if ((rc = ensure_spare(G, G->nnz))) return rc;
  if ((rc = ensure_pcap(G, P))) return rc;
  if ((rc = upload_bases(G))) return rc;
  int32_t* visited = G->pending;
  int32_t* order = G->child;
  int32_t* F = G->fr0;
  int32_t* Fn = G->fr1;
  // the problems' x_init slots
  std::vector<int32_t> roots((size_t)P);
  for (int32_t i = 0; i < P; ++i) roots[(size_t)i] = G->hslot[(size_t)G->pbase[(size_t)i]];
  HIP_OR_FAIL(G, hipMemcpyAsync(Fn, roots.data(), sizeof(int32_t) * (size_t)P, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(G, hipMemsetAsync(visited, 0, sizeof(int32_t) * (size_t)n, s));
  launch_bfs_init(P, Fn, G->dbase, order, visited, G->pscratch, F, &G->dcount[0], s);
  HIP_OR_FAIL(G, hipGetLastError());
  // scratch of the level ordering (all free until the permutation below)
  int32_t* key = G->add;
  int32_t* cand = G->deg;
  int32_t* hist = G->lvl;
  int32_t* cursor = G->child_ptr;
  int64_t* off = G->rp2;
  launch_fill_i32(0, n, INT32_MAX, key, s);
  int32_t fsize = P, tag = 2, levels = 0;
  while (fsize > 0) {
    HIP_OR_FAIL(G, hipMemsetAsync(&G->dcount[1], 0, sizeof(int32_t), s));
    launch_bfs_discover(fsize, F, tag, G->rp, G->col, visited, key, cand, &G->dcount[1], s);
    HIP_OR_FAIL(G, hipGetLastError());
    HIP_OR_FAIL(G, hipMemcpyAsync(&G->host->count[1], &G->dcount[1], sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(G, hipStreamSynchronize(s));
    const int32_t m = G->host->count[1];
    if (m > n || ++levels > n) return fail_device(G, hipErrorUnknown, "renumbering visited too many vertices");
    launch_bfs_order_level(fsize, m, cand, key, hist, off, cursor, Fn, problem_map(G), G->pstart, G->pscratch, order,
                           G->scan_scratch, s);
    HIP_OR_FAIL(G, hipGetLastError());
    fsize = m;
    ++tag;
    std::swap(F, Fn);
  }
  launch_append_unvisited(n, visited, order, problem_map(G), G->pscratch, s);
  HIP_OR_FAIL(G, hipGetLastError());
  // every problem's range must be exactly full
  std::vector<int32_t> cnt((size_t)P);
  HIP_OR_FAIL(G, hipMemcpyAsync(cnt.data(), G->pscratch, sizeof(int32_t) * (size_t)P, hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(G, hipStreamSynchronize(s));
  for (int32_t i = 0; i < P; ++i)
    if (cnt[(size_t)i] != G->pbase[(size_t)i + 1]) return fail_device(G, hipErrorUnknown, "renumbering lost vertices");
  if (G->clustered_order) {
    // seeds by Luby rounds, then clusters in the breadth-first order of their seeds
    int32_t* state = G->pending;
    int32_t* win = G->add;
    HIP_OR_FAIL(G, hipMemsetAsync(state, 0, sizeof(int32_t) * (size_t)n, s));
    for (int round = 0;; ++round) {
      HIP_OR_FAIL(G, hipMemsetAsync(&G->dcount[1], 0, sizeof(int32_t), s));
      launch_mis_round(n, G->rp, G->col, state, win, &G->dcount[1], s);
      HIP_OR_FAIL(G, hipGetLastError());
      HIP_OR_FAIL(G, hipMemcpyAsync(&G->host->count[1], &G->dcount[1], sizeof(int32_t), hipMemcpyDeviceToHost, s));
      HIP_OR_FAIL(G, hipStreamSynchronize(s));
      if (G->host->count[1] == 0) break;
      if (round > n) return fail_device(G, hipErrorUnknown, "independent-set rounds did not finish");
    }
    launch_cluster_order(n, G->rp, G->col, state, order, G->fr1, G->fr0, G->deg, G->rp2, G->child_ptr, G->lvl,
                         G->scan_scratch, s);
    HIP_OR_FAIL(G, hipGetLastError());
    order = G->lvl;
  }
  PermuteArgs a;
  a.n = n;
  a.order = order;
  a.newslot = G->child_ptr;
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
  // every problem now fills its slot range (grown problems held slots past it before)
  if (G->batched) launch_problem_map(n, P, G->dbase, G->prob, s);
  HIP_OR_FAIL(G, hipGetLastError());
  G->hslot.resize((size_t)n);
  HIP_OR_FAIL(G, hipMemcpyAsync(G->hslot.data(), G->slot_of, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(G, hipStreamSynchronize(s));
  G->reorder_n = n;
  G->renumber_pending = false;
  G->adj_version++;
  G->snap_n = -1;  // a snapshot in the old order is no longer valid
  drop_loops(G);
  return PIRRT_OK;
}

// Insertion-time policy of the n_new vertices appended after slot n_old, one
// dependency level at a time (staged rows in brp / bcol / bslot / bcost, the new
// adjacency built).  insert_root: the slot that becomes a root (g = 0), or -1.
int insert_levels(pirrt_graph* G, int32_t n_new, int64_t n_old, int32_t insert_root, const int64_t* brp,
                  const int32_t* bcol, const float* bcost) {
  hipStream_t s = G->stream;
  // dcount[0] / dcount[1]: the frontier sizes of alternate levels; dcount[2]: vertices
  // placed.  Levels go out kLevelsPerCheck at a time (a level past the last one finds
  // an empty frontier and does nothing), then one read-back tells whether more remain.
  constexpr int kLevelsPerCheck = 4;
  HIP_OR_FAIL(G, hipMemsetAsync(G->dcount, 0, 3 * sizeof(int32_t), s));
  launch_pending(n_new, n_old, brp, bcol, G->pending, G->fr0, &G->dcount[0], s);
  HIP_OR_FAIL(G, hipGetLastError());
  if (n_new <= kInsertBlockMax) {  // a small batch: every level in one single-workgroup launch
    launch_insert_block(&G->dcount[0], &G->dcount[2], G->fr0, G->fr1, n_old, n_new, insert_root, brp, bcol, G->bslot,
                        bcost, G->rp, G->col, G->g, G->parent, G->pcost, G->pending, s);
    HIP_OR_FAIL(G, hipGetLastError());
    HIP_OR_FAIL(G, hipMemcpyAsync(G->host->count, G->dcount, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(G, hipStreamSynchronize(s));
    if (G->host->count[2] != n_new)
      return fail_device(G, hipErrorUnknown, "insertion levels did not cover the batch");
    return PIRRT_OK;
  }
  for (int64_t level = 0;;) {
    for (int i = 0; i < kLevelsPerCheck; ++i, ++level) {
      const int cur = (int)(level & 1), nxt = cur ^ 1;
      HIP_OR_FAIL(G, hipMemsetAsync(&G->dcount[nxt], 0, sizeof(int32_t), s));
      launch_insert_level(n_new, &G->dcount[cur], &G->dcount[2], cur ? G->fr1 : G->fr0, n_old, insert_root, brp, bcol,
                          G->bslot, bcost, G->rp, G->col, G->g, G->parent, G->pcost, G->pending,
                          nxt ? G->fr1 : G->fr0, &G->dcount[nxt], s);
      HIP_OR_FAIL(G, hipGetLastError());
    }
    HIP_OR_FAIL(G, hipMemcpyAsync(G->host->count, G->dcount, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(G, hipStreamSynchronize(s));
    if (G->host->count[level & 1] == 0) break;  // the next level's frontier is empty
    if (G->host->count[2] > n_new || level > (int64_t)n_new + kLevelsPerCheck)
      return fail_device(G, hipErrorUnknown, "insertion levels exceed the batch");
  }
  if (G->host->count[2] != n_new) return fail_device(G, hipErrorUnknown, "insertion levels did not cover the batch");
  return PIRRT_OK;
}

// Appends n_new vertices with forward rows.  With new_problem the block starts a
// new problem of a batch and its rows use ids local to the block; otherwise the
// rows use global ids and extend the last (only) problem.
int insert_rows(pirrt_graph* G, int32_t n_new, const int64_t* row_ptr, const int32_t* col, const float* cost,
                int mem_kind, bool new_problem) {
  if (mem_kind != PIRRT_MEM_HOST && mem_kind != PIRRT_MEM_DEVICE) return fail(G, PIRRT_EINVAL, "bad mem_kind");
  if (n_new < 0) return fail(G, PIRRT_EINVAL, "n_new < 0");
  if (n_new == 0 && !new_problem) return PIRRT_OK;
  if (n_new == 0) return fail(G, PIRRT_EINVAL, "a problem needs at least one vertex");
  if (!row_ptr) return fail(G, PIRRT_EINVAL, "row_ptr is NULL");
  if (G->n + (int64_t)n_new > (int64_t)INT32_MAX - 1) return fail(G, PIRRT_EINVAL, "vertex ids beyond INT32_MAX");
  hipStream_t s = G->stream;
  int rc;
  int64_t nnz_b = 0;
  const int64_t n_old = G->n, n1 = G->n + n_new;
  // Device rows of a single graph are read where they are (the call is synchronous):
  // their entry count and their validation come back in one round trip.
  const bool direct = mem_kind == PIRRT_MEM_DEVICE && !new_problem && col && cost;
  const int64_t* brp = G->brp;
  const int32_t* bcol = G->bcol;
  const float* bcost = G->bcost;
  int32_t bad = 0;
  if (direct) {
    HIP_OR_FAIL(G, hipMemsetAsync(G->dflag, 0, sizeof(int32_t), s));
    launch_validate_rows(n_new, n_old, 0, row_ptr, col, cost, 0, G->dflag, s, row_ptr + n_new);
    HIP_OR_FAIL(G, hipGetLastError());
    HIP_OR_FAIL(G, hipMemcpyAsync(&G->host->word, row_ptr + n_new, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(&G->host->flag, G->dflag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(G, hipStreamSynchronize(s));
    nnz_b = G->host->word;
    bad = G->host->flag;
    if (!bad && (rc = ensure_staging(G, n_new, nnz_b))) return rc;  // the slot translation's room
    brp = row_ptr;
    bcol = col;
    bcost = cost;
  } else {
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
    brp = G->brp;
    bcol = G->bcol;
    bcost = G->bcost;
    HIP_OR_FAIL(G, hipMemcpyAsync(G->brp, row_ptr, sizeof(int64_t) * (size_t)(n_new + 1), in_kind(mem_kind), s));
    if (nnz_b > 0) {
      HIP_OR_FAIL(G, hipMemcpyAsync(G->bcol, col, sizeof(int32_t) * (size_t)nnz_b, in_kind(mem_kind), s));
      HIP_OR_FAIL(G, hipMemcpyAsync(G->bcost, cost, sizeof(float) * (size_t)nnz_b, in_kind(mem_kind), s));
    }
    if (new_problem) launch_offset_ids(nnz_b, (int32_t)n_old, G->bcol, s);  // local -> global ids
    HIP_OR_FAIL(G, hipMemsetAsync(G->dflag, 0, sizeof(int32_t), s));
    launch_validate_rows(n_new, n_old, new_problem ? n_old : 0, G->brp, G->bcol, G->bcost, nnz_b, G->dflag, s);
    HIP_OR_FAIL(G, hipGetLastError());
    if ((rc = read_flag(G, &bad))) return rc;
  }
  if (bad) {
    std::string m = "invalid batch:";
    if (bad & 1) m += " row_ptr not 0-based / non-decreasing / bounded;";
    if (bad & 2) m += new_problem ? " col outside [0, own local id);" : " col outside [0, own id);";
    if (bad & 4) m += " cost not finite, negative or -0.0;";
    return fail(G, PIRRT_EINVAL, m);
  }
  if ((rc = ensure_vcap(G, n1))) return rc;
  if (new_problem) {
    if ((rc = ensure_adjacency(G, G->nnz + 2 * nnz_b))) return rc;
  } else if ((rc = ensure_spare(G, G->nnz + 2 * nnz_b))) {
    return rc;
  }
  // new vertices take the slots after the existing ones; neighbours to slots
  launch_identity_ids(n_old, n1, G->ext_of, G->slot_of, s, G->prob, new_problem ? (int32_t)G->pbase.size() - 1 : 0);
  launch_translate(nnz_b, bcol, G->slot_of, G->bslot, s);
  if (new_problem) {
    // a new problem shares no edge with the older ones: its rows are appended
    launch_append(n_new, n_old, G->nnz, G->brp, G->bslot, G->bcost, G->rp, G->col, G->cst, G->add, G->deg, G->rp2,
                  G->scan_scratch, s);
    HIP_OR_FAIL(G, hipGetLastError());
  } else {
    // adjacency rebuild into the spare arrays, then swap
    launch_rebuild(n_new, n_old, brp, G->bslot, bcost, G->rp, G->col, G->cst, G->rp2, G->col2, G->cst2, G->add,
                   G->add0, G->deg, G->scan_scratch, s);
    HIP_OR_FAIL(G, hipGetLastError());
    std::swap(G->rp, G->rp2);
    std::swap(G->col, G->col2);
    std::swap(G->cst, G->cst2);
    std::swap(G->ecap, G->ecap2);
  }
  G->n = n1;
  G->nnz += 2 * nnz_b;
  G->adj_version++;
  G->hslot.resize((size_t)n1);
  for (int64_t v = n_old; v < n1; ++v) G->hslot[(size_t)v] = (int32_t)v;
  if (new_problem)
    G->pbase.push_back(n1);
  else
    G->pbase.back() = n1;
  drop_loops(G);
  const int32_t insert_root = new_problem ? (int32_t)n_old : (n_old == 0 ? 0 : -1);
  if ((rc = insert_levels(G, n_new, n_old, insert_root, brp, bcol, bcost))) return rc;
  if (new_problem) {
    G->renumber_pending = true;
  } else if (G->reorder_growth > 0.0 && (double)n1 >= G->reorder_growth * (double)G->reorder_n &&
             (n1 >= G->reorder_min || (double)n_new >= (1.0 - 1.0 / G->reorder_growth) * (double)n1)) {
    if ((rc = renumber(G))) return rc;
  }
  return PIRRT_OK;
}

// Grows problems of a batch: block k appends n_new[k] vertices (forward rows in the
// problem's local ids) to problem problems[k].  The new vertices are first appended
// after every existing slot with temporary "append ids", the adjacency rebuilt and
// their insertion-time policy computed exactly as for a single graph (the
// tie-breaking order inside each problem is the order of its local ids under both id
// sets); then every vertex takes its final caller id, the problems' bases move, and
// the next Replan renumbers the slots (the layout is no longer one range per problem).
int grow_problems(pirrt_graph* G, int32_t count, const int32_t* problems, const int32_t* n_new,
                  const int64_t* row_ptr, const int32_t* col, const float* cost, int mem_kind) {
  if (mem_kind != PIRRT_MEM_HOST && mem_kind != PIRRT_MEM_DEVICE) return fail(G, PIRRT_EINVAL, "bad mem_kind");
  if (count < 0) return fail(G, PIRRT_EINVAL, "count < 0");
  if (count == 0) return PIRRT_OK;
  if (!problems || !n_new) return fail(G, PIRRT_EINVAL, "problems or n_new is NULL");
  const int32_t P = (int32_t)G->pbase.size() - 1;
  std::vector<int64_t> grow((size_t)P, 0);
  int64_t total = 0;
  for (int32_t k = 0; k < count; ++k) {
    const int32_t p = problems[k];
    if (p < 0 || p >= P) return fail(G, PIRRT_EINVAL, "problem index out of range");
    if (n_new[k] < 0) return fail(G, PIRRT_EINVAL, "n_new < 0");
    for (int32_t j = 0; j < k; ++j)
      if (problems[j] == p) return fail(G, PIRRT_EINVAL, "a problem is listed twice");
    grow[(size_t)p] = n_new[k];
    total += n_new[k];
  }
  if (total == 0) return PIRRT_OK;
  if (!row_ptr) return fail(G, PIRRT_EINVAL, "row_ptr is NULL");
  if (G->n + total > (int64_t)INT32_MAX - 1) return fail(G, PIRRT_EINVAL, "vertex ids beyond INT32_MAX");
  hipStream_t s = G->stream;
  int rc;
  const int32_t tot = (int32_t)total;
  int64_t nnz_b = 0;
  if (mem_kind == PIRRT_MEM_HOST) {
    nnz_b = row_ptr[tot];
  } else {
    HIP_OR_FAIL(G, hipMemcpyAsync(&G->host->word, row_ptr + tot, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(G, hipStreamSynchronize(s));
    nnz_b = G->host->word;
  }
  if (nnz_b < 0 || nnz_b > ((int64_t)1 << 40)) return fail(G, PIRRT_EINVAL, "row_ptr[total] out of range");
  if (nnz_b > 0 && (!col || !cost)) return fail(G, PIRRT_EINVAL, "col or cost is NULL");
  // the block table (non-empty blocks in row order) and the new bases
  const int64_t n_old = G->n, n1 = n_old + total;
  std::vector<BatchBlock> blk;
  int64_t r = 0;
  for (int32_t k = 0; k < count; ++k) {
    if (n_new[k] == 0) continue;
    const int32_t p = problems[k];
    BatchBlock b;
    b.row_begin = r;
    b.base_old = G->pbase[(size_t)p];
    b.app_base = n_old + r;
    b.problem = p;
    b.n_old = (int32_t)(G->pbase[(size_t)p + 1] - G->pbase[(size_t)p]);
    blk.push_back(b);
    r += n_new[k];
  }
  std::vector<int64_t> pbase_new((size_t)P + 1);
  pbase_new[0] = 0;
  for (int32_t p = 0; p < P; ++p)
    pbase_new[(size_t)p + 1] = pbase_new[(size_t)p] + (G->pbase[(size_t)p + 1] - G->pbase[(size_t)p]) + grow[(size_t)p];
  const int32_t nblk = (int32_t)blk.size();
  const int64_t blk_bytes = (int64_t)sizeof(BatchBlock) * nblk;
  const int64_t need = (blk_bytes + 255) / 256 * 256 + 8 * (int64_t)(P + 1);
  if (need > G->dgrow_cap) {
    char* q = nullptr;
    if (!dalloc(G->A, &q, need)) return fail(G, PIRRT_ENOMEM, "device allocation of the block table failed");
    dfree(G->A, G->dgrow);
    G->dgrow = q;
    G->dgrow_cap = need;
  }
  BatchBlock* dblk = reinterpret_cast<BatchBlock*>(G->dgrow);
  int64_t* dbase_new = reinterpret_cast<int64_t*>(G->dgrow + (blk_bytes + 255) / 256 * 256);
  if ((rc = upload_bases(G))) return rc;  // dbase = the old bases
  if ((rc = ensure_staging(G, tot, nnz_b))) return rc;
  HIP_OR_FAIL(G, hipMemcpyAsync(G->brp, row_ptr, sizeof(int64_t) * (size_t)(tot + 1), in_kind(mem_kind), s));
  if (nnz_b > 0) {
    HIP_OR_FAIL(G, hipMemcpyAsync(G->bcol, col, sizeof(int32_t) * (size_t)nnz_b, in_kind(mem_kind), s));
    HIP_OR_FAIL(G, hipMemcpyAsync(G->bcost, cost, sizeof(float) * (size_t)nnz_b, in_kind(mem_kind), s));
  }
  HIP_OR_FAIL(G, hipMemcpyAsync(dblk, blk.data(), (size_t)blk_bytes, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(G, hipMemcpyAsync(dbase_new, pbase_new.data(), sizeof(int64_t) * (size_t)(P + 1), hipMemcpyHostToDevice,
                                s));
  // row offsets and costs first (local ids are checked per block below)
  HIP_OR_FAIL(G, hipMemsetAsync(G->dflag, 0, sizeof(int32_t), s));
  launch_validate_rows(tot, n_old, 0, G->brp, G->bcol, G->bcost, nnz_b, G->dflag, s);
  HIP_OR_FAIL(G, hipGetLastError());
  int32_t bad = 0;
  if ((rc = read_flag(G, &bad))) return rc;
  if (!(bad & 1)) {
    launch_batch_rows(tot, nblk, dblk, G->brp, G->bcol, G->dflag, s);
    HIP_OR_FAIL(G, hipGetLastError());
    if ((rc = read_flag(G, &bad))) return rc;
  }
  if (bad) {
    std::string m = "invalid rows:";
    if (bad & 1) m += " row_ptr not 0-based / non-decreasing / bounded;";
    if (bad & 2) m += " col outside [0, own local id);";
    if (bad & 4) m += " cost not finite, negative or -0.0;";
    return fail(G, PIRRT_EINVAL, m);
  }
  if ((rc = ensure_vcap(G, n1))) return rc;
  if ((rc = ensure_spare(G, G->nnz + 2 * nnz_b))) return rc;
  launch_identity_ids(n_old, n1, G->ext_of, G->slot_of, s);
  launch_block_problems(n_old, tot, nblk, dblk, G->prob, s);
  launch_translate(nnz_b, G->bcol, G->slot_of, G->bslot, s);
  launch_rebuild(tot, n_old, G->brp, G->bslot, G->bcost, G->rp, G->col, G->cst, G->rp2, G->col2, G->cst2, G->add,
                 G->add0, G->deg, G->scan_scratch, s);
  HIP_OR_FAIL(G, hipGetLastError());
  std::swap(G->rp, G->rp2);
  std::swap(G->col, G->col2);
  std::swap(G->cst, G->cst2);
  std::swap(G->ecap, G->ecap2);
  G->n = n1;
  G->nnz += 2 * nnz_b;
  G->adj_version++;
  drop_loops(G);
  if ((rc = insert_levels(G, tot, n_old, -1, G->brp, G->bcol, G->bcost))) return rc;
  // final caller ids, bases and host mirrors
  launch_reid(n1, n_old, nblk, dblk, G->dbase, dbase_new, G->prob, G->ext_of, G->slot_of, s);
  HIP_OR_FAIL(G, hipGetLastError());
  G->hslot.resize((size_t)n1);
  HIP_OR_FAIL(G, hipMemcpyAsync(G->hslot.data(), G->slot_of, sizeof(int32_t) * (size_t)n1, hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(G, hipStreamSynchronize(s));
  auto moved = [&](int32_t id) {  // an old caller id under the new bases
    const size_t p = (size_t)(std::upper_bound(G->pbase.begin(), G->pbase.end(), (int64_t)id) - G->pbase.begin()) - 1;
    return (int32_t)(pbase_new[p] + (id - G->pbase[p]));
  };
  for (auto& id : G->hroots) id = moved(id);
  if (G->nroots > 0)
    HIP_OR_FAIL(G, hipMemcpyAsync(G->droots, G->hroots.data(), sizeof(int32_t) * (size_t)G->nroots,
                                  hipMemcpyHostToDevice, s));
  G->pbase = pbase_new;
  if ((rc = upload_bases(G))) return rc;
  G->renumber_pending = true;
  G->snap_n = -1;  // a snapshot holds the old layout
  return PIRRT_OK;
}

// ---------------------------------------------------------------------------
// The Replan loop.

struct LoopArgs {
  int32_t P;
  bool prune;
  StepArgs sa;
  WalkArgs wa;
  EvalArgs ea;
};

// A single graph's walk after an Improve takes the finish step itself (one launch
// less per iteration); batches and the level-synchronous Evaluate keep k_finish.
bool walk_finishes(pirrt_graph* G, const LoopArgs& L) {
  return L.sa.prob == nullptr && !(G->eval_levels && !L.wa.truncated);
}

// Enqueues Evaluate for every problem that needs it (walk, or level-synchronous
// for a single problem).  after_improve: the Evaluate of an iteration (not the first
// one of a Replan).
void enqueue_evaluate(pirrt_graph* G, LoopArgs& L, hipStream_t s, bool after_improve) {
  if (G->eval_levels && !L.wa.truncated) {  // the truncated Evaluate is a walk
    launch_evaluate(L.ea, s);
  } else {
    L.wa.finish = after_improve && walk_finishes(G, L);
    launch_eval_walk(L.wa, s);
  }
}

// One iteration of Alg. 2 for every active problem.
// (The thresholds of an iteration come from the after-eval step before it.)
void enqueue_iteration(pirrt_graph* G, LoopArgs& L, hipStream_t s, bool timing) {
  if (timing) (void)hipEventRecord(G->ev[2], s);
  launch_mark(L.sa, G->row_variant, s);
  launch_domain_list(L.sa, s);
  if (timing) (void)hipEventRecord(G->ev[3], s);
  launch_improve(L.sa, G->row_variant, s);
  if (timing) (void)hipEventRecord(G->ev[4], s);
  const bool single = L.sa.prob == nullptr;
  if (!walk_finishes(G, L)) launch_finish(L.P, G->ps, G->ctr, G->ctl, single, s);
  if (timing) (void)hipEventRecord(G->ev[0], s);
  enqueue_evaluate(G, L, s, true);
  if (timing) (void)hipEventRecord(G->ev[1], s);
  // a single graph's promising list (next iteration) takes the thresholds step
  if (!single)
    launch_after_eval(L.P, G->ps, G->g, L.prune ? 1 : 0, G->ctl, (int32_t)G->n, problem_map(G), base_map(G),
                      G->tiles, G->bitmap_tiles, walk_tiles(G), s);
}

LoopKey loop_key(pirrt_graph* G, const LoopArgs& L, int iters) {
  LoopKey k;
  memset(&k, 0, sizeof(k));
  const void* p[17] = {G->rp,     G->col,         G->cst, G->g,   G->parent, G->pcost,  G->stamp,
                       G->word,   G->ext_of,      problem_map(G), base_map(G), G->ps,    G->ctr,
                       G->ctl,    L.sa.h,         G->child,       G->lvl};
  memcpy(k.ptrs, p, sizeof(p));
  k.n = G->n;
  k.nnz = G->nnz;
  k.P = L.P;
  k.prune = L.prune;
  k.variant = G->row_variant;
  k.walk_parts = G->walk_parts;
  k.walk_coherent = G->walk_coherent;
  k.eval_levels = G->eval_levels;
  k.has_h = L.sa.h != nullptr;
  k.iters = iters;
  k.mid = L.ea.mid_launches;
  k.lookahead = L.sa.lookahead;
  k.truncated = L.sa.truncated;
  k.blocks = L.sa.blocks;
  k.bitmap_tiles = G->bitmap_tiles;
  k.walk_rank = G->walk_rank;
  return k;
}

// A captured loop body of 2^k iterations (built on first use, reused while every
// baked pointer and size is unchanged).
int loop_graph(pirrt_graph* G, LoopArgs& L, int k, hipGraphExec_t* out) {
  const int iters = 1 << k;
  const LoopKey key = loop_key(G, L, iters);
  if (G->loop_exec[k] && G->loop_key[k] == key) {
    *out = G->loop_exec[k];
    return PIRRT_OK;
  }
  if (G->loop_exec[k]) {
    (void)hipGraphExecDestroy(G->loop_exec[k]);
    G->loop_exec[k] = nullptr;
  }
  hipGraph_t graph = nullptr;
  HIP_OR_FAIL(G, hipStreamBeginCapture(G->cap_stream, hipStreamCaptureModeThreadLocal));
  for (int i = 0; i < iters; ++i) enqueue_iteration(G, L, G->cap_stream, false);
  hipError_t e = hipStreamEndCapture(G->cap_stream, &graph);
  if (e != hipSuccess) return fail_device(G, e, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail_device(G, e, "hipGraphInstantiate");
  G->loop_exec[k] = exec;
  G->loop_key[k] = key;
  *out = exec;
  return PIRRT_OK;
}

// Caller buffers that receive the final policy (see policy_out).
struct PolicyOut {
  float* g;
  int32_t* parent;
  int mem_kind;
};

// Runs Replan for P problems with the given root ids and root / goal slots.  h is
// a device array in slot order (or NULL).  Fills per-problem stats (P entries,
// nullable).  out (nullable): the policy copy-out is enqueued before the final wait,
// so a call waits for the device once at its end.
int run_replan(pirrt_graph* G, int32_t P, const int32_t* root_ids, const int32_t* root_slots,
               const int32_t* goal_slots, const float* h, bool prune, bool timing, pirrt_stats* stats,
               const PolicyOut* out = nullptr) {
  hipStream_t s = G->stream;
  int rc;
  auto t_start = std::chrono::steady_clock::now();
  if ((rc = ensure_pcap(G, P))) return rc;
  const int32_t n = (int32_t)G->n;
  const int64_t cap_iters = G->max_iters > 0 ? G->max_iters : 4 * (int64_t)n + 8;
  for (int32_t i = 0; i < P; ++i) {
    ProblemState& q = G->hps[i];
    memset(&q, 0, sizeof(q));
    q.root = root_slots[i];
    q.goal = goal_slots[i];
    q.active = 1;
    q.needs_eval = 1;
    q.cap = (int32_t)std::min<int64_t>(cap_iters, INT32_MAX);
  }
  if (P == 1 && !G->batched) {
    // one launch from scalar arguments: no host-to-device copies on the latency path
    launch_replan_init_single(G->ps, root_slots[0], goal_slots[0], G->hps[0].cap, root_ids[0], G->nroots, G->droots,
                              G->slot_of, G->parent, G->pcost, G->ctr, G->ctl, G->g, prune ? 1 : 0, s);
  } else {
    HIP_OR_FAIL(G, hipMemcpyAsync(G->ps, G->hps, sizeof(ProblemState) * (size_t)P, hipMemcpyHostToDevice, s));
    // the previous roots lose their mark; the new roots get it
    launch_unmark_roots(G->nroots, G->droots, G->slot_of, G->parent, s);
    HIP_OR_FAIL(G, hipMemcpyAsync(G->droots, root_ids, sizeof(int32_t) * (size_t)P, hipMemcpyHostToDevice, s));
    launch_replan_init(P, G->ps, G->parent, G->pcost, G->ctr, G->ctl, G->g, prune ? 1 : 0, s);
  }
  G->nroots = P;
  G->hroots.assign(root_ids, root_ids + P);
  HIP_OR_FAIL(G, hipGetLastError());
  if (G->fault_launch) {  // injected failure: behave as a failed launch would
    G->fault_launch = false;
    return fail_device(G, hipErrorLaunchFailure, "Replan launch (injected by PIRRT_FAULT_INJECT)");
  }

  LoopArgs L;
  L.P = P;
  L.prune = prune;
  StepArgs& sa = L.sa;
  sa.n = n;
  sa.nnz = G->nnz;
  sa.prob = problem_map(G);
  sa.ps = G->ps;
  sa.ctl = G->ctl;
  sa.prune = prune ? 1 : 0;
  sa.g = G->g;
  sa.h = h;
  sa.rp = G->rp;
  sa.col = G->col;
  sa.cst = G->cst;
  sa.stamp = G->stamp;
  sa.ext_of = G->ext_of;
  sa.parent = G->parent;
  sa.pcost = G->pcost;
  sa.ctr = G->ctr;
  sa.dlist = G->dlist;
  sa.plist = G->fr1;  // free during a Replan (the level evaluator's frontiers run only between marks)
  sa.tiles = G->tiles;
  sa.lookahead = G->lookahead;
  sa.truncated = G->truncated;
  sa.word = G->word;
  sa.blocks = G->batch_blocks;
  WalkArgs& wa = L.wa;
  wa.n = n;
  wa.prob = problem_map(G);
  wa.ps = G->ps;
  wa.ctl = G->ctl;
  wa.parent = G->parent;
  wa.pcost = G->pcost;
  wa.g = G->g;
  wa.word = G->word;
  wa.hops = G->trace ? G->dhops : nullptr;
  wa.parts = G->walk_parts;
  wa.coherent = G->walk_coherent;
  wa.tiles = walk_tiles(G) ? walk_tiles(G) : G->tiles;
  wa.truncated = G->truncated;
  wa.h = h;
  // the batched walk runs no more workgroups than stay resident at once, so it takes
  // the tiles in their rank order with few climbs through unstamped ancestors
  wa.blocks = std::min(G->batch_blocks, G->cus * kWalkResidentPerCu);
  wa.ctr = G->ctr;
  wa.finish = false;
  EvalArgs& ea = L.ea;
  ea.n = n;
  ea.ps = G->ps;
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
  ea.scan_scratch = G->scan_scratch;
  ea.mid_launches = std::max(0, std::min(std::min(G->mid_hint, kMaxMidLaunches), n));
  int64_t lb = (int64_t)n / 2048;
  ea.level_blocks = (int32_t)(lb < 16 ? 16 : (lb > 1024 ? 1024 : lb));
  if (G->eval_levels && P != 1) return fail(G, PIRRT_EINVAL, "the level-synchronous Evaluate takes one problem");
  if (P == 1 && !G->batched && n <= kSmallMax && G->small_graphs && !timing && !G->trace && !G->eval_levels &&
      !G->truncated) {
    // one workgroup runs the whole loop
    launch_replan_small(n, G->rp, G->col, G->cst, h, G->ext_of, prune, G->lookahead, G->ps, G->parent, G->pcost,
                        G->g, s);
    HIP_OR_FAIL(G, hipGetLastError());
    if (out && (out->g || out->parent) && (rc = policy_out(G, out->g, out->parent, nullptr, out->mem_kind)))
      return rc;
    HIP_OR_FAIL(G, hipMemcpyAsync(G->hps, G->ps, sizeof(ProblemState), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(G, hipStreamSynchronize(s));
    const ProblemState& q = G->hps[0];
    if (stats) {
      pirrt_stats& st = stats[0];
      memset(&st, 0, sizeof(st));
      st.iterations = q.iterations;
      st.edges_examined = (int64_t)q.edges;
      st.sum_P = (int64_t)q.sum_P;
      st.sum_D = (int64_t)q.sum_D;
      st.changed_total = (int64_t)q.changed_total;
      st.mark_edges = (int64_t)q.mark_edges;
      st.evaluate_calls = q.iterations;
      st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    G->last_iterations = q.iterations;
    if (q.status != 0) return fail(G, PIRRT_ENOTCONVERGED, "iteration cap reached");
    return PIRRT_OK;
  }

  // the multi-kernel loop's marks: no stamp older than this Replan
  HIP_OR_FAIL(G, hipMemsetAsync(G->stamp, 0, (size_t)n, s));
  pirrt_stats agg;
  memset(&agg, 0, sizeof(agg));
  // first Evaluate of every problem
  if (timing) HIP_OR_FAIL(G, hipEventRecord(G->ev[0], s));
  if (G->trace) HIP_OR_FAIL(G, hipMemsetAsync(G->dhops, 0, sizeof(unsigned long long), s));
  enqueue_evaluate(G, L, s, false);
  if (timing) HIP_OR_FAIL(G, hipEventRecord(G->ev[1], s));
  if (problem_map(G))  // a single graph's first promising list takes the thresholds step
    launch_after_eval(P, G->ps, G->g, prune ? 1 : 0, G->ctl, n, problem_map(G), base_map(G), G->tiles,
                      G->bitmap_tiles, walk_tiles(G), s);
  HIP_OR_FAIL(G, hipGetLastError());
  if (timing) {
    HIP_OR_FAIL(G, hipStreamSynchronize(s));
    agg.ms_evaluate += elapsed_ms(G->ev[0], G->ev[1]);
    agg.evaluate_calls += 1;
  }

  const bool direct = timing || G->trace || !G->use_graph;
  int64_t done_iters = 0;
  if (direct) {
    for (int it = 0;; ++it) {
      if (G->trace) HIP_OR_FAIL(G, hipMemsetAsync(G->dhops, 0, sizeof(unsigned long long), s));
      enqueue_iteration(G, L, s, timing);
      HIP_OR_FAIL(G, hipGetLastError());
      HIP_OR_FAIL(G, hipMemcpyAsync(&G->host->ctl, G->ctl, sizeof(LoopCtl), hipMemcpyDeviceToHost, s));
      if (G->trace) {
        HIP_OR_FAIL(G, hipMemcpyAsync(&G->host->hops, G->dhops, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        HIP_OR_FAIL(G, hipMemcpyAsync(G->hps, G->ps, sizeof(ProblemState) * (size_t)P, hipMemcpyDeviceToHost, s));
      }
      HIP_OR_FAIL(G, hipStreamSynchronize(s));
      ++done_iters;
      if (timing) {
        agg.ms_mark += elapsed_ms(G->ev[2], G->ev[3]);
        agg.ms_improve += elapsed_ms(G->ev[3], G->ev[4]);
        agg.mark_launches += 1;
        agg.improve_launches += 1;
        if (G->host->ctl.any_active) {  // the Evaluate after the last Improve is a no-op
          agg.ms_evaluate += elapsed_ms(G->ev[0], G->ev[1]);
          agg.evaluate_calls += 1;
        }
      }
      if (G->trace) {
        int active = 0;
        for (int32_t q = 0; q < P; ++q) active += G->hps[q].active != 0;
        fprintf(stderr,
                "pirrt iter %d: problem 0 iterations %d edges %llu sum_P %llu sum_D %llu changed %llu; walk hops "
                "%llu; problems active %d, tiles %d\n",
                it + 1, G->hps[0].iterations, (unsigned long long)G->hps[0].edges,
                (unsigned long long)G->hps[0].sum_P, (unsigned long long)G->hps[0].sum_D,
                (unsigned long long)G->hps[0].changed_total, (unsigned long long)G->host->hops, active,
                G->host->ctl.ntiles);
      }
      if (!G->host->ctl.any_active) break;
      if (done_iters > cap_iters + 1) return fail_device(G, hipErrorUnknown, "Replan loop did not stop");
    }
  } else {
    // Planned launches: as many loop bodies as the previous Replan needed, back to
    // back, then one iteration at a time until every problem has stopped.  The loop
    // bodies are captured graphs when this call's arguments (sizes, arrays) repeat the
    // previous call's; a graph that changes every call (a planner inserting a batch
    // before each Replan) would cost its capture and instantiation every time, so such
    // calls enqueue the same kernels directly.
    const LoopKey key1 = loop_key(G, L, 1);
    const bool graphs = G->have_prev_key && G->prev_key == key1;
    G->prev_key = key1;
    G->have_prev_key = true;
    int64_t plan = G->last_iterations > 0 ? G->last_iterations : 8;
    for (;;) {
      const int k = plan >= 8 ? 3 : plan >= 4 ? 2 : plan >= 2 ? 1 : 0;
      if (graphs) {
        hipGraphExec_t exec = nullptr;
        if ((rc = loop_graph(G, L, k, &exec))) return rc;
        HIP_OR_FAIL(G, hipGraphLaunch(exec, s));
      } else {
        for (int i = 0; i < (1 << k); ++i) enqueue_iteration(G, L, s, false);
        HIP_OR_FAIL(G, hipGetLastError());
      }
      done_iters += 1 << k;
      plan -= 1 << k;
      if (plan > 0) continue;
      HIP_OR_FAIL(G, hipMemcpyAsync(&G->host->ctl, G->ctl, sizeof(LoopCtl), hipMemcpyDeviceToHost, s));
      HIP_OR_FAIL(G, hipStreamSynchronize(s));
      if (!G->host->ctl.any_active) break;
      if (done_iters > cap_iters + 8) return fail_device(G, hipErrorUnknown, "Replan loop did not stop");
      plan = 1;
    }
  }
  if (out && (out->g || out->parent) && (rc = policy_out(G, out->g, out->parent, nullptr, out->mem_kind)))
    return rc;
  HIP_OR_FAIL(G, hipMemcpyAsync(G->hps, G->ps, sizeof(ProblemState) * (size_t)P, hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(G, hipStreamSynchronize(s));
  int32_t most = 0;
  bool capped = false;
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  for (int32_t i = 0; i < P; ++i) {
    const ProblemState& q = G->hps[i];
    most = std::max(most, q.iterations);
    capped = capped || q.status != 0;
    if (stats) {
      pirrt_stats& st = stats[i];
      memset(&st, 0, sizeof(st));
      st.iterations = q.iterations;
      st.edges_examined = (int64_t)q.edges;
      st.sum_P = (int64_t)q.sum_P;
      st.sum_D = (int64_t)q.sum_D;
      st.changed_total = (int64_t)q.changed_total;
      st.mark_edges = (int64_t)q.mark_edges;
      st.ms_total = ms;
      st.evaluate_calls = timing ? agg.evaluate_calls : q.iterations;
      // the phases of a batch serve all of its problems at once
      st.ms_evaluate = agg.ms_evaluate;
      st.ms_mark = agg.ms_mark;
      st.ms_improve = agg.ms_improve;
      st.improve_launches = agg.improve_launches;
      st.mark_launches = agg.mark_launches;
    }
  }
  G->last_iterations = most;
  if (capped) return fail(G, PIRRT_ENOTCONVERGED, "iteration cap reached");
  return PIRRT_OK;
}

// Replan of a small single graph on the host (host_replan.hip): the slot-ordered
// adjacency is copied to the host when it changed since the last such call, the policy
// and h are copied over, the roots re-marked as on the device, and the result goes
// back to the device arrays (which stay the handle's state) and to the caller in
// caller ids.
int run_host_replan(pirrt_graph* G, int32_t root, int32_t goal, const float* h, int mem_kind, bool prune,
                    bool lookahead, float* g_out, int32_t* parent_out, pirrt_stats* stats) {
  auto t_start = std::chrono::steady_clock::now();
  hipStream_t s = G->stream;
  const int32_t n = (int32_t)G->n;
  const size_t m = (size_t)G->nnz;
  if (G->hm_version != G->adj_version) {
    G->hm_rp.resize((size_t)n + 1);
    G->hm_col.resize(m);
    G->hm_cst.resize(m);
    HIP_OR_FAIL(G, hipMemcpyAsync(G->hm_rp.data(), G->rp, sizeof(int64_t) * ((size_t)n + 1), hipMemcpyDeviceToHost, s));
    if (m) {
      HIP_OR_FAIL(G, hipMemcpyAsync(G->hm_col.data(), G->col, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s));
      HIP_OR_FAIL(G, hipMemcpyAsync(G->hm_cst.data(), G->cst, sizeof(float) * m, hipMemcpyDeviceToHost, s));
    }
    G->hm_ext.resize((size_t)n);
    for (int32_t id = 0; id < n; ++id) G->hm_ext[(size_t)G->hslot[(size_t)id]] = id;
  }
  std::vector<float> g((size_t)n), pc((size_t)n), hs;
  std::vector<int32_t> par((size_t)n);
  HIP_OR_FAIL(G, hipMemcpyAsync(par.data(), G->parent, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(G, hipMemcpyAsync(pc.data(), G->pcost, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost, s));
  std::vector<float> hc;
  if (h && mem_kind == PIRRT_MEM_DEVICE) {
    hc.resize((size_t)n);
    HIP_OR_FAIL(G, hipMemcpyAsync(hc.data(), h, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost, s));
  }
  HIP_OR_FAIL(G, hipStreamSynchronize(s));
  G->hm_version = G->adj_version;
  if (h) {
    const float* hsrc = mem_kind == PIRRT_MEM_DEVICE ? hc.data() : h;
    hs.resize((size_t)n);
    for (int32_t id = 0; id < n; ++id) {
      if (!(hsrc[id] >= 0.0f)) return fail(G, PIRRT_EINVAL, "h has a NaN or negative entry");
      hs[(size_t)G->hslot[(size_t)id]] = hsrc[id];
    }
  }
  // the previous roots lose their mark (in order, before the new one gets it)
  for (const int32_t id : G->hroots) {
    const size_t sl = (size_t)G->hslot[(size_t)id];
    if (par[sl] == kRootMark) par[sl] = -1;
  }
  HostReplan p;
  p.n = n;
  p.rp = G->hm_rp.data();
  p.col = G->hm_col.data();
  p.cst = G->hm_cst.data();
  p.ext = G->hm_ext.data();
  p.h = h ? hs.data() : nullptr;
  p.g = g.data();
  p.parent = par.data();
  p.pcost = pc.data();
  p.root = G->hslot[(size_t)root];
  p.goal = G->hslot[(size_t)goal];
  p.prune = prune;
  p.lookahead = lookahead;
  p.cap = G->max_iters > 0 ? G->max_iters : 4 * (int64_t)n + 8;
  HostReplanStats hst;
  const int capped = host_replan(p, &hst);
  // the device arrays stay the handle's state
  HIP_OR_FAIL(G, hipMemcpyAsync(G->g, g.data(), sizeof(float) * (size_t)n, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(G, hipMemcpyAsync(G->parent, par.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(G, hipMemcpyAsync(G->pcost, pc.data(), sizeof(float) * (size_t)n, hipMemcpyHostToDevice, s));
  int rc;
  if ((rc = ensure_pcap(G, 1))) return rc;
  HIP_OR_FAIL(G, hipMemcpyAsync(G->droots, &root, sizeof(int32_t), hipMemcpyHostToDevice, s));
  G->nroots = 1;
  G->hroots.assign(1, root);
  // the caller's outputs in caller ids (a root reads -1)
  std::vector<float> go;
  std::vector<int32_t> po;
  float* gw = g_out;
  int32_t* pw = parent_out;
  const bool dev = mem_kind == PIRRT_MEM_DEVICE;
  if (dev && g_out) {
    go.resize((size_t)n);
    gw = go.data();
  }
  if (dev && parent_out) {
    po.resize((size_t)n);
    pw = po.data();
  }
  for (int32_t id = 0; id < n; ++id) {
    const size_t sl = (size_t)G->hslot[(size_t)id];
    if (gw) gw[id] = g[sl];
    if (pw) pw[id] = par[sl] >= 0 ? G->hm_ext[(size_t)par[sl]] : -1;
  }
  if (dev && g_out) HIP_OR_FAIL(G, hipMemcpyAsync(g_out, go.data(), sizeof(float) * (size_t)n, hipMemcpyHostToDevice, s));
  if (dev && parent_out)
    HIP_OR_FAIL(G, hipMemcpyAsync(parent_out, po.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(G, hipStreamSynchronize(s));
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->iterations = hst.iterations;
    stats->edges_examined = hst.edges;
    stats->sum_P = hst.sum_P;
    stats->sum_D = hst.sum_D;
    stats->changed_total = hst.changed;
    stats->mark_edges = hst.mark_edges;
    stats->evaluate_calls = hst.iterations;
    stats->on_host = 1;
    stats->ms_total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  }
  return capped ? PIRRT_ENOTCONVERGED : PIRRT_OK;
}

// Copies and validates a caller h (caller order) into slot order in hbuf.
int stage_h(pirrt_graph* G, const float* h, int mem_kind, const float** out) {
  *out = nullptr;
  if (!h) return PIRRT_OK;
  const int32_t n = (int32_t)G->n;
  hipStream_t s = G->stream;
  int rc;
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
  *out = G->hbuf;
  return PIRRT_OK;
}

// Autotuner: the Replan of the call is run for each kernel configuration -- the
// Improve / mark row split (lanes per row x quads in flight) and the scope of the
// walk's Evaluate stamps (device or workgroup) -- each from the same policy, the
// fastest kept.  Each configuration runs twice in a row: the first run loads its
// kernels and launches them directly, the second repeats its arguments, so it runs
// from captured graphs as repeated Replans do, and is the one timed.  A batch then
// tries the workgroup count of its grid-stride launches (kTuneBlocks, the first one
// being the default) with the best of those, one dimension after the other.  The
// policy and the root marks are restored at the end.
constexpr int kTuneConfigs = kRowVariants * 2;
constexpr int kTuneBlocks[4] = {kBatchBlocks, 1024, 4096, 8192};

int tune(pirrt_graph* G, int32_t P, const int32_t* rid, const int32_t* rs, const int32_t* gs, const float* hdev,
         bool prune, int32_t* config) {
  hipStream_t s = G->stream;
  const size_t n = (size_t)G->n;
  // the policy goes to the spare copies (free here: h is staged in hbuf already)
  HIP_OR_FAIL(G, hipMemcpyAsync(G->g2, G->g, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
  HIP_OR_FAIL(G, hipMemcpyAsync(G->parent2, G->parent, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
  HIP_OR_FAIL(G, hipMemcpyAsync(G->pcost2, G->pcost, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
  const std::vector<int32_t> roots0 = G->hroots;
  int rc;
  auto restore = [&]() -> int {
    HIP_OR_FAIL(G, hipMemcpyAsync(G->g, G->g2, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(G->parent, G->parent2, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    HIP_OR_FAIL(G, hipMemcpyAsync(G->pcost, G->pcost2, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
    G->hroots = roots0;
    G->nroots = (int32_t)roots0.size();
    if (G->nroots > 0)
      HIP_OR_FAIL(G, hipMemcpyAsync(G->droots, roots0.data(), sizeof(int32_t) * roots0.size(), hipMemcpyHostToDevice,
                                    s));
    HIP_OR_FAIL(G, hipStreamSynchronize(s));
    return PIRRT_OK;
  };
  double best = 1e300;
  int bestc = 0;
  auto apply = [&](int c) {
    G->row_variant = c % kRowVariants;
    G->walk_coherent = (c / kRowVariants) % 2 == 0;
    G->batch_blocks = kTuneBlocks[c / kTuneConfigs];
  };
  auto trial = [&](int c) -> int {
    apply(c);
    for (int pass = 0; pass < 2; ++pass) {  // the second run repeats the first: graphs
      int r;
      if ((r = restore())) return r;
      const auto t0 = std::chrono::steady_clock::now();
      r = run_replan(G, P, rid, rs, gs, hdev, prune, false, nullptr);
      if (r != PIRRT_OK && r != PIRRT_ENOTCONVERGED) return r;
      const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      if (pass == 1 && ms < best) {
        best = ms;
        bestc = c;
      }
    }
    return PIRRT_OK;
  };
  for (int c = 0; c < kTuneConfigs; ++c)
    if ((rc = trial(c))) return rc;
  if (G->batched) {  // single graphs size their grids to the work
    const int row = bestc;
    for (int b = 1; b < 4; ++b)
      if ((rc = trial(row + kTuneConfigs * b))) return rc;
  }
  apply(bestc);
  if ((rc = restore())) return rc;
  if (config) *config = bestc;
  return PIRRT_OK;
}

pirrt_graph* new_graph(const pirrt_config* cfg, int* rc_out) {
  *rc_out = PIRRT_OK;
  pirrt_config c;
  memset(&c, 0, sizeof(c));
  c.device = -1;
  if (cfg) c = *cfg;
  if (c.vertex_capacity < 0 || c.edge_capacity < 0 || c.max_iters < 0) {
    g_create_error = "negative capacity or iteration cap";
    *rc_out = PIRRT_EINVAL;
    return nullptr;
  }
  if ((c.alloc == nullptr) != (c.free == nullptr)) {
    g_create_error = "alloc and free must be given together";
    *rc_out = PIRRT_EINVAL;
    return nullptr;
  }
  pirrt_graph* G = new (std::nothrow) pirrt_graph();
  if (!G) {
    *rc_out = PIRRT_ENOMEM;
    return nullptr;
  }
  G->A.alloc = c.alloc;
  G->A.free = c.free;
  G->A.ctx = c.alloc_ctx;
  int dev = c.device;
  if (dev < 0) {
    if (hipGetDevice(&dev) != hipSuccess) {
      (void)hipGetLastError();
      delete G;
      g_create_error = "no HIP device";
      *rc_out = PIRRT_EDEVICE;
      return nullptr;
    }
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || dev >= ndev) {
    (void)hipGetLastError();
    delete G;
    g_create_error = "HIP device not available";
    *rc_out = PIRRT_EDEVICE;
    return nullptr;
  }
  G->device = dev;
  G->stream = (hipStream_t)c.hip_stream;
  G->max_iters = c.max_iters;
  if (hipSetDevice(dev) != hipSuccess) {
    (void)hipGetLastError();
    delete G;
    g_create_error = "hipSetDevice failed";
    *rc_out = PIRRT_EDEVICE;
    return nullptr;
  }
  if (hipDeviceGetAttribute(&G->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || G->cus < 1) {
    (void)hipGetLastError();
    G->cus = 256;
  }
  bool ok = dalloc(G->A, &G->info, 1) && dalloc(G->A, &G->dflag, 1) && dalloc(G->A, &G->dcount, 3) && dalloc(G->A, &G->dhops, 1) &&
            dalloc(G->A, &G->ctl, 1);
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
  if (ok && hipStreamCreate(&G->cap_stream) != hipSuccess) {
    (void)hipGetLastError();
    G->cap_stream = nullptr;
    ok = false;
  }
  if (ok && hipMemset(G->ctl, 0, sizeof(LoopCtl)) != hipSuccess) {
    (void)hipGetLastError();
    ok = false;
  }
  int rc = PIRRT_OK;
  if (ok) rc = ensure_vcap(G, c.vertex_capacity > kMinVertexCap ? c.vertex_capacity : kMinVertexCap);
  if (ok && rc == PIRRT_OK && c.edge_capacity > 0) {
    rc = ensure_spare(G, c.edge_capacity);
    if (rc == PIRRT_OK) {
      std::swap(G->col, G->col2);
      std::swap(G->cst, G->cst2);
      std::swap(G->ecap, G->ecap2);
      rc = ensure_spare(G, c.edge_capacity);
    }
  }
  if (ok && rc == PIRRT_OK) rc = ensure_pcap(G, 1);
  if (!ok || rc != PIRRT_OK || hipStreamSynchronize(G->stream) != hipSuccess) {
    (void)hipGetLastError();
    g_create_error = ok ? G->err : "device allocation failed at create";
    release_all(G);
    delete G;
    *rc_out = ok ? (rc ? rc : PIRRT_EDEVICE) : PIRRT_ENOMEM;
    return nullptr;
  }
  const char* growth = getenv("PIRRT_REORDER_GROWTH");
  if (growth) G->reorder_growth = atof(growth);
  const char* rmin = getenv("PIRRT_REORDER_MIN");
  if (rmin) G->reorder_min = atoll(rmin);
  const char* ord = getenv("PIRRT_ORDER");
  if (ord) G->clustered_order = strcmp(ord, "bfs") != 0;
  const char* tr = getenv("PIRRT_TRACE");
  G->trace = tr && atoi(tr) > 0;
  const char* ev = getenv("PIRRT_EVALUATE");
  if (ev && strcmp(ev, "levels") == 0) G->eval_levels = true;
  const char* wp = getenv("PIRRT_WALK_PARTS");
  if (wp && atoi(wp) >= 1) G->walk_parts = atoi(wp);
  const char* wc = getenv("PIRRT_WALK_COHERENT");
  if (wc) G->walk_coherent = atoi(wc) != 0;
  const char* hm = getenv("PIRRT_HOST_MAX");
  if (hm) G->host_max = atoll(hm);
  const char* gr = getenv("PIRRT_GRAPH");
  if (gr) G->use_graph = atoi(gr) != 0;
  const char* sm = getenv("PIRRT_SMALL");
  if (sm) G->small_graphs = atoi(sm) != 0;
  const char* fi = getenv("PIRRT_FAULT_INJECT");
  if (fi) {
    G->fault_launch = strcmp(fi, "launch") == 0;
    G->fault_alloc = strcmp(fi, "alloc") == 0;
  }
  const char* wr = getenv("PIRRT_WALK_ORDER");
  if (wr) G->walk_rank = strcmp(wr, "tiles") != 0;
  const char* tb = getenv("PIRRT_TILE_BITMAP");
  if (tb) G->bitmap_tiles = atoi(tb) < 0 ? 0 : atoi(tb);
  const char* bb = getenv("PIRRT_BATCH_BLOCKS");
  if (bb && atoi(bb) > 0) G->batch_blocks = atoi(bb);
  const char* variant = getenv("PIRRT_ROW_VARIANT");
  if (variant) {
    int v = atoi(variant);
    if (v >= 0 && v < kRowVariants) G->row_variant = v;
  }
  return G;
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
  int rc;
  pirrt_graph* G = new_graph(cfg, &rc);
  if (!G) return rc;
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
  if (G->batched) return fail(G, PIRRT_EINVAL, "this handle holds a batch of problems");
  return insert_rows(G, n_new, row_ptr, col, cost, mem_kind, false);
}

int pirrt_replan(pirrt_graph* G, int32_t root, int32_t goal, const float* h, uint32_t flags, float* g_out,
                 int32_t* parent_out, int mem_kind, pirrt_stats* stats) {
  int rc = guard(G);
  if (rc) return rc;
  if (G->batched) return fail(G, PIRRT_EINVAL, "this handle holds a batch of problems");
  if (mem_kind != PIRRT_MEM_HOST && mem_kind != PIRRT_MEM_DEVICE) return fail(G, PIRRT_EINVAL, "bad mem_kind");
  if ((flags & PIRRT_TRUNCATED) && (flags & PIRRT_LOOKAHEAD))
    return fail(G, PIRRT_EINVAL, "PIRRT_TRUNCATED and PIRRT_LOOKAHEAD cannot be combined");
  if (G->n <= 0) return fail(G, PIRRT_EINVAL, "empty graph");
  if (root < 0 || root >= G->n || goal < 0 || goal >= G->n) return fail(G, PIRRT_EINVAL, "root or goal out of range");
  if (G->n <= G->host_max && !(flags & PIRRT_TRUNCATED)) {  // small: the host finishes first
    pirrt_stats hst;
    rc = run_host_replan(G, root, goal, h, mem_kind, (flags & PIRRT_NO_PRUNE) == 0, (flags & PIRRT_LOOKAHEAD) != 0,
                         g_out, parent_out, &hst);
    if (rc != PIRRT_OK && rc != PIRRT_ENOTCONVERGED) return rc;
    if (stats) *stats = hst;
    return rc;
  }
  const float* hdev = nullptr;
  if ((rc = stage_h(G, h, mem_kind, &hdev))) return rc;
  const int32_t rslot = G->hslot[(size_t)root], gslot = G->hslot[(size_t)goal];
  pirrt_stats st;
  G->lookahead = (flags & PIRRT_LOOKAHEAD) != 0;
  G->truncated = (flags & PIRRT_TRUNCATED) != 0;
  const PolicyOut po{g_out, parent_out, mem_kind};
  rc = run_replan(G, 1, &root, &rslot, &gslot, hdev, (flags & PIRRT_NO_PRUNE) == 0, (flags & PIRRT_TIMING) != 0,
                  &st, &po);
  if (rc != PIRRT_OK && rc != PIRRT_ENOTCONVERGED) return rc;
  if (stats) *stats = st;
  return rc;
}

int pirrt_tune(pirrt_graph* G, int32_t root, int32_t goal, const float* h, uint32_t flags, int mem_kind,
               int32_t* config) {
  int rc = guard(G);
  if (rc) return rc;
  if (G->batched) return fail(G, PIRRT_EINVAL, "this handle holds a batch of problems");
  if (mem_kind != PIRRT_MEM_HOST && mem_kind != PIRRT_MEM_DEVICE) return fail(G, PIRRT_EINVAL, "bad mem_kind");
  if ((flags & PIRRT_TRUNCATED) && (flags & PIRRT_LOOKAHEAD))
    return fail(G, PIRRT_EINVAL, "PIRRT_TRUNCATED and PIRRT_LOOKAHEAD cannot be combined");
  if (G->n <= 0) return fail(G, PIRRT_EINVAL, "empty graph");
  if (root < 0 || root >= G->n || goal < 0 || goal >= G->n) return fail(G, PIRRT_EINVAL, "root or goal out of range");
  const float* hdev = nullptr;
  if ((rc = stage_h(G, h, mem_kind, &hdev))) return rc;
  const int32_t rslot = G->hslot[(size_t)root], gslot = G->hslot[(size_t)goal];
  G->lookahead = (flags & PIRRT_LOOKAHEAD) != 0;
  G->truncated = (flags & PIRRT_TRUNCATED) != 0;
  return tune(G, 1, &root, &rslot, &gslot, hdev, (flags & PIRRT_NO_PRUNE) == 0, config);
}

int pirrt_get_policy(pirrt_graph* G, float* g_out, int32_t* parent_out, float* pcost_out, int mem_kind) {
  int rc = guard(G);
  if (rc) return rc;
  if (mem_kind != PIRRT_MEM_HOST && mem_kind != PIRRT_MEM_DEVICE) return fail(G, PIRRT_EINVAL, "bad mem_kind");
  if (G->batched && (rc = upload_bases(G))) return rc;
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
  if (G->batched && (rc = upload_bases(G))) return rc;
  if (mem_kind == PIRRT_MEM_HOST) {
    size_t pi = 0;
    for (int32_t v = 0; v < n; ++v) {
      while (G->batched && v >= G->pbase[pi + 1]) ++pi;
      const int64_t b = G->batched ? G->pbase[pi] : 0, len = G->batched ? G->pbase[pi + 1] - b : n;
      uint32_t w;
      memcpy(&w, &pcost_in[v], 4);
      if (parent_in[v] < -1 || parent_in[v] >= len || parent_in[v] == v - b) return fail(G, PIRRT_EINVAL, "bad parent");
      if ((w >> 31) != 0 || (w & 0x7f800000u) == 0x7f800000u) return fail(G, PIRRT_EINVAL, "bad pcost");
    }
  } else {
    HIP_OR_FAIL(G, hipMemsetAsync(G->dflag, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(k_check_policy, dim3(grid_for(n)), dim3(256), 0, s, n, parent_in, pcost_in, problem_map(G),
                       base_map(G), G->dflag);
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
  launch_policy_from_ext(n, G->slot_of, problem_map(G), base_map(G), gs, ps, cs, G->g, G->parent, G->pcost, s);
  HIP_OR_FAIL(G, hipGetLastError());
  HIP_OR_FAIL(G, hipStreamSynchronize(s));
  G->nroots = 0;  // the new policy carries no root marks
  G->hroots.clear();
  return PIRRT_OK;
}

int pirrt_snapshot_save(pirrt_graph* G) {
  int rc = guard(G);
  if (rc) return rc;
  if (G->batched && G->renumber_pending && (rc = renumber(G))) return rc;
  const int64_t n = G->n;
  if (n > G->snap_cap) {
    float* a = nullptr;
    int32_t* b = nullptr;
    float* c = nullptr;
    if (!dalloc(G->A, &a, n) || !dalloc(G->A, &b, n) || !dalloc(G->A, &c, n)) {
      dfree(G->A, a);
      dfree(G->A, b);
      dfree(G->A, c);
      return fail(G, PIRRT_ENOMEM, "device allocation for the snapshot failed");
    }
    dfree(G->A, G->sg);
    dfree(G->A, G->sparent);
    dfree(G->A, G->spcost);
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
  G->snap_roots = G->hroots;
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
  // the restored parents carry the snapshot's root marks
  const int32_t m = (int32_t)G->snap_roots.size();
  if ((rc = ensure_pcap(G, m))) return rc;
  if (m > 0)
    HIP_OR_FAIL(G, hipMemcpyAsync(G->droots, G->snap_roots.data(), sizeof(int32_t) * (size_t)m,
                                  hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(G, hipStreamSynchronize(s));
  G->nroots = m;
  G->hroots = G->snap_roots;
  return PIRRT_OK;
}

int pirrt_promising_count(pirrt_graph* G, int32_t goal, const float* h, int64_t first, int64_t count, int mem_kind,
                          int64_t* out) {
  int rc = guard(G);
  if (rc) return rc;
  if (G->batched) return fail(G, PIRRT_EINVAL, "pirrt_promising_count takes a single graph");
  if (mem_kind != PIRRT_MEM_HOST && mem_kind != PIRRT_MEM_DEVICE) return fail(G, PIRRT_EINVAL, "bad mem_kind");
  if (!out) return fail(G, PIRRT_EINVAL, "out is NULL");
  const int64_t n = G->n;
  if (goal < 0 || goal >= n) return fail(G, PIRRT_EINVAL, "goal out of range");
  if (first < 0 || count < 0 || first + count > n) return fail(G, PIRRT_EINVAL, "id range outside the graph");
  *out = 0;
  if (count == 0) return PIRRT_OK;
  hipStream_t s = G->stream;
  const float* hd = nullptr;
  if (h) {
    if (mem_kind == PIRRT_MEM_HOST) {
      for (int64_t i = first; i < first + count; ++i)
        if (!(h[i] >= 0.0f)) return fail(G, PIRRT_EINVAL, "h must be >= 0 and not NaN");
      HIP_OR_FAIL(G, hipMemcpyAsync(G->hbuf, h + first, sizeof(float) * (size_t)count, hipMemcpyHostToDevice, s));
      hd = G->hbuf;
    } else {
      hd = h + first;
    }
  }
  HIP_OR_FAIL(G, hipMemsetAsync(G->dhops, 0, sizeof(unsigned long long), s));
  launch_count_promising(first, count, G->hslot[(size_t)goal], G->slot_of, G->g, hd, G->dhops, s);
  HIP_OR_FAIL(G, hipGetLastError());
  HIP_OR_FAIL(G, hipMemcpyAsync(&G->host->hops, G->dhops, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(G, hipStreamSynchronize(s));
  *out = (int64_t)G->host->hops;
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

// Checkpoint blob: header, forward rows (each vertex's lower-id neighbours, the
// pirrt_insert_batch format), then the policy in caller ids.
namespace {
constexpr uint64_t kBlobMagic = 0x3154535452524950ull;  // "PIRRTST1"
struct BlobHeader {
  uint64_t magic;
  uint32_t version, header_bytes;
  int64_t n, m;  // vertices, undirected edges (forward entries)
  int64_t reserved[2];
};
static_assert(sizeof(BlobHeader) == 48, "blob header layout");

int64_t blob_bytes(int64_t n, int64_t m) {
  return (int64_t)sizeof(BlobHeader) + 8 * (n + 1) + 8 * m + 12 * n;
}
}  // namespace

int64_t pirrt_state_size(pirrt_graph* G) {
  if (!G || G->poisoned || G->batched) return -1;
  return blob_bytes(G->n, G->nnz / 2);
}

int pirrt_state_save(pirrt_graph* G, void* blob, int64_t size) {
  int rc = guard(G);
  if (rc) return rc;
  if (G->batched) return fail(G, PIRRT_EINVAL, "a batch has no state blob");
  const int64_t n = G->n, m = G->nnz / 2;
  if (!blob || size < blob_bytes(n, m)) return fail(G, PIRRT_EINVAL, "blob is NULL or smaller than pirrt_state_size");
  std::vector<int64_t> ptr((size_t)n + 1);
  std::vector<int32_t> nbr((size_t)G->nnz);
  std::vector<float> cst((size_t)G->nnz);
  if ((rc = pirrt_get_adjacency(G, ptr.data(), nbr.data(), cst.data(), PIRRT_MEM_HOST))) return rc;
  char* out = static_cast<char*>(blob);
  BlobHeader h{};
  h.magic = kBlobMagic;
  h.version = 1;
  h.header_bytes = (uint32_t)sizeof(BlobHeader);
  h.n = n;
  h.m = m;
  memcpy(out, &h, sizeof(h));
  int64_t* rp = reinterpret_cast<int64_t*>(out + sizeof(BlobHeader));
  int32_t* col = reinterpret_cast<int32_t*>(rp + n + 1);
  float* cost = reinterpret_cast<float*>(col + m);
  float* g = cost + m;
  int32_t* parent = reinterpret_cast<int32_t*>(g + n);
  float* pcost = reinterpret_cast<float*>(parent + n);
  int64_t k = 0;
  rp[0] = 0;
  for (int64_t v = 0; v < n; ++v) {
    for (int64_t j = ptr[(size_t)v]; j < ptr[(size_t)v + 1]; ++j)
      if (nbr[(size_t)j] < v) {
        if (k >= m) return fail(G, PIRRT_EDEVICE, "adjacency is not symmetric");
        col[k] = nbr[(size_t)j];
        cost[k] = cst[(size_t)j];
        ++k;
      }
    rp[v + 1] = k;
  }
  if (k != m) return fail(G, PIRRT_EDEVICE, "adjacency is not symmetric");
  return pirrt_get_policy(G, g, parent, pcost, PIRRT_MEM_HOST);
}

int pirrt_state_restore(pirrt_graph* G, const void* blob, int64_t size) {
  int rc = guard(G);
  if (rc) return rc;
  if (G->batched) return fail(G, PIRRT_EINVAL, "a batch has no state blob");
  BlobHeader h;
  if (!blob || size < (int64_t)sizeof(h)) return fail(G, PIRRT_EINVAL, "blob is NULL or too small");
  memcpy(&h, blob, sizeof(h));
  if (h.magic != kBlobMagic || h.version != 1 || h.header_bytes != sizeof(h) || h.n < 0 || h.m < 0 ||
      h.n > (int64_t)INT32_MAX - 1 || h.m > ((int64_t)1 << 40) || size < blob_bytes(h.n, h.m))
    return fail(G, PIRRT_EINVAL, "not a state blob of this library, or truncated");
  const char* in = static_cast<const char*>(blob);
  const int64_t* rp = reinterpret_cast<const int64_t*>(in + sizeof(BlobHeader));
  const int32_t* col = reinterpret_cast<const int32_t*>(rp + h.n + 1);
  const float* cost = reinterpret_cast<const float*>(col + h.m);
  const float* g = cost + h.m;
  const int32_t* parent = reinterpret_cast<const int32_t*>(g + h.n);
  const float* pcost = reinterpret_cast<const float*>(parent + h.n);
  if (h.n == 0) return G->n == 0 ? PIRRT_OK : fail(G, PIRRT_EINVAL, "the blob holds an empty graph");
  // the policy is checked before anything changes (the rows by insert_rows itself)
  for (int64_t v = 0; v < h.n; ++v) {
    uint32_t w;
    memcpy(&w, &pcost[v], 4);
    if (parent[v] < -1 || parent[v] >= h.n || parent[v] == v || (w >> 31) != 0 || (w & 0x7f800000u) == 0x7f800000u)
      return fail(G, PIRRT_EINVAL, "blob policy has a bad parent or pcost");
  }
  if (G->n == 0) {
    // a fresh handle: the saved graph, then the saved policy
    if (rp[h.n] != h.m) return fail(G, PIRRT_EINVAL, "blob row offsets do not match its edge count");
    if ((rc = insert_rows(G, (int32_t)h.n, rp, col, cost, PIRRT_MEM_HOST, false))) return rc;
  } else if (G->n != h.n || G->nnz != 2 * h.m) {
    return fail(G, PIRRT_EINVAL, "the handle holds another graph (vertex or edge count differs)");
  }
  return pirrt_set_policy(G, g, parent, pcost, PIRRT_MEM_HOST);
}

// ---------------------------------------------------------------------------
// Batches of independent problems.

int pirrt_batch_create(pirrt_batch** out, const pirrt_config* cfg) {
  if (!out) return PIRRT_EINVAL;
  *out = nullptr;
  int rc;
  pirrt_graph* G = new_graph(cfg, &rc);
  if (!G) return rc;
  G->batched = true;
  G->pbase.assign(1, 0);
  pirrt_batch* B = new (std::nothrow) pirrt_batch();
  if (!B) {
    pirrt_graph_destroy(G);
    return PIRRT_ENOMEM;
  }
  B->G = G;
  *out = B;
  return PIRRT_OK;
}

int pirrt_batch_destroy(pirrt_batch* B) {
  if (!B) return PIRRT_OK;
  pirrt_graph_destroy(B->G);
  delete B;
  return PIRRT_OK;
}

int pirrt_batch_add_problem(pirrt_batch* B, int32_t n, const int64_t* row_ptr, const int32_t* col, const float* cost,
                            int mem_kind, int32_t* index) {
  if (!B) return PIRRT_EINVAL;
  pirrt_graph* G = B->G;
  int rc = guard(G);
  if (rc) return rc;
  if (n <= 0) return fail(G, PIRRT_EINVAL, "a problem needs at least one vertex");
  const int32_t id = (int32_t)G->pbase.size() - 1;
  if ((rc = insert_rows(G, n, row_ptr, col, cost, mem_kind, true))) return rc;
  if (index) *index = id;
  return PIRRT_OK;
}

int pirrt_batch_insert(pirrt_batch* B, int32_t count, const int32_t* problems, const int32_t* n_new,
                       const int64_t* row_ptr, const int32_t* col, const float* cost, int mem_kind) {
  if (!B) return PIRRT_EINVAL;
  pirrt_graph* G = B->G;
  int rc = guard(G);
  if (rc) return rc;
  return grow_problems(G, count, problems, n_new, row_ptr, col, cost, mem_kind);
}

int32_t pirrt_batch_num_problems(const pirrt_batch* B) { return B ? (int32_t)B->G->pbase.size() - 1 : -1; }
int64_t pirrt_batch_num_vertices(const pirrt_batch* B) { return B ? B->G->n : -1; }
int64_t pirrt_batch_num_edges(const pirrt_batch* B) { return B ? B->G->nnz : -1; }

int64_t pirrt_batch_problem_offset(const pirrt_batch* B, int32_t problem) {
  if (!B || problem < 0 || problem >= (int32_t)B->G->pbase.size()) return -1;
  return B->G->pbase[(size_t)problem];
}

int pirrt_batch_replan(pirrt_batch* B, const int32_t* roots, const int32_t* goals, const float* h, uint32_t flags,
                       float* g_out, int32_t* parent_out, int mem_kind, pirrt_stats* stats) {
  if (!B) return PIRRT_EINVAL;
  pirrt_graph* G = B->G;
  int rc = guard(G);
  if (rc) return rc;
  const int32_t P = (int32_t)G->pbase.size() - 1;
  if (P <= 0) return fail(G, PIRRT_EINVAL, "empty batch");
  if (!roots || !goals) return fail(G, PIRRT_EINVAL, "roots or goals is NULL");
  if (flags & PIRRT_TRUNCATED) return fail(G, PIRRT_EINVAL, "the truncated Evaluate takes a single graph");
  if (mem_kind != PIRRT_MEM_HOST && mem_kind != PIRRT_MEM_DEVICE) return fail(G, PIRRT_EINVAL, "bad mem_kind");
  for (int32_t i = 0; i < P; ++i) {
    const int64_t b = G->pbase[(size_t)i], len = G->pbase[(size_t)i + 1] - b;
    if (roots[i] < 0 || roots[i] >= len || goals[i] < 0 || goals[i] >= len)
      return fail(G, PIRRT_EINVAL, "root or goal out of range in problem " + std::to_string(i));
  }
  if (G->renumber_pending && (rc = renumber(G))) return rc;
  if ((rc = upload_bases(G))) return rc;
  std::vector<int32_t> rid((size_t)P), rs((size_t)P), gs((size_t)P);
  for (int32_t i = 0; i < P; ++i) {
    const int64_t b = G->pbase[(size_t)i];
    rid[(size_t)i] = (int32_t)(b + roots[i]);
    rs[(size_t)i] = G->hslot[(size_t)(b + roots[i])];
    gs[(size_t)i] = G->hslot[(size_t)(b + goals[i])];
  }
  const float* hdev = nullptr;
  if ((rc = stage_h(G, h, mem_kind, &hdev))) return rc;
  G->lookahead = (flags & PIRRT_LOOKAHEAD) != 0;
  G->truncated = false;
  const PolicyOut po{g_out, parent_out, mem_kind};
  rc = run_replan(G, P, rid.data(), rs.data(), gs.data(), hdev, (flags & PIRRT_NO_PRUNE) == 0,
                  (flags & PIRRT_TIMING) != 0, stats, &po);
  if (rc != PIRRT_OK && rc != PIRRT_ENOTCONVERGED) return rc;
  return rc;
}

int pirrt_batch_tune(pirrt_batch* B, const int32_t* roots, const int32_t* goals, const float* h, uint32_t flags,
                     int mem_kind, int32_t* config) {
  if (!B) return PIRRT_EINVAL;
  pirrt_graph* G = B->G;
  int rc = guard(G);
  if (rc) return rc;
  const int32_t P = (int32_t)G->pbase.size() - 1;
  if (P <= 0) return fail(G, PIRRT_EINVAL, "empty batch");
  if (!roots || !goals) return fail(G, PIRRT_EINVAL, "roots or goals is NULL");
  if (flags & PIRRT_TRUNCATED) return fail(G, PIRRT_EINVAL, "the truncated Evaluate takes a single graph");
  if (mem_kind != PIRRT_MEM_HOST && mem_kind != PIRRT_MEM_DEVICE) return fail(G, PIRRT_EINVAL, "bad mem_kind");
  for (int32_t i = 0; i < P; ++i) {
    const int64_t b = G->pbase[(size_t)i], len = G->pbase[(size_t)i + 1] - b;
    if (roots[i] < 0 || roots[i] >= len || goals[i] < 0 || goals[i] >= len)
      return fail(G, PIRRT_EINVAL, "root or goal out of range in problem " + std::to_string(i));
  }
  if (G->renumber_pending && (rc = renumber(G))) return rc;
  if ((rc = upload_bases(G))) return rc;
  std::vector<int32_t> rid((size_t)P), rs((size_t)P), gs((size_t)P);
  for (int32_t i = 0; i < P; ++i) {
    const int64_t b = G->pbase[(size_t)i];
    rid[(size_t)i] = (int32_t)(b + roots[i]);
    rs[(size_t)i] = G->hslot[(size_t)(b + roots[i])];
    gs[(size_t)i] = G->hslot[(size_t)(b + goals[i])];
  }
  const float* hdev = nullptr;
  if ((rc = stage_h(G, h, mem_kind, &hdev))) return rc;
  G->lookahead = (flags & PIRRT_LOOKAHEAD) != 0;
  G->truncated = false;
  return tune(G, P, rid.data(), rs.data(), gs.data(), hdev, (flags & PIRRT_NO_PRUNE) == 0, config);
}

int pirrt_batch_get_policy(pirrt_batch* B, float* g_out, int32_t* parent_out, float* pcost_out, int mem_kind) {
  return B ? pirrt_get_policy(B->G, g_out, parent_out, pcost_out, mem_kind) : PIRRT_EINVAL;
}

int pirrt_batch_snapshot_save(pirrt_batch* B) { return B ? pirrt_snapshot_save(B->G) : PIRRT_EINVAL; }

int pirrt_batch_snapshot_restore(pirrt_batch* B) { return B ? pirrt_snapshot_restore(B->G) : PIRRT_EINVAL; }

const char* pirrt_batch_last_error(const pirrt_batch* B) { return B ? B->G->err.c_str() : g_create_error.c_str(); }

}  // extern "C"
