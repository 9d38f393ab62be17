// Internal interfaces between the host runtime (capi.hip) and the kernel files.
#pragma once

#include "common.h"

namespace pirrt {

// ---- scan.hip ----
size_t scan_scratch_bytes(int64_t n);
void scan_i32_to_i64(const int32_t* in, int64_t n, int64_t* out, void* scratch, hipStream_t s);
void scan_i32_to_i32(const int32_t* in, int64_t n, int32_t* out, void* scratch, hipStream_t s);

// ---- store.hip ----
// Neighbour ids of row i must lie in [lo_bound, n_old + i).
// nnz_dev (nullable): read the entry count from the device (row_ptr[n_new]) instead of nnz.
void launch_validate_rows(int32_t n_new, int64_t n_old, int64_t lo_bound, const int64_t* rp, const int32_t* col,
                          const float* cost, int64_t nnz, int* err, hipStream_t s,
                          const int64_t* nnz_dev = nullptr);
void launch_offset_ids(int64_t m, int32_t offset, int32_t* ids, hipStream_t s);
// Growing problems of a batch: one block of appended rows per grown problem.
struct BatchBlock {
  int64_t row_begin;  // first row of the block among all appended rows
  int64_t base_old;   // the problem's first caller id before the growth
  int64_t app_base;   // append id of the block's first vertex (n_old + row_begin)
  int32_t problem;
  int32_t n_old;      // the problem's vertex count before the growth
};
void launch_batch_rows(int32_t total, int32_t nblk, const BatchBlock* blk, const int64_t* brp, int32_t* bcol, int* err,
                       hipStream_t s);
void launch_block_problems(int64_t n_old, int32_t total, int32_t nblk, const BatchBlock* blk, int32_t* prob,
                           hipStream_t s);
void launch_reid(int64_t n1, int64_t n_old, int32_t nblk, const BatchBlock* blk, const int64_t* pbase_old,
                 const int64_t* pbase_new, const int32_t* prob, int32_t* ext_of, int32_t* slot_of, hipStream_t s);
// add0: int32 per slot, all zero on entry and on return (the per-row counts of new
// entries are gathered there and cleared when read).
void launch_rebuild(int32_t n_new, int64_t n_old, const int64_t* brp, const int32_t* bcol, const float* bcost,
                    const int64_t* rp_old, const int32_t* col_old, const float* cst_old, int64_t* rp_new,
                    int32_t* col_new, float* cst_new, int32_t* add, int32_t* add0, int32_t* deg, void* scan_scratch,
                    hipStream_t s);
// Appends a block whose entries all lie inside it (a new problem of a batch): its
// rows go after the nnz_old existing entries of rp / col / cst, which must have room
// for nnz_old + 2 * brp[n_new] entries; older rows are untouched.  tmp: n_new + 1.
void launch_append(int32_t n_new, int64_t n_old, int64_t nnz_old, const int64_t* brp, const int32_t* bcol,
                   const float* bcost, int64_t* rp, int32_t* col, float* cst, int32_t* add, int32_t* deg,
                   int64_t* tmp, void* scan_scratch, hipStream_t s);
void launch_pending(int32_t n_new, int64_t n_old, const int64_t* brp, const int32_t* bcol, int32_t* pending,
                    int32_t* frontier, int32_t* fcount, hipStream_t s);
// bcol: neighbour ids as given (tie-break keys); bslot: the same in storage slots.
// insert_root: the new vertex that gets g = 0 (x_init), or -1.  The level's frontier
// size is read on the device from *fsize (the grid covers max_size threads), and
// *done accumulates the sizes, so several levels go out without a host round trip.
// Every dependency level of a small batch in one single-workgroup launch (the first
// frontier in f0, its size at fsize0; f1 the other frontier buffer).
constexpr int32_t kInsertBlockMax = 2048;
void launch_insert_block(const int32_t* fsize0, int32_t* done, int32_t* f0, int32_t* f1, int64_t n_old, int32_t n_new,
                         int32_t insert_root, const int64_t* brp, const int32_t* bcol, const int32_t* bslot,
                         const float* bcost, const int64_t* rp, const int32_t* col, float* g, int32_t* parent,
                         float* pcost, int32_t* pending, hipStream_t s);
void launch_insert_level(int32_t max_size, const int32_t* fsize, int32_t* done, const int32_t* frontier,
                         int64_t n_old, int32_t insert_root, const int64_t* brp, const int32_t* bcol,
                         const int32_t* bslot, const float* bcost, const int64_t* rp, const int32_t* col, float* g,
                         int32_t* parent, float* pcost, int32_t* pending, int32_t* next, int32_t* ncount,
                         hipStream_t s);

// ---- reorder.hip ----
struct PermuteArgs {
  int32_t n;
  const int32_t* order;    // order[k] = old slot of new slot k
  int32_t* newslot;        // out: new slot of each old slot
  int32_t* deg;            // scratch, n
  const int64_t* rp;
  const int32_t* col;
  const float* cst;
  int64_t* rp_new;
  int32_t* col_new;
  float* cst_new;
  const float* g;
  const int32_t* parent;
  const float* pcost;
  const int32_t* ext_of;
  float* g2;
  int32_t* parent2;
  float* pcost2;
  int32_t* ext2;
  int32_t* slot_of;        // updated in place
  void* scan_scratch;
};
// Slots [lo, hi) take the same caller ids; with prob, they join problem `problem`.
void launch_identity_ids(int64_t lo, int64_t hi, int32_t* ext_of, int32_t* slot_of, hipStream_t s,
                         int32_t* prob = nullptr, int32_t problem = 0);
void launch_translate(int64_t m, const int32_t* ids, const int32_t* slot_of, int32_t* out, hipStream_t s);
void launch_fill_i32(int64_t lo, int64_t hi, int32_t value, int32_t* a, hipStream_t s);
// prob[s] for s < n from the problems' slot ranges (base: P + 1 device offsets).
void launch_problem_map(int64_t n, int32_t P, const int64_t* base, int32_t* prob, hipStream_t s);
void launch_unmark_roots(int32_t m, const int32_t* ids, const int32_t* slot_of, int32_t* parent, hipStream_t s);
void launch_bfs_init(int32_t P, const int32_t* roots, const int64_t* base, int32_t* order, int32_t* visited,
                     int32_t* pcnt, int32_t* frontier, int32_t* fcount, hipStream_t s);
// One level of the renumbering BFS.  discover lists the newly reached vertices in
// cand (unordered, *ccount of them) with key = lowest discovering frontier index;
// order_level groups them by key into next (the next frontier) and appends each
// problem's part to its range of order.  visited: 0 = unreached, else the tag of
// the level that reached the vertex.  key starts at INT32_MAX for every vertex.
void launch_bfs_discover(int32_t fsize, const int32_t* frontier, int32_t tag, const int64_t* rp, const int32_t* col,
                         int32_t* visited, int32_t* key, int32_t* cand, int32_t* ccount, hipStream_t s);
void launch_bfs_order_level(int32_t fsize, int32_t m, const int32_t* cand, const int32_t* key, int32_t* hist,
                            int64_t* off, int32_t* cursor, int32_t* next, const int32_t* prob, int32_t* pstart,
                            int32_t* pcnt, int32_t* order, void* scan_scratch, hipStream_t s);
// Clustered order: Luby rounds (state 0 undecided / 1 seed / 2 covered; *undecided
// counts the vertices left), then out = the vertices grouped by their seed's rank in
// `order`.
void launch_mis_round(int32_t n, const int64_t* rp, const int32_t* col, int32_t* state, int32_t* win,
                      int32_t* undecided, hipStream_t s);
void launch_cluster_order(int32_t n, const int64_t* rp, const int32_t* col, const int32_t* state, const int32_t* order,
                          int32_t* rank, int32_t* key, int32_t* hist, int64_t* off, int32_t* cursor, int32_t* out,
                          void* scan_scratch, hipStream_t s);
void launch_append_unvisited(int32_t n, const int32_t* visited, int32_t* order, const int32_t* prob, int32_t* pcnt,
                             hipStream_t s);
void launch_permute(const PermuteArgs& a, hipStream_t s);
void launch_gather_by_slot(int32_t n, const int32_t* ext_of, const float* src_ext, float* dst_slot, hipStream_t s);
// prob/base (nullable): parents are reported relative to the first id of the
// vertex's problem.
void launch_policy_to_ext(int32_t n, const int32_t* slot_of, const int32_t* ext_of, const int32_t* prob,
                          const int64_t* base, const float* g, const int32_t* parent, const float* pcost,
                          float* g_ext, int32_t* parent_ext, float* pcost_ext, hipStream_t s);
void launch_policy_from_ext(int32_t n, const int32_t* slot_of, const int32_t* prob, const int64_t* base,
                            const float* g_ext, const int32_t* parent_ext, const float* pcost_ext, float* g,
                            int32_t* parent, float* pcost, hipStream_t s);

// ---- evaluate.hip ----
struct EvalArgs {
  int32_t n;
  const ProblemState* ps;  // one problem (its root); the walk runs only when ps->needs_eval
  int32_t* parent;
  float* pcost;
  float* g;
  int32_t* child_cnt;   // n, all zero on entry and on exit
  int32_t* child_ptr;   // n + 1
  int32_t* child;       // n
  int32_t* fr0;         // n
  int32_t* fr1;         // n
  int32_t* lvl;         // level sizes, n + kMaxMidLaunches + 4
  EvalInfo* info;
  void* scan_scratch;
  int32_t mid_launches; // wide level launches between head and tail
  int32_t level_blocks; // grid of each wide level launch
};
constexpr int32_t kMaxMidLaunches = 1024;
void launch_evaluate(const EvalArgs& a, hipStream_t s);
// Walk evaluation of every problem with needs_eval (see evaluate.hip).
struct WalkArgs {
  int32_t n;
  const int32_t* prob;     // problem of each slot, or NULL for a single problem
  ProblemState* ps;
  LoopCtl* ctl;            // eval_epoch, any_eval
  // Single graphs, the walk after an Improve: the walk also takes the finish step (sums
  // the iteration's counters, which accumulate over the Replan, applies the convergence
  // test and the cap) and runs only if a parent switched.
  bool finish;
  IterCounters* ctr;
  const int32_t* parent;   // roots carry kRootMark
  const float* pcost;
  float* g;
  unsigned long long* word;  // n {epoch, g bits} stamps
  unsigned long long* hops;  // nullable: total parent links walked
  int parts;               // launches over consecutive slot ranges (single graphs)
  const int32_t* tiles;    // batches: active tile list
  bool coherent;           // device-scope stamp accesses
  // Truncated Evaluate (single graphs): only the children of vertices with
  // fl(g + h) < ps[0].thr are visited; unvisited vertices keep their g.
  bool truncated;
  const float* h;          // nullable (h = 0)
  int blocks;              // batches: workgroups of the grid-stride launch
};
void launch_eval_walk(const WalkArgs& a, hipStream_t s);
// Workgroups of the batched walk resident on one compute unit (256 threads and 16 KB
// of LDS each: 8 waves per SIMD).
constexpr int kWalkResidentPerCu = 8;

// ---- host_replan.hip ----
// One Replan of a small graph on the host, on slot-ordered host copies (see the file).
struct HostReplan {
  int32_t n;
  const int64_t* rp;   // adjacency: row offsets [n + 1], neighbour slots, costs
  const int32_t* col;
  const float* cst;
  const int32_t* ext;  // caller id of each slot (tie-break key)
  const float* h;      // slot order, or NULL (h = 0)
  float* g;            // out
  int32_t* parent;     // in / out (the root gets kRootMark)
  float* pcost;        // in / out
  int32_t root, goal;  // slots
  bool prune, lookahead;
  int64_t cap;         // iteration cap
};
struct HostReplanStats {
  int32_t iterations;
  int64_t edges, sum_P, sum_D, changed, mark_edges;
};
// 0 at the fixed point, 1 at the iteration cap (the state is consistent either way).
int host_replan(const HostReplan& p, HostReplanStats* st);

// ---- driver.hip ----
// Also sets each problem's threshold to g(goal) as stored (+inf without pruning): the
// threshold the truncated Evaluate reads in the first walk.
void launch_replan_init(int32_t P, ProblemState* ps, int32_t* parent, float* pcost, IterCounters* ctr,
                        LoopCtl* ctl, const float* g, int prune, hipStream_t s);
// A single graph's set-up from scalar arguments (no host copies): unmarks the nold
// previous roots listed in droots (caller ids), marks root (a slot), writes root_id to
// droots[0] and initialises ps[0] with goal (a slot) and cap.
void launch_replan_init_single(ProblemState* ps, int32_t root, int32_t goal, int32_t cap, int32_t root_id,
                               int32_t nold, int32_t* droots, const int32_t* slot_of, int32_t* parent, float* pcost,
                               IterCounters* ctr, LoopCtl* ctl, const float* g, int prune, hipStream_t s);
// single: one graph (P == 1, no problem map); see launch_after_eval.
void launch_finish(int32_t P, ProblemState* ps, IterCounters* ctr, LoopCtl* ctl, bool single, hipStream_t s);
// prob / base / tiles: a batch's problem map, its problems' slot ranges (P + 1
// offsets) and the active tile list it rebuilds (NULL for a single graph).  Up to
// bitmap_tiles tiles (and the LDS bitmap's capacity) the list is read off a tile
// bitmap; beyond, each tile's first and last problem are looked up.  Only batches
// launch it: a single graph's promising list does the same work for its one problem at
// the start of the next iteration.
// tiles_walk (nullable): the same tiles ordered by their rank inside their problem,
// for the Evaluate walk.
void launch_after_eval(int32_t P, ProblemState* ps, const float* g, int prune, LoopCtl* ctl, int32_t n,
                       const int32_t* prob, const int64_t* base, int32_t* tiles, int32_t bitmap_tiles,
                       int32_t* tiles_walk, hipStream_t s);

// ---- improve.hip ----
struct StepArgs {
  int32_t n;
  int64_t nnz;               // adjacency entries (selects 32-bit offsets when they fit)
  const int32_t* prob;       // problem of each slot, or NULL for a single problem
  ProblemState* ps;          // thresholds and roots
  LoopCtl* ctl;              // epoch, any_active, ndomain
  int prune;                 // single graphs: threshold g(goal) (1) or +inf (0)
  const float* g;
  const float* h;            // nullable
  const int64_t* rp;
  const int32_t* col;
  const float* cst;
  uint8_t* stamp;            // low byte of the mark epoch per slot
  const int32_t* ext_of;     // caller id of each slot (tie-break key)
  int32_t* parent;
  float* pcost;
  IterCounters* ctr;         // kCounterSlots copies per problem
  int32_t* dlist;            // compacted Improve domain (n entries of room)
  int32_t* plist;            // single graphs: compacted promising set (n entries of room)
  const int32_t* tiles;      // batches: active tile list (see LoopCtl::ntiles)
  bool lookahead;            // narrowed domain: stamp a neighbour only for a promising offer
  // Truncated Evaluate (single graphs): P is the set the last walk queued (read from
  // the walk stamps), and Improve counts a switch only when it changes the policy.
  bool truncated;
  const unsigned long long* word;  // the walk stamps
  int blocks;                // batches: workgroups of each grid-stride launch
};
constexpr int kRowVariants = 4;
// One small graph (n <= kSmallMax vertices; the single workgroup is faster than the
// multi-kernel loop up to about 1,700 vertices of a 2D graph) replanned by a single workgroup with its
// vertex state in LDS: the whole loop in one launch (small.hip).  Reads the root,
// goal and cap from ps[0] and leaves the counters and status there; parent / pcost
// are read and written in place (the root's entries untouched), g written.
constexpr int32_t kSmallMax = 1536;
void launch_replan_small(int32_t n, const int64_t* rp, const int32_t* col, const float* cst, const float* h,
                         const int32_t* ext_of, bool prune, bool lookahead, ProblemState* ps, int32_t* parent,
                         float* pcost, float* g, hipStream_t s);
void launch_mark(const StepArgs& a, int variant, hipStream_t s);
// Compacts the stamped slots into dlist / ctl->ndomain (and clears every stamp when
// the next mark epoch wraps its low byte).
void launch_domain_list(const StepArgs& a, hipStream_t s);
// out += number of ids in [first, first + count) with fl(g + h) < g(goal); h is indexed
// from `first` (nullable).
void launch_count_promising(int64_t first, int64_t count, int32_t goal_slot, const int32_t* slot_of, const float* g,
                            const float* h, unsigned long long* out, hipStream_t s);
void launch_improve(const StepArgs& a, int variant, hipStream_t s);

}  // namespace pirrt
