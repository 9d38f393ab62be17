/*
 * pirrt.h -- C ABI of the MI355X (gfx950) implementation of PI-RRT#'s exploitation
 * phase ("Replan": policy evaluation and policy improvement to a fixed point over the
 * random geometric graph that exploration grows), after "GPU Parallelization of
 * Policy Iteration RRT#" (arXiv 2003.04920).
 *
 * Problem statement (Sec. III): a graph G = (V, E) with a cached, symmetric edge cost
 * c : E -> R+ (Sec. IV-A: the only edge property, computed once by Extend), a policy
 * pi : V -> E giving each vertex a parent, the cost-to-come g under that policy, an
 * admissible heuristic h, and the promising set B = { v : g(v) + h(v) < g(x_goal) }.
 * Replan (Alg. 2) alternates Improve (each vertex of the domain takes the neighbour
 * minimising g(n) + c(n, v)) and Evaluate (a breadth-first walk of the policy tree
 * from x_init recomputing g) until no parent changes.
 *
 * Conventions shared by every entry point:
 *   - Vertices are 0 .. n-1 in insertion order.  Vertex 0 is x_init for the
 *     insertion-time policy (it gets g = 0); x_goal is any vertex (vertex 1 by the
 *     usual construction of Alg. 1, which starts from V = {x_init, x_goal}).
 *   - Costs and g are IEEE-754 binary32; every g is one binary32 addition
 *     (round to nearest even) of the parent's g and the parent-edge cost, in
 *     root-to-leaf order.  Unreachable vertices have g = +inf.
 *   - Ties in any minimum go to the lowest neighbour index; Improve switches a
 *     parent only on a strict decrease (Alg. 2's strict comparison).
 *   - mem_kind says where caller buffers live: PIRRT_MEM_HOST (pageable or pinned
 *     host memory) or PIRRT_MEM_DEVICE (device memory on the graph's device).
 *     Inputs are copied before the call returns; the library never keeps caller
 *     pointers.
 *   - Every entry point returns PIRRT_OK (0) or a negative error code; no exception
 *     crosses the ABI.  Arguments are validated before any state changes, so on
 *     PIRRT_EINVAL the graph is unchanged.  After PIRRT_EDEVICE (a HIP runtime error)
 *     the handle is poisoned: every later call except destroy returns PIRRT_EDEVICE.
 *     pirrt_last_error gives a message for the last failure on a handle.
 *   - A handle is not thread safe: use one handle per host thread (or serialise).
 *     All device work of a handle is enqueued on the stream named in its config and
 *     every entry point returns only after its results are complete.
 */
#ifndef PIRRT_H
#define PIRRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PIRRT_OK = 0,
  PIRRT_EINVAL = -1,        /* bad argument; state unchanged */
  PIRRT_ENOMEM = -2,        /* device or host allocation failed; state unchanged */
  PIRRT_EDEVICE = -3,       /* HIP runtime error; handle poisoned */
  PIRRT_ENOTCONVERGED = -4  /* iteration cap reached; policy and g are consistent */
};

enum { PIRRT_MEM_HOST = 0, PIRRT_MEM_DEVICE = 1 };

/* Replan flags. */
enum {
  PIRRT_NO_PRUNE = 1u << 0, /* threshold G = +inf instead of g(goal): every reachable
                               vertex is promising */
  PIRRT_TIMING = 1u << 1,   /* time each phase with HIP events (fills the ms_* and
                               per-kernel fields of pirrt_stats; adds event overhead) */
  PIRRT_LOOKAHEAD = 1u << 2, /* narrowed Improve domain, a work-reduction variant of Sec.
                               IV-C's domain (promising vertices plus their neighbours):
                               a neighbour w of a promising u joins the domain only
                               if fl(fl(g(u) + c(u,w)) + h(w)) < G, i.e. if the candidate u
                               offers could be promising; promising vertices stay in.
                               Improve itself is unchanged.  The fixed point differs from
                               the default's in general; g(goal) keeps the default's
                               optimality argument under a consistent h.  Without
                               pruning both rules coincide. */
  PIRRT_TRUNCATED = 1u << 3 /* truncated Evaluate, Alg. 2's Evaluate as printed (single
                               graphs only; not with PIRRT_LOOKAHEAD, EINVAL otherwise).
                               Every Evaluate of the call walks the policy tree
                               breadth-first from the root with G0 = g(goal) as held
                               when the walk starts (+inf with PIRRT_NO_PRUNE): a child
                               of a queued vertex gets its fresh g and is queued only
                               when fl(g + h) < G0; the root is never queued.  Vertices
                               the walk does not reach keep their previous g (they are
                               not reset to +inf).  P of the next iteration is the set
                               the walk queued; D, Improve and the cap as above, except
                               that a minimum equal to a vertex's own parent and cost
                               is not a switch (a skipped vertex's stale g could
                               otherwise keep the loop going forever).  The result may
                               stop above the full mode's fixed point, and g holds
                               stale values on skipped vertices. */
};

typedef struct pirrt_graph pirrt_graph;

typedef struct {
  int64_t vertex_capacity; /* initial reservation in vertices (0 = library default);
                              storage grows on demand */
  int64_t edge_capacity;   /* initial reservation in directed adjacency entries */
  void* hip_stream;        /* hipStream_t for all device work; NULL = the null stream */
  int32_t max_iters;       /* Replan iteration cap; 0 = 4n + 8 */
  int32_t device;          /* HIP device ordinal; -1 = the device current at create */
  /* Optional device-memory callbacks (both or neither; NULL = hipMalloc / hipFree),
     e.g. a framework's caching allocator.  alloc(bytes, alloc_ctx) returns device
     memory on the handle's device, aligned to at least 256 bytes, or NULL (the call
     then fails with ENOMEM and the handle is unchanged); free(ptr, alloc_ctx) returns
     a block alloc gave.  Both are called on the thread that calls the library, with
     the handle's device current, at create, when storage grows and at destroy; the
     memory is used on hip_stream, and every block is freed before destroy returns.
     The callbacks must not call back into this handle. */
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* alloc_ctx;
} pirrt_config;

typedef struct {
  int32_t iterations;     /* Improve passes, including the last one with no change */
  int32_t on_host;        /* 1 when the call replanned on the host (small graphs), else 0 */
  int64_t edges_examined; /* sum over iterations of the degrees of the Improve domain */
  int64_t sum_P;          /* sum over iterations of |promising set| */
  int64_t sum_D;          /* sum over iterations of |Improve domain| */
  int64_t changed_total;  /* sum over iterations of parents switched */
  /* wall time of the call and, with PIRRT_TIMING, of its phases (milliseconds); the
     phases of a batch run for all of its problems at once, so every problem's entry
     holds the batch's phase times and launch counts */
  double ms_total;
  double ms_evaluate;
  double ms_mark;
  double ms_improve;
  int32_t improve_launches; /* launches of the Improve kernel timed in ms_improve */
  int32_t mark_launches;
  int32_t evaluate_calls;
  int32_t reserved;
  int64_t mark_edges;     /* sum over iterations of the promising set's degrees (the rows
                             streamed to mark the Improve domain) */
} pirrt_stats;

/* Fills *cfg with defaults (capacities 0, NULL stream, cap 0, device -1, no allocator
   callbacks). */
int pirrt_config_init(pirrt_config* cfg);

/* Creates an empty graph (no vertices) on the configured device.  cfg may be NULL
   (defaults).  *out receives the handle, owned by the caller until destroy. */
int pirrt_graph_create(pirrt_graph** out, const pirrt_config* cfg);

/* Releases the handle and all its device memory.  NULL is allowed. */
int pirrt_graph_destroy(pirrt_graph* g);

/*
 * Extend for a batch (Sec. III; Alg. 1 with S = 1, Alg. 3 with batch size S):
 * appends n_new vertices with ids n_old .. n_old + n_new - 1 (n_old = current
 * count).  Row i (entries row_ptr[i] .. row_ptr[i+1]-1 of col/cost) lists the
 * neighbours j of vertex n_old + i with j < n_old + i, each undirected edge given
 * once from its higher endpoint, with its cached cost c (Sec. IV-A).
 *   row_ptr : int64[n_new + 1], row_ptr[0] == 0, non-decreasing.
 *   col     : int32[row_ptr[n_new]], 0 <= col < own id.  Repeated entries are kept
 *             as parallel edges.
 *   cost    : float[row_ptr[n_new]], finite and >= 0.
 * The library stores each edge in both endpoints' adjacency, then sets the
 * insertion-time policy of each new vertex in ascending id order (Extend's local
 * relaxation): (g, parent) = the smallest (g(u) + c, u) over its neighbours u below
 * it, or an orphan (g = +inf, parent = -1) if none is finite; vertex 0 gets g = 0.
 * Errors: EINVAL (n_new < 0, bad row_ptr/col/cost, ids beyond INT32_MAX), ENOMEM,
 * EDEVICE.
 */
int pirrt_insert_batch(pirrt_graph* g, int32_t n_new, const int64_t* row_ptr, const int32_t* col,
                       const float* cost, int mem_kind);

/*
 * Replan (Alg. 2) from the stored policy to its fixed point, with root = x_init and
 * goal = x_goal.  Sets parent(root) = -1, runs Evaluate, then repeats
 *   G = g(goal) (or +inf with PIRRT_NO_PRUNE);  P = { v : g(v) + h(v) < G };
 *   D = P and every neighbour of a vertex of P, minus the root (Sec. IV-C);
 *   Improve over D against the g of the last Evaluate (Jacobi, Sec. IV);
 * re-evaluating after each Improve that switched a parent, until one switches none.
 *   h          : float[n] admissible heuristic (>= 0, not NaN), or NULL for h = 0.
 *   g_out      : float[n] or NULL; receives g.
 *   parent_out : int32[n] or NULL; receives the parent of each vertex (-1 for the
 *                root and for vertices never attached); the final tree is
 *                { (parent(v), v) } (Alg. 1 output).
 *   mem_kind   : location of h, g_out and parent_out.
 *   stats      : optional.
 * Adaptive placement (the CPU/GPU choice the paper's break-even size motivates,
 * Sec. VI-VII): a graph of at most 512 vertices (environment PIRRT_HOST_MAX at create;
 * 0 = always the device) replans on the calling host thread, with the same steps and
 * the same binary32 arithmetic, so the results and counters are identical either way;
 * stats->on_host says which ran, and its phase timings stay 0.  PIRRT_TRUNCATED always
 * runs on the device.
 * Errors: EINVAL (root/goal out of range, bad h, PIRRT_TRUNCATED with
 * PIRRT_LOOKAHEAD), ENOTCONVERGED (cap reached; the state is a consistent policy with
 * its g -- with PIRRT_TRUNCATED, except for the stale g the mode leaves on vertices its
 * walks skip), EDEVICE.
 */
int pirrt_replan(pirrt_graph* g, int32_t root, int32_t goal, const float* h, uint32_t flags,
                 float* g_out, int32_t* parent_out, int mem_kind, pirrt_stats* stats);

/*
 * Autotuner: runs the Replan this call describes (arguments as pirrt_replan) once
 * per kernel configuration -- the Improve / promising-set row split (lanes per row
 * x 16-byte quads in flight: 16x1, 8x2, 4x4, 8x1) and the scope of the walk
 * Evaluate's stamps (device, workgroup) -- each from the current policy, keeps the
 * fastest for later calls on this handle and restores the policy (results never
 * depend on the configuration).  *config (nullable) receives the index chosen,
 * row split + 4 x (workgroup-scope stamps).  Without a tuning call a handle uses
 * configuration 5 (8x2, workgroup-scope stamps).
 */
int pirrt_tune(pirrt_graph* g, int32_t root, int32_t goal, const float* h, uint32_t flags, int mem_kind,
               int32_t* config);

/* Copies the stored policy out: g, parent and parent-edge cost (each may be NULL). */
int pirrt_get_policy(pirrt_graph* g, float* g_out, int32_t* parent_out, float* pcost_out, int mem_kind);

/* Replaces the stored policy (for starting Replan from an arbitrary policy, Sec. V).
   parent[v] must be -1 or a vertex id other than v; pcost must be finite and >= 0.
   g is stored as given (Replan recomputes it from the tree). */
int pirrt_set_policy(pirrt_graph* g, const float* g_in, const int32_t* parent_in, const float* pcost_in,
                     int mem_kind);

/* Keeps a device-side copy of the policy (g, parent, pcost) / restores it.  Restore
   fails with EINVAL if no snapshot exists or the vertex count changed since. */
int pirrt_snapshot_save(pirrt_graph* g);
int pirrt_snapshot_restore(pirrt_graph* g);

/*
 * Alg. 3's replan test |B'| > |B|: after an Extend batch, the number of vertices among
 * ids [first, first + count) that are promising under the stored policy (their
 * insertion-time g), i.e. fl(g(v) + h(v)) < g(goal) with the stored g(goal) (an
 * unreachable goal, g = +inf, makes every reachable vertex promising).  Replan is due
 * when it is nonzero.  h: float[n] over all vertices in caller ids at mem_kind, or
 * NULL (h = 0); only [first, first + count) is read (and, from host memory, checked:
 * >= 0, not NaN).  *out: host int64.  EINVAL for a batch's graph, a goal or range
 * outside the graph.  Synchronous.
 */
int pirrt_promising_count(pirrt_graph* g, int32_t goal, const float* h, int64_t first, int64_t count, int mem_kind,
                          int64_t* out);

/* Copies the adjacency out as CSR: ptr int64[n+1], nbr int32[nnz], cost float[nnz]
   (any may be NULL).  The order of entries inside a row is unspecified. */
int pirrt_get_adjacency(pirrt_graph* g, int64_t* ptr, int32_t* nbr, float* cost, int mem_kind);

/*
 * Checkpoint and resume of a graph handle (the state Replan of Alg. 2 works on: the
 * graph with its cached costs, Sec. IV-A, and the policy with its g) through caller
 * memory.  The blob is host memory the caller owns: a 48-byte header, the graph as
 * forward rows (row_ptr int64[n+1], then each vertex's lower-id neighbours col
 * int32[m] with their costs float[m], m = nnz / 2, the pirrt_insert_batch format),
 * then g float[n], parent int32[n] and pcost float[n] in caller ids.
 *   pirrt_state_size: bytes of the blob for the handle's current state (-1 for NULL,
 *     a poisoned handle or a batch's graph).
 *   pirrt_state_save: writes the blob into `blob` (size >= pirrt_state_size, else
 *     EINVAL); the handle is unchanged.
 *   pirrt_state_restore: reads a blob of pirrt_state_save.  Into an empty handle it
 *     inserts the saved graph and sets the saved policy, so the handle then holds
 *     exactly the saved graph and policy; into a handle holding the same vertex and
 *     edge counts it replaces the policy only (the caller vouches that the graph is
 *     the saved one).  A blob that is not one, is truncated, or holds a bad policy
 *     or rows, or a handle holding another graph, gives EINVAL with the handle
 *     unchanged.  Root marks are not saved: parents of roots read -1 either way.
 */
int64_t pirrt_state_size(pirrt_graph* g);
int pirrt_state_save(pirrt_graph* g, void* blob, int64_t size);
int pirrt_state_restore(pirrt_graph* g, const void* blob, int64_t size);

int64_t pirrt_num_vertices(const pirrt_graph* g);
int64_t pirrt_num_edges(const pirrt_graph* g); /* directed entries = 2 x undirected */

const char* pirrt_last_error(const pirrt_graph* g);
const char* pirrt_strerror(int code);

/*
 * Batches of independent planning problems (many robots or many queries, each with
 * its own RRG; the data-parallel form of Sec. IV applied across graphs).  One
 * handle stores every problem's graph side by side in one device store, and one
 * pirrt_batch_replan runs Alg. 2 for all of them at once: each iteration's
 * threshold, promising set, domain, Improve, Evaluate and convergence test are per
 * problem, and a problem that reached its fixed point takes no further part.  The
 * result of each problem is exactly that of pirrt_replan on a graph holding that
 * problem alone.
 *
 * Ids are local to a problem: vertex k of problem i is 0 <= k < n_i, and parents
 * in policies are local ids.  Arrays of per-vertex values (h, g, parent, pcost)
 * are concatenations of the problems in index order, problem i starting at
 * pirrt_batch_problem_offset(b, i).  Error conventions are those of the graph
 * handle above.
 */
typedef struct pirrt_batch pirrt_batch;

/* Creates an empty batch on the configured device (cfg as for pirrt_graph_create;
   max_iters caps every problem). */
int pirrt_batch_create(pirrt_batch** out, const pirrt_config* cfg);

/* Releases the batch and its device memory.  NULL is allowed. */
int pirrt_batch_destroy(pirrt_batch* b);

/*
 * Adds a problem with n >= 1 vertices given as forward rows exactly as in
 * pirrt_insert_batch, with local ids (row i lists neighbours j < i).  Local vertex
 * 0 is the problem's x_init for the insertion-time policy.  *index (nullable)
 * receives the problem's index (0, 1, ... in order of addition).
 * Errors: EINVAL (n < 1, bad rows, total ids beyond INT32_MAX), ENOMEM, EDEVICE.
 */
int pirrt_batch_add_problem(pirrt_batch* b, int32_t n, const int64_t* row_ptr, const int32_t* col,
                            const float* cost, int mem_kind, int32_t* index);

/*
 * Grows problems of the batch: Alg. 3's exploration step for many planners at once
 * (each extends its own graph by a batch of vertices, Sec. III Extend), before one
 * pirrt_batch_replan replans them all.  For k in [0, count), n_new[k] >= 0 vertices
 * are appended to problem problems[k] (host arrays; indices distinct).  The rows of
 * all blocks are concatenated in k order: row_ptr int64[T + 1] (T = sum of n_new),
 * col int32 / cost float indexed by it, at mem_kind.  Row i of block k is the new
 * local vertex n_p + i of its problem p (n_p = p's vertex count before the call) and
 * lists its neighbours j < n_p + i in p's local ids, each undirected edge once, as
 * in pirrt_insert_batch.  Each new vertex takes the insertion-time policy of
 * pirrt_insert_batch.  Afterwards problem p holds n_p + n_new vertices with local ids
 * unchanged for the old ones, and the per-vertex offsets of the problems move
 * (pirrt_batch_problem_offset gives the new ones).  A snapshot taken before the call
 * is dropped.  Errors: EINVAL (bad count, index, repeated problem, rows or costs;
 * the batch unchanged), ENOMEM, EDEVICE.  Work: one pass over the batch's adjacency
 * plus the new rows.
 */
int pirrt_batch_insert(pirrt_batch* b, int32_t count, const int32_t* problems, const int32_t* n_new,
                       const int64_t* row_ptr, const int32_t* col, const float* cost, int mem_kind);

int32_t pirrt_batch_num_problems(const pirrt_batch* b);
int64_t pirrt_batch_num_vertices(const pirrt_batch* b); /* all problems together */
int64_t pirrt_batch_num_edges(const pirrt_batch* b);    /* directed entries, all problems */
/* First position of problem i in concatenated per-vertex arrays (i == count gives
   the total); -1 if out of range. */
int64_t pirrt_batch_problem_offset(const pirrt_batch* b, int32_t problem);

/*
 * Replan (Alg. 2) for every problem.  roots / goals: host int32[P] local ids.  h,
 * g_out, parent_out: concatenated per-vertex arrays (nullable) at mem_kind.  flags:
 * as pirrt_replan, except that PIRRT_TRUNCATED is rejected (EINVAL).  stats: host
 * pirrt_stats[P] or NULL (with PIRRT_TIMING the phase timings cover all problems
 * together and are copied into every entry).
 * Returns ENOTCONVERGED if any problem reached the cap (each problem's state is
 * still a consistent policy with its g).
 */
int pirrt_batch_replan(pirrt_batch* b, const int32_t* roots, const int32_t* goals, const float* h,
                       uint32_t flags, float* g_out, int32_t* parent_out, int mem_kind, pirrt_stats* stats);

/* As pirrt_tune for the batch's Replan of every problem, with one more dimension: the
   workgroups of the batch's grid-stride launches (2048, 1024, 4096, 8192), tried with
   the best configuration of the others.  *config = row split + 4 x (workgroup-scope
   stamps) + 8 x (index of the workgroup count in that list). */
int pirrt_batch_tune(pirrt_batch* b, const int32_t* roots, const int32_t* goals, const float* h, uint32_t flags,
                     int mem_kind, int32_t* config);

/* Policy of every problem (concatenated, local parent ids). */
int pirrt_batch_get_policy(pirrt_batch* b, float* g_out, int32_t* parent_out, float* pcost_out, int mem_kind);

/* As pirrt_snapshot_save / pirrt_snapshot_restore for the whole batch. */
int pirrt_batch_snapshot_save(pirrt_batch* b);
int pirrt_batch_snapshot_restore(pirrt_batch* b);

const char* pirrt_batch_last_error(const pirrt_batch* b);

/*
 * Exploration support: growing the random geometric graph on the device (Sec. III,
 * Extend: sample a state, connect it to the earlier vertices within the connection
 * radius by collision-free straight segments, cache each edge's cost; Alg. 3 does
 * this for batches of S samples).  A pirrt_rrg handle holds a scene (the unit cube
 * [0,1]^d with sphere and axis-aligned box obstacles, all closed sets) and a list of
 * points in binary64, row-major, d per point, kept in device memory.  Its rows go
 * into a pirrt_graph or a pirrt_batch without leaving the device.
 *
 * Definitions (bit-exact contract):
 *   - Sampling: candidate k of stream s under seed q has coordinate i equal to
 *     (w_i >> 8) * 2^-24, where w_0..w_3 = Philox4x32-10(counter {k mod 2^32,
 *     k >> 32, s, 0}, key {q mod 2^32, q >> 32}) and w_4..w_7 the same with counter
 *     word 3 = 1 (Salmon et al., SC'11).  A candidate inside or on an obstacle is
 *     rejected; free candidates are appended in order of k.
 *   - Obstacles: sphere = sum over axes (x_k - c_k)^2 <= R^2; box = every
 *     |x_k - c_k| <= s_k.
 *   - Edge u-v (u < v): d2 = sum over axes in order of (x_u - x_v)^2 in binary64 with
 *     0 < d2 <= r*r, and the closed segment from x_u to x_v meets no obstacle (sphere:
 *     the segment point closest to the centre, parameter ((c - x_u).e)/(e.e) clamped
 *     to [0, 1] with e = x_v - x_u, lies within R; box: slab test).  Cost = binary32
 *     rounding of sqrt(d2).  Rows list u ascending.
 *   - Heuristic: binary32 rounding of the binary64 distance to the goal point.
 */
typedef struct pirrt_rrg pirrt_rrg;

typedef struct {
  int32_t d;              /* dimension, 1..8 */
  int32_t n_obstacles;    /* >= 0 */
  const int32_t* kind;    /* host int32[n_obstacles]: 0 = sphere, 1 = box; copied */
  const double* centre;   /* host float64[n_obstacles * d]; copied */
  const double* size;     /* host float64[n_obstacles * d]: sphere radius in entry 0,
                             box half-sides; finite, >= 0; copied */
  int64_t point_capacity; /* initial reservation in points (grows on demand) */
  void* hip_stream;       /* hipStream_t for all device work; NULL = the null stream */
  int32_t device;         /* HIP device ordinal; -1 = the device current at create */
} pirrt_rrg_config;

/* Creates a handle with no points.  Errors: EINVAL (d outside 1..8, bad obstacle),
   ENOMEM, EDEVICE. */
int pirrt_rrg_create(pirrt_rrg** out, const pirrt_rrg_config* cfg);
int pirrt_rrg_destroy(pirrt_rrg* r);
int64_t pirrt_rrg_num_points(const pirrt_rrg* r);

/* Appends count given points (float64[count * d], finite; e.g. x_init and x_goal). */
int pirrt_rrg_add_points(pirrt_rrg* r, int32_t count, const double* pts, int mem_kind);

/* Appends count free samples of stream `stream` under `seed`, starting at candidate
   *counter; on return *counter is one past the last candidate taken, so successive
   calls continue the same sequence.  EINVAL if no free sample turns up. */
int pirrt_rrg_sample(pirrt_rrg* r, uint64_t seed, uint32_t stream, uint64_t* counter, int32_t count);

/* Copies points first .. first+count-1 out (float64[count * d]). */
int pirrt_rrg_get_points(pirrt_rrg* r, int64_t first, int64_t count, double* out, int mem_kind);

/* Forward rows of points n_old .. n-1 against all earlier points at the given
   radius: row_ptr int64[n - n_old + 1], col int32 / cost float[*nnz] (col and cost
   may be NULL).  *nnz receives the entry count; EINVAL if it exceeds capacity. */
int pirrt_rrg_rows(pirrt_rrg* r, int64_t n_old, double radius, int64_t* row_ptr, int32_t* col, float* cost,
                   int64_t capacity, int64_t* nnz, int mem_kind);

/* Builds the rows of points n_old .. n-1 and inserts them into g, which must hold
   exactly the points 0 .. n_old-1 as its vertices (pirrt_insert_batch on device
   buffers; g and r on the same device). */
int pirrt_rrg_connect(pirrt_rrg* r, int64_t n_old, double radius, pirrt_graph* g);

/* Builds the rows of all points and adds them to b as one new problem
   (pirrt_batch_add_problem); *index (nullable) receives its index. */
int pirrt_rrg_connect_problem(pirrt_rrg* r, double radius, pirrt_batch* b, int32_t* index);

/* h_out float[n]: heuristic of every point towards point `goal`. */
int pirrt_rrg_heuristic(pirrt_rrg* r, int64_t goal, float* h_out, int mem_kind);

const char* pirrt_rrg_last_error(const pirrt_rrg* r);

/*
 * Learned sampling proposal (not in the paper: a network that scores candidate
 * samples by how likely they are to lie near the optimal path; the planner mixes
 * its picks 50/50 with uniform samples, so Replan stays exact on whatever graph
 * results).  Network: features (in_dim <= 288 binary32 values per sample, e.g. the
 * sample's coordinates then the obstacle encoding) -> 256 -> 256 -> 1 logit, ReLU
 * hidden layers.  Parameters are binary32 masters laid out as one array:
 *   W1 [288 x 256] row-major (rows >= in_dim stay 0), b1 [256],
 *   W2 [256 x 256] row-major, b2 [256], w3 [256], b3 [1]
 * (pirrt_mlp_num_params() floats).  Every product uses bfloat16 (round to nearest
 * even) copies of the weights and bfloat16 activations with binary32 accumulation:
 *   X = bf16(features); A1 = bf16(relu(X W1 + b1)); A2 = bf16(relu(A1 W2 + b2));
 *   logit = A2 bf16(w3) + b3.
 * Training minimises the mean BCE-with-logits loss with Adam; the backward pass
 * rounds dZ2 = dz w3^T [Z2 > 0] and dZ1 = dZ2 W2^T [Z1 > 0] to bfloat16 before its
 * products.  x: float[B * in_dim] row-major; y: float[B] labels in {0, 1}.
 */
typedef struct pirrt_mlp pirrt_mlp;

typedef struct {
  int32_t in_dim;    /* feature width, 1..288 */
  int32_t max_batch; /* largest B of any call */
  float lr, beta1, beta2, eps; /* Adam constants (lr > 0, 0 <= beta < 1, eps > 0) */
  void* hip_stream;  /* hipStream_t; NULL = the null stream */
  int32_t device;    /* HIP device ordinal; -1 = current */
} pirrt_mlp_config;

int64_t pirrt_mlp_num_params(void);
int32_t pirrt_mlp_in_dim(const pirrt_mlp* net); /* -1 for NULL */
/* Creates a network with all parameters 0 (set them with pirrt_mlp_set_params). */
int pirrt_mlp_create(pirrt_mlp** out, const pirrt_mlp_config* cfg);
int pirrt_mlp_destroy(pirrt_mlp* net);
/* Replaces the binary32 parameters (finite) and resets the Adam state. */
int pirrt_mlp_set_params(pirrt_mlp* net, const float* params, int mem_kind);
int pirrt_mlp_get_params(pirrt_mlp* net, float* params, int mem_kind);
/* logits: float[B]. */
int pirrt_mlp_forward(pirrt_mlp* net, int32_t B, const float* x, float* logits, int mem_kind);
/*
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the forward pass of
 * pirrt_mlp_forward with the same kernels and the same logits bit for bit, with its
 * staged features and hidden activations in a fixed array inside the library
 * (12.5 MiB per GPU, allocated with the code object and held until the process ends)
 * instead of the handle's buffers.  It calls no hipMalloc, hipFree or other
 * allocating routine.
 *   x: device float[B * in_dim] (row-major features); logits: device float[B].
 *   1 <= B <= PIRRT_MLP_NOALLOC_MAX_BATCH (any max_batch of the handle); a larger B,
 *   or a NULL pointer, returns PIRRT_EINVAL with nothing enqueued.
 * Asynchronous: the work is enqueued on the handle's stream and the call returns
 * without waiting (it makes no stream or device synchronisation, so it may be
 * captured); logits are valid once the stream reaches that point.  Every call on a
 * GPU shares that GPU's array: calls on one stream are ordered, but calls that
 * overlap on one GPU (other streams, other threads, other handles) race and may
 * return wrong logits.  EDEVICE if the array's device address cannot be obtained.
 */
#define PIRRT_MLP_NOALLOC_MAX_BATCH 8192
int pirrt_mlp_forward_noalloc(pirrt_mlp* net, int32_t B, const float* x, float* logits);
/* Gradient of the mean loss into grads (parameter layout, nullable) and the loss
   into *loss (host, nullable); parameters unchanged. */
int pirrt_mlp_gradients(pirrt_mlp* net, int32_t B, const float* x, const float* y, float* grads, float* loss,
                        int mem_kind);
/* One Adam step on one batch; *loss (host, nullable) = the batch loss before it. */
int pirrt_mlp_train_step(pirrt_mlp* net, int32_t B, const float* x, const float* y, float* loss, int mem_kind);
const char* pirrt_mlp_last_error(const pirrt_mlp* net);

/*
 * Learned proposal sampling: appends to r the `count` best of n_candidates free
 * uniform candidates (<= 8192) of stream `stream` under `seed` from *counter on
 * (advanced past them), scored by net on features = the candidate's coordinates
 * (binary32), then enc[enc_len] (host, e.g. the obstacle encoding); d + enc_len must
 * equal the network's in_dim and n_candidates may not exceed its max_batch.  Higher
 * logit wins, the earlier candidate among equal logits; the chosen ones are appended
 * in candidate order.  The planner mixes these with pirrt_rrg_sample draws.
 */
int pirrt_rrg_sample_learned(pirrt_rrg* r, pirrt_mlp* net, const float* enc, int32_t enc_len, uint64_t seed,
                             uint32_t stream, uint64_t* counter, int32_t n_candidates, int32_t count);

#ifdef __cplusplus
}
#endif

#endif /* PIRRT_H */
