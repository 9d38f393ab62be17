/*
 * ORACLE -- test infrastructure only.  A plain, slow, serial CPU statement of what
 * PI-RRT#'s exploitation phase computes, used by the tests, the smoke check and the
 * CPU baseline of the benchmark to check the GPU library.  It shares no code with
 * the GPU path and is never part of the product path.
 *
 * Source: Arslan-style PI-RRT# as restated in "GPU Parallelization of Policy
 * Iteration RRT#" (arXiv 2003.04920): Sec. III (problem statement, Alg. 1 and the
 * Replan / Improve / Evaluate procedures of Alg. 2), Sec. IV-A (cached edge cost,
 * SoA vertex properties g, h, p, b), Sec. IV-B and IV-C (Jacobi improvement over
 * the promising set and its neighbours; breadth-first tree evaluation), Sec. V
 * (batched extension: Replan over the whole graph from any initial policy).
 *
 * Arithmetic: IEEE-754 binary32.  Every g value is produced by exactly one binary32
 * addition of two binary32 operands (round to nearest even); nothing is fused,
 * reassociated or widened.  Build with -O2 -ffp-contract=off on x86-64 (SSE, no
 * excess precision).
 *
 * Readings of the paper taken here (each documented with the design notes):
 *   - Extend's local relaxation (Sec. III) picks, for a new vertex v, the existing
 *     neighbour u < v minimising (g(u) + c(u,v), u, c) lexicographically (the cost
 *     only separates parallel edges); with no finite candidate v is an orphan
 *     (g = +inf, parent = -1).  Vertex 0 is x_init and gets g = 0.  Costs must be
 *     finite, >= 0 and not -0.0.
 *   - Evaluate (Alg. 2) is taken in full: every vertex whose parent chain reaches
 *     the root gets g(v) = g(parent) + c(parent, v) in breadth-first order from the
 *     root; every other vertex gets +inf.  The promising set is rebuilt after the
 *     traversal from each vertex's own fresh value: B = { v : g(v) + h(v) < G },
 *     G = g(x_goal) (or +inf with pruning off).
 *   - Improve (Alg. 2, Sec. IV-B) runs over the promising vertices and their
 *     neighbours (Sec. IV-C), excluding the root, as a Jacobi step: every candidate
 *     reads the g of the last Evaluate.  Among the neighbours it takes the
 *     lexicographic minimum of (g(n) + c(n,v), n, c) and switches only when that value
 *     is strictly below g(v), as the strict comparison of Alg. 2 does.
 *   - The convergence test dJ < eps is taken with eps at its limit: stop when no
 *     parent changed (then dJ = 0); an iteration cap guards termination.
 *   - A separate mode keeps Evaluate truncated as Alg. 2 prints it (children of
 *     vertices that fail the promising test are not visited and keep their old g),
 *     with the threshold read once before each walk.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENOTCONVERGED (-4)

typedef struct {
  int32_t iterations;
  int64_t edges_examined; /* sum over Improve domains of the vertex degree */
  int64_t sum_P;          /* sum over iterations of |promising set| */
  int64_t sum_D;          /* sum over iterations of |Improve domain| */
  int64_t changed_total;  /* sum over iterations of parents switched */
  int64_t mark_edges;     /* sum over iterations of the degrees of the promising set
                             (the rows walked to build D = P u N(P)) */
} orc_stats;

typedef struct {
  int64_t n;
  int64_t nnz; /* directed adjacency entries (2 x undirected edges) */
  int32_t* deg;
  int32_t* cap;
  int32_t** nbr;
  float** cst;
  float* g;
  int32_t* parent;
  float* pcost;
} orc_graph;

orc_graph* orc_create(void) { return (orc_graph*)calloc(1, sizeof(orc_graph)); }

void orc_destroy(orc_graph* G) {
  if (!G) return;
  for (int64_t v = 0; v < G->n; ++v) {
    free(G->nbr[v]);
    free(G->cst[v]);
  }
  free(G->deg); free(G->cap); free(G->nbr); free(G->cst);
  free(G->g); free(G->parent); free(G->pcost);
  free(G);
}

int64_t orc_num_vertices(const orc_graph* G) { return G->n; }
int64_t orc_num_edges(const orc_graph* G) { return G->nnz; }

static int push_adj(orc_graph* G, int64_t v, int32_t u, float c) {
  if (G->deg[v] == G->cap[v]) {
    int32_t nc = G->cap[v] ? 2 * G->cap[v] : 8;
    int32_t* nn = (int32_t*)realloc(G->nbr[v], sizeof(int32_t) * (size_t)nc);
    if (!nn) return ORC_ENOMEM;
    G->nbr[v] = nn;
    float* cc = (float*)realloc(G->cst[v], sizeof(float) * (size_t)nc);
    if (!cc) return ORC_ENOMEM;
    G->cst[v] = cc;
    G->cap[v] = nc;
  }
  G->nbr[v][G->deg[v]] = u;
  G->cst[v][G->deg[v]] = c;
  G->deg[v]++;
  return ORC_OK;
}

/*
 * Extend for a batch of new vertices (Sec. III; Alg. 1 / Alg. 3 inner loop).
 * Row i of (row_ptr, col, cost) lists the existing neighbours u < n_old + i of the
 * new vertex n_old + i with the cached edge cost c(u, v) (Sec. IV-A).  The edge is
 * stored in both adjacency lists (the graph is undirected).  Then, in ascending
 * vertex order, the local relaxation sets g, parent and pcost of the new vertex.
 */
int orc_insert(orc_graph* G, int32_t n_new, const int64_t* row_ptr, const int32_t* col,
               const float* cost) {
  if (n_new < 0) return ORC_EINVAL;
  int64_t n0 = G->n, n1 = G->n + n_new;
  if (row_ptr[0] != 0) return ORC_EINVAL;
  for (int32_t i = 0; i < n_new; ++i) {
    if (row_ptr[i + 1] < row_ptr[i]) return ORC_EINVAL;
    for (int64_t j = row_ptr[i]; j < row_ptr[i + 1]; ++j) {
      float c = cost[j];
      if (col[j] < 0 || col[j] >= n0 + i) return ORC_EINVAL;
      if (!(c >= 0.0f) || isinf(c) || signbit(c)) return ORC_EINVAL;
    }
  }
  /* grow the per-vertex arrays */
  int32_t* deg = (int32_t*)realloc(G->deg, sizeof(int32_t) * (size_t)(n1 > 0 ? n1 : 1));
  if (!deg) return ORC_ENOMEM;
  G->deg = deg;
  int32_t* cap = (int32_t*)realloc(G->cap, sizeof(int32_t) * (size_t)(n1 > 0 ? n1 : 1));
  if (!cap) return ORC_ENOMEM;
  G->cap = cap;
  int32_t** nbr = (int32_t**)realloc(G->nbr, sizeof(int32_t*) * (size_t)(n1 > 0 ? n1 : 1));
  if (!nbr) return ORC_ENOMEM;
  G->nbr = nbr;
  float** cst = (float**)realloc(G->cst, sizeof(float*) * (size_t)(n1 > 0 ? n1 : 1));
  if (!cst) return ORC_ENOMEM;
  G->cst = cst;
  float* g = (float*)realloc(G->g, sizeof(float) * (size_t)(n1 > 0 ? n1 : 1));
  if (!g) return ORC_ENOMEM;
  G->g = g;
  int32_t* parent = (int32_t*)realloc(G->parent, sizeof(int32_t) * (size_t)(n1 > 0 ? n1 : 1));
  if (!parent) return ORC_ENOMEM;
  G->parent = parent;
  float* pcost = (float*)realloc(G->pcost, sizeof(float) * (size_t)(n1 > 0 ? n1 : 1));
  if (!pcost) return ORC_ENOMEM;
  G->pcost = pcost;
  for (int64_t v = n0; v < n1; ++v) {
    G->deg[v] = 0;
    G->cap[v] = 0;
    G->nbr[v] = NULL;
    G->cst[v] = NULL;
  }
  G->n = n1;
  for (int32_t i = 0; i < n_new; ++i) {
    int64_t v = n0 + i;
    for (int64_t j = row_ptr[i]; j < row_ptr[i + 1]; ++j) {
      if (push_adj(G, v, col[j], cost[j]) != ORC_OK) return ORC_ENOMEM;
      if (push_adj(G, col[j], (int32_t)v, cost[j]) != ORC_OK) return ORC_ENOMEM;
      G->nnz += 2;
    }
  }
  /* Local relaxation of each new vertex over its existing (lower-index)
     neighbours, in insertion order. */
  for (int32_t i = 0; i < n_new; ++i) {
    int64_t v = n0 + i;
    if (v == 0) {
      G->g[v] = 0.0f;
      G->parent[v] = -1;
      G->pcost[v] = 0.0f;
      continue;
    }
    float best = INFINITY;
    int32_t best_u = -1;
    float best_c = 0.0f;
    for (int64_t j = row_ptr[i]; j < row_ptr[i + 1]; ++j) {
      int32_t u = col[j];
      float cand = G->g[u] + cost[j];
      if (cand < best || (cand == best && best_u >= 0 && (u < best_u || (u == best_u && cost[j] < best_c)))) {
        if (cand < INFINITY) {
          best = cand;
          best_u = u;
          best_c = cost[j];
        }
      }
    }
    G->g[v] = best;
    G->parent[v] = best_u;
    G->pcost[v] = best_u >= 0 ? best_c : 0.0f;
  }
  return ORC_OK;
}

/* Overwrites the policy (for tests that start Replan from an arbitrary policy). */
int orc_set_state(orc_graph* G, const float* g, const int32_t* parent, const float* pcost) {
  for (int64_t v = 0; v < G->n; ++v) {
    if (parent[v] < -1 || parent[v] >= G->n) return ORC_EINVAL;
  }
  memcpy(G->g, g, sizeof(float) * (size_t)G->n);
  memcpy(G->parent, parent, sizeof(int32_t) * (size_t)G->n);
  memcpy(G->pcost, pcost, sizeof(float) * (size_t)G->n);
  return ORC_OK;
}

void orc_get_state(const orc_graph* G, float* g, int32_t* parent, float* pcost) {
  if (g) memcpy(g, G->g, sizeof(float) * (size_t)G->n);
  if (parent) memcpy(parent, G->parent, sizeof(int32_t) * (size_t)G->n);
  if (pcost) memcpy(pcost, G->pcost, sizeof(float) * (size_t)G->n);
}

/* Adjacency export (for tests): out_ptr[n+1], out_nbr[nnz], out_cost[nnz]. */
void orc_get_adjacency(const orc_graph* G, int64_t* out_ptr, int32_t* out_nbr, float* out_cost) {
  int64_t k = 0;
  for (int64_t v = 0; v < G->n; ++v) {
    out_ptr[v] = k;
    for (int32_t j = 0; j < G->deg[v]; ++j) {
      if (out_nbr) out_nbr[k] = G->nbr[v][j];
      if (out_cost) out_cost[k] = G->cst[v][j];
      ++k;
    }
  }
  out_ptr[G->n] = k;
}

/*
 * Evaluate (Alg. 2; Sec. IV-C): a breadth-first walk of the policy tree from the
 * root with a FIFO queue; each child n of a popped vertex v gets
 * g(n) = g(v) + c(v, n).  Vertices not reached keep +inf.  Returns the number of
 * tree levels visited.
 */
static int64_t evaluate(orc_graph* G, int32_t root, int32_t* child_ptr, int32_t* child, int32_t* queue,
                        int32_t* depth) {
  int64_t n = G->n;
  /* children lists from the parent pointers */
  for (int64_t v = 0; v <= n; ++v) child_ptr[v] = 0;
  for (int64_t v = 0; v < n; ++v)
    if (v != root && G->parent[v] >= 0) child_ptr[G->parent[v] + 1]++;
  for (int64_t v = 0; v < n; ++v) child_ptr[v + 1] += child_ptr[v];
  for (int64_t v = 0; v < n; ++v) depth[v] = child_ptr[v]; /* fill cursor */
  for (int64_t v = 0; v < n; ++v)
    if (v != root && G->parent[v] >= 0) child[depth[G->parent[v]]++] = (int32_t)v;

  for (int64_t v = 0; v < n; ++v) G->g[v] = INFINITY;
  G->g[root] = 0.0f;
  int64_t head = 0, tail = 0, levels = 0;
  queue[tail++] = root;
  depth[root] = 0;
  while (head < tail) {
    int32_t v = queue[head++];
    if (depth[v] + 1 > levels) levels = depth[v] + 1;
    for (int32_t k = child_ptr[v]; k < child_ptr[v + 1]; ++k) {
      int32_t c = child[k];
      G->g[c] = G->g[v] + G->pcost[c];
      depth[c] = depth[v] + 1;
      queue[tail++] = c;
    }
  }
  return levels;
}

/*
 * Truncated Evaluate: Alg. 2's Evaluate as printed, with two readings.  A child is
 * tested on its own fresh value (not its parent's), and the threshold G0 is the
 * g(x_goal) held when the walk starts (the printed test reads g(x_goal) while the walk
 * may still be changing it).  Breadth-first from the root with a FIFO queue: every
 * child n of a popped vertex v gets g(n) = g(v) + c(v, n); n joins the queue and B
 * only when g(n) + h(n) < G0.  The root is never in B.  Vertices the walk does not
 * reach keep the g they held before it.  Fills inB and returns |B|.
 */
static int64_t evaluate_truncated(orc_graph* G, int32_t root, const float* h, float G0, int32_t* child_ptr,
                                  int32_t* child, int32_t* queue, int32_t* cursor, unsigned char* inB) {
  int64_t n = G->n;
  for (int64_t v = 0; v <= n; ++v) child_ptr[v] = 0;
  for (int64_t v = 0; v < n; ++v)
    if (v != root && G->parent[v] >= 0) child_ptr[G->parent[v] + 1]++;
  for (int64_t v = 0; v < n; ++v) child_ptr[v + 1] += child_ptr[v];
  for (int64_t v = 0; v < n; ++v) cursor[v] = child_ptr[v];
  for (int64_t v = 0; v < n; ++v)
    if (v != root && G->parent[v] >= 0) child[cursor[G->parent[v]]++] = (int32_t)v;

  for (int64_t v = 0; v < n; ++v) inB[v] = 0;
  int64_t nb = 0, head = 0, tail = 0;
  G->g[root] = 0.0f;
  queue[tail++] = root;
  while (head < tail) {
    int32_t v = queue[head++];
    for (int32_t k = child_ptr[v]; k < child_ptr[v + 1]; ++k) {
      int32_t c = child[k];
      G->g[c] = G->g[v] + G->pcost[c];
      float f = G->g[c] + (h ? h[c] : 0.0f);
      if (f < G0) {
        queue[tail++] = c;
        inB[c] = 1;
        ++nb;
      }
    }
  }
  return nb;
}

/*
 * Replan (Alg. 2) from the stored policy: Evaluate, then repeat
 *   promising set  P = { v : g(v) + h(v) < G }          (G = g(goal) or +inf)
 *   Improve domain D = (P and every neighbour of P) minus the root
 *   Improve over D (Jacobi, strict improvement, lowest index on ties)
 * until no parent changes, re-evaluating after every step that changed one.
 * h may be NULL (h = 0).  max_iters <= 0 selects 4n + 8.
 *
 * lookahead != 0 narrows the domain (a work-reduction variant of Sec. IV-C, not the
 * paper's own rule): a neighbour w of a promising u joins D only when the candidate
 * that u offers it could itself be promising, (g(u) + c(u,w)) + h(w) < G, each sum
 * one binary32 addition.  Promising vertices stay in D.  Improve over D is unchanged
 * (every neighbour is a candidate).  With pruning off (G = +inf) the filter keeps
 * every neighbour of a finite-g vertex, so the two modes coincide.
 *
 * mode: bit 0 (ORC_MODE_LOOKAHEAD) is the narrowed domain above; bit 1
 * (ORC_MODE_TRUNCATED) replaces every Evaluate, the first one included, by the
 * truncated Evaluate, and the promising set of each iteration by the B that walk
 * returned (G0 = g(goal) just before the walk, or +inf without pruning).  The two
 * bits together are rejected (EINVAL).  Truncation leaves stale g on the vertices the
 * walk skips; Improve then compares against them, so the loop may stop on a policy
 * that the full mode would still improve.  A stale vertex can also find its own
 * parent below its stale g (dJ > 0) in every iteration, since no walk refreshes it;
 * so in this mode an iteration counts as a change only when some parent or
 * parent-edge cost actually changes, and the loop stops at the first Improve that
 * leaves the policy as it was -- then Evaluate and Improve would repeat themselves
 * exactly.  (In the full mode the two tests agree: a fresh g equals the offer of its
 * own parent, so a strict decrease always moves the parent or the cost.)
 */
#define ORC_MODE_LOOKAHEAD 1
#define ORC_MODE_TRUNCATED 2
int orc_replan_mode(orc_graph* G, int32_t root, int32_t goal, const float* h, int prune, int mode,
                    int32_t max_iters, orc_stats* st);

int orc_replan(orc_graph* G, int32_t root, int32_t goal, const float* h, int prune, int32_t max_iters,
               orc_stats* st) {
  return orc_replan_mode(G, root, goal, h, prune, 0, max_iters, st);
}

int orc_replan_mode(orc_graph* G, int32_t root, int32_t goal, const float* h, int prune, int mode,
                    int32_t max_iters, orc_stats* st) {
  int64_t n = G->n;
  orc_stats local;
  if (!st) st = &local;
  memset(st, 0, sizeof(*st));
  const int lookahead = (mode & ORC_MODE_LOOKAHEAD) != 0, truncated = (mode & ORC_MODE_TRUNCATED) != 0;
  if (mode & ~(ORC_MODE_LOOKAHEAD | ORC_MODE_TRUNCATED)) return ORC_EINVAL;
  if (lookahead && truncated) return ORC_EINVAL;
  if (root < 0 || root >= n || goal < 0 || goal >= n) return ORC_EINVAL;
  if (h) {
    for (int64_t v = 0; v < n; ++v)
      if (!(h[v] >= 0.0f)) return ORC_EINVAL;
  }
  int64_t cap = max_iters > 0 ? max_iters : 4 * n + 8;
  int32_t* child_ptr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t* child = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t* depth = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  unsigned char* inP = (unsigned char*)malloc((size_t)(n > 0 ? n : 1));
  unsigned char* inD = (unsigned char*)malloc((size_t)(n > 0 ? n : 1));
  int32_t* newpar = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  float* newpc = (float*)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
  int rc = ORC_OK;
  if (!child_ptr || !child || !queue || !depth || !inP || !inD || !newpar || !newpc) {
    rc = ORC_ENOMEM;
    goto done;
  }
  G->parent[root] = -1;
  G->pcost[root] = 0.0f;
  int64_t nb = 0; /* |B| of the last truncated Evaluate (inP holds B) */
  if (truncated)
    nb = evaluate_truncated(G, root, h, prune ? G->g[goal] : INFINITY, child_ptr, child, queue, depth, inP);
  else
    evaluate(G, root, child_ptr, child, queue, depth);
  for (;;) {
    float thr = prune ? G->g[goal] : INFINITY;
    int64_t np = 0, nd = 0, ex = 0, nchg = 0, pe = 0;
    if (truncated) {
      np = nb;
      for (int64_t v = 0; v < n; ++v) inD[v] = 0;
    } else {
      for (int64_t v = 0; v < n; ++v) {
        float hv = h ? h[v] : 0.0f;
        float f = G->g[v] + hv;
        inP[v] = f < thr;
        np += inP[v];
        inD[v] = 0;
      }
    }
    for (int64_t v = 0; v < n; ++v) {
      if (!inP[v]) continue;
      inD[v] = 1;
      pe += G->deg[v];
      for (int32_t j = 0; j < G->deg[v]; ++j) {
        int32_t w = G->nbr[v][j];
        if (lookahead) {
          float offer = G->g[v] + G->cst[v][j];
          float f = offer + (h ? h[w] : 0.0f);
          if (!(f < thr)) continue;
        }
        inD[w] = 1;
      }
    }
    inD[root] = 0;
    for (int64_t v = 0; v < n; ++v) {
      newpar[v] = G->parent[v];
      newpc[v] = G->pcost[v];
      if (!inD[v]) continue;
      ++nd;
      ex += G->deg[v];
      float best = INFINITY;
      int32_t best_u = -1;
      float best_c = 0.0f;
      for (int32_t j = 0; j < G->deg[v]; ++j) {
        int32_t u = G->nbr[v][j];
        float cand = G->g[u] + G->cst[v][j];
        if (cand < best || (cand == best && best_u >= 0 && (u < best_u || (u == best_u && G->cst[v][j] < best_c)))) {
          best = cand;
          best_u = u;
          best_c = G->cst[v][j];
        }
      }
      /* Truncated mode: a vertex the last walk skipped may offer its own parent below
         its stale g; that keeps the policy as it is and is not a switch. */
      if (best_u >= 0 && best < G->g[v] && (!truncated || best_u != G->parent[v] || best_c != G->pcost[v])) {
        newpar[v] = best_u;
        newpc[v] = best_c;
        ++nchg;
      }
    }
    st->iterations += 1;
    st->edges_examined += ex;
    st->sum_P += np;
    st->sum_D += nd;
    st->changed_total += nchg;
    st->mark_edges += pe;
    if (nchg == 0) break;
    memcpy(G->parent, newpar, sizeof(int32_t) * (size_t)n);
    memcpy(G->pcost, newpc, sizeof(float) * (size_t)n);
    if (truncated)
      nb = evaluate_truncated(G, root, h, prune ? G->g[goal] : INFINITY, child_ptr, child, queue, depth, inP);
    else
      evaluate(G, root, child_ptr, child, queue, depth);
    if (st->iterations >= cap) {
      rc = ORC_ENOTCONVERGED;
      break;
    }
  }
done:
  free(child_ptr); free(child); free(queue); free(depth);
  free(inP); free(inD); free(newpar); free(newpc);
  return rc;
}

/* Evaluate alone (for the closed-form pin): returns the number of tree levels. */
int64_t orc_evaluate(orc_graph* G, int32_t root) {
  int64_t n = G->n;
  int32_t* child_ptr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t* child = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t* depth = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int64_t levels = -1;
  if (child_ptr && child && queue && depth) {
    G->parent[root] = -1;
    G->pcost[root] = 0.0f;
    levels = evaluate(G, root, child_ptr, child, queue, depth);
  }
  free(child_ptr); free(child); free(queue); free(depth);
  return levels;
}
