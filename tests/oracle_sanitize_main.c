/*
 * Host-only driver for the oracle under AddressSanitizer and UndefinedBehavior-
 * Sanitizer (built and run by tests/test_oracle_sanitize.py).  It drives every
 * entry point of oracle/pirrt_oracle.c and oracle/rrg_oracle.c over small seeded
 * graphs -- batches grown from sampled points, every Replan mode with and without
 * pruning and heuristic, the iteration cap, a policy of orphans, degenerate graphs
 * -- and over each invalid-argument path.  It checks no results (the pin tests do);
 * it exists so that an out-of-bounds access, a leak, a use after free or undefined
 * arithmetic in the oracle stops the run.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t iterations;
  int64_t edges_examined, sum_P, sum_D, changed_total, mark_edges;
} orc_stats;
typedef struct orc_graph orc_graph;

orc_graph* orc_create(void);
void orc_destroy(orc_graph* G);
int64_t orc_num_vertices(const orc_graph* G);
int64_t orc_num_edges(const orc_graph* G);
int orc_insert(orc_graph* G, int32_t n_new, const int64_t* row_ptr, const int32_t* col, const float* cost);
int orc_set_state(orc_graph* G, const float* g, const int32_t* parent, const float* pcost);
void orc_get_state(const orc_graph* G, float* g, int32_t* parent, float* pcost);
void orc_get_adjacency(const orc_graph* G, int64_t* out_ptr, int32_t* out_nbr, float* out_cost);
int orc_replan_mode(orc_graph* G, int32_t root, int32_t goal, const float* h, int prune, int mode,
                    int32_t max_iters, orc_stats* st);
int64_t orc_evaluate(orc_graph* G, int32_t root);
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]);
int orc_sample(int d, uint64_t seed, uint32_t stream, uint64_t* counter, int64_t count, int n_obs,
               const int32_t* kind, const double* centre, const double* size, int64_t max_candidates, double* pts);
int orc_segment_blocked(int d, const double* a, const double* b, int n_obs, const int32_t* kind,
                        const double* centre, const double* size);
int64_t orc_build_rows(int d, int64_t n_old, int64_t n, const double* pts, double r, int n_obs,
                       const int32_t* kind, const double* centre, const double* size, int64_t* row_ptr,
                       int32_t* col, float* cost, int64_t cap);
void orc_heuristic(int d, int64_t n, const double* pts, const double* goal, float* h);

static uint64_t lcg = 88172645463325252ull;
static double unif(void) {
  lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

#define CHECK(cond)                                                 \
  do {                                                              \
    if (!(cond)) {                                                  \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      exit(2);                                                      \
    }                                                               \
  } while (0)

/* One scene: points sampled by the exploration oracle, rows built in three
   batches, every Replan mode after each batch. */
static void scene(int d, int n_obs, int n_total, uint64_t seed) {
  int32_t kind[16];
  double centre[16 * 8], size[16 * 8];
  for (int o = 0; o < n_obs; ++o) {
    kind[o] = o & 1;
    for (int k = 0; k < d; ++k) {
      centre[o * d + k] = 0.2 + 0.6 * unif();
      size[o * d + k] = 0.04 + 0.06 * unif();
    }
  }
  double* pts = (double*)malloc(sizeof(double) * (size_t)n_total * (size_t)d);
  CHECK(pts);
  for (int k = 0; k < d; ++k) {
    pts[k] = 0.05;
    pts[d + k] = 0.95;
  }
  uint64_t counter = 0;
  CHECK(orc_sample(d, seed, 0, &counter, n_total - 2, n_obs, kind, centre, size, 100000000, pts + 2 * d) == 0);
  orc_graph* G = orc_create();
  CHECK(G);
  const int64_t cuts[4] = {0, n_total / 3, (2 * n_total) / 3, n_total};
  for (int b = 0; b < 3; ++b) {
    const int64_t n_old = cuts[b], n = cuts[b + 1];
    const double r = pow(log((double)n) / (double)n, 1.0 / d) * 1.2;
    const int64_t cap = (n - n_old) * n + 1;
    int64_t* rp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n - n_old + 1));
    int32_t* col = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
    float* cost = (float*)malloc(sizeof(float) * (size_t)cap);
    CHECK(rp && col && cost);
    const int64_t m = orc_build_rows(d, n_old, n, pts, r, n_obs, kind, centre, size, rp, col, cost, cap);
    CHECK(m >= 0);
    CHECK(orc_insert(G, (int32_t)(n - n_old), rp, m ? col : NULL, m ? cost : NULL) == 0);
    free(rp);
    free(col);
    free(cost);
    float* h = (float*)malloc(sizeof(float) * (size_t)n);
    CHECK(h);
    orc_heuristic(d, n, pts, pts + d, h);
    for (int mode = 0; mode < 3; ++mode)
      for (int prune = 0; prune < 2; ++prune)
        for (int hh = 0; hh < 2; ++hh) {
          orc_stats st;
          const int rc = orc_replan_mode(G, 0, 1, hh ? h : NULL, prune, mode, 0, &st);
          CHECK(rc == 0);
          const int rc2 = orc_replan_mode(G, 1, 0, NULL, prune, mode, 2, NULL);
          CHECK(rc2 == 0 || rc2 == -4);
        }
    free(h);
  }
  const int64_t n = orc_num_vertices(G), nnz = orc_num_edges(G);
  int64_t* ptr = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int32_t* nbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz + 1));
  float* cst = (float*)malloc(sizeof(float) * (size_t)(nnz + 1));
  float* g = (float*)malloc(sizeof(float) * (size_t)n);
  int32_t* par = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  float* pc = (float*)malloc(sizeof(float) * (size_t)n);
  CHECK(ptr && nbr && cst && g && par && pc);
  orc_get_adjacency(G, ptr, nbr, cst);
  orc_get_adjacency(G, ptr, NULL, NULL);
  orc_get_state(G, g, par, pc);
  orc_get_state(G, NULL, NULL, NULL);
  /* a policy of orphans, then Replan from it; Evaluate alone */
  for (int64_t v = 0; v < n; ++v) {
    g[v] = INFINITY;
    par[v] = -1;
    pc[v] = 0.0f;
  }
  CHECK(orc_set_state(G, g, par, pc) == 0);
  CHECK(orc_replan_mode(G, 0, 1, NULL, 1, 0, 0, NULL) == 0);
  CHECK(orc_evaluate(G, 1) >= 1);
  /* invalid arguments */
  par[0] = (int32_t)n;
  CHECK(orc_set_state(G, g, par, pc) == -1);
  CHECK(orc_replan_mode(G, -1, 1, NULL, 1, 0, 0, NULL) == -1);
  CHECK(orc_replan_mode(G, 0, (int32_t)n, NULL, 1, 0, 0, NULL) == -1);
  CHECK(orc_replan_mode(G, 0, 1, NULL, 1, 3, 0, NULL) == -1);
  CHECK(orc_replan_mode(G, 0, 1, NULL, 1, 4, 0, NULL) == -1);
  float hbad[1];
  (void)hbad;
  free(ptr); free(nbr); free(cst); free(g); free(par); free(pc);
  orc_destroy(G);
  free(pts);
}

static void invalid_batches(void) {
  orc_graph* G = orc_create();
  CHECK(G);
  const int64_t rp0[3] = {0, 0, 1};
  const int32_t col0[1] = {0};
  const float cost0[1] = {1.0f};
  CHECK(orc_insert(G, 2, rp0, col0, cost0) == 0);
  const int64_t rp_bad[2] = {1, 1};
  CHECK(orc_insert(G, 1, rp_bad, col0, cost0) == -1);
  const int64_t rp_dec[3] = {0, 1, 0};
  CHECK(orc_insert(G, 2, rp_dec, col0, cost0) == -1);
  const int64_t rp1[2] = {0, 1};
  const int32_t col_self[1] = {2};
  CHECK(orc_insert(G, 1, rp1, col_self, cost0) == -1);
  const int32_t col_neg[1] = {-1};
  CHECK(orc_insert(G, 1, rp1, col_neg, cost0) == -1);
  const float bad_costs[4] = {NAN, INFINITY, -1.0f, -0.0f};
  for (int k = 0; k < 4; ++k) CHECK(orc_insert(G, 1, rp1, col0, &bad_costs[k]) == -1);
  CHECK(orc_insert(G, -1, rp1, col0, cost0) == -1);
  const int64_t rp_empty[1] = {0};
  CHECK(orc_insert(G, 0, rp_empty, NULL, NULL) == 0);
  CHECK(orc_num_vertices(G) == 2);
  /* zero-cost and parallel edges, a lone vertex */
  const int64_t rp2[3] = {0, 2, 2};
  const int32_t col2[2] = {1, 1};
  const float cost2[2] = {0.0f, 0.5f};
  CHECK(orc_insert(G, 2, rp2, col2, cost2) == 0);
  CHECK(orc_replan_mode(G, 0, 3, NULL, 1, 0, 0, NULL) == 0);
  CHECK(orc_replan_mode(G, 0, 0, NULL, 0, 2, 0, NULL) == 0);
  orc_destroy(G);
  orc_graph* E = orc_create();
  CHECK(E);
  orc_destroy(E);
  orc_destroy(NULL);
}

int main(void) {
  const uint32_t ctr[4] = {0, 0, 0, 0}, key[2] = {0, 0};
  uint32_t out[4];
  orc_philox4x32_10(ctr, key, out);
  const double a[2] = {0.0, 0.0}, b[2] = {1.0, 1.0};
  const int32_t kind[2] = {0, 1};
  const double centre[4] = {0.5, 0.5, 0.2, 0.8}, size[4] = {0.1, 0.0, 0.05, 0.05};
  (void)orc_segment_blocked(2, a, b, 2, kind, centre, size);
  invalid_batches();
  scene(2, 8, 600, 1);
  scene(3, 10, 500, 2);
  scene(6, 12, 400, 3);
  printf("oracle sanitizer run ok\n");
  return 0;
}
