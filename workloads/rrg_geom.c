/*
 * Geometry for the seeded synthetic workloads: radius-r neighbour search over a
 * uniform grid and exact segment-versus-obstacle tests in d dimensions.
 *
 * This file builds the planner's INPUT (the random geometric graph that the
 * exploration phase of PI-RRT# grows, Sec. III): for every new vertex v it lists
 * the lower-index vertices u < v within distance r whose straight segment u-v
 * touches no obstacle, with the FP32 rounding of the FP64 Euclidean length as the
 * edge cost.  It holds no part of policy evaluation or improvement and is shared,
 * as data, by the oracle tests and the GPU path.
 *
 * Conventions (closed sets throughout):
 *   sphere  : |x - c| <= R blocks the point; a segment whose closest approach to c
 *             is <= R is in collision.
 *   box     : centre c, half-sides s; |x_k - c_k| <= s_k on every axis blocks; a
 *             segment that meets the closed box (slab test) is in collision.
 *   edge    : kept if |u - v| <= r (FP64), |u - v| > 0, and no obstacle is hit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int64_t nnz;
  int64_t* row_ptr; /* n_new + 1 */
  int32_t* col;     /* nnz, ascending within a row */
  float* cost;      /* nnz */
} rrg_rows;

static int seg_hits_sphere(int d, const double* a, const double* b, const double* c, double rad) {
  double ab2 = 0.0, acab = 0.0;
  for (int k = 0; k < d; ++k) {
    double e = b[k] - a[k];
    ab2 += e * e;
    acab += (c[k] - a[k]) * e;
  }
  double t = ab2 > 0.0 ? acab / ab2 : 0.0;
  if (t < 0.0) t = 0.0;
  if (t > 1.0) t = 1.0;
  double dist2 = 0.0;
  for (int k = 0; k < d; ++k) {
    double p = a[k] + t * (b[k] - a[k]) - c[k];
    dist2 += p * p;
  }
  return dist2 <= rad * rad;
}

static int seg_hits_box(int d, const double* a, const double* b, const double* c, const double* half) {
  double t0 = 0.0, t1 = 1.0;
  for (int k = 0; k < d; ++k) {
    double lo = c[k] - half[k], hi = c[k] + half[k];
    double e = b[k] - a[k];
    if (e == 0.0) {
      if (a[k] < lo || a[k] > hi) return 0;
      continue;
    }
    double ta = (lo - a[k]) / e, tb = (hi - a[k]) / e;
    if (ta > tb) {
      double s = ta;
      ta = tb;
      tb = s;
    }
    if (ta > t0) t0 = ta;
    if (tb < t1) t1 = tb;
    if (t0 > t1) return 0;
  }
  return 1;
}

/* 1 if the segment a-b meets any obstacle.  A cheap bounding-sphere reject runs
   first: the segment lies within |b-a|/2 of its midpoint. */
static int seg_blocked(int d, const double* a, const double* b, int n_obs, const int32_t* kind,
                       const double* centre, const double* size, const double* bound) {
  double mid[16];
  double half_len2 = 0.0;
  for (int k = 0; k < d; ++k) {
    mid[k] = 0.5 * (a[k] + b[k]);
    double e = 0.5 * (b[k] - a[k]);
    half_len2 += e * e;
  }
  double half_len = sqrt(half_len2);
  for (int o = 0; o < n_obs; ++o) {
    const double* c = centre + (int64_t)o * d;
    double dm2 = 0.0;
    for (int k = 0; k < d; ++k) {
      double e = mid[k] - c[k];
      dm2 += e * e;
    }
    double reach = bound[o] + half_len;
    if (dm2 > reach * reach * (1.0 + 1e-12) + 1e-300) continue;
    int hit = kind[o] == 0 ? seg_hits_sphere(d, a, b, c, size[(int64_t)o * d])
                           : seg_hits_box(d, a, b, c, size + (int64_t)o * d);
    if (hit) return 1;
  }
  return 0;
}

/* 1 where point x is inside (or on) an obstacle. */
int rrg_point_blocked(int d, const double* x, int n_obs, const int32_t* kind, const double* centre,
                      const double* size) {
  for (int o = 0; o < n_obs; ++o) {
    const double* c = centre + (int64_t)o * d;
    const double* s = size + (int64_t)o * d;
    if (kind[o] == 0) {
      double d2 = 0.0;
      for (int k = 0; k < d; ++k) d2 += (x[k] - c[k]) * (x[k] - c[k]);
      if (d2 <= s[0] * s[0]) return 1;
    } else {
      int in = 1;
      for (int k = 0; k < d; ++k)
        if (fabs(x[k] - c[k]) > s[k]) in = 0;
      if (in) return 1;
    }
  }
  return 0;
}

static int cmp_pair(const void* pa, const void* pb) {
  int64_t a = *(const int64_t*)pa, b = *(const int64_t*)pb;
  return a < b ? -1 : (a > b ? 1 : 0);
}

/*
 * Builds the forward rows of vertices n_old .. n_old+n_new-1 over the points
 * pts[(n_old+n_new) x d] (all in [0,1]^d).  Returns 0, or -1 on bad arguments,
 * -2 on allocation failure.  The caller frees the result with rrg_free_rows.
 */
int rrg_build_rows(int d, int64_t n_old, int64_t n_new, const double* pts, double r, int n_obs,
                   const int32_t* kind, const double* centre, const double* size, int nthreads,
                   rrg_rows* out) {
  memset(out, 0, sizeof(*out));
  if (d < 1 || d > 16 || n_old < 0 || n_new < 0 || !(r > 0.0)) return -1;
  int64_t n = n_old + n_new;
  /* grid of m^d cells with side 1/m >= r */
  int64_t m = (int64_t)floor(1.0 / r);
  if (m < 1) m = 1;
  while (1) {
    double cells = pow((double)m, (double)d);
    if (cells <= (double)(1 << 24)) break;
    --m;
  }
  int64_t ncell = 1;
  for (int k = 0; k < d; ++k) ncell *= m;
  int64_t* cell_of = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t* cstart = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
  int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  double* spts = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * d);
  double* bound = (double*)malloc(sizeof(double) * (size_t)(n_obs > 0 ? n_obs : 1));
  int64_t* counts = (int64_t*)calloc((size_t)n_new + 1, sizeof(int64_t));
  if (!cell_of || !cstart || !order || !spts || !bound || !counts) {
    free(cell_of); free(cstart); free(order); free(spts); free(bound); free(counts);
    return -2;
  }
  for (int o = 0; o < n_obs; ++o) {
    const double* s = size + (int64_t)o * d;
    if (kind[o] == 0) {
      bound[o] = s[0];
    } else {
      double b2 = 0.0;
      for (int k = 0; k < d; ++k) b2 += s[k] * s[k];
      bound[o] = sqrt(b2);
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    int64_t id = 0;
    for (int k = d - 1; k >= 0; --k) {
      int64_t q = (int64_t)floor(pts[i * d + k] * (double)m);
      if (q < 0) q = 0;
      if (q >= m) q = m - 1;
      id = id * m + q;
    }
    cell_of[i] = id;
    cstart[id + 1]++;
  }
  for (int64_t c = 0; c < ncell; ++c) cstart[c + 1] += cstart[c];
  {
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)ncell);
    if (!fill) {
      free(cell_of); free(cstart); free(order); free(spts); free(bound); free(counts);
      return -2;
    }
    memcpy(fill, cstart, sizeof(int64_t) * (size_t)ncell);
    for (int64_t i = 0; i < n; ++i) order[fill[cell_of[i]]++] = i; /* ascending id per cell */
    free(fill);
  }
  for (int64_t j = 0; j < n; ++j)
    for (int k = 0; k < d; ++k) spts[j * d + k] = pts[order[j] * d + k];

  int64_t noff = 1;
  for (int k = 0; k < d; ++k) noff *= 3;
  const double r2 = r * r;
  /* Rows are produced block by block; each block owns a buffer of (u, cost). */
  const int64_t block = 512;
  int64_t nblocks = (n_new + block - 1) / block;
  int64_t** bcol = (int64_t**)calloc((size_t)(nblocks > 0 ? nblocks : 1), sizeof(int64_t*));
  float** bcost = (float**)calloc((size_t)(nblocks > 0 ? nblocks : 1), sizeof(float*));
  int failed = 0;
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
  {
    int64_t cap = 1024;
    int64_t* cand = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap);
    int64_t lcap = 4096;
    int64_t* lcol = (int64_t*)malloc(sizeof(int64_t) * (size_t)lcap);
    float* lcost = (float*)malloc(sizeof(float) * (size_t)lcap);
    if (!cand || !lcol || !lcost) failed = 1;
#pragma omp for schedule(dynamic, 1)
    for (int64_t b = 0; b < nblocks; ++b) {
      if (failed) continue;
      int64_t lnnz = 0;
      int64_t v_lo = n_old + b * block, v_hi = v_lo + block;
      if (v_hi > n) v_hi = n;
      for (int64_t v = v_lo; v < v_hi; ++v) {
        const double* xv = pts + v * d;
        int64_t cv[16];
        for (int k = 0; k < d; ++k) {
          int64_t q = (int64_t)floor(xv[k] * (double)m);
          if (q < 0) q = 0;
          if (q >= m) q = m - 1;
          cv[k] = q;
        }
        int64_t nc = 0;
        for (int64_t t = 0; t < noff; ++t) {
          int64_t tt = t, id = 0, mul = 1;
          int ok = 1;
          for (int k = 0; k < d; ++k) {
            int64_t q = cv[k] + (tt % 3) - 1;
            tt /= 3;
            if (q < 0 || q >= m) {
              ok = 0;
              break;
            }
            id += q * mul;
            mul *= m;
          }
          if (!ok) continue;
          for (int64_t j = cstart[id]; j < cstart[id + 1]; ++j) {
            int64_t u = order[j];
            if (u >= v) continue;
            const double* xu = spts + j * d;
            double d2 = 0.0;
            for (int k = 0; k < d; ++k) {
              double e = xu[k] - xv[k];
              d2 += e * e;
            }
            if (d2 <= r2 && d2 > 0.0) {
              if (nc == cap) {
                cap *= 2;
                int64_t* nb = (int64_t*)realloc(cand, sizeof(int64_t) * (size_t)cap);
                if (!nb) {
                  failed = 1;
                  break;
                }
                cand = nb;
              }
              cand[nc++] = u;
            }
          }
        }
        if (failed) break;
        qsort(cand, (size_t)nc, sizeof(int64_t), cmp_pair);
        int64_t kept = 0;
        for (int64_t i = 0; i < nc; ++i) {
          int64_t u = cand[i];
          const double* xu = pts + u * d;
          if (seg_blocked(d, xu, xv, n_obs, kind, centre, size, bound)) continue;
          double d2 = 0.0;
          for (int k = 0; k < d; ++k) {
            double e = xu[k] - xv[k];
            d2 += e * e;
          }
          if (lnnz == lcap) {
            lcap *= 2;
            int64_t* nb = (int64_t*)realloc(lcol, sizeof(int64_t) * (size_t)lcap);
            float* nf = (float*)realloc(lcost, sizeof(float) * (size_t)lcap);
            if (nb) lcol = nb;
            if (nf) lcost = nf;
            if (!nb || !nf) {
              failed = 1;
              break;
            }
          }
          lcol[lnnz] = u;
          lcost[lnnz] = (float)sqrt(d2);
          ++lnnz;
          ++kept;
        }
        counts[v - n_old] = kept;
      }
      if (!failed) {
        bcol[b] = (int64_t*)malloc(sizeof(int64_t) * (size_t)(lnnz > 0 ? lnnz : 1));
        bcost[b] = (float*)malloc(sizeof(float) * (size_t)(lnnz > 0 ? lnnz : 1));
        if (!bcol[b] || !bcost[b]) {
          failed = 1;
        } else {
          memcpy(bcol[b], lcol, sizeof(int64_t) * (size_t)lnnz);
          memcpy(bcost[b], lcost, sizeof(float) * (size_t)lnnz);
        }
      }
    }
    free(cand);
    free(lcol);
    free(lcost);
  }
  int rc = failed ? -2 : 0;
  if (!failed) {
    out->row_ptr = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_new + 1));
    if (!out->row_ptr) rc = -2;
  }
  if (rc == 0) {
    out->row_ptr[0] = 0;
    for (int64_t i = 0; i < n_new; ++i) out->row_ptr[i + 1] = out->row_ptr[i] + counts[i];
    out->nnz = out->row_ptr[n_new];
    out->col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(out->nnz > 0 ? out->nnz : 1));
    out->cost = (float*)malloc(sizeof(float) * (size_t)(out->nnz > 0 ? out->nnz : 1));
    if (!out->col || !out->cost) rc = -2;
  }
  if (rc == 0) {
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 4)
    for (int64_t b = 0; b < nblocks; ++b) {
      int64_t off = out->row_ptr[b * block];
      int64_t len = out->row_ptr[(b + 1) * block < n_new ? (b + 1) * block : n_new] - off;
      for (int64_t i = 0; i < len; ++i) {
        out->col[off + i] = (int32_t)bcol[b][i];
        out->cost[off + i] = bcost[b][i];
      }
    }
  }
  for (int64_t b = 0; b < nblocks; ++b) {
    free(bcol[b]);
    free(bcost[b]);
  }
  free(bcol); free(bcost);
  free(cell_of); free(cstart); free(order); free(spts); free(bound); free(counts);
  if (rc != 0) {
    free(out->row_ptr); free(out->col); free(out->cost);
    memset(out, 0, sizeof(*out));
  }
  return rc;
}

void rrg_free_rows(rrg_rows* r) {
  free(r->row_ptr);
  free(r->col);
  free(r->cost);
  memset(r, 0, sizeof(*r));
}
