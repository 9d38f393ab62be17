/*
 * Oracle for the exploration support of the planner (test infrastructure: only the
 * tests, the smoke check and the benchmark's CPU baseline use it).
 *
 * Plain serial definitions of what Extend needs to grow the random geometric graph
 * (Sec. III: sample a free state, connect it to every earlier vertex within the
 * connection radius whose straight segment is collision free, cache the edge
 * cost), written for checking, not speed:
 *
 *   philox4x32-10 : the counter-based generator of Salmon, Moraes, Dror and Shaw
 *                   (SC'11), 10 rounds, multipliers 0xD2511F53 / 0xCD9E8D57, key
 *                   increments 0x9E3779B9 / 0xBB67AE85.
 *   sampling      : candidate k of stream s under seed q is the point whose
 *                   coordinate i is (w_i >> 8) * 2^-24, w_0..w_3 = philox(counter
 *                   {lo(k), hi(k), s, 0}, key {lo(q), hi(q)}), w_4..w_7 the same
 *                   with counter word 3 = 1.  A candidate inside or on an obstacle
 *                   is rejected; free candidates are taken in order of k.
 *   obstacles     : closed sets.  Sphere: sum_k (x_k - c_k)^2 <= R^2.  Box: every
 *                   |x_k - c_k| <= s_k.
 *   edge u-v      : u < v, d2 = sum over axes in order of (x_u - x_v)^2 in binary64,
 *                   0 < d2 <= r*r, and the closed segment from x_u to x_v meets no
 *                   obstacle.  Sphere: the segment point closest to c (parameter
 *                   t = ((c - x_u).e) / (e.e), e = x_v - x_u, clamped to [0, 1])
 *                   lies within R.  Box: the slab intersection of the parameter
 *                   intervals over all axes is not empty.  Cost = binary32 rounding
 *                   of sqrt(d2).
 *   heuristic     : h(v) = binary32 rounding of the binary64 Euclidean distance to
 *                   the goal.
 *
 * Every neighbour search here is brute force over all earlier vertices; no grid,
 * no pre-rejection.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* One Philox4x32 round function application, 10 rounds. */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n1 = lo1;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    const uint32_t n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* Candidate k as a point (d <= 8). */
void orc_candidate(int d, uint64_t seed, uint32_t stream, uint64_t k, double* x) {
  uint32_t w[8];
  for (int half = 0; half < 2 && 4 * half < d; ++half) {
    const uint32_t ctr[4] = {(uint32_t)k, (uint32_t)(k >> 32), stream, (uint32_t)half};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, w + 4 * half);
  }
  for (int i = 0; i < d; ++i) x[i] = (double)(w[i] >> 8) * (1.0 / 16777216.0);
}

int orc_point_blocked(int d, const double* x, int n_obs, const int32_t* kind, const double* centre,
                      const double* size) {
  for (int o = 0; o < n_obs; ++o) {
    const double* c = centre + (int64_t)o * d;
    const double* s = size + (int64_t)o * d;
    if (kind[o] == 0) {
      double d2 = 0.0;
      for (int k = 0; k < d; ++k) {
        const double e = x[k] - c[k];
        d2 += e * e;
      }
      if (d2 <= s[0] * s[0]) return 1;
    } else {
      int inside = 1;
      for (int k = 0; k < d; ++k)
        if (fabs(x[k] - c[k]) > s[k]) inside = 0;
      if (inside) return 1;
    }
  }
  return 0;
}

/* Appends `count` free samples to pts (row-major, d per point) from candidate
   *counter on; *counter ends one past the last candidate taken.  Gives up (returns
   -1) after max_candidates candidates. */
int orc_sample(int d, uint64_t seed, uint32_t stream, uint64_t* counter, int64_t count, int n_obs,
               const int32_t* kind, const double* centre, const double* size, int64_t max_candidates,
               double* pts) {
  if (d < 1 || d > 8 || count < 0) return -1;
  uint64_t k = *counter;
  int64_t got = 0;
  for (int64_t tried = 0; got < count; ++tried, ++k) {
    if (tried >= max_candidates) return -1;
    double x[8];
    orc_candidate(d, seed, stream, k, x);
    if (orc_point_blocked(d, x, n_obs, kind, centre, size)) continue;
    memcpy(pts + got * d, x, sizeof(double) * (size_t)d);
    ++got;
  }
  *counter = k;
  return 0;
}

static int hits_sphere(int d, const double* a, const double* b, const double* c, double rad) {
  double ee = 0.0, ce = 0.0;
  for (int k = 0; k < d; ++k) {
    const double e = b[k] - a[k];
    ee += e * e;
    ce += (c[k] - a[k]) * e;
  }
  double t = ee > 0.0 ? ce / ee : 0.0;
  if (t < 0.0) t = 0.0;
  if (t > 1.0) t = 1.0;
  double q2 = 0.0;
  for (int k = 0; k < d; ++k) {
    const double q = a[k] + t * (b[k] - a[k]) - c[k];
    q2 += q * q;
  }
  return q2 <= rad * rad;
}

static int hits_box(int d, const double* a, const double* b, const double* c, const double* half) {
  double lo_t = 0.0, hi_t = 1.0;
  for (int k = 0; k < d; ++k) {
    const double lo = c[k] - half[k], hi = c[k] + half[k];
    const double e = b[k] - a[k];
    if (e == 0.0) {
      if (a[k] < lo || a[k] > hi) return 0;
      continue;
    }
    double t_lo = (lo - a[k]) / e, t_hi = (hi - a[k]) / e;
    if (t_lo > t_hi) {
      const double s = t_lo;
      t_lo = t_hi;
      t_hi = s;
    }
    if (t_lo > lo_t) lo_t = t_lo;
    if (t_hi < hi_t) hi_t = t_hi;
    if (lo_t > hi_t) return 0;
  }
  return 1;
}

int orc_segment_blocked(int d, const double* a, const double* b, int n_obs, const int32_t* kind,
                        const double* centre, const double* size) {
  for (int o = 0; o < n_obs; ++o) {
    const double* c = centre + (int64_t)o * d;
    const double* s = size + (int64_t)o * d;
    if (kind[o] == 0 ? hits_sphere(d, a, b, c, s[0]) : hits_box(d, a, b, c, s)) return 1;
  }
  return 0;
}

/*
 * Forward rows of vertices n_old .. n-1 over pts[n x d]: row v lists every u < v
 * joined to v by an edge, ascending, with its cost.  row_ptr has n - n_old + 1
 * entries; col / cost have room for cap entries.  Returns the entry count, or -1
 * if cap is too small.
 */
int64_t orc_build_rows(int d, int64_t n_old, int64_t n, const double* pts, double r, int n_obs,
                       const int32_t* kind, const double* centre, const double* size, int64_t* row_ptr,
                       int32_t* col, float* cost, int64_t cap) {
  const double r2 = r * r;
  int64_t m = 0;
  row_ptr[0] = 0;
  for (int64_t v = n_old; v < n; ++v) {
    const double* xv = pts + v * d;
    for (int64_t u = 0; u < v; ++u) {
      const double* xu = pts + u * d;
      double d2 = 0.0;
      for (int k = 0; k < d; ++k) {
        const double e = xu[k] - xv[k];
        d2 += e * e;
      }
      if (!(d2 <= r2 && d2 > 0.0)) continue;
      if (orc_segment_blocked(d, xu, xv, n_obs, kind, centre, size)) continue;
      if (m >= cap) return -1;
      col[m] = (int32_t)u;
      cost[m] = (float)sqrt(d2);
      ++m;
    }
    row_ptr[v - n_old + 1] = m;
  }
  return m;
}

void orc_heuristic(int d, int64_t n, const double* pts, const double* goal, float* h) {
  for (int64_t v = 0; v < n; ++v) {
    double d2 = 0.0;
    for (int k = 0; k < d; ++k) {
      const double e = pts[v * d + k] - goal[k];
      d2 += e * e;
    }
    h[v] = (float)sqrt(d2);
  }
}
