// Replan on the host for small graphs (the adaptive choice of Sec. VII: below the
// size where a launch costs more than the work, one host thread finishes first).
//
// The same steps and the same arithmetic as the device loop, on host copies of the
// graph's slot-ordered arrays: Evaluate (every g the binary32 left fold of the
// parent-edge costs down its root path, breadth-first from the root; vertices it does
// not reach get +inf), the promising set fl(g + h) < G with G = g(goal) after the
// Evaluate (or +inf without pruning), the domain D = P u N(P) minus the root (with the
// narrowed domain a neighbour w of a promising u only for fl(fl(g(u) + c) + h(w)) < G),
// and a Jacobi Improve: for v in D the lexicographic minimum of (fl(g(u) + c), caller
// id of u, c) over v's row, a switch only below g(v).  The loop stops when nothing
// switched or at the iteration cap.  This file is compiled with -ffp-contract=off, so
// every addition is one binary32 addition rounded to nearest even.
#include <string.h>

#include <cmath>
#include <limits>
#include <vector>

#include "internal.h"

namespace pirrt {

namespace {

// g of every slot from the policy: children lists by a counting pass, then a FIFO
// walk from the root.
void host_evaluate(const HostReplan& p, std::vector<int32_t>& head, std::vector<int32_t>& kids,
                   std::vector<int32_t>& fifo) {
  const int32_t n = p.n;
  const float inf = std::numeric_limits<float>::infinity();
  head.assign((size_t)n + 1, 0);
  for (int32_t v = 0; v < n; ++v)
    if (v != p.root && p.parent[v] >= 0) ++head[(size_t)p.parent[v] + 1];
  for (int32_t v = 0; v < n; ++v) head[(size_t)v + 1] += head[(size_t)v];
  kids.resize((size_t)n);
  std::vector<int32_t> fill(head.begin(), head.end() - 1);
  for (int32_t v = 0; v < n; ++v)
    if (v != p.root && p.parent[v] >= 0) kids[(size_t)fill[(size_t)p.parent[v]]++] = v;
  for (int32_t v = 0; v < n; ++v) p.g[v] = inf;
  p.g[p.root] = 0.0f;
  fifo.resize((size_t)n);
  int32_t qh = 0, qt = 0;
  fifo[(size_t)qt++] = p.root;
  while (qh < qt) {
    const int32_t u = fifo[(size_t)qh++];
    for (int32_t k = head[(size_t)u]; k < head[(size_t)u + 1]; ++k) {
      const int32_t c = kids[(size_t)k];
      p.g[c] = p.g[u] + p.pcost[c];
      fifo[(size_t)qt++] = c;
    }
  }
}

}  // namespace

int host_replan(const HostReplan& p, HostReplanStats* st) {
  const int32_t n = p.n;
  const float inf = std::numeric_limits<float>::infinity();
  memset(st, 0, sizeof(*st));
  p.parent[p.root] = kRootMark;
  p.pcost[p.root] = 0.0f;
  std::vector<int32_t> head, kids, fifo, dom;
  std::vector<uint8_t> inP((size_t)n), inD((size_t)n);
  std::vector<int32_t> np((size_t)n);
  std::vector<float> nc((size_t)n);
  host_evaluate(p, head, kids, fifo);
  for (;;) {
    const float G = p.prune ? p.g[p.goal] : inf;
    int64_t sp = 0, sd = 0, ed = 0, pe = 0, ch = 0;
    std::fill(inD.begin(), inD.end(), (uint8_t)0);
    for (int32_t v = 0; v < n; ++v) {
      const float f = p.g[v] + (p.h ? p.h[v] : 0.0f);
      inP[(size_t)v] = f < G;
      sp += inP[(size_t)v];
    }
    for (int32_t u = 0; u < n; ++u) {
      if (!inP[(size_t)u]) continue;
      inD[(size_t)u] = 1;
      pe += p.rp[u + 1] - p.rp[u];
      for (int64_t j = p.rp[u]; j < p.rp[u + 1]; ++j) {
        const int32_t w = p.col[j];
        if (p.lookahead && !((p.g[u] + p.cst[j]) + (p.h ? p.h[w] : 0.0f) < G)) continue;
        inD[(size_t)w] = 1;
      }
    }
    inD[(size_t)p.root] = 0;
    dom.clear();
    for (int32_t v = 0; v < n; ++v)
      if (inD[(size_t)v]) dom.push_back(v);
    for (const int32_t v : dom) {  // Jacobi: every minimum reads the g of the last Evaluate
      ++sd;
      ed += p.rp[v + 1] - p.rp[v];
      float bm = inf;
      int32_t bu = -1, be = 0;
      float bc = 0.0f;
      for (int64_t j = p.rp[v]; j < p.rp[v + 1]; ++j) {
        const int32_t u = p.col[j];
        const float m = p.g[u] + p.cst[j];
        const int32_t e = p.ext[u];
        if (bu < 0 ? m < inf : (m < bm || (m == bm && (e < be || (e == be && p.cst[j] < bc))))) {
          bm = m;
          bu = u;
          be = e;
          bc = p.cst[j];
        }
      }
      np[(size_t)v] = -1;
      if (bu >= 0 && bm < p.g[v]) {
        np[(size_t)v] = bu;
        nc[(size_t)v] = bc;
        ++ch;
      }
    }
    st->iterations += 1;
    st->sum_P += sp;
    st->sum_D += sd;
    st->edges += ed;
    st->mark_edges += pe;
    st->changed += ch;
    if (ch == 0) return 0;
    for (const int32_t v : dom)
      if (np[(size_t)v] >= 0) {
        p.parent[v] = np[(size_t)v];
        p.pcost[v] = nc[(size_t)v];
      }
    host_evaluate(p, head, kids, fifo);
    if (st->iterations >= p.cap) return 1;
  }
}

}  // namespace pirrt
