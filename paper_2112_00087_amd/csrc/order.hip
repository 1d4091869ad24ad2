// Internal node numberings of the operator rows (host code).
//
// Reverse Cuthill-McKee: breadth-first search of the matrix graph from a
// pseudo-peripheral node (the George-Liu search: restart from a
// minimum-degree node of the last level while the number of levels grows),
// each node's unvisited neighbours taken in ascending degree, then the whole
// sequence reversed (Cuthill and McKee 1969; reversal by George 1971).
// Neighbours of one level then sit within about two level widths of each
// other, so an unstructured mesh gets the narrow band that a structured
// lexicographic numbering has by construction.
//
// Length sort (SELL-C-sigma, Kreutzer et al. 2014): within windows of sigma
// consecutive rows, rows are stably sorted by length, longest first.  The
// sliced-ELL storage pads each 64-row slice to its longest row; on a mesh
// whose rows range from 15 to 75 entries almost every slice of an
// unsorted numbering would be padded to the maximum.
#include <algorithm>
#include <numeric>

#include "ctx.h"

namespace {

struct Graph {
  const std::vector<int64_t>& ptr;
  const std::vector<int32_t>& col;
  int64_t deg(int64_t i) const { return ptr[i + 1] - ptr[i]; }
};

// Level structure of the component of s: nodes in breadth-first order
// (written to q), returns the number of levels and the start of the last.
int64_t levels(const Graph& g, int32_t s, std::vector<int32_t>& mark, int32_t stamp, std::vector<int32_t>& q,
               int64_t* last_begin, int64_t* size) {
  q.clear();
  q.push_back(s);
  mark[s] = stamp;
  int64_t head = 0, nlev = 0, lb = 0;
  while (head < int64_t(q.size())) {
    const int64_t end = int64_t(q.size());
    lb = head;
    ++nlev;
    for (; head < end; ++head) {
      const int32_t u = q[head];
      for (int64_t t = g.ptr[u]; t < g.ptr[u + 1]; ++t) {
        const int32_t v = g.col[t];
        if (mark[v] != stamp) {
          mark[v] = stamp;
          q.push_back(v);
        }
      }
    }
  }
  *last_begin = lb;
  *size = int64_t(q.size());
  return nlev;
}

int32_t pseudo_peripheral(const Graph& g, int32_t s, std::vector<int32_t>& mark, int32_t* stamp,
                          std::vector<int32_t>& q) {
  int64_t lb = 0, sz = 0;
  int64_t ecc = levels(g, s, mark, ++*stamp, q, &lb, &sz);
  for (int it = 0; it < 16; ++it) {
    int32_t x = q[lb];
    for (int64_t t = lb; t < sz; ++t)
      if (g.deg(q[t]) < g.deg(x) || (g.deg(q[t]) == g.deg(x) && q[t] < x)) x = q[t];
    const int64_t ex = levels(g, x, mark, ++*stamp, q, &lb, &sz);
    if (ex <= ecc) break;
    s = x;
    ecc = ex;
  }
  return s;
}

}  // namespace

void node_order(int64_t n, const std::vector<int64_t>& rowptr, const std::vector<int32_t>& col, int order,
                int sigma, std::vector<int32_t>* perm) {
  std::vector<int32_t>& P = *perm;
  P.resize(n);
  std::iota(P.begin(), P.end(), 0);
  const Graph g{rowptr, col};
  if (order == HZ_ORDER_RCM && n > 0) {
    // component starts: nodes by ascending degree (then id)
    std::vector<int32_t> by_deg(n);
    std::iota(by_deg.begin(), by_deg.end(), 0);
    std::stable_sort(by_deg.begin(), by_deg.end(), [&](int32_t a, int32_t b) { return g.deg(a) < g.deg(b); });
    std::vector<int32_t> mark(n, 0), q;
    std::vector<uint8_t> seen(n, 0);
    int32_t stamp = 0;
    int64_t filled = 0, next = 0;
    std::vector<int32_t> nb;
    while (filled < n) {
      while (seen[by_deg[next]]) ++next;
      const int32_t s = pseudo_peripheral(g, by_deg[next], mark, &stamp, q);
      // Cuthill-McKee sweep of this component, appended to P
      int64_t head = filled;
      P[filled++] = s;
      seen[s] = 1;
      while (head < filled) {
        const int32_t u = P[head++];
        nb.clear();
        for (int64_t t = rowptr[u]; t < rowptr[u + 1]; ++t) {
          const int32_t v = col[t];
          if (!seen[v]) {
            seen[v] = 1;
            nb.push_back(v);
          }
        }
        std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) {
          return g.deg(a) != g.deg(b) ? g.deg(a) < g.deg(b) : a < b;
        });
        for (int32_t v : nb) P[filled++] = v;
      }
    }
    std::reverse(P.begin(), P.end());
  }
  if (sigma > 0)
    for (int64_t w = 0; w < n; w += sigma) {
      auto b = P.begin() + w, e = P.begin() + std::min<int64_t>(n, w + sigma);
      std::stable_sort(b, e, [&](int32_t a, int32_t c) { return g.deg(a) > g.deg(c); });
    }
}
