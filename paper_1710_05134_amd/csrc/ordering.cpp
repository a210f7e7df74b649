// Fill-reducing order Q for the shared pattern of A and B (Section 3.3 uses a
// nested-dissection order for the sparse direct solver).  Written for the
// pencils of electronic-structure calculations, where the orbitals of one atom
// have identical rows:
//   1. supervariable compression (rows with identical pattern -> one vertex);
//   2. recursive bisection of the compressed graph, each cut found by a
//      multilevel scheme: heavy-edge matching coarsening, greedy growing on the
//      coarsest graph, Fiduccia-Mattheyses refinement while projecting back;
//      the cut edges' minimum vertex cover (Konig) is the vertex separator,
//      thinned by greedy vertex moves; parts are ordered before their separator;
//   3. disconnected pieces are ordered independently; small pieces keep their
//      order.
#include <algorithm>
#include <cstdio>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "analysis.hpp"

namespace kth {

std::string check_pattern(const Pattern& p, bool check_symmetry) {
  if (p.n <= 0) return "n must be positive";
  if (!p.rowptr || !p.col) return "null pattern pointer";
  if (p.rowptr[0] != 0) return "rowptr[0] must be 0";
  for (int64_t i = 0; i < p.n; i++) {
    if (p.rowptr[i + 1] < p.rowptr[i]) return "rowptr is not non-decreasing";
    bool diag = false;
    for (int64_t q = p.rowptr[i]; q < p.rowptr[i + 1]; q++) {
      int64_t c = p.col[q];
      if (c < 0 || c >= p.n) return "column index out of range in row " + std::to_string(i);
      if (q > p.rowptr[i] && p.col[q - 1] >= c)
        return "columns not strictly increasing in row " + std::to_string(i);
      if (c == i) diag = true;
    }
    if (!diag) return "missing diagonal entry in row " + std::to_string(i);
  }
  if (check_symmetry) {
    for (int64_t i = 0; i < p.n; i++)
      for (int64_t q = p.rowptr[i]; q < p.rowptr[i + 1]; q++) {
        int64_t c = p.col[q];
        const int32_t* b = p.col + p.rowptr[c];
        const int32_t* e = p.col + p.rowptr[c + 1];
        if (!std::binary_search(b, e, (int32_t)i))
          return "pattern is not symmetric at (" + std::to_string(i) + "," + std::to_string(c) + ")";
      }
  }
  return "";
}

namespace {

struct Graph {
  int64_t n = 0;
  std::vector<int64_t> xadj;
  std::vector<int32_t> adj;
  std::vector<int64_t> w;  // vertex weights (supervariable sizes)
};

// Group rows with identical patterns (each row's pattern contains the row).
static void compress(const Pattern& p, Graph& g, std::vector<int32_t>& sv_of,
                     std::vector<int64_t>& sv_ptr, std::vector<int32_t>& sv_rows) {
  const int64_t n = p.n;
  std::vector<uint64_t> h(n);
  for (int64_t i = 0; i < n; i++) {
    uint64_t x = 1469598103934665603ull ^ (uint64_t)(p.rowptr[i + 1] - p.rowptr[i]);
    for (int64_t q = p.rowptr[i]; q < p.rowptr[i + 1]; q++) {
      x ^= (uint64_t)p.col[q] + 0x9e3779b97f4a7c15ull;
      x *= 1099511628211ull;
    }
    h[i] = x;
  }
  std::vector<int64_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
    return h[a] != h[b] ? h[a] < h[b] : a < b;
  });
  sv_of.assign(n, -1);
  std::vector<int64_t> rep;  // representative row of each supervariable
  auto same = [&](int64_t a, int64_t b) {
    int64_t la = p.rowptr[a + 1] - p.rowptr[a], lb = p.rowptr[b + 1] - p.rowptr[b];
    if (la != lb) return false;
    return std::memcmp(p.col + p.rowptr[a], p.col + p.rowptr[b], sizeof(int32_t) * la) == 0;
  };
  for (int64_t s = 0; s < n;) {
    int64_t e = s;
    while (e < n && h[idx[e]] == h[idx[s]]) e++;
    for (int64_t q = s; q < e; q++) {
      int64_t r = idx[q];
      if (sv_of[r] != -1) continue;
      int32_t id = (int32_t)rep.size();
      rep.push_back(r);
      sv_of[r] = id;
      for (int64_t t = q + 1; t < e; t++)
        if (sv_of[idx[t]] == -1 && same(r, idx[t])) sv_of[idx[t]] = id;
    }
    s = e;
  }
  // renumber supervariables in order of their smallest member (deterministic, local)
  const int64_t m = (int64_t)rep.size();
  std::vector<int32_t> first(m, -1), ren(m);
  int32_t cnt = 0;
  for (int64_t i = 0; i < n; i++)
    if (first[sv_of[i]] == -1) { first[sv_of[i]] = (int32_t)i; ren[sv_of[i]] = cnt++; }
  for (int64_t i = 0; i < n; i++) sv_of[i] = ren[sv_of[i]];
  sv_ptr.assign(m + 1, 0);
  for (int64_t i = 0; i < n; i++) sv_ptr[sv_of[i] + 1]++;
  for (int64_t s = 0; s < m; s++) sv_ptr[s + 1] += sv_ptr[s];
  sv_rows.assign(n, 0);
  std::vector<int64_t> fill(sv_ptr.begin(), sv_ptr.end() - 1);
  for (int64_t i = 0; i < n; i++) sv_rows[fill[sv_of[i]]++] = (int32_t)i;
  g.n = m;
  g.w.assign(m, 0);
  g.xadj.assign(m + 1, 0);
  std::vector<int32_t> mark(m, -1);
  std::vector<int32_t> tmp;
  g.adj.clear();
  for (int64_t s = 0; s < m; s++) {
    g.w[s] = sv_ptr[s + 1] - sv_ptr[s];
    int64_t r = sv_rows[sv_ptr[s]];
    mark[s] = (int32_t)s;
    for (int64_t q = p.rowptr[r]; q < p.rowptr[r + 1]; q++) {
      int32_t t = sv_of[p.col[q]];
      if (mark[t] != (int32_t)s) { mark[t] = (int32_t)s; g.adj.push_back(t); }
    }
    std::sort(g.adj.begin() + g.xadj[s], g.adj.end());
    g.xadj[s + 1] = (int64_t)g.adj.size();
  }
}

// ---------------------------------------------------------------------------
// Multilevel edge bisection (heavy-edge matching, greedy growing, FM refinement)
// ---------------------------------------------------------------------------
struct WGraph {
  int32_t n = 0;
  std::vector<int64_t> xadj;
  std::vector<int32_t> adj;
  std::vector<int32_t> ew;   // edge weights
  std::vector<int64_t> vw;   // vertex weights
  int64_t total() const { int64_t t = 0; for (int64_t x : vw) t += x; return t; }
};

struct Rng {
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed * 2654435761ull + 88172645463325252ull) {}
  uint64_t next() { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; }
};

static void coarsen(const WGraph& g, WGraph& c, std::vector<int32_t>& cmap, Rng& rng) {
  std::vector<int32_t> order(g.n), match(g.n, -1);
  std::iota(order.begin(), order.end(), 0);
  for (int32_t i = g.n - 1; i > 0; i--) std::swap(order[i], order[(int32_t)(rng.next() % (uint64_t)(i + 1))]);
  for (int32_t v : order) {
    if (match[v] != -1) continue;
    int32_t best = -1, bw = -1;
    for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; e++) {
      int32_t u = g.adj[e];
      if (match[u] == -1 && u != v && g.ew[e] > bw) { bw = g.ew[e]; best = u; }
    }
    if (best == -1) match[v] = v;
    else { match[v] = best; match[best] = v; }
  }
  cmap.assign(g.n, -1);
  int32_t nc = 0;
  for (int32_t v = 0; v < g.n; v++) {
    if (cmap[v] != -1) continue;
    cmap[v] = nc;
    if (match[v] != v) cmap[match[v]] = nc;
    nc++;
  }
  c = WGraph();
  c.n = nc;
  c.vw.assign(nc, 0);
  for (int32_t v = 0; v < g.n; v++) c.vw[cmap[v]] += g.vw[v];
  std::vector<int32_t> members(g.n), mptr(nc + 1, 0);
  for (int32_t v = 0; v < g.n; v++) mptr[cmap[v] + 1]++;
  for (int32_t i = 0; i < nc; i++) mptr[i + 1] += mptr[i];
  {
    std::vector<int32_t> f(mptr.begin(), mptr.end() - 1);
    for (int32_t v = 0; v < g.n; v++) members[f[cmap[v]]++] = v;
  }
  std::vector<int32_t> slot(nc, -1);
  c.xadj.assign(nc + 1, 0);
  for (int32_t cv = 0; cv < nc; cv++) {
    int64_t start = (int64_t)c.adj.size();
    for (int32_t q = mptr[cv]; q < mptr[cv + 1]; q++) {
      int32_t v = members[q];
      for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; e++) {
        int32_t cu = cmap[g.adj[e]];
        if (cu == cv) continue;
        if (slot[cu] == -1) {
          slot[cu] = (int32_t)c.adj.size();
          c.adj.push_back(cu);
          c.ew.push_back(g.ew[e]);
        } else {
          c.ew[slot[cu]] += g.ew[e];
        }
      }
    }
    for (int64_t e = start; e < (int64_t)c.adj.size(); e++) slot[c.adj[e]] = -1;
    c.xadj[cv + 1] = (int64_t)c.adj.size();
  }
}

static int64_t edge_cut(const WGraph& g, const std::vector<int8_t>& part) {
  int64_t cut = 0;
  for (int32_t v = 0; v < g.n; v++)
    for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; e++)
      if (part[g.adj[e]] != part[v]) cut += g.ew[e];
  return cut / 2;
}

// Two-way Fiduccia-Mattheyses passes with rollback to the best prefix.
static void fm_refine(const WGraph& g, std::vector<int8_t>& part, double eps, int passes) {
  const int64_t tot = g.total();
  const int64_t maxw = (int64_t)((0.5 + eps) * (double)tot) + 1;
  std::vector<int64_t> gain(g.n);
  std::vector<int8_t> locked(g.n);
  std::vector<int32_t> ver(g.n, 0);
  for (int pass = 0; pass < passes; pass++) {
    int64_t W[2] = {0, 0};
    for (int32_t v = 0; v < g.n; v++) W[part[v]] += g.vw[v];
    std::vector<std::pair<int64_t, int64_t>> heap[2];   // (gain, v | version << 32)
    auto push = [&](int32_t v) {
      heap[part[v]].push_back({gain[v], (int64_t)v | ((int64_t)ver[v] << 32)});
      std::push_heap(heap[part[v]].begin(), heap[part[v]].end());
    };
    for (int32_t v = 0; v < g.n; v++) {
      int64_t ext = 0, in = 0;
      bool bnd = false;
      for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; e++) {
        if (part[g.adj[e]] != part[v]) { ext += g.ew[e]; bnd = true; } else in += g.ew[e];
      }
      gain[v] = ext - in;
      locked[v] = 0;
      ver[v]++;
      if (bnd) push(v);
    }
    int64_t cut = edge_cut(g, part);
    int64_t best_cut = cut, best_imb = std::llabs(W[0] - W[1]);
    std::vector<int32_t> moves;
    size_t best_len = 0;
    int since = 0;
    const int limit = std::max<int>(50, g.n / 50);
    while (since < limit) {
      int side = -1;
      int32_t pick[2] = {-1, -1};
      for (int s = 0; s < 2; s++) {
        auto& h = heap[s];
        while (!h.empty()) {
          int32_t v = (int32_t)(h.front().second & 0xffffffff);
          int32_t vv = (int32_t)(h.front().second >> 32);
          if (locked[v] || vv != ver[v] || part[v] != s) { std::pop_heap(h.begin(), h.end()); h.pop_back(); continue; }
          pick[s] = v;
          break;
        }
      }
      // candidate sides allowed by balance
      int64_t bg = INT64_MIN;
      for (int s = 0; s < 2; s++) {
        if (pick[s] < 0) continue;
        if (W[1 - s] + g.vw[pick[s]] > maxw) continue;
        int64_t gv = gain[pick[s]];
        if (gv > bg || (gv == bg && W[s] > W[1 - s])) { bg = gv; side = s; }
      }
      if (side < 0) break;
      int32_t v = pick[side];
      std::pop_heap(heap[side].begin(), heap[side].end());
      heap[side].pop_back();
      part[v] = (int8_t)(1 - side);
      W[side] -= g.vw[v];
      W[1 - side] += g.vw[v];
      cut -= gain[v];
      locked[v] = 1;
      moves.push_back(v);
      gain[v] = -gain[v];
      for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; e++) {
        int32_t u = g.adj[e];
        if (locked[u]) continue;
        gain[u] += (part[u] == part[v]) ? -2 * g.ew[e] : 2 * g.ew[e];
        ver[u]++;
        push(u);
      }
      int64_t imb = std::llabs(W[0] - W[1]);
      if (cut < best_cut || (cut == best_cut && imb < best_imb)) {
        best_cut = cut; best_imb = imb; best_len = moves.size(); since = 0;
      } else {
        since++;
      }
    }
    for (size_t q = moves.size(); q > best_len; q--) part[moves[q - 1]] ^= 1;
    if (best_len == 0) break;
  }
}

// Greedy graph growing from a seed vertex (breadth first) to half the weight.
static void grow(const WGraph& g, int32_t seed, std::vector<int8_t>& part) {
  const int64_t half = g.total() / 2;
  part.assign(g.n, 1);
  std::vector<int32_t> q;
  q.reserve(g.n);
  q.push_back(seed);
  part[seed] = 0;
  int64_t w = g.vw[seed];
  size_t h = 0;
  while (w < half) {
    if (h == q.size()) {   // disconnected: take any remaining vertex
      int32_t v = -1;
      for (int32_t u = 0; u < g.n; u++) if (part[u] == 1) { v = u; break; }
      if (v < 0) break;
      part[v] = 0; w += g.vw[v]; q.push_back(v);
      continue;
    }
    int32_t v = q[h++];
    for (int64_t e = g.xadj[v]; e < g.xadj[v + 1] && w < half; e++) {
      int32_t u = g.adj[e];
      if (part[u] == 1) { part[u] = 0; w += g.vw[u]; q.push_back(u); }
    }
  }
}

static void multilevel_bisect(const WGraph& g0, std::vector<int8_t>& part, uint64_t seed) {
  Rng rng(seed);
  std::vector<WGraph> G;
  std::vector<std::vector<int32_t>> maps;
  G.push_back(g0);
  while (G.back().n > 160) {
    WGraph c;
    std::vector<int32_t> cm;
    coarsen(G.back(), c, cm, rng);
    if (c.n > (int32_t)(0.92 * G.back().n)) break;
    maps.push_back(std::move(cm));
    G.push_back(std::move(c));
  }
  const WGraph& gc = G.back();
  std::vector<int8_t> best, trial;
  int64_t best_cut = INT64_MAX;
  for (int t = 0; t < 10; t++) {
    int32_t s = (int32_t)(rng.next() % (uint64_t)gc.n);
    grow(gc, s, trial);
    fm_refine(gc, trial, 0.03, 8);
    int64_t c = edge_cut(gc, trial);
    if (c < best_cut) { best_cut = c; best = trial; }
  }
  part = best;
  for (int64_t l = (int64_t)maps.size() - 1; l >= 0; l--) {
    const WGraph& fine = G[l];
    std::vector<int8_t> fp(fine.n);
    for (int32_t v = 0; v < fine.n; v++) fp[v] = part[maps[l][v]];
    part.swap(fp);
    fm_refine(fine, part, 0.03, 6);
  }
}

// Minimum vertex cover of the cut edges (Konig: from a maximum matching of the
// bipartite boundary graph): an optimal vertex separator for the edge cut.
static void cover_separator(const WGraph& g, std::vector<int8_t>& part) {
  std::vector<int32_t> L, R, lid(g.n, -1), rid(g.n, -1);
  for (int32_t v = 0; v < g.n; v++) {
    bool b = false;
    for (int64_t e = g.xadj[v]; e < g.xadj[v + 1] && !b; e++) if (part[g.adj[e]] != part[v]) b = true;
    if (!b) continue;
    if (part[v] == 0) { lid[v] = (int32_t)L.size(); L.push_back(v); }
    else { rid[v] = (int32_t)R.size(); R.push_back(v); }
  }
  std::vector<int32_t> mL(L.size(), -1), mR(R.size(), -1), seen(R.size(), -1);
  // greedy start
  for (size_t i = 0; i < L.size(); i++) {
    int32_t v = L[i];
    for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; e++) {
      int32_t u = g.adj[e];
      if (part[u] == 1 && mR[rid[u]] == -1) { mL[i] = rid[u]; mR[rid[u]] = (int32_t)i; break; }
    }
  }
  // augmenting paths (iterative DFS)
  std::vector<std::pair<int32_t, int64_t>> st;
  for (size_t i0 = 0; i0 < L.size(); i0++) {
    if (mL[i0] != -1) continue;
    st.clear();
    st.push_back({(int32_t)i0, g.xadj[L[i0]]});
    bool found = false;
    std::vector<int32_t> path_r;
    while (!st.empty() && !found) {
      auto& top = st.back();
      int32_t li = top.first;
      int32_t v = L[li];
      if (top.second >= g.xadj[v + 1]) { st.pop_back(); if (!path_r.empty()) path_r.pop_back(); continue; }
      int32_t u = g.adj[top.second++];
      if (part[u] != 1) continue;
      int32_t ri = rid[u];
      if (seen[ri] == (int32_t)i0) continue;
      seen[ri] = (int32_t)i0;
      if (mR[ri] == -1) {
        // augment along the stack
        path_r.push_back(ri);
        for (size_t d = 0; d < st.size(); d++) {
          int32_t l = st[d].first, r = path_r[d];
          mL[l] = r; mR[r] = l;
        }
        found = true;
      } else {
        path_r.push_back(ri);
        st.push_back({mR[ri], g.xadj[L[mR[ri]]]});
      }
    }
  }
  // Konig: Z = vertices reachable from unmatched left vertices by alternating paths
  std::vector<int8_t> zL(L.size(), 0), zR(R.size(), 0);
  std::vector<int32_t> q;
  for (size_t i = 0; i < L.size(); i++) if (mL[i] == -1) { zL[i] = 1; q.push_back((int32_t)i); }
  for (size_t h = 0; h < q.size(); h++) {
    int32_t v = L[q[h]];
    for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; e++) {
      int32_t u = g.adj[e];
      if (part[u] != 1) continue;
      int32_t ri = rid[u];
      if (zR[ri]) continue;
      zR[ri] = 1;
      int32_t l = mR[ri];
      if (l != -1 && !zL[l]) { zL[l] = 1; q.push_back(l); }
    }
  }
  for (size_t i = 0; i < L.size(); i++) if (!zL[i]) part[L[i]] = 2;
  for (size_t i = 0; i < R.size(); i++) if (zR[i]) part[R[i]] = 2;
}

// Vertex-separator Fiduccia-Mattheyses: a separator vertex moves to side s and
// its neighbours on the other side join the separator; gain = its weight minus
// the weight pulled in.  Negative moves are allowed within a pass, which is
// rolled back to its lightest separator.
static void node_fm(const WGraph& g, std::vector<int8_t>& part, double eps, int passes) {
  const int64_t tot = g.total();
  const int64_t maxw = (int64_t)((0.5 + eps) * (double)tot) + 1;
  std::vector<int32_t> ver(g.n, 0);
  std::vector<int8_t> locked(g.n, 0);
  auto gain_to = [&](int32_t v, int s) {
    int64_t pulled = 0;
    for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; e++) {
      int32_t u = g.adj[e];
      if (part[u] == 1 - s) pulled += g.vw[u];
    }
    return g.vw[v] - pulled;
  };
  for (int pass = 0; pass < passes; pass++) {
    int64_t W[3] = {0, 0, 0};
    for (int32_t v = 0; v < g.n; v++) W[part[v]] += g.vw[v];
    std::vector<std::pair<int64_t, int64_t>> heap[2];
    auto push = [&](int32_t v) {
      ver[v]++;
      for (int s = 0; s < 2; s++) {
        heap[s].push_back({gain_to(v, s), (int64_t)v | ((int64_t)ver[v] << 32)});
        std::push_heap(heap[s].begin(), heap[s].end());
      }
    };
    for (int32_t v = 0; v < g.n; v++) { locked[v] = 0; if (part[v] == 2) push(v); }
    struct Move { int32_t v; int8_t side; int32_t first, count; };
    std::vector<Move> moves;
    std::vector<int32_t> pulled_log;
    int64_t best_sep = W[2], best_imb = std::llabs(W[0] - W[1]);
    size_t best_len = 0;
    int since = 0;
    const int limit = std::max<int>(100, g.n / 100);
    while (since < limit) {
      int32_t pick[2] = {-1, -1};
      int64_t pg[2] = {INT64_MIN, INT64_MIN};
      for (int s = 0; s < 2; s++) {
        auto& h = heap[s];
        while (!h.empty()) {
          int32_t v = (int32_t)(h.front().second & 0xffffffff);
          int32_t vv = (int32_t)(h.front().second >> 32);
          if (locked[v] || vv != ver[v] || part[v] != 2) { std::pop_heap(h.begin(), h.end()); h.pop_back(); continue; }
          pick[s] = v; pg[s] = h.front().first;
          break;
        }
      }
      int side = -1;
      int64_t bg = INT64_MIN;
      for (int s = 0; s < 2; s++) {
        if (pick[s] < 0) continue;
        if (W[s] + g.vw[pick[s]] > maxw) continue;
        if (pg[s] > bg || (pg[s] == bg && W[s] < W[1 - s])) { bg = pg[s]; side = s; }
      }
      if (side < 0) break;
      int32_t v = pick[side];
      std::pop_heap(heap[side].begin(), heap[side].end());
      heap[side].pop_back();
      Move mv{v, (int8_t)side, (int32_t)pulled_log.size(), 0};
      part[v] = (int8_t)side;
      W[2] -= g.vw[v];
      W[side] += g.vw[v];
      locked[v] = 1;
      std::vector<int32_t> touched;
      for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; e++) {
        int32_t u = g.adj[e];
        if (part[u] == 1 - side) {
          part[u] = 2;
          W[1 - side] -= g.vw[u];
          W[2] += g.vw[u];
          pulled_log.push_back(u);
          mv.count++;
          touched.push_back(u);
        } else if (part[u] == 2) {
          touched.push_back(u);
        }
      }
      // separator neighbours of pulled vertices change their gains as well
      size_t nt = touched.size();
      for (size_t q = 0; q < nt; q++) {
        int32_t u = touched[q];
        if (part[u] != 2) continue;
        for (int64_t e = g.xadj[u]; e < g.xadj[u + 1]; e++)
          if (part[g.adj[e]] == 2) touched.push_back(g.adj[e]);
      }
      std::sort(touched.begin(), touched.end());
      touched.erase(std::unique(touched.begin(), touched.end()), touched.end());
      for (int32_t u : touched) if (!locked[u] && part[u] == 2) push(u);
      moves.push_back(mv);
      int64_t imb = std::llabs(W[0] - W[1]);
      if (W[2] < best_sep || (W[2] == best_sep && imb < best_imb)) {
        best_sep = W[2]; best_imb = imb; best_len = moves.size(); since = 0;
      } else {
        since++;
      }
    }
    for (size_t q = moves.size(); q > best_len; q--) {
      const Move& mv = moves[q - 1];
      for (int32_t t = mv.count - 1; t >= 0; t--) part[pulled_log[mv.first + t]] = (int8_t)(1 - mv.side);
      part[mv.v] = 2;
    }
    if (best_len == 0) break;
  }
}

// Multilevel vertex separator: coarsen, bisect the coarsest graph (edge FM,
// vertex cover; halves within 5% of balance), then project the three-way
// partition back level by level with vertex FM at each level. The projected
// refinement may unbalance the halves up to 15%: on the 3-D lattice pencils a
// smaller separator outweighs the uneven halves (about 25% fewer factor flops
// than with a 5% limit).
static void multilevel_separator(const WGraph& g0, std::vector<int8_t>& part, uint64_t seed) {
  Rng rng(seed);
  std::vector<WGraph> G;
  std::vector<std::vector<int32_t>> maps;
  G.push_back(g0);
  while (G.back().n > 200) {
    WGraph c;
    std::vector<int32_t> cm;
    coarsen(G.back(), c, cm, rng);
    if (c.n > (int32_t)(0.92 * G.back().n)) break;
    maps.push_back(std::move(cm));
    G.push_back(std::move(c));
  }
  const WGraph& gc = G.back();
  std::vector<int8_t> best, trial;
  int64_t best_sep = INT64_MAX;
  for (int t = 0; t < 8; t++) {
    int32_t s = (int32_t)(rng.next() % (uint64_t)gc.n);
    grow(gc, s, trial);
    fm_refine(gc, trial, 0.05, 8);
    cover_separator(gc, trial);
    node_fm(gc, trial, 0.05, 6);
    int64_t w2 = 0;
    for (int32_t v = 0; v < gc.n; v++) if (trial[v] == 2) w2 += gc.vw[v];
    if (w2 < best_sep) { best_sep = w2; best = trial; }
  }
  part = best;
  for (int64_t l = (int64_t)maps.size() - 1; l >= 0; l--) {
    const WGraph& fine = G[l];
    std::vector<int8_t> fp(fine.n);
    for (int32_t v = 0; v < fine.n; v++) fp[v] = part[maps[l][v]];
    part.swap(fp);
    node_fm(fine, part, 0.15, 4);
  }
}

struct ND {
  const Graph& g;
  int64_t leaf;
  std::vector<int32_t> stamp;   // membership stamp of the current vertex set
  std::vector<int32_t> local;   // global -> local index in the current set
  std::vector<int32_t> d1;
  std::vector<int32_t> queue;
  std::vector<int32_t> out;
  int32_t cur = 0;
  uint64_t calls = 0;

  explicit ND(const Graph& gg, int64_t lf)
      : g(gg), leaf(lf), stamp(gg.n, 0), local(gg.n, -1), d1(gg.n, -1), queue(gg.n) {}

  int64_t bfs(int32_t src, const std::vector<int32_t>& V) {
    for (int32_t v : V) d1[v] = -1;
    int64_t qh = 0, qt = 0;
    queue[qt++] = src;
    d1[src] = 0;
    while (qh < qt) {
      int32_t v = queue[qh++];
      for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; e++) {
        int32_t u = g.adj[e];
        if (stamp[u] != cur || d1[u] != -1) continue;
        d1[u] = d1[v] + 1;
        queue[qt++] = u;
      }
    }
    return qt;
  }

  void run(std::vector<int32_t> V) {
    if ((int64_t)V.size() <= leaf) {
      out.insert(out.end(), V.begin(), V.end());
      return;
    }
    ++cur;
    for (int32_t v : V) stamp[v] = cur;
    if (bfs(V[0], V) < (int64_t)V.size()) {
      // split into connected pieces and order each on its own
      std::vector<std::vector<int32_t>> comps;
      std::vector<int32_t> pending(V);
      while (!pending.empty()) {
        bfs(pending[0], pending);
        std::vector<int32_t> comp, rest;
        for (int32_t v : pending) (d1[v] >= 0 ? comp : rest).push_back(v);
        for (int32_t v : comp) stamp[v] = 0;   // drop from the current set
        comps.push_back(std::move(comp));
        pending.swap(rest);
      }
      for (auto& c : comps) run(std::move(c));
      return;
    }
    // local weighted graph of V
    WGraph w;
    w.n = (int32_t)V.size();
    for (int32_t i = 0; i < w.n; i++) local[V[i]] = i;
    w.xadj.assign(w.n + 1, 0);
    w.vw.resize(w.n);
    for (int32_t i = 0; i < w.n; i++) {
      int32_t v = V[i];
      w.vw[i] = g.w[v];
      for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; e++) {
        int32_t u = g.adj[e];
        if (u == v || stamp[u] != cur) continue;
        w.adj.push_back(local[u]);
        w.ew.push_back(1);
      }
      w.xadj[i + 1] = (int64_t)w.adj.size();
    }
    // several multilevel trials; keep the lightest separator (ties: better balance)
    std::vector<int8_t> part, trial;
    int64_t best_sep = INT64_MAX, best_imb = INT64_MAX;
    const int trials = w.n > 20000 ? 3 : w.n > 2000 ? 3 : 2;
    for (int t = 0; t < trials; t++) {
      multilevel_separator(w, trial, 0x5eed + 7919 * (calls++));
      refine(w, trial);
      int64_t W[3] = {0, 0, 0};
      for (int32_t i = 0; i < w.n; i++) W[trial[i]] += w.vw[i];
      int64_t imb = std::llabs(W[0] - W[1]);
      if (W[2] < best_sep || (W[2] == best_sep && imb < best_imb)) {
        best_sep = W[2]; best_imb = imb; part = trial;
      }
    }
    std::vector<int32_t> P0, P1, S;
    for (int32_t i = 0; i < w.n; i++) (part[i] == 0 ? P0 : part[i] == 1 ? P1 : S).push_back(V[i]);
    for (int32_t v : V) local[v] = -1;
    if (P0.empty() || P1.empty()) {  // no useful split
      out.insert(out.end(), V.begin(), V.end());
      return;
    }
    run(std::move(P0));
    run(std::move(P1));
    out.insert(out.end(), S.begin(), S.end());
  }

  // Greedy vertex-separator thinning: a separator vertex with no neighbour on
  // one side moves to the other side; a move that pulls fewer (by weight)
  // neighbours into the separator than it removes is taken if balance allows.
  static void refine(const WGraph& g, std::vector<int8_t>& part) {
    int64_t W[3] = {0, 0, 0};
    for (int32_t v = 0; v < g.n; v++) W[part[v]] += g.vw[v];
    const int64_t tot = W[0] + W[1] + W[2];
    for (int pass = 0; pass < 6; pass++) {
      bool improved = false;
      for (int32_t v = 0; v < g.n; v++) {
        if (part[v] != 2) continue;
        int64_t n0 = 0, n1 = 0;
        for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; e++) {
          int32_t u = g.adj[e];
          if (part[u] == 0) n0 += g.vw[u];
          else if (part[u] == 1) n1 += g.vw[u];
        }
        int side = -1;
        if (n1 == 0) side = 0;
        else if (n0 == 0) side = 1;
        else {
          int64_t g0 = g.vw[v] - n1, g1 = g.vw[v] - n0;
          int best = g0 >= g1 ? 0 : 1;
          int64_t gain = best == 0 ? g0 : g1;
          if (gain > 0) {
            int64_t nw0 = W[0] + (best == 0 ? g.vw[v] : -n0);
            int64_t nw1 = W[1] + (best == 1 ? g.vw[v] : -n1);
            if (std::llabs(nw0 - nw1) <= tot / 5) side = best;
          }
        }
        if (side < 0) continue;
        int other = 1 - side;
        part[v] = (int8_t)side;
        W[2] -= g.vw[v];
        W[side] += g.vw[v];
        for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; e++) {
          int32_t u = g.adj[e];
          if (part[u] == other) { part[u] = 2; W[other] -= g.vw[u]; W[2] += g.vw[u]; }
        }
        improved = true;
      }
      if (!improved) break;
    }
  }
};

}  // namespace

std::vector<int64_t> nested_dissection(const Pattern& p, const AnalysisOpts& o,
                                       int64_t* n_supervars) {
  Graph g;
  std::vector<int32_t> sv_of, sv_rows;
  std::vector<int64_t> sv_ptr;
  compress(p, g, sv_of, sv_ptr, sv_rows);
  if (n_supervars) *n_supervars = g.n;
  ND nd(g, o.leaf_size);
  std::vector<int32_t> all(g.n);
  std::iota(all.begin(), all.end(), 0);
  nd.run(std::move(all));
  std::vector<int64_t> perm;
  perm.reserve(p.n);
  for (int32_t s : nd.out)
    for (int64_t q = sv_ptr[s]; q < sv_ptr[s + 1]; q++) perm.push_back(sv_rows[q]);
  return perm;
}

}  // namespace kth
