// Symbolic factorization for the multifrontal LDL^T of Q (A - sigma B) Q^T.
// Works on the supervariable-compressed graph (the orbitals of one atom form a
// dense block with one shared structure) and expands to degrees of freedom:
// elimination tree, postorder, column structures, fundamental supernodes,
// relaxed amalgamation, tree levels, extend-add maps and assembly maps.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>
#include <stdexcept>
#include <vector>

#include "analysis.hpp"

namespace kth {

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct SNode {
  int64_t first, last;        // compressed column range [first, last]
  std::vector<int32_t> rows;  // compressed row list (starts with the columns)
  int64_t exact_nnz;          // exact structural entries of its columns' L (dof units, incl. diag)
  int64_t parent;
  bool alive;
};

}  // namespace

void analyze(const Pattern& p, const AnalysisOpts& o, Symbolic& S) {
  const int64_t n = p.n;
  S = Symbolic();
  S.n = n;
  S.nnz = p.rowptr[n];
  double t0 = now_s();
  S.perm = nested_dissection(p, o, &S.n_supervars);
  S.t_order = now_s() - t0;
  t0 = now_s();

  // ---- supervariables in elimination order (consecutive dofs of perm) ----
  // Rebuild the grouping from perm: a supervariable is a maximal run of
  // consecutive perm entries with identical row patterns.
  std::vector<int64_t> svp;   // compressed vertex c -> dof range in elimination order [svp[c], svp[c+1])
  svp.push_back(0);
  for (int64_t k = 1; k < n; k++) {
    int64_t a = S.perm[k - 1], b = S.perm[k];
    int64_t la = p.rowptr[a + 1] - p.rowptr[a], lb = p.rowptr[b + 1] - p.rowptr[b];
    bool same = la == lb &&
                std::memcmp(p.col + p.rowptr[a], p.col + p.rowptr[b], sizeof(int32_t) * la) == 0;
    if (!same) svp.push_back(k);
  }
  svp.push_back(n);
  const int64_t m = (int64_t)svp.size() - 1;
  S.iperm.assign(n, 0);
  for (int64_t k = 0; k < n; k++) S.iperm[S.perm[k]] = k;
  std::vector<int32_t> cof(n);  // elimination position -> compressed vertex
  for (int64_t c = 0; c < m; c++)
    for (int64_t k = svp[c]; k < svp[c + 1]; k++) cof[k] = (int32_t)c;
  auto wt = [&](int64_t c) { return svp[c + 1] - svp[c]; };
  // compressed adjacency in elimination numbering
  std::vector<int64_t> xadj(m + 1, 0);
  std::vector<int32_t> adj;
  {
    std::vector<int32_t> mark(m, -1);
    for (int64_t c = 0; c < m; c++) {
      int64_t r = S.perm[svp[c]];
      mark[c] = (int32_t)c;
      for (int64_t q = p.rowptr[r]; q < p.rowptr[r + 1]; q++) {
        int32_t t = cof[S.iperm[p.col[q]]];
        if (mark[t] != (int32_t)c) { mark[t] = (int32_t)c; adj.push_back(t); }
      }
      std::sort(adj.begin() + xadj[c], adj.end());
      xadj[c + 1] = (int64_t)adj.size();
    }
  }

  // ---- elimination tree of the compressed graph ----
  std::vector<int64_t> parent(m, -1), anc(m, -1);
  for (int64_t i = 0; i < m; i++) {
    for (int64_t e = xadj[i]; e < xadj[i + 1]; e++) {
      int64_t j = adj[e];
      while (j != -1 && j < i) {
        int64_t nx = anc[j];
        anc[j] = i;
        if (nx == -1) { parent[j] = i; break; }
        j = nx;
      }
    }
  }
  // ---- postorder (children visited in increasing order) ----
  std::vector<int64_t> post;
  post.reserve(m);
  {
    std::vector<int64_t> head(m, -1), next(m, -1), stack;
    for (int64_t i = m - 1; i >= 0; i--)
      if (parent[i] != -1) { next[i] = head[parent[i]]; head[parent[i]] = i; }
    for (int64_t r = 0; r < m; r++) {
      if (parent[r] != -1) continue;
      stack.push_back(r);
      while (!stack.empty()) {
        int64_t v = stack.back();
        int64_t c = head[v];
        if (c != -1) { head[v] = next[c]; stack.push_back(c); }
        else { post.push_back(v); stack.pop_back(); }
      }
    }
  }
  // relabel compressed vertices by postorder and rebuild perm / svp / adjacency
  {
    std::vector<int64_t> newpos(m);
    for (int64_t k = 0; k < m; k++) newpos[post[k]] = k;
    std::vector<int64_t> perm2;
    perm2.reserve(n);
    std::vector<int64_t> svp2(m + 1, 0);
    for (int64_t k = 0; k < m; k++) {
      int64_t c = post[k];
      for (int64_t q = svp[c]; q < svp[c + 1]; q++) perm2.push_back(S.perm[q]);
      svp2[k + 1] = svp2[k] + wt(c);
    }
    std::vector<int64_t> par2(m);
    for (int64_t k = 0; k < m; k++) par2[k] = parent[post[k]] == -1 ? -1 : newpos[parent[post[k]]];
    std::vector<int64_t> xadj2(m + 1, 0);
    std::vector<int32_t> adj2;
    adj2.reserve(adj.size());
    for (int64_t k = 0; k < m; k++) {
      int64_t c = post[k];
      for (int64_t e = xadj[c]; e < xadj[c + 1]; e++) adj2.push_back((int32_t)newpos[adj[e]]);
      std::sort(adj2.begin() + xadj2[k], adj2.end());
      xadj2[k + 1] = (int64_t)adj2.size();
    }
    S.perm.swap(perm2);
    svp.swap(svp2);
    parent.swap(par2);
    xadj.swap(xadj2);
    adj.swap(adj2);
    for (int64_t k = 0; k < n; k++) S.iperm[S.perm[k]] = k;
  }

  // ---- column structures (compressed), fundamental supernodes ----
  std::vector<int64_t> nchild(m, 0);
  for (int64_t j = 0; j < m; j++) if (parent[j] != -1) nchild[parent[j]]++;
  std::vector<int64_t> chead(m, -1), cnext(m, -1);
  for (int64_t j = m - 1; j >= 0; j--)
    if (parent[j] != -1) { cnext[j] = chead[parent[j]]; chead[parent[j]] = j; }
  std::vector<std::vector<int32_t>> st(m);
  std::vector<int64_t> cnt(m, 0);
  std::vector<int32_t> mark(m, -1), tmp;
  std::vector<SNode> sn;
  S.flops = 0;
  S.nnz_l = 0;
  for (int64_t j = 0; j < m; j++) {
    tmp.clear();
    for (int64_t e = xadj[j]; e < xadj[j + 1]; e++) {
      int32_t i = adj[e];
      if (i > j && mark[i] != (int32_t)j) { mark[i] = (int32_t)j; tmp.push_back(i); }
    }
    for (int64_t c = chead[j]; c != -1; c = cnext[c]) {
      for (int32_t i : st[c])
        if (i > j && mark[i] != (int32_t)j) { mark[i] = (int32_t)j; tmp.push_back(i); }
      std::vector<int32_t>().swap(st[c]);
    }
    std::sort(tmp.begin(), tmp.end());
    cnt[j] = (int64_t)tmp.size();
    int64_t below = 0;  // dofs below this compressed column's block
    for (int32_t i : tmp) below += wt(i);
    // exact counts for the w dof columns of this supervariable
    int64_t w = wt(j);
    int64_t colnnz = 0;
    for (int64_t q = 0; q < w; q++) {
      double c = (double)(below + (w - 1 - q));
      S.flops += c * c + 2 * c;
      S.nnz_l += (int64_t)c;
      colnnz += (int64_t)c + 1;
    }
    bool join = j > 0 && parent[j - 1] == j && nchild[j] == 1 && cnt[j - 1] == cnt[j] + 1;
    if (join) {
      sn.back().last = j;
      sn.back().exact_nnz += colnnz;
    } else {
      SNode s;
      s.first = s.last = j;
      s.rows.reserve(tmp.size() + 1);
      s.rows.push_back((int32_t)j);
      s.rows.insert(s.rows.end(), tmp.begin(), tmp.end());
      s.exact_nnz = colnnz;
      s.parent = -1;
      s.alive = true;
      sn.push_back(std::move(s));
    }
    if (parent[j] != -1) st[j] = tmp;
  }
  st.clear();
  S.nsup_fundamental = (int64_t)sn.size();
  // supernode of each compressed column, supernodal parents
  std::vector<int64_t> snode(m);
  for (int64_t s = 0; s < (int64_t)sn.size(); s++)
    for (int64_t j = sn[s].first; j <= sn[s].last; j++) snode[j] = s;
  for (int64_t s = 0; s < (int64_t)sn.size(); s++) {
    int64_t pj = parent[sn[s].last];
    sn[s].parent = pj == -1 ? -1 : snode[pj];
  }

  // ---- relaxed amalgamation: merge the child ending right before a node ----
  auto dofs_of_cols = [&](const SNode& s) { return svp[s.last + 1] - svp[s.first]; };
  auto dof_rows = [&](const SNode& s) {
    int64_t t = 0;
    for (int32_t r : s.rows) t += wt(r);
    return t;
  };
  std::vector<int64_t> ending(m, -1);   // compressed column -> alive node ending there
  for (int64_t s = 0; s < (int64_t)sn.size(); s++) ending[sn[s].last] = s;
  std::vector<int64_t> merged_into(sn.size(), -1);
  auto find = [&](int64_t x) {
    while (x != -1 && merged_into[x] != -1) x = merged_into[x];
    return x;
  };
  for (int64_t s = 0; s < (int64_t)sn.size(); s++) {
    while (sn[s].first > 0) {
      int64_t d = ending[sn[s].first - 1];
      if (d < 0 || !sn[d].alive || find(sn[d].parent) != s) break;
      int64_t ns_d = dofs_of_cols(sn[d]), ns_s = dofs_of_cols(sn[s]);
      int64_t nf_s = dof_rows(sn[s]);
      int64_t ns_m = ns_d + ns_s, nf_m = ns_d + nf_s;
      double tot = (double)ns_m * nf_m - (double)ns_m * (ns_m - 1) / 2.0;
      double ex = (double)(sn[d].exact_nnz + sn[s].exact_nnz);
      double zf = 1.0 - ex / tot;
      bool ok = ns_m <= o.relax_small || (ns_m <= 64 && zf <= o.relax_frac_mid) ||
                (ns_m <= o.max_amalg && zf <= o.relax_frac_big);
      if (!ok) break;
      // merge d into s
      std::vector<int32_t> rows;
      rows.reserve(sn[d].last - sn[d].first + 1 + sn[s].rows.size());
      for (int64_t c = sn[d].first; c <= sn[d].last; c++) rows.push_back((int32_t)c);
      rows.insert(rows.end(), sn[s].rows.begin(), sn[s].rows.end());
      sn[s].rows.swap(rows);
      sn[s].first = sn[d].first;
      sn[s].exact_nnz += sn[d].exact_nnz;
      sn[d].alive = false;
      merged_into[d] = s;
      std::vector<int32_t>().swap(sn[d].rows);
      ending[sn[d].last] = -1;
    }
  }
  // compact alive nodes (already in increasing column order = topological order)
  std::vector<int64_t> newid(sn.size(), -1);
  int64_t ns_alive = 0;
  for (int64_t s = 0; s < (int64_t)sn.size(); s++) if (sn[s].alive) newid[s] = ns_alive++;
  // parent of a node: the alive node containing the etree parent of its last column
  std::vector<int64_t> node_of_col(m, -1);
  for (int64_t s = 0; s < (int64_t)sn.size(); s++)
    if (sn[s].alive) for (int64_t c = sn[s].first; c <= sn[s].last; c++) node_of_col[c] = newid[s];

  // ---- expand to dofs ----
  S.nsup = ns_alive;
  S.sfirst.assign(S.nsup + 1, 0);
  S.rptr.assign(S.nsup + 1, 0);
  S.sparent.assign(S.nsup, -1);
  S.rows.clear();
  S.flops_padded = 0;
  S.nnz_l_padded = 0;
  S.max_front = 0;
  S.max_ns = 0;
  for (int64_t s = 0; s < (int64_t)sn.size(); s++) {
    if (!sn[s].alive) continue;
    int64_t id = newid[s];
    S.sfirst[id] = svp[sn[s].first];
    S.rptr[id] = (int64_t)S.rows.size();
    for (int32_t r : sn[s].rows)
      for (int64_t k = svp[r]; k < svp[r + 1]; k++) S.rows.push_back((int32_t)k);
    int64_t pj = parent[sn[s].last];
    S.sparent[id] = pj == -1 ? -1 : node_of_col[pj];
  }
  S.sfirst[S.nsup] = n;
  S.rptr[S.nsup] = (int64_t)S.rows.size();
  S.lptr.assign(S.nsup + 1, 0);
  S.front_bytes = 0;
  for (int64_t s = 0; s < S.nsup; s++) {
    int64_t nf = S.nf(s), ns = S.ns(s);
    if (S.sparent[s] != -1 && S.sparent[s] <= s) throw std::logic_error("supernodal tree not topological");
    S.max_front = std::max(S.max_front, nf);
    S.max_ns = std::max(S.max_ns, ns);
    for (int64_t q = 0; q < ns; q++) {
      double c = (double)(nf - 1 - q);
      S.flops_padded += c * c + 2 * c;
      S.nnz_l_padded += (int64_t)c;
    }
    S.lptr[s + 1] = S.lptr[s] + nf * ns;
    S.front_bytes += 8.0 * nf * nf;
  }
  S.cptr.assign(S.nsup + 1, 0);
  for (int64_t s = 0; s < S.nsup; s++) if (S.sparent[s] != -1) S.cptr[S.sparent[s] + 1]++;
  for (int64_t s = 0; s < S.nsup; s++) S.cptr[s + 1] += S.cptr[s];
  S.clist.assign(S.cptr[S.nsup], 0);
  {
    std::vector<int64_t> f(S.cptr.begin(), S.cptr.end() - 1);
    for (int64_t s = 0; s < S.nsup; s++) if (S.sparent[s] != -1) S.clist[f[S.sparent[s]]++] = (int32_t)s;
  }
  // levels (height)
  S.level.assign(S.nsup, 0);
  for (int64_t s = 0; s < S.nsup; s++)
    if (S.sparent[s] != -1)
      S.level[S.sparent[s]] = std::max(S.level[S.sparent[s]], S.level[s] + 1);
  S.nlevels = 0;
  for (int64_t s = 0; s < S.nsup; s++) S.nlevels = std::max(S.nlevels, S.level[s] + 1);

  // ---- update-block pool: liveness over levels, first-fit ----
  {
    S.uptr.assign(S.nsup, -1);
    std::vector<std::vector<int64_t>> bylevel(S.nlevels);
    for (int64_t s = 0; s < S.nsup; s++) bylevel[S.level[s]].push_back(s);
    std::vector<std::pair<int64_t, int64_t>> freel;   // (offset, size), sorted by offset
    int64_t top = 0;
    auto alloc = [&](int64_t sz) {
      for (size_t q = 0; q < freel.size(); q++) {
        if (freel[q].second >= sz) {
          int64_t off = freel[q].first;
          freel[q].first += sz;
          freel[q].second -= sz;
          if (freel[q].second == 0) freel.erase(freel.begin() + q);
          return off;
        }
      }
      int64_t off = top;
      top += sz;
      return off;
    };
    auto release = [&](int64_t off, int64_t sz) {
      auto it = std::lower_bound(freel.begin(), freel.end(), std::make_pair(off, (int64_t)0));
      it = freel.insert(it, {off, sz});
      size_t q = it - freel.begin();
      if (q + 1 < freel.size() && freel[q].first + freel[q].second == freel[q + 1].first) {
        freel[q].second += freel[q + 1].second;
        freel.erase(freel.begin() + q + 1);
      }
      if (q > 0 && freel[q - 1].first + freel[q - 1].second == freel[q].first) {
        freel[q - 1].second += freel[q].second;
        freel.erase(freel.begin() + q);
      }
      if (!freel.empty() && freel.back().first + freel.back().second == top) {
        top = freel.back().first;
        freel.pop_back();
      }
    };
    int64_t peak = 0;
    for (int64_t L = 0; L < S.nlevels; L++) {
      for (int64_t s : bylevel[L]) {
        int64_t nu = S.nf(s) - S.ns(s);
        if (S.sparent[s] != -1 && nu > 0) S.uptr[s] = alloc(nu * nu);
      }
      peak = std::max(peak, top);
      for (int64_t s : bylevel[L])
        for (int64_t q = S.cptr[s]; q < S.cptr[s + 1]; q++) {
          int64_t c = S.clist[q];
          if (S.uptr[c] >= 0) { int64_t nu = S.nf(c) - S.ns(c); release(S.uptr[c], nu * nu); }
        }
    }
    S.pool_size = std::max<int64_t>(peak, 1);
  }
  // ---- extend-add maps ----
  S.eptr.assign(S.nsup + 1, 0);
  for (int64_t s = 0; s < S.nsup; s++) S.eptr[s + 1] = S.eptr[s] + (S.sparent[s] == -1 ? 0 : S.nf(s) - S.ns(s));
  S.emap.assign(S.eptr[S.nsup], 0);
  for (int64_t s = 0; s < S.nsup; s++) {
    int64_t pa = S.sparent[s];
    if (pa == -1) continue;
    const int32_t* cr = S.rows.data() + S.rptr[s] + S.ns(s);
    const int32_t* pr = S.rows.data() + S.rptr[pa];
    int64_t nu = S.nf(s) - S.ns(s), pnf = S.nf(pa), q = 0;
    for (int64_t a = 0; a < nu; a++) {
      while (q < pnf && pr[q] < cr[a]) q++;
      if (q >= pnf || pr[q] != cr[a]) throw std::logic_error("child row missing from parent front");
      S.emap[S.eptr[s] + a] = (int32_t)q;
    }
  }
  // ---- assembly maps: lower-triangle entries by elimination column ----
  std::vector<int64_t> snode_dof(n);
  for (int64_t s = 0; s < S.nsup; s++)
    for (int64_t k = S.sfirst[s]; k < S.sfirst[s + 1]; k++) snode_dof[k] = s;
  S.acptr.assign(n + 1, 0);
  for (int64_t r = 0; r < n; r++)
    for (int64_t q = p.rowptr[r]; q < p.rowptr[r + 1]; q++) {
      int64_t i = S.iperm[r], j = S.iperm[p.col[q]];
      if (i >= j) S.acptr[j + 1]++;
    }
  for (int64_t j = 0; j < n; j++) S.acptr[j + 1] += S.acptr[j];
  S.asrc.assign(S.acptr[n], 0);
  S.adst.assign(S.acptr[n], 0);
  std::vector<int64_t> fill(S.acptr.begin(), S.acptr.end() - 1);
  for (int64_t r = 0; r < n; r++)
    for (int64_t q = p.rowptr[r]; q < p.rowptr[r + 1]; q++) {
      int64_t i = S.iperm[r], j = S.iperm[p.col[q]];
      if (i < j) continue;
      int64_t s = snode_dof[j];
      const int32_t* R = S.rows.data() + S.rptr[s];
      int64_t nf = S.nf(s);
      const int32_t* it = std::lower_bound(R, R + nf, (int32_t)i);
      if (it == R + nf || *it != i) throw std::logic_error("entry outside its front");
      int64_t e = fill[j]++;
      S.asrc[e] = q;
      S.adst[e] = (int64_t)(it - R) + (j - S.sfirst[s]) * nf;
    }
  S.t_symbolic = now_s() - t0;
}

}  // namespace kth
