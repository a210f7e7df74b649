// Driver of the host analysis (ordering.cpp, symbolic.cpp) for the sanitizer test:
// reads a CSR pattern (binary: n, nnz as int64, rowptr int64[n+1], col int32[nnz]),
// validates it, runs the analysis, checks the structural invariants of the result
// and prints "nsup flops nnz_l max_front nlevels".  Any failed invariant exits 2;
// the address and undefined-behaviour sanitizers abort on their own findings.
#include <cstdint>
#include <cstdio>
#include <fstream>
#include <vector>

#include "analysis.hpp"

using namespace kth;

#define CHECK(c)                                                    \
  do {                                                              \
    if (!(c)) {                                                     \
      std::fprintf(stderr, "invariant failed: %s (line %d)\n", #c, __LINE__); \
      return 2;                                                     \
    }                                                               \
  } while (0)

int main(int argc, char** argv) {
  if (argc < 2) return 1;
  std::ifstream f(argv[1], std::ios::binary);
  int64_t n = 0, nnz = 0;
  f.read(reinterpret_cast<char*>(&n), 8);
  f.read(reinterpret_cast<char*>(&nnz), 8);
  std::vector<int64_t> rp(n + 1);
  std::vector<int32_t> col(nnz);
  f.read(reinterpret_cast<char*>(rp.data()), 8 * (n + 1));
  f.read(reinterpret_cast<char*>(col.data()), 4 * nnz);
  if (!f) return 1;
  Pattern p;
  p.n = n;
  p.rowptr = rp.data();
  p.col = col.data();
  const std::string msg = check_pattern(p, true);
  if (!msg.empty()) {
    std::printf("rejected: %s\n", msg.c_str());
    return 0;
  }
  AnalysisOpts o;
  Symbolic S;
  analyze(p, o, S);
  // the order is a permutation and iperm its inverse
  std::vector<char> seen(n, 0);
  for (int64_t k = 0; k < n; k++) {
    CHECK(S.perm[k] >= 0 && S.perm[k] < n && !seen[S.perm[k]]);
    seen[S.perm[k]] = 1;
    CHECK(S.iperm[S.perm[k]] == k);
  }
  // supernodes partition the columns; row lists start with the columns, then
  // increasing rows beyond them; parents come later and sit one level up or more
  CHECK(S.sfirst[0] == 0 && S.sfirst[S.nsup] == n);
  for (int64_t s = 0; s < S.nsup; s++) {
    const int64_t ns = S.ns(s), nf = S.nf(s);
    CHECK(ns >= 1 && nf >= ns);
    for (int64_t a = 0; a < ns; a++) CHECK(S.rows[S.rptr[s] + a] == S.sfirst[s] + a);
    for (int64_t a = ns; a < nf; a++) {
      CHECK(S.rows[S.rptr[s] + a] >= S.sfirst[s + 1] && S.rows[S.rptr[s] + a] < n);
      if (a > ns) CHECK(S.rows[S.rptr[s] + a] > S.rows[S.rptr[s] + a - 1]);
    }
    const int64_t par = S.sparent[s];
    CHECK(par == -1 || (par > s && par < S.nsup && S.level[par] > S.level[s]));
    CHECK(S.level[s] >= 0 && S.level[s] < S.nlevels);
    CHECK(S.lptr[s + 1] - S.lptr[s] == nf * ns);
    // the extend-add map sends the update rows into the parent's row list
    if (par >= 0) {
      for (int64_t a = 0; a < nf - ns; a++) {
        const int32_t m = S.emap[S.eptr[s] + a];
        CHECK(m >= 0 && m < S.nf(par));
        CHECK(S.rows[S.rptr[par] + m] == S.rows[S.rptr[s] + ns + a]);
      }
    }
  }
  // original entries land inside their column's panel
  for (int64_t j = 0; j < n; j++) {
    for (int64_t e = S.acptr[j]; e < S.acptr[j + 1]; e++) {
      CHECK(S.asrc[e] >= 0 && S.asrc[e] < nnz);
      CHECK(S.adst[e] >= 0);
    }
  }
  std::printf("%lld %.17g %lld %lld %lld\n", (long long)S.nsup, S.flops, (long long)S.nnz_l,
              (long long)S.max_front, (long long)S.nlevels);
  return 0;
}
