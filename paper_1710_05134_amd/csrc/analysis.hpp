// Host analysis of the sparsity pattern shared by A and B: fill-reducing
// nested-dissection order Q, elimination tree, supernodes and the frontal
// maps used by the numeric factorization.  Everything here depends on the
// pattern only, so it is computed once and reused for B and for every shift
// sigma (Section 3.3: Q and the symbolic factorization are sigma-independent).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace kth {

struct Pattern {
  int64_t n = 0;
  const int64_t* rowptr = nullptr;  // [n+1]
  const int32_t* col = nullptr;     // [nnz], sorted per row, both triangles
};

// Options of the analysis.
struct AnalysisOpts {
  int64_t leaf_size = 48;     // nested dissection stops at this many supervariables
  int64_t relax_small = 8;    // always amalgamate when the merged node has <= this many columns
  double relax_frac_mid = 0.20;  // allowed explicit-zero fraction for merged ns <= 64
  double relax_frac_big = 0.04;  // ... for merged ns <= max_amalg
  int64_t max_amalg = 256;
};

struct Symbolic {
  int64_t n = 0, nnz = 0;
  std::vector<int64_t> perm;    // elimination position -> original index
  std::vector<int64_t> iperm;   // original index -> elimination position
  // supernodes (after relaxed amalgamation), in a postorder of the supernodal tree
  int64_t nsup = 0;
  std::vector<int64_t> sfirst;  // [nsup+1] first elimination column
  std::vector<int64_t> rptr;    // [nsup+1] offsets into rows
  std::vector<int32_t> rows;    // row lists (elimination indices); first ns are the columns
  std::vector<int64_t> sparent; // -1 for roots
  std::vector<int64_t> level;   // height in the supernodal tree (leaves 0)
  int64_t nlevels = 0;
  // child -> parent extend-add maps: for child c, emap[eptr[c] + a] = position of
  // the child's a-th update row in the parent's row list
  std::vector<int64_t> eptr;
  std::vector<int32_t> emap;
  // children of each supernode (increasing order)
  std::vector<int64_t> cptr;    // [nsup+1]
  std::vector<int32_t> clist;
  // factor panel offsets: panel s is nf x ns doubles, column-major, ld = nf
  std::vector<int64_t> lptr;    // [nsup+1]
  // update (contribution) block of s: nu x nu doubles, ld = nu, at pool offset
  // uptr[s] (-1 for roots); offsets planned by liveness over tree levels
  std::vector<int64_t> uptr;
  int64_t pool_size = 0;        // doubles
  // original entries of the lower triangle of Q C Q^T by elimination column:
  // entries acptr[j]..acptr[j+1] of column j: input CSR value index asrc[e] goes
  // to local panel offset adst[e] (row + col*nf) of column j's supernode
  std::vector<int64_t> acptr;   // [n+1]
  std::vector<int64_t> asrc;
  std::vector<int64_t> adst;
  // statistics
  double flops = 0;          // algorithmic count sum_j (c_j^2 + 2 c_j), exact structure
  double flops_padded = 0;   // same count over the amalgamated (padded) structure
  int64_t nnz_l = 0;         // exact structural nonzeros below the diagonal
  int64_t nnz_l_padded = 0;
  int64_t max_front = 0;
  int64_t max_ns = 0;
  int64_t n_supervars = 0;
  int64_t nsup_fundamental = 0;
  double front_bytes = 0;    // sum nf^2 * 8 (if every front were kept whole)
  double t_order = 0, t_symbolic = 0;

  int64_t nf(int64_t s) const { return rptr[s + 1] - rptr[s]; }
  int64_t ns(int64_t s) const { return sfirst[s + 1] - sfirst[s]; }
};

// Validates the pattern (sorted, in range, structurally symmetric, diagonal
// present).  Returns an empty string when valid, else a message.
std::string check_pattern(const Pattern& p, bool check_symmetry);

// Nested-dissection order of the pattern (elimination position -> original).
std::vector<int64_t> nested_dissection(const Pattern& p, const AnalysisOpts& o,
                                       int64_t* n_supervars);

// Full analysis: ordering, symbolic factorization, maps.
void analyze(const Pattern& p, const AnalysisOpts& o, Symbolic& S);

}  // namespace kth
