// Three-stage k-th eigenpair algorithm (Alg. 4) on the device engine.
//
//   stage 1 (Alg. 2): B-orthonormal Lanczos on (A, B) from a random v1; at step j
//     the extreme Ritz value theta_1 or theta_j of T_j becomes the shift sigma^(j)
//     and nu(sigma^(j)) is counted, until two consecutive shifts bracket lambda_k;
//   stage 2 (Alg. 1'): bisection of [sigma_l, sigma_u) with the inertia count until
//     it holds at most m_max eigenvalues (or is shorter than tau_len);
//   stage 3 (Alg. 3): shift-and-invert Lanczos at the midpoint with full
//     reorthogonalisation; from step m on, Ritz pairs (eq. (13), eq. (15)),
//     error bounds (Prop. 3), inclusion / disjointness, residual (eq. (res2)) and
//     relative-difference tests; the l = k - nu_l -th pair of the interval is
//     returned with its index validated.
// Readings of points the paper leaves open are the same as the oracle's:
// starting vectors (caller-provided rows, else the library's own generator),
// CGS2 in both Lanczos processes, V = B^{-1} V~ kept with V~ = B V, the m pairs of
// largest |theta~| (ties: larger theta~), closed bounds inside [sigma_l, sigma_u),
// relative differences matched in ascending order after sign alignment.
#include "driver.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <atomic>
#include <mutex>
#include <numeric>
#include <thread>

#include "blas.hpp"

namespace kth {

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// splitmix64 + Box-Muller: the library's own N(0,1) start vectors when the caller gives none.
void gen_start(int64_t n, uint64_t seed, int row, std::vector<double>& out) {
  out.resize(n);
  uint64_t s = seed * 0x9E3779B97F4A7C15ull + 0xD1B54A32D192ED03ull * (uint64_t)(row + 1);
  auto next = [&]() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  for (int64_t i = 0; i < n; i += 2) {
    double u1 = ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    double u2 = ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    double r = std::sqrt(-2.0 * std::log(u1)), t = 6.283185307179586 * u2;
    out[i] = r * std::cos(t);
    if (i + 1 < n) out[i + 1] = r * std::sin(t);
  }
}

struct Work {
  Ctx* c = nullptr;
  int64_t n = 0;
  int cap = 0;
  DBuf<double> V, Vt;           // basis and its B-image (n x cap each)
  DBuf<double> w, Bw, ya, yb;   // n-vectors
  DBuf<double> partial, h, h2, sc;
  DBuf<double> alpha_d, beta_d, theta_d, Y_d, twork;
  DBuf<double> C_d, cu_d, f_d, X, Xn, Prev, Dif;
  DBuf<int32_t> perm_d;
  int tcap = 0, mcap = 0;

  void init(Ctx* ctx, int64_t nn) {
    c = ctx;
    n = nn;
    w.alloc(c, n);
    Bw.alloc(c, n);
    ya.alloc(c, n);
    yb.alloc(c, n);
    sc.alloc(c, 4096);
    ensure_cols(64);
  }
  void ensure_cols(int need) {
    if (need <= cap) return;
    int nc = std::max(need, cap * 2);
    DBuf<double> V2, Vt2;
    V2.alloc(c, (size_t)n * nc);
    Vt2.alloc(c, (size_t)n * nc);
    if (cap) {
      KTH_HIP(hipMemcpyAsync(V2.get(), V.get(), sizeof(double) * n * cap, hipMemcpyDeviceToDevice, c->stream));
      KTH_HIP(hipMemcpyAsync(Vt2.get(), Vt.get(), sizeof(double) * n * cap, hipMemcpyDeviceToDevice, c->stream));
    }
    V.swap(V2);
    Vt.swap(Vt2);
    cap = nc;
    partial.alloc(c, (size_t)multidot_blocks(n) * (cap + 72));
    h.alloc(c, cap + 8);
    h2.alloc(c, cap + 8);
  }
  void ensure_tri(int j) {
    if (j <= tcap) return;
    int nc = std::max(j, 2 * tcap);
    alpha_d.alloc(c, nc);
    beta_d.alloc(c, nc);
    theta_d.alloc(c, nc);
    Y_d.alloc(c, (size_t)nc * nc);
    twork.alloc(c, (size_t)5 * nc * nc);
    tcap = nc;
  }
  void ensure_m(int m, int j) {
    if (m > mcap) {
      int nm = std::max(m, 8);
      X.alloc(c, (size_t)n * nm);
      Xn.alloc(c, (size_t)n * nm);
      Prev.alloc(c, (size_t)n * nm);
      Dif.alloc(c, (size_t)n * nm);
      f_d.alloc(c, nm);
      cu_d.alloc(c, nm);
      perm_d.alloc(c, nm);
      mcap = nm;
    }
    C_d.alloc(c, (size_t)std::max(j, 1) * std::max(m, 1));
  }
  double* v(int col) { return V.get() + (size_t)n * col; }
  double* vt(int col) { return Vt.get() + (size_t)n * col; }
};

template <typename T>
void d2h(Ctx* c, T* host, const T* dev, size_t count) {
  KTH_HIP(hipMemcpyAsync(host, dev, sizeof(T) * count, hipMemcpyDeviceToHost, c->stream));
  c->sync();
}
template <typename T>
void h2d(Ctx* c, T* dev, const T* host, size_t count) {
  KTH_HIP(hipMemcpyAsync(dev, host, sizeof(T) * count, hipMemcpyHostToDevice, c->stream));
}

double dot_dev(Work& W, const double* a, const double* b) {
  multidot(W.n, 1, a, W.n, b, W.partial.get(), W.sc.get(), 1.0, W.c->stream);
  double r;
  d2h(W.c, &r, W.sc.get(), 1);
  return r;
}

double bits_to_double(unsigned long long b) {
  double d;
  std::memcpy(&d, &b, sizeof(d));
  return d;
}

// nu(sigma) with the pencil's scratch factor; returns neg, sets the zero count,
// min |pivot| and max |L_ij|
int64_t count_nu(Pencil& P, double sigma, int64_t* zero, double* mind, double* maxl) {
  NumFactor& F = *P.scratch;
  factor_enqueue(P, F, sigma, false);
  factor_read_stats(P, F);
  if (zero) *zero = (int64_t)F.hs.zero;
  if (mind) *mind = bits_to_double(F.hs.min_d_bits);
  if (maxl) *maxl = bits_to_double(F.hs.max_l_bits);
  return (int64_t)F.hs.neg;
}

struct Shifts {
  std::vector<double> s;
  std::vector<int64_t> nu;
  double min_pivot_rel = INFINITY;
  double max_abs_l = 0;
  int nudges = 0;      // shifts moved for a zero or weak pivot or large growth
  int weak_kept = 0;   // counts accepted with a weak pivot after the nudges ran out
};

// A count is trusted when no pivot is zero, the smallest pivot is not below
// kWeakPivotRel * ||A - sigma B||_inf and no multiplier exceeds kGrowthMax: the
// count is exact for A - sigma B + E with E of the size of the factorization's
// backward error, so a shift within that distance of an eigenvalue, or a
// factorization with large element growth (pivoting is restricted to the
// fully-summed block), could count an eigenvalue on the wrong side.
constexpr double kWeakPivotRel = 1e-13;
constexpr double kGrowthMax = 1e8;
bool weak_count(int64_t zero, double md, double maxl, double scale) {
  return zero != 0 || md < kWeakPivotRel * scale || !(maxl <= kGrowthMax);
}

// nu at sigma; a shift with a zero or weak pivot, or with large growth, moves by
// `nudge` (growing with the attempt) and is counted again.  Zero pivots that
// persist are an error; a weak but nonzero pivot that persists is accepted (and
// reported) after kWeakAttempts moves.
constexpr int kWeakAttempts = 3;
int64_t nu_checked(Pencil& P, double& sigma, double nudge, Shifts& log, int64_t* nfac) {
  for (int attempt = 0; attempt < 8; attempt++) {
    int64_t zero = 0;
    double md = 0, ml = 0;
    int64_t nu = count_nu(P, sigma, &zero, &md, &ml);
    (*nfac)++;
    double scale = P.normA_inf + std::fabs(sigma) * P.normB_inf;
    bool weak = weak_count(zero, md, ml, scale);
    if (zero == 0 && (!weak || attempt >= kWeakAttempts)) {
      if (scale > 0) log.min_pivot_rel = std::min(log.min_pivot_rel, md / scale);
      log.max_abs_l = std::max(log.max_abs_l, ml);
      if (weak) log.weak_kept++;
      log.s.push_back(sigma);
      log.nu.push_back(nu);
      return nu;
    }
    log.nudges++;
    sigma += nudge * (attempt + 1);
  }
  throw Error(KTH_ESINGULAR, "repeated zero pivots near sigma");
}

// Next shift of the interpolating stage 2 (a bracketing root-finder on the
// eigenvalue count; Section 2.1 and Section 5 name such methods as alternatives
// to bisection): the count is modelled as linear between the bracket ends and the
// shift aims at the count that brings the farther end to within m_max / 2 of k
// (k - m_max/2 below, k + m_max/2 - 1 above, + 1/2 to land inside the count's
// step), at a fraction of the bracket kept inside [1/64, 63/64].  The arithmetic
// is written out operation by operation, uncontracted, so the shifts are the same
// doubles as the oracle's.
double interp_shift(int64_t k, double sl, double su, int64_t nl, int64_t nu_, int64_t m_max) {
#pragma clang fp contract(off)
  double c;
  if ((k - nl) >= (nu_ - k)) c = (double)k - (double)m_max / 2.0 + 0.5;
  else c = (double)k + (double)m_max / 2.0 - 1.0 + 0.5;
  double t = (c - (double)nl) / (double)(nu_ - nl);
  t = std::min(std::max(t, 1.0 / 64.0), 63.0 / 64.0);
  return sl + t * (su - sl);
}

// Stage-2 stopping count from measured costs (Section 3.4 and Section 5 leave
// m_max, which trades bisection steps against Lanczos steps, to tuning).  The
// validated shift-and-invert iteration of Alg. 3 takes about 2.6 m + 8 steps for
// m eigenvalues in the interval (measured on the tight-binding workloads), each
// step about 1.15 solves.  Bisection halves m for one more factorization, which
// pays while 2.6 (m / 2) t_step > t_fact, i.e. down to m = 2 t_fact / (2.6 t_step).
// The interpolating root-finder lands its last shifts within about one count of
// their targets, so narrowing costs it no extra steps down to m_max = 2 (the
// bracket [lambda_{k-1}, lambda_{k+1}]); it takes 2.  Clamped to [2, 20].
int64_t auto_m_max(int root_finder, double t_fact, double t_solve) {
  if (root_finder == 1) return 2;
  if (!(t_fact > 0) || !(t_solve > 0)) return 20;
  const double m = 2.0 * t_fact / (2.6 * 1.15 * t_solve);
  return std::min<int64_t>(20, std::max<int64_t>(2, (int64_t)std::lround(m)));
}


// Eigenvalues (ascending, w) and eigenvectors (columns of Z, column-major) of a
// symmetric N x N matrix A (column-major, both triangles) by the cyclic Jacobi
// method: rotations annihilate a(p, q) in turn until the off-diagonal part is
// below 1e-16 of the Frobenius norm (at most 60 sweeps).
void sym_eig_jacobi(int N, std::vector<double> A, std::vector<double>& w, std::vector<double>& Z) {
  Z.assign((size_t)N * N, 0.0);
  for (int i = 0; i < N; i++) Z[(size_t)i * N + i] = 1.0;
  auto a = [&](int r, int c) -> double& { return A[(size_t)c * N + r]; };
  double fro = 0;
  for (double v : A) fro += v * v;
  fro = std::sqrt(fro);
  for (int sweep = 0; sweep < 60; sweep++) {
    double off = 0;
    for (int c = 0; c < N; c++)
      for (int r = 0; r < c; r++) off += 2.0 * a(r, c) * a(r, c);
    if (std::sqrt(off) <= 1e-16 * fro || fro == 0) break;
    for (int p = 0; p < N - 1; p++)
      for (int q = p + 1; q < N; q++) {
        const double apq = a(p, q);
        if (apq == 0.0) continue;
        const double th = (a(q, q) - a(p, p)) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(1.0 + th * th));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = t * cs;
        for (int r = 0; r < N; r++) {   // columns p, q
          const double x = a(r, p), y = a(r, q);
          a(r, p) = cs * x - sn * y;
          a(r, q) = sn * x + cs * y;
        }
        for (int c = 0; c < N; c++) {   // rows p, q
          const double x = a(p, c), y = a(q, c);
          a(p, c) = cs * x - sn * y;
          a(q, c) = sn * x + cs * y;
        }
        for (int r = 0; r < N; r++) {
          const double x = Z[(size_t)p * N + r], y = Z[(size_t)q * N + r];
          Z[(size_t)p * N + r] = cs * x - sn * y;
          Z[(size_t)q * N + r] = sn * x + cs * y;
        }
      }
  }
  std::vector<int> ord(N);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return a(x, x) < a(y, y); });
  std::vector<double> Zs((size_t)N * N);
  w.resize(N);
  for (int i = 0; i < N; i++) {
    w[i] = a(ord[i], ord[i]);
    std::copy(Z.begin() + (size_t)ord[i] * N, Z.begin() + (size_t)(ord[i] + 1) * N, Zs.begin() + (size_t)i * N);
  }
  Z.swap(Zs);
}

// Largest singular value of the p x c matrix M (column-major).
double norm2_mat(int p, int c, const std::vector<double>& M) {
  std::vector<double> G((size_t)c * c, 0.0), w, Z;
  for (int a = 0; a < c; a++)
    for (int b = 0; b < c; b++) {
      double t = 0;
      for (int r = 0; r < p; r++) t += M[(size_t)a * p + r] * M[(size_t)b * p + r];
      G[(size_t)b * c + a] = t;
    }
  sym_eig_jacobi(c, G, w, Z);
  return std::sqrt(std::max(w.back(), 0.0));
}

// Upper-triangular Cholesky factor R (column-major, G = R^T R) of a symmetric
// positive definite p x p matrix; false if a pivot is not positive.
bool cholesky_upper(int p, const std::vector<double>& G, std::vector<double>& R) {
  R.assign((size_t)p * p, 0.0);
  for (int j = 0; j < p; j++) {
    for (int i = 0; i <= j; i++) {
      double t = G[(size_t)j * p + i];
      for (int q = 0; q < i; q++) t -= R[(size_t)i * p + q] * R[(size_t)j * p + q];
      if (i == j) {
        if (!(t > 0)) return false;
        R[(size_t)j * p + j] = std::sqrt(t);
      } else {
        R[(size_t)j * p + i] = t / R[(size_t)i * p + i];
      }
    }
  }
  return true;
}

// Inverse of an upper-triangular p x p matrix (column-major).
std::vector<double> inv_upper(int p, const std::vector<double>& R) {
  std::vector<double> X((size_t)p * p, 0.0);
  for (int c = 0; c < p; c++) {
    X[(size_t)c * p + c] = 1.0 / R[(size_t)c * p + c];
    for (int r = c - 1; r >= 0; r--) {
      double t = 0;
      for (int q = r + 1; q <= c; q++) t += R[(size_t)q * p + r] * X[(size_t)c * p + q];
      X[(size_t)c * p + r] = -t / R[(size_t)r * p + r];
    }
  }
  return X;
}

// Result of the block shift-and-invert Lanczos.
struct BlockOut {
  kth_status st = KTH_ENOCONV;
  double lam = 0, eta = 0;
  int steps = 0, it_bound = 0, it_res = 0, it_diff = 0;
  int xcol = -1;        // column of W.X holding the returned x_{l,2}
};

// Block shift-and-invert Lanczos for an interval that may hold multiple or
// clustered eigenvalues (the modification Section 3.4 proposes; block size p).
// With V = B^{-1} V~ kept B-orthonormal and V~ = B V, block by block:
//   (A - sigma B)^{-1} B V_j = V_j T_j + V_{j+1} B_j E_j^T,
// T_j block tridiagonal (diagonal blocks A_i from the first reorthogonalisation
// pass, subdiagonal blocks B_i from the twice-repeated Cholesky B-orthonormalisation
// of each new block).  A Ritz pair (theta, y) gives lambda = sigma + 1/theta and
// x_2 = theta V_j y + V_{j+1} B_j E_j^T y, whose residual is -V~_{j+1} s with
// s = B_j E_j^T y / theta, so the bound of Prop. 3 holds with ||s||_2 for |s|.
// Validation: the m pairs of largest |theta|; all bounds inside [sigma_l,
// sigma_u); overlapping bounds form a cluster C whose B-orthonormal Ritz block
// has residual norm rho = ||B_j E_j^T Y_C||_2, so |C| eigenvalues lie within
// rho / (|theta| (|theta| - rho)) of its lambdas (Kahan's theorem for the
// operator (A - sigma B)^{-1} B, self-adjoint in the B inner product); single
// bounds and cluster intervals must be pairwise disjoint.  Residual test per
// pair; relative difference per single pair (as in Alg. 3), per cluster on its
// eigenvalues (|lambda^(j) - lambda^(j-1)| <= tau_diff max(1, |lambda|)), with the
// same cluster shape as the step before.  Bounds and cluster radii are not taken
// below 64 eps (||A||_inf + |sigma| ||B||_inf), the rounding level of the solves.
BlockOut si_block_run(Pencil& P, NumFactor& FS, Work& W, int64_t k, double sl, double su,
                      int64_t nl, int64_t nu_, double sigma, int p, const kth_opts& o,
                      const std::function<void(int, std::vector<double>&)>& start_vec,
                      const std::function<void()>& refactor_fp64) {
  Ctx* c = P.ctx;
  hipStream_t st = c->stream;
  const int64_t n = P.n;
  const int64_t l = k - nl;
  const int m = (int)(nu_ - nl);
  const double floor_b = 64.0 * 2.220446049250313e-16 * (P.normA_inf + std::fabs(sigma) * P.normB_inf);
  BlockOut out;
  DBuf<double> zero, zcu, Cb;
  zero.alloc(c, n);
  KTH_HIP(hipMemsetAsync(zero.get(), 0, sizeof(double) * n, st));
  zcu.alloc(c, 4096);
  KTH_HIP(hipMemsetAsync(zcu.get(), 0, sizeof(double) * 4096, st));
  W.ensure_m(std::max(m, p), 1);
  // X := X * C for a block of q columns at column c0 of V or Vt (through W.X)
  auto times_small = [&](double* base, int q, const std::vector<double>& C) {
    Cb.alloc(c, C.size());
    h2d(c, Cb.get(), C.data(), C.size());
    ritz_vectors(n, q, q, base, n, Cb.get(), zero.get(), zcu.get(), W.X.get(), n, st);
    KTH_HIP(hipMemcpyAsync(base, W.X.get(), sizeof(double) * n * q, hipMemcpyDeviceToDevice, st));
    c->sync();   // Cb is released on the next call
  };
  // Gram matrix X^T Y of two blocks of q columns
  auto gram = [&](const double* X, const double* Y, int q) {
    std::vector<double> G((size_t)q * q);
    for (int b = 0; b < q; b++) {
      multidot(n, q, X, n, Y + (size_t)b * n, W.partial.get(), W.h.get(), 1.0, st);
      d2h(c, G.data() + (size_t)b * q, W.h.get(), q);
    }
    return G;
  };
  // B-orthonormalise the block at column c0 (twice); R: the total factor
  auto borth = [&](int c0, std::vector<double>& R) -> bool {
    R.assign((size_t)p * p, 0.0);
    for (int i = 0; i < p; i++) R[(size_t)i * p + i] = 1.0;
    for (int pass = 0; pass < 2; pass++) {
      std::vector<double> G = gram(W.v(c0), W.vt(c0), p), Rc;
      for (int a = 0; a < p; a++)
        for (int b = 0; b < a; b++) {
          const double t = 0.5 * (G[(size_t)a * p + b] + G[(size_t)b * p + a]);
          G[(size_t)a * p + b] = G[(size_t)b * p + a] = t;
        }
      if (!cholesky_upper(p, G, Rc)) return false;
      const std::vector<double> Ri = inv_upper(p, Rc);
      times_small(W.v(c0), p, Ri);
      times_small(W.vt(c0), p, Ri);
      std::vector<double> Rn((size_t)p * p, 0.0);   // Rc * R
      for (int a = 0; a < p; a++)
        for (int b = 0; b < p; b++) {
          double t = 0;
          for (int q = 0; q < p; q++) t += Rc[(size_t)q * p + a] * R[(size_t)b * p + q];
          Rn[(size_t)b * p + a] = t;
        }
      R.swap(Rn);
    }
    return true;
  };
  W.ensure_cols(2 * p);
  std::vector<double> hv;
  for (int q = 0; q < p; q++) {
    start_vec(q == 0 ? 1 : 3 + q, hv);
    h2d(c, W.v(q), hv.data(), n);
    spmv2(n, P.rowptr.get(), P.col.get(), P.aval.get(), P.bval.get(), W.v(q), nullptr, W.vt(q), st);
  }
  std::vector<double> R0;
  if (!borth(0, R0)) throw Error(KTH_ENOCONV, "block Lanczos: the start block is rank deficient");
  std::vector<std::vector<double>> Ab, Bb;
  std::vector<int> prev_shape;
  std::vector<double> prev_la;
  bool have_prev = false;
  for (int j = 1; j <= o.max_lanczos; j++) {
    const int base = (j - 1) * p, nxt = j * p;
    W.ensure_cols(nxt + p);
    for (int q = 0; q < p; q++) {
      SolveOutcome so = solve_refined(P, FS, W.vt(base + q), W.v(nxt + q), o.ir_tol > 0 ? o.ir_tol : kIrTol);
      if (!so.converged) {
        refactor_fp64();
        solve_enqueue_f(P, FS, W.vt(base + q), W.v(nxt + q));
      }
      spmv2(n, P.rowptr.get(), P.col.get(), P.aval.get(), P.bval.get(), W.v(nxt + q), nullptr,
            W.vt(nxt + q), st);
    }
    std::vector<double> Aj((size_t)p * p);
    for (int q = 0; q < p; q++) {
      double* w = W.v(nxt + q);
      double* bw = W.vt(nxt + q);
      multidot(n, nxt, W.Vt.get(), n, w, W.partial.get(), W.h.get(), 1.0, st);
      d2h(c, Aj.data() + (size_t)q * p, W.h.get() + base, p);
      multiaxpy(n, nxt, W.V.get(), n, W.h.get(), w, W.Vt.get(), bw, st);
      multidot(n, nxt, W.Vt.get(), n, w, W.partial.get(), W.h2.get(), 1.0, st);
      multiaxpy(n, nxt, W.V.get(), n, W.h2.get(), w, W.Vt.get(), bw, st);
    }
    for (int a = 0; a < p; a++)
      for (int b = 0; b < a; b++) {
        const double t = 0.5 * (Aj[(size_t)a * p + b] + Aj[(size_t)b * p + a]);
        Aj[(size_t)a * p + b] = Aj[(size_t)b * p + a] = t;
      }
    Ab.push_back(Aj);
    std::vector<double> Rj;
    if (!borth(nxt, Rj)) throw Error(KTH_ENOCONV, "block Lanczos: a new block is rank deficient");
    out.steps = j;
    if ((int64_t)j * p >= m) {
      const int N = j * p;
      std::vector<double> T((size_t)N * N, 0.0);
      for (int i = 0; i < j; i++)
        for (int a = 0; a < p; a++)
          for (int b = 0; b < p; b++) {
            T[(size_t)(i * p + b) * N + i * p + a] = Ab[i][(size_t)b * p + a];
            if (i + 1 < j) {
              const double v = Bb[i][(size_t)b * p + a];   // rows (i+1) p + a, columns i p + b
              T[(size_t)(i * p + b) * N + (i + 1) * p + a] = v;
              T[(size_t)((i + 1) * p + a) * N + i * p + b] = v;
            }
          }
      std::vector<double> th, Y;
      sym_eig_jacobi(N, T, th, Y);
      std::vector<int> ord(N);
      std::iota(ord.begin(), ord.end(), 0);
      std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
        if (std::fabs(th[a]) != std::fabs(th[b])) return std::fabs(th[a]) > std::fabs(th[b]);
        return th[a] > th[b];
      });
      ord.resize(m);
      std::vector<double> lam(m), eta(m), S((size_t)p * m), RY((size_t)p * m);
      for (int q = 0; q < m; q++) {
        const int i = ord[q];
        const double ts = th[i];
        lam[q] = sigma + 1.0 / ts;
        double sn = 0;
        for (int a = 0; a < p; a++) {   // (B_j E_j^T y)_a
          double t = 0;
          for (int b = a; b < p; b++) t += Rj[(size_t)b * p + a] * Y[(size_t)i * N + (N - p) + b];
          RY[(size_t)q * p + a] = t;
          S[(size_t)q * p + a] = t / ts;
          sn += (t / ts) * (t / ts);
        }
        sn = std::sqrt(sn);
        eta[q] = std::max((1.0 / std::fabs(ts)) * sn / std::sqrt(1.0 + sn * sn), floor_b);
      }
      bool incl = true;
      for (int q = 0; q < m; q++) incl = incl && (lam[q] - eta[q] >= sl) && (lam[q] + eta[q] < su);
      std::vector<int> asc(m);
      std::iota(asc.begin(), asc.end(), 0);
      std::stable_sort(asc.begin(), asc.end(), [&](int a, int b) { return lam[a] < lam[b]; });
      std::vector<std::vector<int>> comps{{asc[0]}};
      for (int q = 1; q < m; q++) {
        const int a = asc[q - 1], b = asc[q];
        if (lam[a] + eta[a] >= lam[b] - eta[b]) comps.back().push_back(b);
        else comps.push_back({b});
      }
      bool ok = incl;
      std::vector<std::pair<double, double>> iv;
      for (const auto& C : comps) {
        if (C.size() == 1) {
          iv.push_back({lam[C[0]] - eta[C[0]], lam[C[0]] + eta[C[0]]});
          continue;
        }
        std::vector<double> M((size_t)p * C.size());
        double tmin = INFINITY;
        for (size_t q = 0; q < C.size(); q++) {
          std::copy(RY.begin() + (size_t)C[q] * p, RY.begin() + (size_t)(C[q] + 1) * p,
                    M.begin() + q * p);
          tmin = std::min(tmin, std::fabs(th[ord[C[q]]]));
        }
        const double rho = norm2_mat(p, (int)C.size(), M);
        if (!(rho < tmin)) { ok = false; break; }
        double lo = INFINITY, hi = -INFINITY;
        for (int q : C) {
          const double tc = std::fabs(th[ord[q]]);
          const double e = std::max(rho / (tc * (tc - rho)), floor_b);
          lo = std::min(lo, lam[q] - e);
          hi = std::max(hi, lam[q] + e);
        }
        iv.push_back({lo, hi});
      }
      if (ok)
        for (size_t q = 0; q < iv.size(); q++)
          ok = ok && iv[q].first >= sl && iv[q].second < su && (q == 0 || iv[q - 1].second < iv[q].first);
      // Ritz vectors x_2 = [V_j, V_{j+1}] [theta y; B_j E_j^T y], in column groups
      const int J = N + p;
      const int mg = std::max(1, std::min(m, 8000 / (J + 1)));
      for (int g0 = 0; g0 < m; g0 += mg) {
        const int cnt = std::min(mg, m - g0);
        std::vector<double> C((size_t)J * cnt);
        for (int q = 0; q < cnt; q++) {
          const int i = ord[g0 + q];
          for (int r = 0; r < N; r++) C[(size_t)q * J + r] = th[i] * Y[(size_t)i * N + r];
          for (int a = 0; a < p; a++) C[(size_t)q * J + N + a] = RY[(size_t)(g0 + q) * p + a];
        }
        Cb.alloc(c, C.size());
        h2d(c, Cb.get(), C.data(), C.size());
        ritz_vectors(n, J, cnt, W.V.get(), n, Cb.get(), zero.get(), zcu.get(), W.X.get() + (size_t)g0 * n, n, st);
        c->sync();
      }
      std::vector<double> xn2(m);
      multidot2(n, m, W.X.get(), n, W.X.get(), n, W.partial.get(), W.sc.get(), 1.0, st);
      d2h(c, xn2.data(), W.sc.get(), m);
      const std::vector<double> Gt = gram(W.vt(nxt), W.vt(nxt), p);
      bool res_ok = true;
      for (int q = 0; q < m; q++) {
        double rr = 0;
        for (int a = 0; a < p; a++)
          for (int b = 0; b < p; b++) rr += S[(size_t)q * p + a] * Gt[(size_t)b * p + a] * S[(size_t)q * p + b];
        res_ok = res_ok && (std::sqrt(std::max(rr, 0.0)) / std::sqrt(xn2[q]) < o.tau_res);
      }
      std::vector<int> shape;
      for (const auto& C : comps) shape.push_back((int)C.size());
      std::vector<double> la(m);
      std::vector<int32_t> pa(m);
      std::vector<double> fa(m);
      for (int q = 0; q < m; q++) {
        la[q] = lam[asc[q]];
        pa[q] = asc[q];
        fa[q] = 1.0 / std::sqrt(xn2[asc[q]]);
      }
      h2d(c, W.perm_d.get(), pa.data(), m);
      h2d(c, W.f_d.get(), fa.data(), m);
      gather_cols(n, m, W.X.get(), n, W.perm_d.get(), W.f_d.get(), W.Xn.get(), n, st);
      bool diff_ok = false;
      if (have_prev && shape == prev_shape) {
        std::vector<double> dd(m), sg(m);
        multidot2(n, m, W.Xn.get(), n, W.Prev.get(), n, W.partial.get(), W.sc.get(), 1.0, st);
        d2h(c, dd.data(), W.sc.get(), m);
        for (int q = 0; q < m; q++) sg[q] = dd[q] < 0 ? -1.0 : 1.0;
        h2d(c, W.f_d.get(), sg.data(), m);
        diff_cols(n, m, W.Xn.get(), n, W.f_d.get(), W.Prev.get(), n, W.Dif.get(), n, st);
        multidot2(n, m, W.Dif.get(), n, W.Dif.get(), n, W.partial.get(), W.sc.get(), 1.0, st);
        d2h(c, dd.data(), W.sc.get(), m);
        diff_ok = true;
        int pos = 0;
        for (int sz : shape) {
          for (int q = pos; q < pos + sz; q++)
            diff_ok = diff_ok && (sz == 1 ? std::sqrt(dd[q]) < o.tau_diff
                                          : std::fabs(la[q] - prev_la[q]) <= o.tau_diff * std::max(1.0, std::fabs(la[q])));
          pos += sz;
        }
      }
      W.Xn.swap(W.Prev);
      have_prev = true;
      prev_shape = shape;
      prev_la = la;
      if (ok && !out.it_bound) out.it_bound = j;
      if (res_ok && !out.it_res) out.it_res = j;
      if (diff_ok && !out.it_diff) out.it_diff = j;
      if (ok && res_ok && diff_ok) {
        const int q = asc[l - 1];
        out.st = KTH_OK;
        out.lam = lam[q];
        out.eta = eta[q];
        out.xcol = q;
        return out;
      }
    }
    Bb.push_back(Rj);
  }
  return out;
}

}  // namespace

void numeric_factor(Pencil& P, NumFactor& F, double sigma, kth_precision prec) {
  if (prec != KTH_FP64 && prec != KTH_FP32_IR) throw Error(KTH_EINVAL, "unknown precision");
  factor_alloc(P, F, 1, prec);
  factor_enqueue(P, F, sigma, false);
  factor_read_stats(P, F);
}

SolveOutcome solve_refined(Pencil& P, NumFactor& F, const double* b, double* x, double tol) {
  SolveOutcome out;
  solve_enqueue_f(P, F, b, x);
  if (F.prec == KTH_FP64) return out;
  Ctx* c = P.ctx;
  hipStream_t st = c->stream;
  const int64_t n = P.n;
  const int mk = kGmresMax;
  if (!F.ir_r.p) {
    F.ir_r.alloc(c, n);
    F.ir_V.alloc(c, (size_t)n * (mk + 1));
    F.ir_part.alloc(c, (size_t)multidot_blocks(n) * (mk + 1));
    F.ir_out.alloc(c, 2 * (mk + 1) + 4);
  }
  double* r = F.ir_r.get();
  double* V = F.ir_V.get();
  double* part = F.ir_part.get();
  double* h1 = F.ir_out.get();            // [mk + 1]
  double* h2 = h1 + (mk + 1);             // [mk + 1]
  double* nrm = h2 + (mk + 1);            // [4]: ||r||_inf, ||x||_inf, ||b||_inf, ||w||_2^2
  auto col = [&](int j) { return V + (size_t)j * n; };
  auto norm2sq = [&](const double* v) {
    multidot(n, 1, v, n, v, part, nrm + 3, 1.0, st);
    double t;
    d2h(c, &t, nrm + 3, 1);
    return t;
  };
  // ||A - sigma B||_inf bounded by ||A||_inf + |sigma| ||B||_inf
  const double normM = P.normA_inf + std::fabs(F.sigma) * P.normB_inf;
  const double* A = P.aval.get();
  const double* Bv = P.bval.get();
  absmax(n, b, part, nrm + 2, st);
  double prev = INFINITY;
  int slow = 0;
  std::vector<double> y(mk);   // outlives the asynchronous upload below
  for (int outer = 0;; outer++) {
    shifted_residual(n, P.rowptr.get(), P.col.get(), A, Bv, F.sigma, x, b, r, st);
    absmax(n, r, part, nrm, st);
    absmax(n, x, part, nrm + 1, st);
    double hn[3];
    d2h(c, hn, nrm, 3);
    const double den = normM * hn[1] + hn[2];
    out.berr = den > 0 ? hn[0] / den : 0.0;
    if (!std::isfinite(out.berr)) { out.converged = false; return out; }
    if (out.berr <= tol) return out;
    if (hn[0] > 0.5 * prev) {
      if (++slow >= 2) { out.converged = false; return out; }
    } else {
      slow = 0;
    }
    if (outer >= kIrMaxOuter) { out.converged = false; return out; }
    prev = hn[0];
    // GMRES on M32^{-1} M d = M32^{-1} r from d = 0 (CGS2 Arnoldi, Givens QR of H)
    solve_enqueue_f(P, F, r, col(0));
    out.steps++;
    const double beta = std::sqrt(norm2sq(col(0)));
    if (!(beta > 0) || !std::isfinite(beta)) { out.converged = false; return out; }
    scale_copy(n, 1.0 / beta, col(0), col(0), st);
    std::vector<double> H((size_t)(mk + 1) * mk, 0.0), cs(mk), sn(mk), g(mk + 1, 0.0);
    g[0] = beta;
    int k = 0;
    for (int j = 0; j < mk; j++) {
      // w = M32^{-1} (M v_j), stored in column j + 1
      shifted_residual(n, P.rowptr.get(), P.col.get(), A, Bv, F.sigma, col(j), nullptr, r, st);
      solve_enqueue_f(P, F, r, col(j + 1));
      out.steps++;
      double* w = col(j + 1);
      multidot(n, j + 1, V, n, w, part, h1, 1.0, st);
      multiaxpy(n, j + 1, V, n, h1, w, nullptr, nullptr, st);
      multidot(n, j + 1, V, n, w, part, h2, 1.0, st);
      multiaxpy(n, j + 1, V, n, h2, w, nullptr, nullptr, st);
      std::vector<double> ha(j + 1), hb(j + 1);
      d2h(c, ha.data(), h1, j + 1);
      d2h(c, hb.data(), h2, j + 1);
      const double hw = std::sqrt(std::max(norm2sq(w), 0.0));
      double* hc = &H[(size_t)j * (mk + 1)];
      for (int i = 0; i <= j; i++) hc[i] = ha[i] + hb[i];
      hc[j + 1] = hw;
      if (hw > 0) scale_copy(n, 1.0 / hw, w, w, st);
      for (int i = 0; i < j; i++) {   // earlier rotations
        const double t = cs[i] * hc[i] + sn[i] * hc[i + 1];
        hc[i + 1] = -sn[i] * hc[i] + cs[i] * hc[i + 1];
        hc[i] = t;
      }
      const double rho = std::hypot(hc[j], hc[j + 1]);
      cs[j] = rho > 0 ? hc[j] / rho : 1.0;
      sn[j] = rho > 0 ? hc[j + 1] / rho : 0.0;
      hc[j] = rho;
      hc[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      k = j + 1;
      if (std::fabs(g[j + 1]) <= kGmresTol * beta || !(hw > 0)) break;
    }
    // y = R^{-1} g, x += V y  (as x -= V (-y))
    for (int i = k - 1; i >= 0; i--) {
      double t = g[i];
      for (int q = i + 1; q < k; q++) t -= H[(size_t)q * (mk + 1) + i] * y[q];
      const double d = H[(size_t)i * (mk + 1) + i];
      y[i] = d != 0 ? t / d : 0.0;
    }
    for (int i = 0; i < k; i++) y[i] = -y[i];
    h2d(c, h1, y.data(), k);
    multiaxpy(n, k, V, n, h1, x, nullptr, nullptr, st);
  }
}

void solve_many(Pencil& P, NumFactor& F, int32_t nrhs, const double* r, int64_t ldr, double* x,
                int64_t ldx, bool device_ptrs, bool unrefined) {
  auto one = [&](const double* b, double* xx) {
    if (!unrefined) return solve_refined(P, F, b, xx);
    solve_enqueue_f(P, F, b, xx);
    return SolveOutcome{};
  };
  Ctx* c = P.ctx;
  DBuf<double> rb, xb;
  if (!device_ptrs) {
    rb.alloc(c, P.n);
    xb.alloc(c, P.n);
  }
  for (int32_t q = 0; q < nrhs; q++) {
    const double* rq = r + (size_t)q * ldr;
    double* xq = x + (size_t)q * ldx;
    SolveOutcome so;
    if (device_ptrs) {
      so = one(rq, xq);
    } else {
      h2d(c, rb.get(), rq, P.n);
      so = one(rb.get(), xb.get());
      d2h(c, xq, xb.get(), P.n);
    }
    if (!so.converged) {
      c->sync();
      throw Error(KTH_ENOCONV, "iterative refinement of the FP32 factor stalled at backward error " +
                                   std::to_string(so.berr) + " (column " + std::to_string(q) + ")");
    }
  }
  c->sync();
}

// nu at many shifts: batches of factorizations advancing together through the
// level schedule (one launch sequence per batch); returns the zero-pivot count.
// weak (may be null): per shift, whether the count fails the trust test of
// nu_checked (zero or weak pivot, or large growth).
int64_t inertia_batch_counts(Pencil& P, int32_t nsigma, const double* sigmas, int64_t* nu,
                             int64_t* nzero, uint8_t* weak = nullptr) {
  if (nsigma <= 0) return 0;
  const int cap = factor_batch_capacity(P, nsigma);
  if (!P.batchF || P.batchF->nb < cap) {
    P.batchF.reset(new NumFactor());
    factor_alloc(P, *P.batchF, cap);
  }
  NumFactor& F = *P.batchF;
  int64_t zeros = 0;
  for (int32_t i = 0; i < nsigma; i += F.nb) {
    const int nb = std::min<int32_t>(F.nb, nsigma - i);
    factor_enqueue_batch(P, F, sigmas + i, nb, false);
    factor_read_stats(P, F, nb);
    for (int q = 0; q < nb; q++) {
      const FactStats& h = F.hsb[q];
      nu[i + q] = (int64_t)h.neg;
      if (nzero) nzero[i + q] = (int64_t)h.zero;
      if (weak) {
        const double scale = P.normA_inf + std::fabs(sigmas[i + q]) * P.normB_inf;
        weak[i + q] = weak_count((int64_t)h.zero, bits_to_double(h.min_d_bits),
                                 bits_to_double(h.max_l_bits), scale);
      }
      zeros += (int64_t)h.zero;
    }
  }
  return zeros;
}

void inertia_batch(Pencil& P, int32_t nsigma, const double* sigmas, int64_t* nu) {
  for (int32_t i = 0; i < nsigma; i++)
    if (!std::isfinite(sigmas[i])) throw Error(KTH_EINVAL, "sigma must be finite");
  if (inertia_batch_counts(P, nsigma, sigmas, nu, nullptr) > 0)
    throw Error(KTH_ESINGULAR, "a shift gives an exactly zero pivot");
}

kth_status three_stage(Pencil& P, int64_t k, const kth_opts& o, double* lambda, double* xout,
                       kth_info* info) {
  Ctx* c = P.ctx;
  hipStream_t st = c->stream;
  const int64_t n = P.n;
  const double nA = P.normA_inf;
  Work W;
  W.init(c, n);
  Shifts log;
  int64_t nfac = 0;
  double t_task[7] = {P.S.t_order + P.S.t_symbolic, 0, 0, 0, 0, 0, 0};
  const int n_sv = o.start_vectors ? (o.n_start_vectors > 0 ? o.n_start_vectors : 4) : 0;
  std::function<void(int, std::vector<double>&)> start_vec = [&](int row, std::vector<double>& v) {
    if (row < n_sv) v.assign(o.start_vectors + (size_t)row * n, o.start_vectors + (size_t)(row + 1) * n);
    else gen_start(n, o.seed, row, v);
  };
  std::vector<double> hv;

  // ---- task (ii): factor of B (its inertia must be (0, 0, n)) ----
  // With b_solver = 1 and B strictly diagonally dominant with a positive diagonal
  // (symmetric positive definite by Gershgorin's theorem), B is not factored:
  // the stage-1 B-solves run Jacobi-preconditioned conjugate gradients.
  const bool b_cg = o.b_solver == 1 && P.b_diag_dominant;
  double t0 = now_s();
  // the factor of B and the shift-and-invert factor are kept by the pencil, so
  // later calls replay their captured launch sequences
  if (!P.fb) { P.fb.reset(new NumFactor()); P.fb->replay = true; }
  NumFactor& FB = *P.fb;
  if (!b_cg) {
    factor_alloc(P, FB);
    factor_enqueue(P, FB, 0.0, true);
    factor_read_stats(P, FB);
    nfac++;
    if (FB.hs.neg != 0 || FB.hs.zero != 0) throw Error(KTH_ENOTPD, "B is not positive definite");
  }
  t_task[1] = now_s() - t0;
  // x = B^{-1} rhs (device vectors): the factor's solve, or conjugate gradients
  // to a relative residual of 1e-14
  DBuf<double> cg_r, cg_z, cg_p, cg_q;
  int cg_iters = 0;
  auto bsolve = [&](const double* rhs, double* x) {
    if (!b_cg) {
      solve_enqueue_f(P, FB, rhs, x);
      return;
    }
    if (!cg_r.p) {
      cg_r.alloc(c, n); cg_z.alloc(c, n); cg_p.alloc(c, n); cg_q.alloc(c, n);
    }
    const double* dinv = P.b_dinv.get();
    double* r = cg_r.get();
    double* z = cg_z.get();
    double* p = cg_p.get();
    double* q = cg_q.get();
    vmul(n, dinv, rhs, x, st);                         // x0 = D^{-1} rhs
    spmv2(n, P.rowptr.get(), P.col.get(), P.aval.get(), P.bval.get(), x, nullptr, q, st);
    KTH_HIP(hipMemcpyAsync(r, rhs, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    axpy(n, -1.0, q, r, st);
    vmul(n, dinv, r, z, st);
    KTH_HIP(hipMemcpyAsync(p, z, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    const double bb = dot_dev(W, rhs, rhs);
    double rz = dot_dev(W, r, z);
    for (int it = 0;; it++) {
      if (it >= 1000) throw Error(KTH_ENOCONV, "conjugate gradients on B did not converge");
      spmv2(n, P.rowptr.get(), P.col.get(), P.aval.get(), P.bval.get(), p, nullptr, q, st);
      const double pq = dot_dev(W, p, q);
      if (!(pq > 0)) throw Error(KTH_ENOTPD, "B is not positive definite (conjugate gradients)");
      const double al = rz / pq;
      axpy(n, al, p, x, st);
      axpy(n, -al, q, r, st);
      cg_iters++;
      const double rr = dot_dev(W, r, r);
      if (rr <= 1e-28 * bb) break;
      vmul(n, dinv, r, z, st);
      const double rz2 = dot_dev(W, r, z);
      scale_copy(n, rz2 / rz, p, p, st);
      axpy(n, 1.0, z, p, st);
      rz = rz2;
    }
  };

  double sl, su;
  int64_t nl, nu_;
  int s1 = 0, s2 = 0, s1_restarts = 0;
  // cost model of the stage-2 stopping count (opts.m_max = 0): measured time of
  // one factorization and of one solve in stage 1
  double t_fact_meas = 0, t_solve_meas = 0;
  int64_t m_eff = o.m_max;
  if (o.warm_interval && o.warm_counts) {
    sl = o.warm_interval[0];
    su = o.warm_interval[1];
    nl = o.warm_counts[0];
    nu_ = o.warm_counts[1];
    if (!(sl < su) || !(nl < k && k <= nu_)) throw Error(KTH_EINVAL, "warm interval does not bracket k");
  } else {
    // ---- stage 1: Alg. 2 ----
    int restart = 0;
    bool done = false;
    while (!done) {
      start_vec(restart == 0 ? 0 : 1 + restart, hv);
      h2d(c, W.v(0), hv.data(), n);
      spmv2(n, P.rowptr.get(), P.col.get(), P.aval.get(), P.bval.get(), W.v(0), nullptr, W.vt(0), st);
      double nb = std::sqrt(dot_dev(W, W.v(0), W.vt(0)));
      scale_copy(n, 1.0 / nb, W.v(0), W.v(0), st);
      scale_copy(n, 1.0 / nb, W.vt(0), W.vt(0), st);
      std::vector<double> al, be;
      int64_t nu_prev = 0;
      double sig_prev = 0;
      for (int j = 1;; j++) {
        W.ensure_cols(j + 1);
        // A v_j, alpha_j, w = B^{-1} A v_j
        spmv2(n, P.rowptr.get(), P.col.get(), P.aval.get(), P.bval.get(), W.v(j - 1), W.ya.get(), nullptr, st);
        al.push_back(dot_dev(W, W.v(j - 1), W.ya.get()));
        if (j == 1 && o.m_max == 0 && o.root_finder == 0 && !b_cg) {
          // time of one solve with a factor of the pencil's structure (cost model)
          c->sync();
          const double ts0 = now_s();
          bsolve(W.ya.get(), W.w.get());
          c->sync();
          t_solve_meas = now_s() - ts0;
        } else {
          bsolve(W.ya.get(), W.w.get());
        }
        KTH_HIP(hipMemcpyAsync(W.Bw.get(), W.ya.get(), sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        for (int pass = 0; pass < 2; pass++) {   // CGS2 in the B inner product: h = V^T (B w)
          multidot(n, j, W.V.get(), n, W.Bw.get(), W.partial.get(), W.h.get(), 1.0, st);
          multiaxpy(n, j, W.V.get(), n, W.h.get(), W.w.get(), W.Vt.get(), W.Bw.get(), st);
        }
        // Ritz values of T_j (task iii)
        double tr0 = now_s();
        W.ensure_tri(j);
        h2d(c, W.alpha_d.get(), al.data(), j);
        if (j > 1) h2d(c, W.beta_d.get(), be.data(), j - 1);
        tridiag_eig(j, W.alpha_d.get(), W.beta_d.get(), W.theta_d.get(), W.Y_d.get(), W.twork.get(), st);
        std::vector<double> th(j);
        d2h(c, th.data(), W.theta_d.get(), j);
        t_task[2] += now_s() - tr0;
        double sig = (k <= nu_prev) ? th[0] : th[j - 1];
        double tf = now_s();
        int64_t nu = nu_checked(P, sig, 1e-12 * std::max(nA, 1.0), log, &nfac);
        t_fact_meas = now_s() - tf;
        t_task[3] += t_fact_meas;
        s1 = j;
        if (j != 1 && ((nu < k && k <= nu_prev) || (nu_prev < k && k <= nu))) {
          sl = std::min(sig_prev, sig);
          su = std::max(sig_prev, sig);
          nl = std::min(nu_prev, nu);
          nu_ = std::max(nu_prev, nu);
          done = true;
          break;
        }
        sig_prev = sig;
        nu_prev = nu;
        double beta = std::sqrt(std::max(dot_dev(W, W.w.get(), W.Bw.get()), 0.0));
        if (!(beta > 1e-14 * std::max(1.0, std::fabs(al.back())))) {
          if (++restart > 2) throw Error(KTH_ENOCONV, "stage-1 Lanczos broke down repeatedly");
          s1_restarts = restart;
          break;   // restart with the next seeded vector
        }
        be.push_back(beta);
        scale_copy(n, 1.0 / beta, W.w.get(), W.v(j), st);
        scale_copy(n, 1.0 / beta, W.Bw.get(), W.vt(j), st);
        if (j > n + 1) throw Error(KTH_ENOCONV, "stage 1 exceeded n steps");
      }
    }
    // ---- stage 2: Alg. 1' (repeat-until: at least one bisection step) ----
    double tb = now_s();
    const int ms = std::max(1, o.multisection);
    m_eff = o.m_max > 0 ? o.m_max : auto_m_max(o.root_finder, t_fact_meas, t_solve_meas);
    // interpolating stage 2: two consecutive interpolated steps that each failed to
    // halve the count in the bracket make the next step a bisection (bounds the
    // worst case)
    bool slow[2] = {false, false};
    int nslow = 0;
    while (true) {
      if (ms == 1) {
        const bool bisect = o.root_finder == 0 || (nslow >= 2 && slow[0] && slow[1]);
        double sig = bisect ? 0.5 * (sl + su) : interp_shift(k, sl, su, nl, nu_, m_eff);
        const int64_t gap = nu_ - nl;
        int64_t nu = nu_checked(P, sig, 1e-3 * (su - sl), log, &nfac);
        s2++;
        if (k <= nu) { su = sig; nu_ = nu; } else { sl = sig; nl = nu; }
        if (bisect) {
          nslow = 0;
        } else {
          slow[0] = slow[1];
          slow[1] = 2 * (nu_ - nl) > gap;
          nslow++;
        }
      } else {
        std::vector<double> sg(ms);
        std::vector<int64_t> cnt(ms), zc(ms);
        std::vector<uint8_t> wk(ms);
        for (int i = 0; i < ms; i++) sg[i] = sl + (su - sl) * (double)(i + 1) / (double)(ms + 1);
        inertia_batch_counts(P, ms, sg.data(), cnt.data(), zc.data(), wk.data());
        nfac += ms;
        for (int i = 0; i < ms; i++) {
          if (wk[i]) {   // move that shift and count again on its own
            nfac--;
            cnt[i] = nu_checked(P, sg[i], 1e-3 * (su - sl) / (ms + 1), log, &nfac);
          } else {
            log.s.push_back(sg[i]);
            log.nu.push_back(cnt[i]);
          }
        }
        s2++;
        double nsl = sl, nsu = su;
        int64_t nnl = nl, nnu = nu_;
        for (int i = 0; i < ms; i++) {
          if (k <= cnt[i]) { nsu = sg[i]; nnu = cnt[i]; break; }
          nsl = sg[i];
          nnl = cnt[i];
        }
        sl = nsl; su = nsu; nl = nnl; nu_ = nnu;
      }
      if (nu_ - nl <= m_eff) break;
      if (o.tau_len > 0 && (su - sl) < o.tau_len) break;
      if (s2 > 200) throw Error(KTH_ECLUSTER, "bisection did not isolate a small interval");
    }
    t_task[4] = now_s() - tb;
  }

  // ---- stage 3: Alg. 3 ----
  const int64_t l = k - nl;
  const int m = (int)(nu_ - nl);
  double sigma = 0.5 * (sl + su);
  double tsi = now_s();
  if (!P.fs) { P.fs.reset(new NumFactor()); P.fs->replay = true; }
  NumFactor& FS = *P.fs;
  // the shift-and-invert factor: FP64, or FP32 with FP64 refinement of every solve
  // (falls back to FP64 at the same shift if a refinement stalls)
  auto si_factor = [&](kth_precision prec) {
    factor_alloc(P, FS, 1, prec);
    for (int attempt = 0;; attempt++) {
      factor_enqueue(P, FS, sigma, false);
      factor_read_stats(P, FS);
      nfac++;
      const double md = bits_to_double(FS.hs.min_d_bits), ml = bits_to_double(FS.hs.max_l_bits);
      const double scale = P.normA_inf + std::fabs(sigma) * P.normB_inf;
      // the FP64 factor's count is checked against the interval below, so a weak
      // pivot or large growth there moves the shift too (FP32: zero pivots only)
      const bool weak = prec == KTH_FP64 ? weak_count((int64_t)FS.hs.zero, md, ml, scale)
                                         : FS.hs.zero != 0;
      if (FS.hs.zero == 0 && (!weak || attempt >= kWeakAttempts)) {
        if (prec == KTH_FP64) {
          if (scale > 0) log.min_pivot_rel = std::min(log.min_pivot_rel, md / scale);
          log.max_abs_l = std::max(log.max_abs_l, ml);
          if (weak) log.weak_kept++;
        }
        break;
      }
      if (attempt > 6) throw Error(KTH_ESINGULAR, "shift-and-invert factor keeps hitting zero pivots");
      log.nudges++;
      sigma += 1e-3 * (su - sl);
    }
    // the FP64 count is exact; the FP32 one only serves the factor itself
    if (prec == KTH_FP64 && ((int64_t)FS.hs.neg < nl || (int64_t)FS.hs.neg > nu_))
      throw Error(KTH_EDEVICE, "inertia at the interval midpoint is outside [nu_l, nu_u]");
  };
  si_factor(o.si_precision == KTH_FP32_IR ? KTH_FP32_IR : KTH_FP64);
  int ir_steps = 0, ir_fallback = 0;
  double ir_max_berr = 0;
  t_task[5] = now_s() - tsi;
  double t3 = now_s();
  start_vec(1, hv);
  h2d(c, W.v(0), hv.data(), n);
  spmv2(n, P.rowptr.get(), P.col.get(), P.aval.get(), P.bval.get(), W.v(0), nullptr, W.vt(0), st);
  {
    double nb = std::sqrt(dot_dev(W, W.v(0), W.vt(0)));
    scale_copy(n, 1.0 / nb, W.v(0), W.v(0), st);
    scale_copy(n, 1.0 / nb, W.vt(0), W.vt(0), st);
  }
  std::vector<double> al, be;
  bool have_prev = false;
  int it_bound = 0, it_res = 0, it_diff = 0, j_done = 0;
  bool ever_incl_not_disj = false;
  kth_status result = KTH_ENOCONV;
  double lam_out = 0, eta_out = 0;
  // x = x_{l,2}, B-normalised, largest-|.| entry positive; explicit residual
  auto finish = [&](double* xq) {
    spmv2(n, P.rowptr.get(), P.col.get(), P.aval.get(), P.bval.get(), xq, W.ya.get(), W.yb.get(), st);
    double xbx = dot_dev(W, xq, W.yb.get());
    double xx = dot_dev(W, xq, xq);
    residual(n, lam_out, W.ya.get(), W.yb.get(), W.w.get(), st);
    double rr = dot_dev(W, W.w.get(), W.w.get());
    const double scale = 1.0 / std::sqrt(xbx);
    std::vector<double> hx(n);
    d2h(c, hx.data(), xq, n);
    int64_t imax = 0;
    for (int64_t i = 1; i < n; i++) if (std::fabs(hx[i]) > std::fabs(hx[imax])) imax = i;
    const double sgn = hx[imax] < 0 ? -1.0 : 1.0;
    if (xout) for (int64_t i = 0; i < n; i++) xout[i] = sgn * scale * hx[i];
    info->rel_residual = std::sqrt(rr) / std::sqrt(xx);
    info->rel_residual_normA = info->rel_residual / (nA > 0 ? nA : 1.0);
  };
  // block size: si_block > 1 as given; 0 (automatic) the block method with p = m
  // when stage 2 stopped with more than m_max eigenvalues (a cluster), else
  // Alg. 3 for at most 3 m + 30 steps and the block method after that
  const int64_t mcap = m_eff > 0 ? m_eff : 20;
  int block_p = o.si_block > 1 ? o.si_block : 0;
  if (o.si_block == 0 && m > mcap) block_p = m;
  const int single_cap = o.si_block == 1 ? o.max_lanczos : std::min(o.max_lanczos, 3 * m + 30);
  for (int j = 1; j <= (block_p ? 0 : single_cap); j++) {
    W.ensure_cols(j + 1);
    // w = (A - sigma B)^{-1} v~_j, Bw = B w
    {
      SolveOutcome so = solve_refined(P, FS, W.vt(j - 1), W.w.get(), o.ir_tol > 0 ? o.ir_tol : kIrTol);
      if (!so.converged) {
        // refinement stalled: refactor in FP64 at the same shift and redo this solve
        const double ts = now_s();
        const double sig_keep = sigma;
        si_factor(KTH_FP64);
        if (sigma != sig_keep)
          throw Error(KTH_ESINGULAR, "FP64 fallback factor hit a zero pivot at the FP32 shift");
        t_task[5] += now_s() - ts;
        ir_fallback = 1;
        solve_enqueue_f(P, FS, W.vt(j - 1), W.w.get());
      } else {
        ir_steps += so.steps;
        ir_max_berr = std::max(ir_max_berr, so.berr);
      }
    }
    spmv2(n, P.rowptr.get(), P.col.get(), P.aval.get(), P.bval.get(), W.w.get(), nullptr, W.Bw.get(), st);
    // CGS2 in the B inner product: h = V~^T w = V^T B w
    multidot(n, j, W.Vt.get(), n, W.w.get(), W.partial.get(), W.h.get(), 1.0, st);
    multiaxpy(n, j, W.V.get(), n, W.h.get(), W.w.get(), W.Vt.get(), W.Bw.get(), st);
    multidot(n, j, W.Vt.get(), n, W.w.get(), W.partial.get(), W.h2.get(), 1.0, st);
    multiaxpy(n, j, W.V.get(), n, W.h2.get(), W.w.get(), W.Vt.get(), W.Bw.get(), st);
    double alpha;
    d2h(c, &alpha, W.h.get() + (j - 1), 1);
    al.push_back(alpha);
    double beta = std::sqrt(std::max(dot_dev(W, W.w.get(), W.Bw.get()), 0.0));
    if (beta > 0) {
      scale_copy(n, 1.0 / beta, W.w.get(), W.v(j), st);
      scale_copy(n, 1.0 / beta, W.Bw.get(), W.vt(j), st);
    } else {
      KTH_HIP(hipMemsetAsync(W.v(j), 0, sizeof(double) * n, st));
      KTH_HIP(hipMemsetAsync(W.vt(j), 0, sizeof(double) * n, st));
    }
    j_done = j;
    if (j >= m) {
      W.ensure_tri(j);
      h2d(c, W.alpha_d.get(), al.data(), j);
      if (j > 1) h2d(c, W.beta_d.get(), be.data(), j - 1);
      tridiag_eig(j, W.alpha_d.get(), W.beta_d.get(), W.theta_d.get(), W.Y_d.get(), W.twork.get(), st);
      std::vector<double> th(j), Y((size_t)j * j);
      d2h(c, th.data(), W.theta_d.get(), j);
      d2h(c, Y.data(), W.Y_d.get(), (size_t)j * j);
      std::vector<int> ord(j);
      std::iota(ord.begin(), ord.end(), 0);
      std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
        if (std::fabs(th[a]) != std::fabs(th[b])) return std::fabs(th[a]) > std::fabs(th[b]);
        return th[a] > th[b];
      });
      ord.resize(m);
      std::vector<double> lam(m), s(m), eta(m), C((size_t)j * m), cu(m);
      for (int q = 0; q < m; q++) {
        const int i = ord[q];
        const double yl = Y[(size_t)i * j + (j - 1)];
        lam[q] = sigma + 1.0 / th[i];
        s[q] = beta * yl / th[i];
        eta[q] = (1.0 / std::fabs(th[i])) * std::fabs(s[q]) / std::sqrt(1.0 + s[q] * s[q]);
        for (int cc = 0; cc < j; cc++) C[(size_t)q * j + cc] = th[i] * Y[(size_t)i * j + cc];
        cu[q] = beta * yl;
      }
      bool incl = true;
      for (int q = 0; q < m; q++) incl = incl && (lam[q] - eta[q] >= sl) && (lam[q] + eta[q] < su);
      std::vector<int> asc(m);
      std::iota(asc.begin(), asc.end(), 0);
      std::stable_sort(asc.begin(), asc.end(), [&](int a, int b) { return lam[a] < lam[b]; });
      bool disj = true;
      for (int q = 0; q + 1 < m; q++)
        disj = disj && (lam[asc[q]] + eta[asc[q]] < lam[asc[q + 1]] - eta[asc[q + 1]]);
      if (incl && !disj) ever_incl_not_disj = true;
      // Ritz vectors x_{i,2} (eq. (15)), their norms, residual test (eq. (res2))
      W.ensure_m(m, j);
      h2d(c, W.C_d.get(), C.data(), C.size());
      h2d(c, W.cu_d.get(), cu.data(), m);
      ritz_vectors(n, j, m, W.V.get(), n, W.C_d.get(), W.v(j), W.cu_d.get(), W.X.get(), n, st);
      std::vector<double> xn2(m);
      multidot2(n, m, W.X.get(), n, W.X.get(), n, W.partial.get(), W.sc.get(), 1.0, st);
      d2h(c, xn2.data(), W.sc.get(), m);
      double vtn = std::sqrt(dot_dev(W, W.vt(j), W.vt(j)));
      bool res_ok = true;
      for (int q = 0; q < m; q++) res_ok = res_ok && (std::fabs(s[q]) * vtn / std::sqrt(xn2[q]) < o.tau_res);
      // normalised, ascending copies and the relative difference to the previous step
      std::vector<int32_t> pa(m);
      std::vector<double> fa(m);
      for (int q = 0; q < m; q++) { pa[q] = asc[q]; fa[q] = 1.0 / std::sqrt(xn2[asc[q]]); }
      h2d(c, W.perm_d.get(), pa.data(), m);
      h2d(c, W.f_d.get(), fa.data(), m);
      gather_cols(n, m, W.X.get(), n, W.perm_d.get(), W.f_d.get(), W.Xn.get(), n, st);
      bool diff_ok = false;
      if (have_prev) {
        std::vector<double> dd(m), sg(m);
        multidot2(n, m, W.Xn.get(), n, W.Prev.get(), n, W.partial.get(), W.sc.get(), 1.0, st);
        d2h(c, dd.data(), W.sc.get(), m);
        for (int q = 0; q < m; q++) sg[q] = dd[q] < 0 ? -1.0 : 1.0;
        h2d(c, W.f_d.get(), sg.data(), m);
        diff_cols(n, m, W.Xn.get(), n, W.f_d.get(), W.Prev.get(), n, W.Dif.get(), n, st);
        multidot2(n, m, W.Dif.get(), n, W.Dif.get(), n, W.partial.get(), W.sc.get(), 1.0, st);
        d2h(c, dd.data(), W.sc.get(), m);
        diff_ok = true;
        for (int q = 0; q < m; q++) diff_ok = diff_ok && (std::sqrt(dd[q]) < o.tau_diff);
      }
      W.Xn.swap(W.Prev);
      have_prev = true;
      if (incl && disj && !it_bound) it_bound = j;
      if (res_ok && !it_res) it_res = j;
      if (diff_ok && !it_diff) it_diff = j;
      if (incl && disj && res_ok && diff_ok) {
        const int q = asc[l - 1];
        lam_out = lam[q];
        eta_out = eta[q];
        finish(W.X.get() + (size_t)n * q);
        result = KTH_OK;
        break;
      }
    }
    if (beta == 0) break;
    be.push_back(beta);
  }
  if (result != KTH_OK && o.si_block == 0 && block_p == 0) block_p = m;
  int block_steps = 0;
  if (result != KTH_OK && block_p > 0) {
    auto refactor64 = [&]() {
      const double ts = now_s();
      const double sig_keep = sigma;
      si_factor(KTH_FP64);
      if (sigma != sig_keep)
        throw Error(KTH_ESINGULAR, "FP64 fallback factor hit a zero pivot at the FP32 shift");
      t_task[5] += now_s() - ts;
      ir_fallback = 1;
    };
    BlockOut bo = si_block_run(P, FS, W, k, sl, su, nl, nu_, sigma, block_p, o, start_vec, refactor64);
    block_steps = bo.steps;
    it_bound = bo.it_bound;
    it_res = bo.it_res;
    it_diff = bo.it_diff;
    if (bo.st == KTH_OK) {
      lam_out = bo.lam;
      eta_out = bo.eta;
      finish(W.X.get() + (size_t)n * bo.xcol);
      result = KTH_OK;
    } else {
      ever_incl_not_disj = true;   // the interval's eigenvalues were not resolved
    }
  }
  t_task[6] = now_s() - t3;
  if (result != KTH_OK && ever_incl_not_disj) result = KTH_ECLUSTER;
  *lambda = lam_out;
  info->k_validated = result == KTH_OK ? k : 0;
  info->nu_lower = nl;
  info->nu_upper = nu_;
  info->sigma_lower = sl;
  info->sigma_upper = su;
  info->sigma_si = sigma;
  info->stage1_steps = s1;
  info->bisection_steps = s2;
  info->si_steps = j_done + block_steps;
  info->si_block = block_p > 0 ? block_p : 1;
  info->it_bound = it_bound;
  info->it_residual = it_res;
  info->it_difference = it_diff;
  info->eta = eta_out;
  info->min_pivot_rel = log.min_pivot_rel;
  info->max_abs_l = log.max_abs_l;
  info->weak_pivot_nudges = log.nudges;
  info->weak_pivot_kept = log.weak_kept;
  info->stage1_restarts = s1_restarts;
  info->m_max_used = m_eff;
  info->b_cg_iterations = cg_iters;
  info->n_factorizations = nfac;
  info->flops_factor = P.S.flops;
  for (int q = 0; q < 7; q++) info->t_task[q] = t_task[q];
  info->peak_device_bytes = c->peak_bytes;
  info->n_sigmas = (int32_t)std::min<size_t>(log.s.size(), 128);
  for (int q = 0; q < info->n_sigmas; q++) {
    info->sigmas[q] = log.s[q];
    info->nus[q] = log.nu[q];
  }
  info->si_precision = FS.prec;
  info->ir_steps = ir_steps;
  info->ir_fallback = ir_fallback;
  info->ir_max_berr = ir_max_berr;
  if (result != KTH_OK) {
    c->last_error = result == KTH_ECLUSTER ? "error bounds never became disjoint"
                                           : "shift-and-invert Lanczos did not converge";
  }
  return result;
}

void eig_batch(Ctx& c, const std::vector<Pencil*>& ps, const int64_t* k, const kth_opts& o,
               double* lambda, double* const* x, kth_info* info, kth_status* per) {
  const int np = (int)ps.size();
  // pencils are independent: worker threads, each on its own streams, take them in
  // turn so that the short, latency-bound launches of several pencils overlap
  const int nw = std::min(np, o.batch_workers > 0 ? (int)o.batch_workers : 8);
  std::mutex err_mu;
  auto run_one = [&](int i, Ctx* wc) {
    kth_info tmp;
    kth_info* inf = info ? info + i : &tmp;
    std::memset(inf, 0, sizeof(*inf));
    Pencil& P = *ps[i];
    Ctx* keep = P.ctx;
    if (wc) P.ctx = wc;
    try {
      if (k[i] < 1 || k[i] > P.n) throw Error(KTH_EINVAL, "k out of range");
      per[i] = three_stage(P, k[i], o, lambda + i, x ? x[i] : nullptr, inf);
    } catch (const std::exception& e) {
      const Error* ke = dynamic_cast<const Error*>(&e);
      per[i] = ke ? ke->status : KTH_EDEVICE;
      std::lock_guard<std::mutex> g(err_mu);
      c.last_error = e.what();
    }
    if (wc) {
      (void)hipStreamSynchronize(wc->stream);
      P.ctx = keep;
    }
  };
  if (nw <= 1) {
    for (int i = 0; i < np; i++) run_one(i, nullptr);
    return;
  }
  c.ensure_workers(nw);
  for (int w = 0; w < nw; w++) {
    // the workers' kernels must not start before work the caller queued on its stream
    c.workers[w]->ensure_aux();
    KTH_HIP(hipEventRecord(c.workers[w]->ev_diag, c.stream));
    KTH_HIP(hipStreamWaitEvent(c.workers[w]->stream, c.workers[w]->ev_diag, 0));
  }
  std::atomic<int> next(0);
  std::vector<std::thread> th;
  for (int w = 0; w < nw; w++)
    th.emplace_back([&, w]() {
      (void)hipSetDevice(c.device);
      for (;;) {
        const int i = next.fetch_add(1);
        if (i >= np) break;
        run_one(i, c.workers[w].get());
      }
    });
  for (auto& t : th) t.join();
}

void hf_backward(Pencil& P, double lambda, const double* x, double g, double* ga, double* gb) {
  Ctx* c = P.ctx;
  DBuf<double> xd, gad, gbd;
  xd.upload(c, x, P.n);
  gad.alloc(c, P.nnz);
  gbd.alloc(c, P.nnz);
  hf_gradient(P.n, P.rowptr.get(), P.col.get(), xd.get(), g, lambda, gad.get(), gbd.get(), c->stream);
  if (P.h_amap.empty()) {
    d2h(c, ga, gad.get(), P.nnz);
    d2h(c, gb, gbd.get(), P.nnz);
    return;
  }
  // union entries back to A's and B's own patterns
  std::vector<double> ua(P.nnz), ub(P.nnz);
  d2h(c, ua.data(), gad.get(), P.nnz);
  d2h(c, ub.data(), gbd.get(), P.nnz);
  for (int64_t q = 0; q < P.nnz_a; q++) ga[q] = ua[P.h_amap[q]];
  for (int64_t q = 0; q < P.nnz_b; q++) gb[q] = ub[P.h_bmap[q]];
}

}  // namespace kth
