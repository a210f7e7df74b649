// Host orchestration of the device path: context (device, stream, allocator),
// pencil (pattern analysis, schedule, device arrays) and numeric factors.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/kth.h"
#include "analysis.hpp"
#include "device.hpp"
#include "solve.hpp"

namespace kth {

struct Error : std::runtime_error {
  kth_status status;
  Error(kth_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define KTH_HIP(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::kth::Error(KTH_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  kth_alloc_fn afn = nullptr;
  kth_free_fn ffn = nullptr;
  void* user = nullptr;
  std::string last_error;
  double cur_bytes = 0, peak_bytes = 0;
  // factorizations replay a captured HIP graph of their launch sequence
  // (environment KTH_GRAPHS=0 at context creation: launch kernel by kernel)
  bool use_graphs = true;
  // second stream for the pivot tiles and the panel solves of their next rows (the
  // critical path), and the events that order it against the context stream
  hipStream_t aux = nullptr;
  hipEvent_t ev_diag = nullptr, ev_tile = nullptr, ev_main = nullptr;
  // contexts of the worker threads of kth_eig_batch (own streams, same device and
  // allocator); they live as long as this context, so buffers they allocate for a
  // pencil stay releasable
  std::vector<std::unique_ptr<Ctx>> workers;
  // released blocks of the default allocator kept for reuse: size -> (pointer, unused)
  std::multimap<size_t, std::pair<void*, int>> cache;
  std::unordered_map<void*, size_t> sizes;   // size of every block handed out
  size_t cache_bytes = 0;
  void* alloc(size_t bytes);
  void release(void* p, size_t bytes);
  void trim_cache(size_t keep);   // hipFree cached blocks (largest first) down to keep bytes
  void sync();
  void ensure_aux();
  void destroy_aux();
  void ensure_workers(int nw);
  void destroy_workers();
};

// Device buffer owned through the context's allocator.
template <typename T>
struct DBuf {
  Ctx* ctx = nullptr;
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { reset(); }
  void reset() {
    if (p) ctx->release(p, n * sizeof(T));
    p = nullptr;
    n = 0;
  }
  void alloc(Ctx* c, size_t count) {
    reset();
    ctx = c;
    n = count ? count : 1;
    p = static_cast<T*>(ctx->alloc(n * sizeof(T)));
  }
  void upload(Ctx* c, const T* host, size_t count) {
    alloc(c, count);
    if (count) KTH_HIP(hipMemcpyAsync(p, host, count * sizeof(T), hipMemcpyHostToDevice, c->stream));
  }
  void upload(Ctx* c, const std::vector<T>& v) { upload(c, v.data(), v.size()); }
  T* get() const { return p; }
  void swap(DBuf& o) {
    std::swap(ctx, o.ctx);
    std::swap(p, o.p);
    std::swap(n, o.n);
  }
};

struct StepPlan {
  int32_t t;
  int32_t nfronts;     // active large fronts (prefix of the level's sorted list)
  int32_t trsm_off, trsm_cnt;        // Int2 (front, row) panel-solve tasks of the next tile's rows
  int32_t trsm2_off, trsm2_cnt;      // ... of the rows below those (offsets in int32 units)
  int32_t ll_rest_off, ll_rest_cnt;  // Int2 (front, row): rows below it (t > 0), after the
                                     // tasks (front, row | kLaFlag) of the next tile's
                                     // diagonal block at the same depth
  int32_t ll_nseg;                   // depth segments of the rows-below update
  int32_t ll_segk;                   // their depth (>= kSegK, a multiple of 16)
};

struct LevelPlan {
  int32_t small_off = 0, small_cnt = 0, small_maxnf = 0;
  int32_t init_off = 0, init_cnt = 0;
  int32_t large_off = 0, large_cnt = 0;
  int32_t cb_off = 0, cb_cnt = 0;    // Int2 (front, lower tile) of the contribution blocks
  int32_t cb128_off = 0, cb128_cnt = 0;  // the same on 128 x 128 tiles (nu >= cb128_min_nu)
  std::vector<StepPlan> steps;
};

struct NumFactor;

struct Pencil {
  Ctx* ctx = nullptr;
  int64_t n = 0, nnz = 0;
  Symbolic S;
  std::vector<int64_t> h_rowptr;   // union of the patterns of A and B
  std::vector<int32_t> h_col;
  // A's and B's own patterns inside the union (empty maps: both patterns equal it)
  int64_t nnz_a = 0, nnz_b = 0;
  std::vector<int64_t> h_amap, h_bmap;
  DBuf<int64_t> d_amap, d_bmap;
  double normA_inf = 0, normB_inf = 0;
  bool b_diag_dominant = false;   // B strictly diagonally dominant, positive diagonal
  DBuf<double> b_dinv;            // 1 / diag(B)
  // device CSR and values
  DBuf<int64_t> rowptr;
  DBuf<int32_t> col;
  DBuf<double> aval, bval, zeros;
  // device metadata
  DBuf<int64_t> d_sfirst, d_rptr, d_lptr, d_uptr, d_tptr, d_eptr, d_cptr, d_acptr, d_asrc,
      d_adst, d_perm;
  DBuf<int32_t> d_rows, d_emap, d_clist, d_tilew, d_sched, d_imap, d_l21base;
  DBuf<int64_t> d_iptr;
  FrontMeta meta{};
  std::vector<LevelPlan> levels;
  int64_t cb128_min_nu = 0;          // contribution blocks of >= this many rows: 128 x 128 tiles
  std::vector<int32_t> h_sched;   // host copy of the schedule array
  SolvePlan splan;
  int64_t wsize = 0;   // W = L D workspace (panel-shaped) elements per factorization
  int64_t tsize = 0;   // tile-inverse doubles per factorization
  int64_t psize = 0;   // split-depth partial products per factorization
  int ws_batches = 0;  // factorizations the workspace below holds
  DBuf<double> U, W;   // update-block pool, W = L D panels (ws_batches copies)
  DBuf<double> Tinv;   // inverses of the current pivot tiles (ws_batches copies)
  DBuf<double> Part;   // partial products of split column-block updates (ws_batches copies)
  std::unique_ptr<NumFactor> scratch;   // factor reused by inertia-only calls
  std::unique_ptr<NumFactor> batchF;    // batched inertia-only factorizations (multisection)
  std::unique_ptr<NumFactor> fb, fs;    // kth_eig's factor of B and shift-and-invert factor
  double flops() const { return S.flops; }
};

// Instantiated graph of one factorization's launch sequence (everything after the
// shifts are written to the device), valid for the buffers it was captured with.
constexpr int kGraphKey = 12;
struct FactorGraph {
  hipGraphExec_t exec = nullptr;
  const void* key[kGraphKey] = {};
  int nb = 0;
};

struct NumFactor {
  NumFactor() = default;
  NumFactor(const NumFactor&) = delete;
  NumFactor& operator=(const NumFactor&) = delete;
  ~NumFactor() {
    for (FactorGraph& g : graphs)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
  }
  FactorGraph graphs[2];      // [factor of B itself]
  bool replay = false;        // factorizations go through a captured graph
  Pencil* p = nullptr;
  int nb = 1;                 // batched factorizations held (solves use batch 0)
  double sigma = 0;
  kth_precision prec = KTH_FP64;
  DBuf<double> L, D, E;
  DBuf<int32_t> tperm;
  DBuf<FactStats> stats;
  DBuf<double> sig;           // [nb] shifts on the device
  FactStats hs{};             // batch 0
  std::vector<FactStats> hsb; // all batches
  bool have_stats = false;
  // solve scratch
  DBuf<double> xe, ye, R, partial;
  // refinement scratch (FP32 factors): residual, Krylov basis, dot partials, small results
  DBuf<double> ir_r, ir_V, ir_part, ir_out;
};

// Per-kernel-class timing of one factorization (HIP events on the context stream).
enum { PROF_SMALL = 0, PROF_INIT, PROF_TILE, PROF_TRSM, PROF_GEMM, PROF_REDUCE, PROF_NCLASS };
struct FactorProfile {
  std::vector<hipEvent_t> ev;       // pairs (start, stop)
  std::vector<int> cls;             // class of each pair
  double time[PROF_NCLASS] = {0};   // seconds
  double flops[PROF_NCLASS] = {0};  // dense-front operation counts of the launches
  double bytes[PROF_NCLASS] = {0};  // algorithmic HBM bytes of the launches (where stated)
  int64_t launches[PROF_NCLASS] = {0};
  // the contribution-block share of PROF_GEMM (seconds, operations, launches, bytes)
  std::vector<char> cb;             // per event pair: a contribution-block launch
  double cb_time = 0, cb_flops = 0, cb_bytes = 0;
  int64_t cb_launches = 0;
  double total = 0;                 // seconds, first to last event
  ~FactorProfile();
};

// Host arrays: A on (arp, acol), B on (brp, bcol); the union pattern is analysed.
void pencil_init(Pencil& P, Ctx* ctx, int64_t n, const int64_t* arp, const int32_t* acol,
                 const double* a, const int64_t* brp, const int32_t* bcol, const double* b,
                 uint32_t flags);
// a: nnz_a values on A's pattern, b: nnz_b on B's (host, or device with device_ptrs).
void pencil_set_values(Pencil& P, const double* a, const double* b, bool device_ptrs);
void factor_alloc(Pencil& P, NumFactor& F, int nb = 1, kth_precision prec = KTH_FP64);
// Largest batch of factorizations that fits in free device memory (<= cap).
int factor_batch_capacity(Pencil& P, int cap);
// Enqueue the numeric factorization of A - sigma B (mode_b: factor B itself).
void factor_enqueue(Pencil& P, NumFactor& F, double sigma, bool mode_b,
                    FactorProfile* prof = nullptr);
// Enqueue nb factorizations A - sigma_i B (i < nb <= F.nb) in one launch sequence.
void factor_enqueue_batch(Pencil& P, NumFactor& F, const double* sigmas, int nb, bool mode_b,
                          FactorProfile* prof = nullptr);
// Resolve the events of a profiled factorization (synchronises the stream).
void factor_profile_finish(Pencil& P, FactorProfile& prof);
// Read back the inertia statistics of batch 0 / of nb batches (synchronises the stream).
void factor_read_stats(Pencil& P, NumFactor& F);
void factor_read_stats(Pencil& P, NumFactor& F, int nb);
// x = (A - sigma B)^{-1} b, device vectors (enqueue only).
void solve_enqueue_f(Pencil& P, NumFactor& F, const double* b, double* x);
// The same for nrhs device columns with the work vectors in the per-GPU fixed array
// (noalloc_scratch): no device allocation; enqueue only.  Throws KTH_EINVAL when
// the factor's solve needs more than kNoAllocScratchBytes.
void solve_noalloc(Pencil& P, NumFactor& F, int32_t nrhs, const double* r, int64_t ldr, double* x,
                   int64_t ldx);

}  // namespace kth
