// Host orchestration: allocation, pattern analysis -> device schedule, and the
// level-by-level launch sequence of the numeric factorization.
#include "engine.hpp"

#include "blas.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

namespace kth {

// Default allocator: blocks released by this context are kept for reuse (on this
// context's stream, so stream order covers any pending use) instead of hipFree,
// which would synchronise the whole device and stall other contexts' streams.
static constexpr size_t kCacheLimit = size_t(16) << 30;

void* Ctx::alloc(size_t bytes) {
  void* p = nullptr;
  if (afn) {
    p = afn(bytes, user);
    if (!p) throw Error(KTH_ENOMEM, "device allocator returned NULL for " + std::to_string(bytes) + " bytes");
  } else {
    // a cached block of at least this size and at most twice it
    auto it = cache.lower_bound(bytes);
    if (it != cache.end() && it->first <= 2 * bytes + 4096) {
      p = it->second.first;
      const size_t got = it->first;
      cache_bytes -= got;
      cache.erase(it);
      sizes[p] = got;
    } else {
      hipError_t e = hipMalloc(&p, bytes);
      if ((e != hipSuccess || !p) && !cache.empty()) {
        (void)hipGetLastError();
        trim_cache(0);
        e = hipMalloc(&p, bytes);
      }
      if (e != hipSuccess || !p)
        throw Error(KTH_ENOMEM, "hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
      sizes[p] = bytes;
    }
  }
  cur_bytes += (double)bytes;
  peak_bytes = std::max(peak_bytes, cur_bytes);
  return p;
}

void Ctx::release(void* p, size_t bytes) {
  if (!p) return;
  cur_bytes -= (double)bytes;
  if (ffn) {
    // the caller's allocator may hand the block out again at once: the work that
    // used it (on this context's stream, or a batch worker's) must be finished
    (void)hipStreamSynchronize(stream);
    ffn(p, user);
    return;
  }
  auto it = sizes.find(p);
  const size_t got = it != sizes.end() ? it->second : bytes;
  if (it != sizes.end()) sizes.erase(it);
  cache.emplace(got, std::make_pair(p, 0));
  cache_bytes += got;
  if (cache_bytes > kCacheLimit) trim_cache(kCacheLimit / 2);
}

void Ctx::trim_cache(size_t keep) {
  // largest blocks first
  while (!cache.empty() && cache_bytes > keep) {
    auto it = std::prev(cache.end());
    (void)hipFree(it->second.first);
    cache_bytes -= it->first;
    cache.erase(it);
  }
}

void Ctx::sync() { KTH_HIP(hipStreamSynchronize(stream)); }

void Ctx::ensure_aux() {
  if (aux) return;
  KTH_HIP(hipStreamCreateWithFlags(&aux, hipStreamNonBlocking));
  KTH_HIP(hipEventCreateWithFlags(&ev_diag, hipEventDisableTiming));
  KTH_HIP(hipEventCreateWithFlags(&ev_tile, hipEventDisableTiming));
  KTH_HIP(hipEventCreateWithFlags(&ev_main, hipEventDisableTiming));
}

void Ctx::ensure_workers(int nw) {
  while ((int)workers.size() < nw) {
    std::unique_ptr<Ctx> w(new Ctx());
    w->device = device;
    w->afn = afn;
    w->ffn = ffn;
    w->user = user;
    // worker threads launch kernel by kernel: graphs replayed from several threads at
    // once gave inertia counts read before all of a replay's kernels had finished
    w->use_graphs = false;
    KTH_HIP(hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking));
    w->own_stream = true;
    workers.push_back(std::move(w));
  }
}

void Ctx::destroy_workers() {
  for (auto& w : workers) {
    (void)hipStreamSynchronize(w->stream);
    w->destroy_aux();
    w->trim_cache(0);
    if (w->own_stream) (void)hipStreamDestroy(w->stream);
  }
  workers.clear();
}

void Ctx::destroy_aux() {
  if (!aux) return;
  (void)hipStreamSynchronize(aux);
  (void)hipEventDestroy(ev_diag);
  (void)hipEventDestroy(ev_tile);
  (void)hipEventDestroy(ev_main);
  (void)hipStreamDestroy(aux);
  aux = nullptr;
}

static double csr_norm_inf(int64_t n, const int64_t* rp, const double* v) {
  double m = 0;
  for (int64_t i = 0; i < n; i++) {
    double s = 0;
    for (int64_t q = rp[i]; q < rp[i + 1]; q++) s += std::fabs(v[q]);
    m = std::max(m, s);
  }
  return m;
}

// Contribution blocks with at least this many rows go to 128 x 128 tiles
// (kCb128MinNu; the environment variable KTH_CB128_MIN_NU overrides it, read when
// a pencil is created: a huge value keeps every block on 64 x 64 tiles).
static int64_t cb128_min_nu() {
  const char* e = std::getenv("KTH_CB128_MIN_NU");
  if (!e || !*e) return kCb128MinNu;
  const long long v = std::atoll(e);
  return v < 1 ? 1 : (int64_t)v;
}

// Workgroups a split-depth left-looking launch aims at (KTH_LL_WGS overrides,
// read when a pencil is created).
static int64_t ll_target_wgs() {
  const char* e = std::getenv("KTH_LL_WGS");
  if (!e || !*e) return kLLTargetWgs;
  const long long v = std::atoll(e);
  return v < 1 ? 1 : (int64_t)v;
}

static void build_schedule(Pencil& P) {
  const Symbolic& S = P.S;
  const int64_t nu_big = cb128_min_nu();
  const int64_t ll_wgs = ll_target_wgs();
  P.cb128_min_nu = nu_big;
  std::vector<int32_t> sched;
  auto align2 = [&]() { if (sched.size() & 1) sched.push_back(0); };
  std::vector<std::vector<int32_t>> bylevel(S.nlevels);
  for (int64_t s = 0; s < S.nsup; s++) bylevel[S.level[s]].push_back((int32_t)s);
  std::vector<int64_t> tptr(S.nsup, -1);
  std::vector<int32_t> tilew(S.nsup, 0);
  P.wsize = std::max<int64_t>(1, S.lptr[S.nsup]);   // W = L D, panel-shaped
  P.psize = 1;
  P.tsize = 1;
  P.splan.partial_size = 1;
  P.levels.assign(S.nlevels, LevelPlan());
  for (int64_t L = 0; L < S.nlevels; L++) {
    LevelPlan& lp = P.levels[L];
    std::vector<int32_t> small, large;
    for (int32_t s : bylevel[L]) (S.nf(s) <= kSmallMaxNf ? small : large).push_back(s);
    lp.small_off = (int32_t)sched.size();
    lp.small_cnt = (int32_t)small.size();
    for (int32_t s : small) {
      sched.push_back(s);
      lp.small_maxnf = std::max<int32_t>(lp.small_maxnf, (int32_t)S.nf(s));
      tilew[s] = (int32_t)std::max<int64_t>(S.ns(s), 1);
    }
    std::stable_sort(large.begin(), large.end(), [&](int32_t a, int32_t b) { return S.ns(a) > S.ns(b); });
    lp.large_off = (int32_t)sched.size();
    lp.large_cnt = (int32_t)large.size();
    int64_t toff = 0;
    for (int32_t s : large) {
      sched.push_back(s);
      tilew[s] = kNB;
      tptr[s] = toff;
      toff += 2 * kNB * kNB;   // tile inverses of even and odd steps
    }
    P.tsize = std::max(P.tsize, toff);
    align2();
    lp.init_off = (int32_t)sched.size();
    // assembly tasks: (front, chunk * nrb + row block) for the column chunks of
    // kAsmCols and the row blocks of kAsmRows that meet the lower triangle
    for (int32_t s : large) {
      const int64_t nf = S.nf(s), nrb = (nf + kAsmRows - 1) / kAsmRows;
      const int64_t nch = (nf + kAsmCols - 1) / kAsmCols;
      if (nch * nrb > INT32_MAX) throw Error(KTH_EINVAL, "front too large for the assembly schedule");
      for (int64_t ch = 0; ch < nch; ch++)
        for (int64_t rb = ch * kAsmCols / kAsmRows; rb < nrb; rb++) {
          sched.push_back(s);
          sched.push_back((int32_t)(ch * nrb + rb));
        }
    }
    lp.init_cnt = (int32_t)((sched.size() - lp.init_off) / 2);
    int64_t tmax = 0;
    for (int32_t s : large) tmax = std::max<int64_t>(tmax, (S.ns(s) + kNB - 1) / kNB);
    for (int64_t t = 0; t < tmax; t++) {
      StepPlan sp{};
      sp.t = (int32_t)t;
      int32_t act = 0;
      while (act < (int32_t)large.size() && S.ns(large[act]) > t * kNB) act++;
      sp.nfronts = act;
      align2();
      // panel solve: the first kTrsmRows rows below the tile (the next tile's rows,
      // which the next diagonal-block update needs) apart from the rest
      sp.trsm_off = (int32_t)sched.size();
      for (int32_t q = 0; q < act; q++) {
        int32_t s = large[q];
        int64_t ns = S.ns(s), nf = S.nf(s);
        int64_t k0 = t * kNB, kb = std::min<int64_t>(kNB, ns - k0);
        if (k0 + kb < nf) { sched.push_back(s); sched.push_back((int32_t)(k0 + kb)); }
      }
      sp.trsm_cnt = (int32_t)((sched.size() - sp.trsm_off) / 2);
      sp.trsm2_off = (int32_t)sched.size();
      for (int32_t q = 0; q < act; q++) {
        int32_t s = large[q];
        int64_t ns = S.ns(s), nf = S.nf(s);
        int64_t k0 = t * kNB, kb = std::min<int64_t>(kNB, ns - k0);
        for (int64_t r = k0 + kb + kTrsmRows; r < nf; r += kTrsmRows) { sched.push_back(s); sched.push_back((int32_t)r); }
      }
      sp.trsm2_cnt = (int32_t)((sched.size() - sp.trsm2_off) / 2);
      // left-looking update at depth t * kNB (steps after the first): the rows below
      // this tile in kTile chunks and, ahead of the next tile, its diagonal block
      // (the columns of tile t reach that block in the panel solve of step t)
      sp.ll_rest_off = (int32_t)sched.size();
      if (t > 0) {
        // the next tile's diagonal block at this depth (the next tile's fronts: a
        // prefix of the list), then the rows below this tile
        int32_t act_next = 0;
        while (act_next < (int32_t)large.size() && S.ns(large[act_next]) > (t + 1) * kNB) act_next++;
        for (int32_t q = 0; q < act_next; q++) {
          sched.push_back(large[q]);
          sched.push_back((int32_t)((t + 1) * kNB) | kLaFlag);
        }
      }
      if (t > 0)
        for (int32_t q = 0; q < act; q++) {
          const int32_t s = large[q];
          for (int64_t r = t * kNB + kTile; r < S.nf(s); r += kTile) { sched.push_back(s); sched.push_back((int32_t)r); }
        }
      sp.ll_rest_cnt = (int32_t)((sched.size() - sp.ll_rest_off) / 2);
      const int64_t depth = (int64_t)t * kNB;
      // as many depth segments (each at least kSegK deep, a multiple of 16) as bring
      // the launch to about ll_wgs workgroups
      {
        const int64_t most = std::max<int64_t>(1, (depth + kSegK - 1) / kSegK);
        const int64_t want = (ll_wgs + std::max<int64_t>(sp.ll_rest_cnt, 1) - 1) /
                             std::max<int64_t>(sp.ll_rest_cnt, 1);
        const int64_t ns_ = std::min(most, std::max<int64_t>(1, want));
        sp.ll_segk = (int32_t)std::max<int64_t>(kSegK, ((depth + ns_ - 1) / ns_ + 15) / 16 * 16);
        sp.ll_nseg = std::max<int32_t>(1, (int32_t)((depth + sp.ll_segk - 1) / sp.ll_segk));
      }
      if (sp.ll_nseg > 1)
        P.psize = std::max<int64_t>(P.psize, (int64_t)sp.ll_rest_cnt * sp.ll_nseg * kTile * kTile);
      lp.steps.push_back(sp);
    }
    // contribution blocks: lower tiles of each nu x nu block (depth ns), 64 x 64 or,
    // for nu >= nu_big, 128 x 128
    align2();
    lp.cb_off = (int32_t)sched.size();
    for (int32_t s : large) {
      const int64_t nu = S.nf(s) - S.ns(s), T = (nu + kTile - 1) / kTile;
      if (nu >= nu_big) continue;
      for (int64_t tl = 0; tl < T * (T + 1) / 2; tl++) { sched.push_back(s); sched.push_back((int32_t)tl); }
    }
    lp.cb_cnt = (int32_t)((sched.size() - lp.cb_off) / 2);
    lp.cb128_off = (int32_t)sched.size();
    for (int32_t s : large) {
      const int64_t nu = S.nf(s) - S.ns(s), T = (nu + 127) / 128;
      if (nu < nu_big) continue;
      if (T * (T + 1) / 2 > INT32_MAX) throw Error(KTH_EINVAL, "front too large for the tile schedule");
      for (int64_t tl = 0; tl < T * (T + 1) / 2; tl++) { sched.push_back(s); sched.push_back((int32_t)tl); }
    }
    lp.cb128_cnt = (int32_t)((sched.size() - lp.cb128_off) / 2);
  }
  std::vector<int32_t> l21base(S.nsup, 0);
  int64_t l21_part = 0;
  // solve plan: small fronts reuse the factorization lists; large fronts get
  // gather tasks of kSolveChunk rows and reuse the panel tasks of each step
  P.splan.levels.assign(S.nlevels, SolveLevel());
  for (int64_t L = 0; L < S.nlevels; L++) {
    const LevelPlan& lp = P.levels[L];
    SolveLevel& sl = P.splan.levels[L];
    sl.small_off = lp.small_off;
    sl.small_cnt = lp.small_cnt;
    sl.large_off = lp.large_off;
    sl.large_cnt = lp.large_cnt;
    align2();
    sl.init_off = (int32_t)sched.size();
    for (int32_t q = 0; q < lp.large_cnt; q++) {
      int32_t s = sched[lp.large_off + q];
      for (int64_t r = 0; r < S.nf(s); r += kSolveChunk) { sched.push_back(s); sched.push_back((int32_t)r); }
    }
    sl.init_cnt = (int32_t)((sched.size() - sl.init_off) / 2);
    // the chain steps take the tiles two at a time (tiles t and t + 1, t even)
    for (size_t qs = 0; qs < lp.steps.size(); qs += 2) {
      const StepPlan& sp = lp.steps[qs];
      SolveStep ss;
      ss.t = sp.t;
      ss.nfronts = sp.nfronts;
      const int64_t k0 = sp.t * (int64_t)kNB;
      // forward: rows below the two tiles inside the pivot block only (the rows
      // below the block take the level's L21 launches)
      align2();
      ss.fwd_off = (int32_t)sched.size();
      for (int32_t q = 0; q < sp.nfronts; q++) {
        const int32_t s = sched[lp.large_off + q];
        const int64_t ns = S.ns(s);
        const int64_t rb = std::min<int64_t>(k0 + 2 * kNB, ns);
        if (rb >= ns) { sched.push_back(s); sched.push_back((int32_t)ns); }
        for (int64_t r = rb; r < ns; r += kNB) { sched.push_back(s); sched.push_back((int32_t)r); }
      }
      ss.fwd_cnt = (int32_t)((sched.size() - ss.fwd_off) / 2);
      // backward: the pivot-block columns before the tile, 64 at a time
      align2();
      ss.bwd_off = (int32_t)sched.size();
      for (int32_t q = 0; q < sp.nfronts; q++) {
        const int32_t s = sched[lp.large_off + q];
        if (k0 == 0) { sched.push_back(s); sched.push_back(0); }
        for (int64_t c = 0; c < k0; c += kNB) { sched.push_back(s); sched.push_back((int32_t)c); }
      }
      ss.bwd_cnt = (int32_t)((sched.size() - ss.bwd_off) / 2);
      sl.steps.push_back(ss);
    }
    // L21 tasks: kL21Rows-row chunks of the rows below each pivot block
    align2();
    sl.l21_off = (int32_t)sched.size();
    for (int32_t q = 0; q < lp.large_cnt; q++) {
      const int32_t s = sched[lp.large_off + q];
      const int64_t ns = S.ns(s), nf = S.nf(s);
      l21base[s] = (int32_t)((sched.size() - sl.l21_off) / 2);
      if (nf <= ns) continue;
      sl.l21_nseg = std::max<int32_t>(sl.l21_nseg, (int32_t)((ns + kL21Cols - 1) / kL21Cols));
      sl.l21_ntile = std::max<int32_t>(sl.l21_ntile, (int32_t)((ns + kNB - 1) / kNB));
      for (int64_t r = ns; r < nf; r += kL21Rows) { sched.push_back(s); sched.push_back((int32_t)r); }
    }
    sl.l21_cnt = (int32_t)((sched.size() - sl.l21_off) / 2);
    l21_part = std::max<int64_t>(l21_part, (int64_t)sl.l21_cnt *
                                               std::max<int64_t>((int64_t)sl.l21_nseg * kL21Rows,
                                                                 (int64_t)sl.l21_ntile * kNB));
  }
  P.splan.l21_part_off = 0;
  P.splan.partial_size = std::max<int64_t>(1, l21_part);
  Ctx* c = P.ctx;
  P.d_sched.upload(c, sched);
  P.h_sched = sched;
  P.d_tptr.upload(c, tptr);
  P.d_tilew.upload(c, tilew);
  P.d_l21base.upload(c, l21base);
  P.splan.sched = P.d_sched.get();
  P.splan.l21base = P.d_l21base.get();
}

// Rows of one CSR pattern: in range, strictly increasing columns.
static void check_rows(int64_t n, const int64_t* rp, const int32_t* col, const char* name) {
  if (!rp || !col) throw Error(KTH_EINVAL, std::string("null pattern of ") + name);
  if (rp[0] != 0) throw Error(KTH_EINVAL, std::string(name) + ": rowptr[0] must be 0");
  for (int64_t i = 0; i < n; i++) {
    if (rp[i + 1] < rp[i]) throw Error(KTH_EINVAL, std::string(name) + ": rowptr is not non-decreasing");
    for (int64_t q = rp[i]; q < rp[i + 1]; q++) {
      if (col[q] < 0 || col[q] >= n)
        throw Error(KTH_EINVAL, std::string(name) + ": column index out of range in row " + std::to_string(i));
      if (q > rp[i] && col[q - 1] >= col[q])
        throw Error(KTH_EINVAL, std::string(name) + ": columns not strictly increasing in row " + std::to_string(i));
    }
  }
}

void pencil_init(Pencil& P, Ctx* ctx, int64_t n, const int64_t* arp, const int32_t* acol,
                 const double* a, const int64_t* brp, const int32_t* bcol, const double* b,
                 uint32_t flags) {
  P.ctx = ctx;
  P.n = n;
  if (n <= 0) throw Error(KTH_EINVAL, "n must be positive");
  check_rows(n, arp, acol, "A");
  check_rows(n, brp, bcol, "B");
  P.nnz_a = arp[n];
  P.nnz_b = brp[n];
  const bool same = (arp == brp && acol == bcol) ||
                    (P.nnz_a == P.nnz_b && std::equal(arp, arp + n + 1, brp) &&
                     std::equal(acol, acol + P.nnz_a, bcol));
  P.h_amap.clear();
  P.h_bmap.clear();
  if (same) {
    P.h_rowptr.assign(arp, arp + n + 1);
    P.h_col.assign(acol, acol + P.nnz_a);
  } else {
    // row-wise merge of the two sorted column lists; maps from each pattern into it
    P.h_rowptr.assign(n + 1, 0);
    P.h_col.clear();
    P.h_col.reserve(std::max(P.nnz_a, P.nnz_b));
    P.h_amap.resize(P.nnz_a);
    P.h_bmap.resize(P.nnz_b);
    for (int64_t i = 0; i < n; i++) {
      int64_t qa = arp[i], qb = brp[i];
      while (qa < arp[i + 1] || qb < brp[i + 1]) {
        const int32_t ca = qa < arp[i + 1] ? acol[qa] : INT32_MAX;
        const int32_t cb = qb < brp[i + 1] ? bcol[qb] : INT32_MAX;
        const int32_t c = std::min(ca, cb);
        const int64_t u = (int64_t)P.h_col.size();
        P.h_col.push_back(c);
        if (ca == c) P.h_amap[qa++] = u;
        if (cb == c) P.h_bmap[qb++] = u;
      }
      P.h_rowptr[i + 1] = (int64_t)P.h_col.size();
    }
  }
  P.nnz = P.h_rowptr[n];
  Pattern pat;
  pat.n = n;
  pat.rowptr = P.h_rowptr.data();
  pat.col = P.h_col.data();
  std::string msg = check_pattern(pat, (flags & KTH_CHECK_SYMMETRY) != 0);
  if (!msg.empty()) throw Error(KTH_EINVAL, msg);
  if (!P.h_amap.empty()) {
    P.d_amap.upload(ctx, P.h_amap);
    P.d_bmap.upload(ctx, P.h_bmap);
  }
  pat.rowptr = P.h_rowptr.data();
  pat.col = P.h_col.data();
  AnalysisOpts o;
  analyze(pat, o, P.S);
  const Symbolic& S = P.S;
  P.rowptr.upload(ctx, P.h_rowptr);
  P.col.upload(ctx, P.h_col);
  P.aval.alloc(ctx, P.nnz);
  P.bval.alloc(ctx, P.nnz);
  P.zeros.alloc(ctx, P.nnz);
  KTH_HIP(hipMemsetAsync(P.zeros.get(), 0, P.nnz * sizeof(double), ctx->stream));
  pencil_set_values(P, a, b, false);
  P.d_sfirst.upload(ctx, S.sfirst);
  P.d_rptr.upload(ctx, S.rptr);
  P.d_rows.upload(ctx, S.rows);
  P.d_lptr.upload(ctx, S.lptr);
  P.d_uptr.upload(ctx, S.uptr);
  P.d_eptr.upload(ctx, S.eptr);
  P.d_emap.upload(ctx, S.emap);
  P.d_cptr.upload(ctx, S.cptr);
  P.d_clist.upload(ctx, S.clist);
  P.d_acptr.upload(ctx, S.acptr);
  P.d_asrc.upload(ctx, S.asrc);
  P.d_adst.upload(ctx, S.adst);
  P.d_perm.upload(ctx, S.perm);
  {
    // inverse extend-add maps of the children of large fronts (assembly by gather)
    std::vector<int64_t> iptr(S.nsup, -1);
    std::vector<int32_t> imap;
    for (int64_t c = 0; c < S.nsup; c++) {
      const int64_t par = S.sparent[c];
      if (par < 0 || S.nf(par) <= kSmallMaxNf) continue;
      const int64_t nuc = S.nf(c) - S.ns(c);
      iptr[c] = (int64_t)imap.size();
      imap.resize(imap.size() + S.nf(par), -1);
      for (int64_t a = 0; a < nuc; a++) imap[iptr[c] + S.emap[S.eptr[c] + a]] = (int32_t)a;
    }
    P.d_iptr.upload(ctx, iptr);
    P.d_imap.upload(ctx, imap);
  }
  build_schedule(P);
  P.meta.sfirst = P.d_sfirst.get();
  P.meta.rptr = P.d_rptr.get();
  P.meta.rows = P.d_rows.get();
  P.meta.lptr = P.d_lptr.get();
  P.meta.uptr = P.d_uptr.get();
  P.meta.eptr = P.d_eptr.get();
  P.meta.emap = P.d_emap.get();
  P.meta.cptr = P.d_cptr.get();
  P.meta.clist = P.d_clist.get();
  P.meta.acptr = P.d_acptr.get();
  P.meta.asrc = P.d_asrc.get();
  P.meta.adst = P.d_adst.get();
  P.meta.tilew = P.d_tilew.get();
  P.meta.tptr = P.d_tptr.get();
  P.meta.iptr = P.d_iptr.get();
  P.meta.imap = P.d_imap.get();
  P.ws_batches = 0;
  P.scratch.reset(new NumFactor());
  P.scratch->replay = true;
  factor_alloc(P, *P.scratch);
  ctx->sync();
}

// B strictly diagonally dominant with a positive diagonal (then symmetric positive
// definite by Gershgorin's theorem), and 1 / diag(B) on the device for the Jacobi
// preconditioner of the conjugate-gradient B-solve.
static void b_dominance(Pencil& P, const double* b) {
  std::vector<double> dinv(P.n, 0.0);
  bool dd = true;
  for (int64_t i = 0; i < P.n; i++) {
    double di = 0, off = 0;
    for (int64_t q = P.h_rowptr[i]; q < P.h_rowptr[i + 1]; q++) {
      if (P.h_col[q] == i) di = b[q];
      else off += std::fabs(b[q]);
    }
    if (!(di > off)) dd = false;
    dinv[i] = di != 0 ? 1.0 / di : 0.0;
  }
  P.b_diag_dominant = dd;
  P.b_dinv.upload(P.ctx, dinv);
}

void pencil_set_values(Pencil& P, const double* a, const double* b, bool device_ptrs) {
  Ctx* c = P.ctx;
  const size_t bytes = P.nnz * sizeof(double);
  if (P.h_amap.empty() && !device_ptrs) {
    KTH_HIP(hipMemcpyAsync(P.aval.get(), a, bytes, hipMemcpyHostToDevice, c->stream));
    KTH_HIP(hipMemcpyAsync(P.bval.get(), b, bytes, hipMemcpyHostToDevice, c->stream));
    P.normA_inf = csr_norm_inf(P.n, P.h_rowptr.data(), a);
    P.normB_inf = csr_norm_inf(P.n, P.h_rowptr.data(), b);
    b_dominance(P, b);
    c->sync();
    return;
  }
  if (!device_ptrs) {
    std::vector<double> ua(P.nnz, 0.0), ub(P.nnz, 0.0);
    for (int64_t q = 0; q < P.nnz_a; q++) ua[P.h_amap[q]] = a[q];
    for (int64_t q = 0; q < P.nnz_b; q++) ub[P.h_bmap[q]] = b[q];
    KTH_HIP(hipMemcpyAsync(P.aval.get(), ua.data(), bytes, hipMemcpyHostToDevice, c->stream));
    KTH_HIP(hipMemcpyAsync(P.bval.get(), ub.data(), bytes, hipMemcpyHostToDevice, c->stream));
    P.normA_inf = csr_norm_inf(P.n, P.h_rowptr.data(), ua.data());
    P.normB_inf = csr_norm_inf(P.n, P.h_rowptr.data(), ub.data());
    b_dominance(P, ub.data());
    c->sync();   // the host staging arrays go out of scope
    return;
  }
  if (P.h_amap.empty()) {
    KTH_HIP(hipMemcpyAsync(P.aval.get(), a, bytes, hipMemcpyDeviceToDevice, c->stream));
    KTH_HIP(hipMemcpyAsync(P.bval.get(), b, bytes, hipMemcpyDeviceToDevice, c->stream));
  } else {
    KTH_HIP(hipMemsetAsync(P.aval.get(), 0, bytes, c->stream));
    KTH_HIP(hipMemsetAsync(P.bval.get(), 0, bytes, c->stream));
    scatter_values(P.nnz_a, P.d_amap.get(), a, P.aval.get(), c->stream);
    scatter_values(P.nnz_b, P.d_bmap.get(), b, P.bval.get(), c->stream);
  }
  // norms on the union arrays as they now sit on the device
  std::vector<double> ha(P.nnz), hb(P.nnz);
  KTH_HIP(hipMemcpyAsync(ha.data(), P.aval.get(), bytes, hipMemcpyDeviceToHost, c->stream));
  KTH_HIP(hipMemcpyAsync(hb.data(), P.bval.get(), bytes, hipMemcpyDeviceToHost, c->stream));
  c->sync();
  P.normA_inf = csr_norm_inf(P.n, P.h_rowptr.data(), ha.data());
  P.normB_inf = csr_norm_inf(P.n, P.h_rowptr.data(), hb.data());
  b_dominance(P, hb.data());
  c->sync();
}

static void ensure_workspace(Pencil& P, int nb) {
  if (nb <= P.ws_batches) return;
  Ctx* c = P.ctx;
  P.U.alloc(c, (size_t)P.S.pool_size * nb);
  P.W.alloc(c, (size_t)P.wsize * nb);
  P.Tinv.alloc(c, (size_t)std::max<int64_t>(P.tsize, 1) * nb);
  P.Part.alloc(c, (size_t)P.psize * nb);
  P.ws_batches = nb;
}

void factor_alloc(Pencil& P, NumFactor& F, int nb, kth_precision prec) {
  Ctx* c = P.ctx;
  if (nb < 1 || nb > kMaxBatch) throw Error(KTH_EINVAL, "batch of factorizations out of range");
  if (F.p == &P && F.nb == nb && F.prec == prec && F.L.p) {   // already laid out
    ensure_workspace(P, nb);
    return;
  }
  // a new layout (pencil, batch or precision): captured launch sequences belong to
  // the old one -- its kernels may be of the other precision even where the new
  // buffers land at the old addresses -- so they are dropped
  if (F.graphs[0].exec || F.graphs[1].exec) {
    KTH_HIP(hipStreamSynchronize(c->stream));
    for (FactorGraph& g : F.graphs)
      if (g.exec) {
        (void)hipGraphExecDestroy(g.exec);
        g.exec = nullptr;
        g.nb = 0;
      }
  }
  F.p = &P;
  F.nb = nb;
  F.prec = prec;
  const size_t lsz = (size_t)P.S.lptr[P.S.nsup] * nb;
  F.L.alloc(c, prec == KTH_FP64 ? lsz : (lsz + 1) / 2);   // float panels in the same buffer type
  F.D.alloc(c, (size_t)P.n * nb);
  F.E.alloc(c, (size_t)P.n * nb);
  F.tperm.alloc(c, (size_t)P.n * nb);
  F.stats.alloc(c, nb);
  F.sig.alloc(c, nb);
  ensure_workspace(P, nb);
}

int factor_batch_capacity(Pencil& P, int cap) {
  size_t fr = 0, tot = 0;
  KTH_HIP(hipMemGetInfo(&fr, &tot));
  const double per = 8.0 * ((double)P.S.lptr[P.S.nsup] + (double)P.S.pool_size + (double)P.wsize +
                            (double)P.tsize + (double)P.psize + 3.0 * (double)P.n);
  // already-held workspace counts as available for the batch it serves
  const double have =
      8.0 * ((double)P.S.pool_size + (double)P.wsize + (double)P.tsize + (double)P.psize) * P.ws_batches;
  int k = (int)((0.8 * (double)fr + have) / per);
  return std::max(1, std::min(k, std::min(cap, kMaxBatch)));
}

FactorProfile::~FactorProfile() {
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
}

namespace {
struct ProfScope {
  FactorProfile* p;
  hipStream_t st;
  int cls;
  ProfScope(FactorProfile* pr, hipStream_t s, int c, double flops, double bytes = 0.0,
            bool cb = false)
      : p(pr), st(s), cls(c) {
    if (!p) return;
    hipEvent_t e;
    KTH_HIP(hipEventCreate(&e));
    KTH_HIP(hipEventRecord(e, st));
    p->ev.push_back(e);
    p->cls.push_back(c);
    p->cb.push_back(cb ? 1 : 0);
    p->flops[c] += flops;
    p->bytes[c] += bytes;
    p->launches[c]++;
    if (cb) { p->cb_flops += flops; p->cb_bytes += bytes; p->cb_launches++; }
  }
  ~ProfScope() {
    if (!p) return;
    hipEvent_t e;
    if (hipEventCreate(&e) == hipSuccess) {
      (void)hipEventRecord(e, st);
      p->ev.push_back(e);
    }
  }
};
}  // namespace

void factor_enqueue(Pencil& P, NumFactor& F, double sigma, bool mode_b, FactorProfile* prof) {
  factor_enqueue_batch(P, F, &sigma, 1, mode_b, prof);
}

template <typename T>
static void factor_body(Pencil& P, NumFactor& F, int nb, const double* av, const double* bv,
                        FactorProfile* prof);

template <typename T>
static void factor_enqueue_t(Pencil& P, NumFactor& F, const double* sigmas, int nb, bool mode_b,
                             FactorProfile* prof) {
  Ctx* c = P.ctx;
  hipStream_t st = c->stream;
  if (nb < 1 || nb > F.nb) throw Error(KTH_EINVAL, "batch larger than the factor storage");
  ensure_workspace(P, nb);
  F.sigma = sigmas[0];
  F.have_stats = false;
  double sv[kMaxBatch];
  for (int i = 0; i < nb; i++) sv[i] = mode_b ? -1.0 : sigmas[i];   // B = fma(-(-1), b, 0)
  const double* av = mode_b ? P.zeros.get() : P.aval.get();
  const double* bv = P.bval.get();
  launch_set_scalars(F.sig.get(), nb, sv, st);
  c->ensure_aux();
  // the rest of the sequence depends on the shifts only through F.sig: for a factor
  // that is used again and again (the pencil's inertia-only factor), captured once
  // into a graph and replayed (not when every launch is timed)
  const bool graph = c->use_graphs && F.replay && !prof;
  const void* key[kGraphKey] = {F.L.get(), P.U.get(), P.W.get(), P.Tinv.get(), P.Part.get(),
                                F.stats.get(), F.sig.get(), av, bv, F.D.get(), F.E.get(), F.tperm.get()};
  FactorGraph& fg = F.graphs[mode_b ? 1 : 0];
  if (graph && fg.exec && fg.nb == nb && std::equal(key, key + kGraphKey, fg.key)) {
    KTH_HIP(hipGraphLaunch(fg.exec, st));
    return;
  }
  if (graph) {
    if (fg.exec) {
      KTH_HIP(hipGraphExecDestroy(fg.exec));
      fg.exec = nullptr;
    }
    KTH_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  }
  try {
    factor_body<T>(P, F, nb, av, bv, prof);
  } catch (...) {
    if (graph) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(st, &g);
      if (g) (void)hipGraphDestroy(g);
    }
    throw;
  }
  if (graph) {
    hipGraph_t g = nullptr;
    KTH_HIP(hipStreamEndCapture(st, &g));
    const hipError_t ie = hipGraphInstantiate(&fg.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    KTH_HIP(ie);
    std::copy(key, key + kGraphKey, fg.key);
    fg.nb = nb;
    KTH_HIP(hipGraphLaunch(fg.exec, st));
  }
}

template <typename T>
static void factor_body(Pencil& P, NumFactor& F, int nb, const double* av, const double* bv,
                        FactorProfile* prof) {
  Ctx* c = P.ctx;
  hipStream_t st = c->stream;
  const Symbolic& S = P.S;
  launch_fill_stats(F.stats.get(), nb, st);
  Batch bt;
  bt.sL = P.S.lptr[P.S.nsup];
  bt.sU = P.S.pool_size;
  bt.sW = P.wsize;
  bt.sT = std::max<int64_t>(P.tsize, 1);
  bt.sP = P.psize;
  bt.sN = P.n;
  bt.sig = F.sig.get();
  const int32_t* sched = P.d_sched.get();
  T* Lf = reinterpret_cast<T*>(F.L.get());
  T* Uf = reinterpret_cast<T*>(P.U.get());
  T* Wf = reinterpret_cast<T*>(P.W.get());
  T* Tf = reinterpret_cast<T*>(P.Tinv.get());
  T* Pf = reinterpret_cast<T*>(P.Part.get());
  const std::vector<int32_t>& hs = P.h_sched;
  for (const LevelPlan& lp : P.levels) {
    if (lp.small_cnt > 0) {
      double fl = 0;
      if (prof)
        for (int32_t q = 0; q < lp.small_cnt; q++) {
          const int32_t s = hs[lp.small_off + q];
          for (int64_t j = 0; j < S.ns(s); j++) { double cc = (double)(S.nf(s) - 1 - j); fl += cc * cc + 2 * cc; }
        }
      ProfScope ps(prof, st, PROF_SMALL, fl);
      launch_small_fronts(P.meta, sched + lp.small_off, lp.small_cnt, lp.small_maxnf, av, bv, bt,
                          nb, Lf, Uf, F.D.get(), F.E.get(), F.tperm.get(),
                          F.stats.get(), st);
    }
    if (lp.large_cnt == 0) continue;
    {
      ProfScope ps(prof, st, PROF_INIT, 0.0);
      launch_front_init(P.meta, reinterpret_cast<const Int2*>(sched + lp.init_off), lp.init_cnt, av,
                        bv, bt, nb, Lf, Uf, st);
    }
    // Left-looking steps with look-ahead: the panel solve of tile q's next rows
    // finishes the diagonal block of tile q+1 (its columns < q*kNB were applied a
    // step earlier); tile q+1 is factored while the rest of tile q's rows are
    // solved and the rows below tile q+1 (and, ahead, the diagonal block of tile
    // q+2) are updated.  Contribution blocks follow the last step.
    // per step: operation counts and, for the column-block update, its algorithmic
    // bytes (each C entry read and written once, the depth-k0 rows of L below and
    // of W in the tile read once; diagonal-block counts are kept apart)
    struct StepCost { double tile = 0, trsm = 0, ll = 0, ll_bytes = 0, lld = 0, lla = 0, lla_bytes = 0; };
    auto step_cost = [&](const StepPlan& sp) {
      StepCost c;
      if (!prof) return c;
      for (int32_t q = 0; q < sp.nfronts; q++) {
        const int32_t s = hs[lp.large_off + q];
        const double ns = (double)S.ns(s), nf = (double)S.nf(s);
        const double k0 = (double)sp.t * kNB, kb = std::min<double>(kNB, ns - k0);
        const double R = nf - k0 - kb;   // rows below the tile
        for (int64_t j = 0; j < (int64_t)kb; j++) { double cc = kb - 1 - j; c.tile += cc * cc + 2 * cc; }
        c.trsm += R * (kb * kb + kb);      // R rows: triangular solve + diagonal scaling
        const double rd = std::min<double>(kTile, nf - k0);   // rows of the diagonal task
        const double ed = kb * rd - kb * (kb - 1) / 2, er = kb * (nf - k0 - rd);
        const double ka = std::max<double>(0.0, k0 - kNB);   // depth of the look-ahead part
        c.lld += 2.0 * k0 * ed;
        c.lla += 2.0 * ka * ed;
        c.ll += 2.0 * k0 * er;
        c.lla_bytes += 16.0 * ed + 8.0 * ka * (rd + kb);
        c.ll_bytes += 16.0 * er + 8.0 * k0 * ((nf - k0 - rd) + kb);
      }
      return c;
    };
    // The chain of a level runs on the auxiliary stream: tile q's factorization,
    // the panel solve of its next rows (which finishes tile q+1's diagonal block),
    // tile q+1's factorization, ...; each next-rows solve also waits for the
    // context stream's previous step (the rows below tile q, the look-ahead
    // diagonal block).  The context stream solves the rest of tile q's rows and
    // updates the rows below tile q+1 (and, ahead, tile q+2's diagonal block).
    KTH_HIP(hipEventRecord(c->ev_main, st));   // the level's fronts assembled
    KTH_HIP(hipStreamWaitEvent(c->aux, c->ev_main, 0));
    if (!lp.steps.empty()) {
      const StepPlan& s0 = lp.steps[0];
      ProfScope ps(prof, c->aux, PROF_TILE, step_cost(s0).tile);
      launch_tile_factor(P.meta, sched + lp.large_off, s0.nfronts, s0.t, bt, nb, Lf,
                         F.D.get(), F.E.get(), F.tperm.get(), Tf, F.stats.get(), c->aux);
    }
    KTH_HIP(hipEventRecord(c->ev_tile, c->aux));
    for (size_t q = 0; q < lp.steps.size(); q++) {
      const StepPlan& sp = lp.steps[q];
      const StepCost cs = step_cost(sp);
      const bool has_next = q + 1 < lp.steps.size();
      const StepCost cn = has_next ? step_cost(lp.steps[q + 1]) : StepCost{};
      if (q > 0) {   // the rows below tile q and tile q+1's earlier depth are in
        KTH_HIP(hipEventRecord(c->ev_main, st));
        KTH_HIP(hipStreamWaitEvent(c->aux, c->ev_main, 0));
      }
      {
        // the next tile's rows, which also apply this tile's columns to the next
        // diagonal block (the rest of its update was applied during this tile)
        ProfScope ps(prof, c->aux, PROF_TRSM, cs.trsm + (cn.lld - cn.lla));
        launch_panel_trsm(P.meta, reinterpret_cast<const Int2*>(sched + sp.trsm_off), sp.trsm_cnt,
                          sp.t, bt, nb, Lf, Wf, F.D.get(), F.E.get(), F.tperm.get(),
                          Tf, F.stats.get(), 1, c->aux);
      }
      KTH_HIP(hipEventRecord(c->ev_diag, c->aux));
      // the rest of the panel solve, after tile q is factored (it reads tile q's
      // inverse from the slot of q's parity while tile q+1's is written)
      KTH_HIP(hipStreamWaitEvent(st, c->ev_tile, 0));
      if (has_next) {
        const StepPlan& nx = lp.steps[q + 1];
        ProfScope ps(prof, c->aux, PROF_TILE, cn.tile);
        launch_tile_factor(P.meta, sched + lp.large_off, nx.nfronts, nx.t, bt, nb, Lf,
                           F.D.get(), F.E.get(), F.tperm.get(), Tf, F.stats.get(), c->aux);
      }
      KTH_HIP(hipEventRecord(c->ev_tile, c->aux));
      {
        ProfScope ps(prof, st, PROF_TRSM, 0.0);
        launch_panel_trsm(P.meta, reinterpret_cast<const Int2*>(sched + sp.trsm2_off), sp.trsm2_cnt,
                          sp.t, bt, nb, Lf, Wf, F.D.get(), F.E.get(), F.tperm.get(),
                          Tf, F.stats.get(), 0, st);
      }
      KTH_HIP(hipStreamWaitEvent(st, c->ev_diag, 0));   // the next rows' L and W
      if (has_next) {
        const StepPlan& nx = lp.steps[q + 1];
        const Int2* rtask = reinterpret_cast<const Int2*>(sched + nx.ll_rest_off);
        {
          // the rows below tile q + 1 and, ahead, the diagonal block of tile q + 2 at
          // the same depth (columns of tiles <= q; tile q's rows there were just solved)
          const StepCost c2 = q + 2 < lp.steps.size() ? step_cost(lp.steps[q + 2]) : StepCost{};
          ProfScope ps(prof, st, PROF_GEMM, cn.ll + c2.lla, cn.ll_bytes + c2.lla_bytes);
          launch_gemm_lt(P.meta, rtask, nx.ll_rest_cnt, nx.t, 1, nx.ll_nseg, nx.ll_segk, bt, nb, Lf, Uf,
                         Wf, Pf, st);
        }
        if (nx.ll_nseg > 1 && nx.ll_rest_cnt > 0) {
          ProfScope ps(prof, st, PROF_REDUCE, 0.0);
          launch_gemm_reduce(P.meta, rtask, nx.ll_rest_cnt, nx.t, nx.ll_nseg, bt, nb, Lf, Pf, st);
        }
      }
    }
    KTH_HIP(hipStreamWaitEvent(st, c->ev_tile, 0));   // everything on the second stream
    // contribution blocks, operation counts and algorithmic bytes: C once; L_u and
    // W_u once
    auto cb_cost = [&](bool big, double& fl, double& by) {
      fl = by = 0;
      if (!prof) return;
      for (int32_t q = 0; q < lp.large_cnt; q++) {
        const int32_t s = hs[lp.large_off + q];
        const double ns = (double)S.ns(s), nu = (double)(S.nf(s) - S.ns(s));
        if ((nu >= (double)P.cb128_min_nu) != big) continue;
        fl += 2.0 * ns * nu * (nu + 1) / 2;
        by += 16.0 * nu * (nu + 1) / 2 + 2.0 * 8.0 * ns * nu;
      }
    };
    if (lp.cb_cnt > 0) {
      double fl_cb, by_cb;
      cb_cost(false, fl_cb, by_cb);
      ProfScope ps(prof, st, PROF_GEMM, fl_cb, by_cb, true);
      launch_gemm_lt(P.meta, reinterpret_cast<const Int2*>(sched + lp.cb_off), lp.cb_cnt, 0, 2, 1, 0,
                     bt, nb, Lf, Uf, Wf, Pf, st);
    }
    if (lp.cb128_cnt > 0) {
      double fl_cb, by_cb;
      cb_cost(true, fl_cb, by_cb);
      ProfScope ps(prof, st, PROF_GEMM, fl_cb, by_cb, true);
      launch_gemm_cb128(P.meta, reinterpret_cast<const Int2*>(sched + lp.cb128_off), lp.cb128_cnt, bt,
                        nb, Lf, Uf, Wf, st);
    }
  }
  KTH_HIP(hipGetLastError());
}

void factor_enqueue_batch(Pencil& P, NumFactor& F, const double* sigmas, int nb, bool mode_b,
                          FactorProfile* prof) {
  if (F.prec == KTH_FP64) factor_enqueue_t<double>(P, F, sigmas, nb, mode_b, prof);
  else factor_enqueue_t<float>(P, F, sigmas, nb, mode_b, prof);
}

void factor_profile_finish(Pencil& P, FactorProfile& prof) {
  P.ctx->sync();
  for (size_t q = 0; q + 1 < prof.ev.size(); q += 2) {
    float ms = 0;
    KTH_HIP(hipEventElapsedTime(&ms, prof.ev[q], prof.ev[q + 1]));
    prof.time[prof.cls[q / 2]] += ms * 1e-3;
    if (prof.cb[q / 2]) prof.cb_time += ms * 1e-3;
  }
  if (prof.ev.size() >= 2) {
    float ms = 0;
    KTH_HIP(hipEventElapsedTime(&ms, prof.ev.front(), prof.ev.back()));
    prof.total = ms * 1e-3;
  }
}

void factor_read_stats(Pencil& P, NumFactor& F, int nb) {
  F.hsb.resize(nb);
  KTH_HIP(hipMemcpyAsync(F.hsb.data(), F.stats.get(), sizeof(FactStats) * nb, hipMemcpyDeviceToHost,
                         P.ctx->stream));
  P.ctx->sync();
  F.hs = F.hsb[0];
  F.have_stats = true;
  for (int i = 0; i < nb; i++) {
    const FactStats& h = F.hsb[i];
    if ((int64_t)(h.neg + h.zero + h.pos) != P.n)
      throw Error(KTH_EDEVICE, "inertia counts do not add up to n (" + std::to_string(h.neg) + "+" +
                                   std::to_string(h.zero) + "+" + std::to_string(h.pos) + ")");
  }
}

void factor_read_stats(Pencil& P, NumFactor& F) { factor_read_stats(P, F, 1); }

void solve_enqueue_f(Pencil& P, NumFactor& F, const double* b, double* x) {
  Ctx* c = P.ctx;
  if (!F.xe.p) {
    F.xe.alloc(c, (size_t)P.n);
    F.ye.alloc(c, (size_t)P.n);
    F.R.alloc(c, P.S.rows.size());
    F.partial.alloc(c, (size_t)P.splan.partial_size);
  }
  if (F.prec == KTH_FP64)
    solve_enqueue<double>(P.splan, P.meta, F.L.get(), F.D.get(), F.E.get(), F.tperm.get(),
                          P.d_perm.get(), P.n, b, x, F.xe.get(), F.ye.get(), F.R.get(),
                          F.partial.get(), c->stream);
  else
    solve_enqueue<float>(P.splan, P.meta, reinterpret_cast<const float*>(F.L.get()), F.D.get(),
                         F.E.get(), F.tperm.get(), P.d_perm.get(), P.n, b, x, F.xe.get(),
                         F.ye.get(), F.R.get(), F.partial.get(), c->stream);
}

void solve_noalloc(Pencil& P, NumFactor& F, int32_t nrhs, const double* r, int64_t ldr, double* x,
                   int64_t ldx) {
  double* base = noalloc_scratch(P.ctx->device);
  if (!base) throw Error(KTH_ESTATE, "no work array address for this device");
  auto up = [](size_t v) { return (v + 31) / 32 * 32; };   // 256-byte pieces
  const size_t n = (size_t)P.n;
  const size_t o_ye = up(n), o_r = o_ye + up(n), o_p = o_r + up(P.S.rows.size());
  const size_t need = o_p + up((size_t)P.splan.partial_size);
  if (need * sizeof(double) > kNoAllocScratchBytes)
    throw Error(KTH_EINVAL, "this factor's solve needs " + std::to_string(need * sizeof(double)) +
                                " bytes of work array; the allocation-free solve has " +
                                std::to_string(kNoAllocScratchBytes));
  for (int32_t q = 0; q < nrhs; q++) {
    const double* b = r + (size_t)q * ldr;
    double* xq = x + (size_t)q * ldx;
    if (F.prec == KTH_FP64)
      solve_enqueue<double>(P.splan, P.meta, F.L.get(), F.D.get(), F.E.get(), F.tperm.get(),
                            P.d_perm.get(), P.n, b, xq, base, base + o_ye, base + o_r, base + o_p,
                            P.ctx->stream);
    else
      solve_enqueue<float>(P.splan, P.meta, reinterpret_cast<const float*>(F.L.get()), F.D.get(),
                           F.E.get(), F.tperm.get(), P.d_perm.get(), P.n, b, xq, base, base + o_ye,
                           base + o_r, base + o_p, P.ctx->stream);
  }
}

}  // namespace kth
