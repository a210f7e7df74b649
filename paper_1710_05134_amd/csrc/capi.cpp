// extern "C" entry points of libkth.so (declared in include/kth.h).  Each call
// converts exceptions into a kth_status and keeps the message on its context.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>

#include "../../include/kth.h"
#include "blas.hpp"
#include "driver.hpp"
#include "engine.hpp"

using namespace kth;

static_assert(KTH_NOALLOC_SCRATCH_BYTES == kNoAllocScratchBytes,
              "the header's work-array size must match the library's");

// Handles are reference counted: a pencil holds its context, a factor its pencil,
// so the device memory of a child is released through a live parent whatever the
// order in which the caller destroys them.
struct kth_ctx_s {
  Ctx c;
  int refs = 1;
};
struct kth_pencil_s {
  kth_ctx_s* ctx;
  Pencil p;
  int refs = 1;
};
struct kth_factor_s {
  kth_pencil_s* pen;
  NumFactor f;
};

namespace {

thread_local std::string g_noctx_error;

template <typename F>
kth_status guarded(Ctx* c, F&& fn) {
  try {
    fn();
    if (c) c->last_error.clear();
    return KTH_OK;
  } catch (const Error& e) {
    if (c) c->last_error = e.what(); else g_noctx_error = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    if (c) c->last_error = "host allocation failed"; else g_noctx_error = "host allocation failed";
    return KTH_ENOMEM;
  } catch (const std::exception& e) {
    if (c) c->last_error = e.what(); else g_noctx_error = e.what();
    return KTH_EINVAL;
  }
}

void set_device(Ctx& c) { KTH_HIP(hipSetDevice(c.device)); }

void check_opts(const kth_opts& o) {
  if (o.m_max < 0) throw Error(KTH_EINVAL, "m_max must be >= 0 (0: automatic)");
  if (!(o.tau_res > 0) || !(o.tau_diff > 0)) throw Error(KTH_EINVAL, "tolerances must be > 0");
  if (!(o.tau_len >= 0)) throw Error(KTH_EINVAL, "tau_len must be >= 0");
  if (o.max_lanczos < 1) throw Error(KTH_EINVAL, "max_lanczos must be >= 1");
  if (o.multisection < 1 || o.multisection > kMaxBatch)
    throw Error(KTH_EINVAL, "multisection must be in [1, 64]");
  if (o.si_precision != KTH_FP64 && o.si_precision != KTH_FP32_IR)
    throw Error(KTH_EINVAL, "unknown si_precision");
  if (!(o.ir_tol >= 0) || !std::isfinite(o.ir_tol)) throw Error(KTH_EINVAL, "ir_tol must be >= 0");
  if (o.batch_workers < 0 || o.batch_workers > 64) throw Error(KTH_EINVAL, "batch_workers must be in [0, 64]");
  if (o.root_finder != 0 && o.root_finder != 1) throw Error(KTH_EINVAL, "root_finder must be 0 or 1");
  if (o.si_block < 0 || o.si_block > 64) throw Error(KTH_EINVAL, "si_block must be in [0, 64]");
  if (o.n_start_vectors < 0) throw Error(KTH_EINVAL, "n_start_vectors must be >= 0");
  if (o.b_solver != 0 && o.b_solver != 1) throw Error(KTH_EINVAL, "b_solver must be 0 or 1");
  if (o.root_finder == 1 && o.multisection != 1)
    throw Error(KTH_EINVAL, "the interpolating root-finder takes one shift per step (multisection = 1)");
}

void ctx_release(kth_ctx_s* c) {
  if (--c->refs > 0) return;
  (void)hipSetDevice(c->c.device);
  c->c.destroy_workers();
  c->c.destroy_aux();
  (void)hipStreamSynchronize(c->c.stream);
  c->c.trim_cache(0);
  if (c->c.own_stream) (void)hipStreamDestroy(c->c.stream);
  delete c;
}

void pencil_release(kth_pencil_s* p) {
  if (--p->refs > 0) return;
  kth_ctx_s* c = p->ctx;
  (void)hipSetDevice(c->c.device);
  (void)hipStreamSynchronize(c->c.stream);
  delete p;
  ctx_release(c);
}

}  // namespace

extern "C" {

const char* kth_status_string(kth_status s) {
  switch (s) {
    case KTH_OK: return "ok";
    case KTH_EINVAL: return "invalid argument";
    case KTH_ENOMEM: return "out of memory";
    case KTH_EDEVICE: return "device error";
    case KTH_ENOTPD: return "B is not positive definite";
    case KTH_ESINGULAR: return "zero pivot (shift is an eigenvalue to working precision)";
    case KTH_ENOCONV: return "no convergence";
    case KTH_ECLUSTER: return "error bounds never disjoint (cluster or multiple eigenvalue)";
    case KTH_ESTATE: return "invalid state";
  }
  return "unknown status";
}

const char* kth_last_error(kth_ctx ctx) { return ctx ? ctx->c.last_error.c_str() : g_noctx_error.c_str(); }

kth_status kth_ctx_create(int device, void* hip_stream, kth_alloc_fn alloc, kth_free_fn free_fn,
                          void* user, kth_ctx* out) {
  if (!out) return KTH_EINVAL;
  *out = nullptr;
  if ((alloc == nullptr) != (free_fn == nullptr)) {
    g_noctx_error = "alloc and free must both be given or both be NULL";
    return KTH_EINVAL;
  }
  std::unique_ptr<kth_ctx_s> c(new kth_ctx_s());
  kth_status st = guarded(nullptr, [&] {
    int ndev = 0;
    KTH_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) throw Error(KTH_EDEVICE, "no HIP device " + std::to_string(device));
    hipDeviceProp_t prop;
    KTH_HIP(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      throw Error(KTH_EDEVICE, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
    c->c.device = device;
    KTH_HIP(hipSetDevice(device));
    // address of this device's work array for kth_solve_noalloc (once per device)
    KTH_HIP(noalloc_scratch_init(device));
    if (hip_stream) {
      c->c.stream = static_cast<hipStream_t>(hip_stream);
    } else {
      KTH_HIP(hipStreamCreateWithFlags(&c->c.stream, hipStreamNonBlocking));
      c->c.own_stream = true;
    }
    c->c.afn = alloc;
    c->c.ffn = free_fn;
    c->c.user = user;
    const char* g = std::getenv("KTH_GRAPHS");
    c->c.use_graphs = !(g && g[0] == '0');
  });
  if (st == KTH_OK) *out = c.release();
  return st;
}

kth_status kth_ctx_destroy(kth_ctx ctx) {
  if (!ctx) return KTH_EINVAL;
  ctx_release(ctx);
  return KTH_OK;
}

kth_status kth_analyze(int64_t n, const int64_t* rowptr, const int32_t* col, uint32_t flags,
                       double* stats, int64_t* perm_out) {
  return guarded(nullptr, [&] {
    if (!rowptr || !col || !stats) throw Error(KTH_EINVAL, "null argument");
    Pattern pat;
    pat.n = n;
    pat.rowptr = rowptr;
    pat.col = col;
    std::string msg = check_pattern(pat, (flags & KTH_CHECK_SYMMETRY) != 0);
    if (!msg.empty()) throw Error(KTH_EINVAL, msg);
    Symbolic S;
    AnalysisOpts o;
    analyze(pat, o, S);
    stats[0] = (double)n;
    stats[1] = (double)rowptr[n];
    stats[2] = (double)S.n_supervars;
    stats[3] = (double)S.nsup_fundamental;
    stats[4] = (double)S.nsup;
    stats[5] = (double)S.max_front;
    stats[6] = (double)S.max_ns;
    stats[7] = (double)S.nlevels;
    stats[8] = S.flops;
    stats[9] = S.flops_padded;
    stats[10] = (double)S.nnz_l;
    stats[11] = (double)S.nnz_l_padded;
    stats[12] = 8.0 * (double)S.pool_size;
    stats[13] = 8.0 * (double)S.lptr[S.nsup];
    stats[14] = S.t_order;
    stats[15] = S.t_symbolic;
    if (perm_out) std::memcpy(perm_out, S.perm.data(), sizeof(int64_t) * n);
  });
}

kth_status kth_pencil_create(kth_ctx ctx, int64_t n, const int64_t* a_rowptr, const int32_t* a_col,
                             const double* a_val, const int64_t* b_rowptr, const int32_t* b_col,
                             const double* b_val, uint32_t flags, kth_pencil* out) {
  if (!ctx || !out) return KTH_EINVAL;
  *out = nullptr;
  std::unique_ptr<kth_pencil_s> p(new kth_pencil_s());
  p->ctx = ctx;
  kth_status st = guarded(&ctx->c, [&] {
    if (!a_rowptr || !a_col || !a_val || !b_rowptr || !b_col || !b_val)
      throw Error(KTH_EINVAL, "null argument");
    if (n <= 0) throw Error(KTH_EINVAL, "n must be positive");
    set_device(ctx->c);
    if (flags & KTH_DEVICE_PTRS) {
      // device inputs: the analysis runs on the host, so bring them over first
      std::vector<int64_t> arp(n + 1), brp(n + 1);
      KTH_HIP(hipMemcpy(arp.data(), a_rowptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
      KTH_HIP(hipMemcpy(brp.data(), b_rowptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
      if (arp[n] < 0 || brp[n] < 0) throw Error(KTH_EINVAL, "rowptr[n] is negative");
      std::vector<int32_t> ac(arp[n]), bc(brp[n]);
      std::vector<double> av(arp[n]), bv(brp[n]);
      KTH_HIP(hipMemcpy(ac.data(), a_col, sizeof(int32_t) * arp[n], hipMemcpyDeviceToHost));
      KTH_HIP(hipMemcpy(bc.data(), b_col, sizeof(int32_t) * brp[n], hipMemcpyDeviceToHost));
      KTH_HIP(hipMemcpy(av.data(), a_val, sizeof(double) * arp[n], hipMemcpyDeviceToHost));
      KTH_HIP(hipMemcpy(bv.data(), b_val, sizeof(double) * brp[n], hipMemcpyDeviceToHost));
      pencil_init(p->p, &ctx->c, n, arp.data(), ac.data(), av.data(), brp.data(), bc.data(), bv.data(),
                  flags);
    } else {
      pencil_init(p->p, &ctx->c, n, a_rowptr, a_col, a_val, b_rowptr, b_col, b_val, flags);
    }
  });
  if (st == KTH_OK) {
    ctx->refs++;
    *out = p.release();
  }
  return st;
}

kth_status kth_pencil_set_values(kth_pencil p, const double* a_val, const double* b_val,
                                 uint32_t flags) {
  if (!p) return KTH_EINVAL;
  return guarded(&p->ctx->c, [&] {
    if (!a_val || !b_val) throw Error(KTH_EINVAL, "null argument");
    set_device(p->ctx->c);
    pencil_set_values(p->p, a_val, b_val, (flags & KTH_DEVICE_PTRS) != 0);
    p->ctx->c.sync();
  });
}

kth_status kth_pencil_destroy(kth_pencil p) {
  if (!p) return KTH_EINVAL;
  pencil_release(p);
  return KTH_OK;
}

kth_status kth_inertia(kth_pencil p, double sigma, int64_t* nu, int64_t* nzero) {
  if (!p || !nu) return KTH_EINVAL;
  kth_status st = guarded(&p->ctx->c, [&] {
    if (!std::isfinite(sigma)) throw Error(KTH_EINVAL, "sigma must be finite");
    set_device(p->ctx->c);
    NumFactor& F = *p->p.scratch;
    factor_enqueue(p->p, F, sigma, false);
    factor_read_stats(p->p, F);
    *nu = (int64_t)F.hs.neg;
    if (nzero) *nzero = (int64_t)F.hs.zero;
  });
  if (st == KTH_OK && p->p.scratch->hs.zero > 0) {
    p->ctx->c.last_error = "zero pivot in LDL^T of A - sigma B";
    return KTH_ESINGULAR;
  }
  return st;
}

kth_status kth_inertia_batch(kth_pencil p, int32_t nsigma, const double* sigmas, int64_t* nu) {
  if (!p || !sigmas || !nu || nsigma < 0) return KTH_EINVAL;
  return guarded(&p->ctx->c, [&] {
    set_device(p->ctx->c);
    inertia_batch(p->p, nsigma, sigmas, nu);
  });
}

kth_status kth_factor(kth_pencil p, double sigma, kth_precision prec, kth_factor_t* out) {
  if (!p || !out) return KTH_EINVAL;
  *out = nullptr;
  std::unique_ptr<kth_factor_s> f(new kth_factor_s());
  f->pen = p;
  kth_status st = guarded(&p->ctx->c, [&] {
    if (!std::isfinite(sigma)) throw Error(KTH_EINVAL, "sigma must be finite");
    if (prec != KTH_FP64 && prec != KTH_FP32_IR) throw Error(KTH_EINVAL, "unknown precision");
    set_device(p->ctx->c);
    numeric_factor(p->p, f->f, sigma, prec);
  });
  if (st == KTH_OK) {
    p->refs++;
    *out = f.release();
  }
  return st;
}

kth_status kth_factor_inertia(kth_factor_t f, int64_t* neg, int64_t* zero, int64_t* pos) {
  if (!f) return KTH_EINVAL;
  if (f->f.prec != KTH_FP64 || !f->f.have_stats) {
    f->pen->ctx->c.last_error = "inertia is only kept for FP64 factors";
    return KTH_ESTATE;
  }
  if (neg) *neg = (int64_t)f->f.hs.neg;
  if (zero) *zero = (int64_t)f->f.hs.zero;
  if (pos) *pos = (int64_t)f->f.hs.pos;
  return KTH_OK;
}

kth_status kth_solve(kth_factor_t f, int32_t nrhs, const double* r, int64_t ldr, double* x,
                     int64_t ldx, uint32_t flags) {
  if (!f || !r || !x || nrhs < 0) return KTH_EINVAL;
  kth_pencil_s* p = f->pen;
  return guarded(&p->ctx->c, [&] {
    if (ldr < p->p.n || ldx < p->p.n) throw Error(KTH_EINVAL, "leading dimension smaller than n");
    set_device(p->ctx->c);
    solve_many(p->p, f->f, nrhs, r, ldr, x, ldx, (flags & KTH_DEVICE_PTRS) != 0,
               (flags & KTH_SOLVE_UNREFINED) != 0);
  });
}

kth_status kth_solve_noalloc(kth_factor_t f, int32_t nrhs, const double* r, int64_t ldr, double* x,
                             int64_t ldx, uint32_t flags) {
  if (!f || !r || !x || nrhs < 0) return KTH_EINVAL;
  kth_pencil_s* p = f->pen;
  return guarded(&p->ctx->c, [&] {
    if (ldr < p->p.n || ldx < p->p.n) throw Error(KTH_EINVAL, "leading dimension smaller than n");
    if (f->f.prec != KTH_FP64 && !(flags & KTH_SOLVE_UNREFINED))
      throw Error(KTH_EINVAL, "an FP32 factor needs KTH_SOLVE_UNREFINED here (refinement allocates)");
    set_device(p->ctx->c);
    solve_noalloc(p->p, f->f, nrhs, r, ldr, x, ldx);
  });
}

kth_status kth_factor_destroy(kth_factor_t f) {
  if (!f) return KTH_EINVAL;
  kth_pencil_s* p = f->pen;
  (void)hipSetDevice(p->ctx->c.device);
  (void)hipStreamSynchronize(p->ctx->c.stream);
  delete f;
  pencil_release(p);
  return KTH_OK;
}

kth_status kth_factor_stats(kth_factor_t f, int64_t* n2x2, double* min_pivot_rel, double* max_abs_l) {
  if (!f) return KTH_EINVAL;
  if (!f->f.have_stats) {
    f->pen->ctx->c.last_error = "factor has no statistics";
    return KTH_ESTATE;
  }
  const FactStats& h = f->f.hs;
  double md, ml;
  std::memcpy(&md, &h.min_d_bits, sizeof(md));
  std::memcpy(&ml, &h.max_l_bits, sizeof(ml));
  const Pencil& P = f->pen->p;
  const double scale = P.normA_inf + std::fabs(f->f.sigma) * P.normB_inf;
  if (n2x2) *n2x2 = (int64_t)h.n2x2;
  if (min_pivot_rel) *min_pivot_rel = scale > 0 ? md / scale : md;
  if (max_abs_l) *max_abs_l = ml;
  return KTH_OK;
}

void kth_opts_default(kth_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->m_max = 20;
  o->tau_res = 1e-10;
  o->tau_diff = 1e-10;
  o->tau_len = 0.0;
  o->max_lanczos = 500;
  o->multisection = 1;
  o->seed = 0;
  o->si_precision = KTH_FP64;
}

kth_status kth_eig(kth_pencil p, int64_t k, const kth_opts* opts, double* lambda, double* x,
                   kth_info* info) {
  if (!p || !lambda) return KTH_EINVAL;
  kth_opts o;
  if (opts) o = *opts; else kth_opts_default(&o);
  kth_info tmp;
  kth_info* inf = info ? info : &tmp;
  std::memset(inf, 0, sizeof(*inf));
  kth_status st = KTH_OK;
  kth_status g = guarded(&p->ctx->c, [&] {
    if (k < 1 || k > p->p.n) throw Error(KTH_EINVAL, "k out of range");
    check_opts(o);
    set_device(p->ctx->c);
    st = three_stage(p->p, k, o, lambda, x, inf);
  });
  return g != KTH_OK ? g : st;
}

kth_status kth_eig_batch(kth_ctx ctx, int32_t np, const kth_pencil* p, const int64_t* k,
                         const kth_opts* opts, double* lambda, double* const* x, kth_info* info,
                         kth_status* per_pencil) {
  if (!ctx || np < 0 || (np > 0 && (!p || !k || !lambda || !per_pencil))) return KTH_EINVAL;
  kth_opts o;
  if (opts) o = *opts; else kth_opts_default(&o);
  std::string batch_msg;
  kth_status st = guarded(&ctx->c, [&] {
    check_opts(o);
    set_device(ctx->c);
    std::vector<Pencil*> ps(np);
    for (int32_t i = 0; i < np; i++) {
      if (!p[i] || p[i]->ctx != ctx) throw Error(KTH_EINVAL, "pencil from another context");
      ps[i] = &p[i]->p;
    }
    // a pencil's workspaces (scratch factor, update pool, panels) serve one run at a time
    std::vector<Pencil*> sorted(ps);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
      throw Error(KTH_EINVAL, "the same pencil appears more than once in the batch");
    ctx->c.last_error.clear();
    eig_batch(ctx->c, ps, k, o, lambda, x, info, per_pencil);
    batch_msg = ctx->c.last_error;
  });
  if (st == KTH_OK) ctx->c.last_error = batch_msg;   // a failing pencil's message, if any
  return st;
}

kth_status kth_eig_backward(kth_pencil p, double lambda, const double* x, double g,
                            double* grad_a, double* grad_b) {
  if (!p || !x || !grad_a || !grad_b) return KTH_EINVAL;
  return guarded(&p->ctx->c, [&] {
    set_device(p->ctx->c);
    hf_backward(p->p, lambda, x, g, grad_a, grad_b);
  });
}

kth_status kth_profile_factor(kth_pencil p, double sigma, double* out, int32_t nout) {
  if (!p || !out || nout < 28) return KTH_EINVAL;
  return guarded(&p->ctx->c, [&] {
    set_device(p->ctx->c);
    FactorProfile prof;
    NumFactor& F = *p->p.scratch;
    factor_enqueue(p->p, F, sigma, false, &prof);
    factor_profile_finish(p->p, prof);
    factor_read_stats(p->p, F);
    for (int q = 0; q < nout; q++) out[q] = 0.0;
    out[0] = prof.total;
    out[1] = p->p.S.flops;
    out[2] = p->p.S.flops_padded;
    for (int c = 0; c < PROF_NCLASS; c++) {
      out[3 + 4 * c] = prof.time[c];
      out[4 + 4 * c] = prof.flops[c];
      out[5 + 4 * c] = (double)prof.launches[c];
      out[6 + 4 * c] = prof.bytes[c];
    }
    out[27] = (double)F.hs.neg;
    if (nout >= 32) {
      out[28] = prof.cb_time;
      out[29] = prof.cb_flops;
      out[30] = (double)prof.cb_launches;
      out[31] = prof.cb_bytes;
    }
  });
}

kth_status kth_profile_solve(kth_factor_t f, int32_t reps, double* out, int32_t nout) {
  if (!f || !out || nout < 6 || reps < 1) return KTH_EINVAL;
  kth_pencil_s* pp = f->pen;
  return guarded(&pp->ctx->c, [&] {
    set_device(pp->ctx->c);
    Pencil& P = pp->p;
    Ctx* c = P.ctx;
    hipStream_t st = c->stream;
    DBuf<double> b, x, y;
    b.alloc(c, P.n);
    x.alloc(c, P.n);
    y.alloc(c, P.n);
    // right-hand side e_1 (the sweeps read the whole factor whatever the vector)
    KTH_HIP(hipMemsetAsync(b.get(), 0, sizeof(double) * P.n, st));
    launch_set_scalar(b.get(), 1.0, st);
    solve_enqueue_f(P, f->f, b.get(), x.get());   // warm
    hipEvent_t e[6];
    for (auto& q : e) KTH_HIP(hipEventCreate(&q));
    KTH_HIP(hipEventRecord(e[0], st));
    for (int r = 0; r < reps; r++) solve_enqueue_f(P, f->f, b.get(), x.get());
    KTH_HIP(hipEventRecord(e[1], st));
    for (int r = 0; r < reps; r++)
      spmv2(P.n, P.rowptr.get(), P.col.get(), P.aval.get(), P.bval.get(), x.get(), nullptr, y.get(), st);
    KTH_HIP(hipEventRecord(e[2], st));
    KTH_HIP(hipEventRecord(e[3], st));
    for (int r = 0; r < reps; r++)
      spmv2(P.n, P.rowptr.get(), P.col.get(), P.aval.get(), P.bval.get(), x.get(), y.get(), b.get(), st);
    KTH_HIP(hipEventRecord(e[4], st));
    c->sync();
    float ms0 = 0, ms1 = 0, ms2 = 0;
    KTH_HIP(hipEventElapsedTime(&ms0, e[0], e[1]));
    KTH_HIP(hipEventElapsedTime(&ms1, e[1], e[2]));
    KTH_HIP(hipEventElapsedTime(&ms2, e[3], e[4]));
    for (auto& q : e) (void)hipEventDestroy(q);
    const double n = (double)P.n, nnz = (double)P.nnz;
    const double tsz = f->f.prec == KTH_FP64 ? 8.0 : 4.0;
    for (int q = 0; q < nout; q++) out[q] = 0.0;
    out[0] = ms0 * 1e-3 / reps;
    out[1] = 2.0 * tsz * (double)P.S.nnz_l + 32.0 * n;   // L read forward and backward; b, x, work vectors
    out[2] = ms1 * 1e-3 / reps;
    out[3] = 12.0 * nnz + 24.0 * n;                      // B x: values + columns, row pointers, x, y
    if (nout > 5) {
      out[4] = ms2 * 1e-3 / reps;
      out[5] = 20.0 * nnz + 32.0 * n;                    // A x and B x together
    }
  });
}

kth_status kth_debug_mfma_probe_f32(const float* A, const float* B, float* D) {
  return guarded(nullptr, [&] {
    float *dA, *dB, *dD;
    KTH_HIP(hipMalloc(&dA, 64 * sizeof(float)));
    KTH_HIP(hipMalloc(&dB, 64 * sizeof(float)));
    KTH_HIP(hipMalloc(&dD, 256 * sizeof(float)));
    KTH_HIP(hipMemcpy(dA, A, 64 * sizeof(float), hipMemcpyHostToDevice));
    KTH_HIP(hipMemcpy(dB, B, 64 * sizeof(float), hipMemcpyHostToDevice));
    launch_mfma_probe_f32(dA, dB, dD, nullptr);
    KTH_HIP(hipDeviceSynchronize());
    KTH_HIP(hipMemcpy(D, dD, 256 * sizeof(float), hipMemcpyDeviceToHost));
    (void)hipFree(dA);
    (void)hipFree(dB);
    (void)hipFree(dD);
  });
}

kth_status kth_debug_mfma_probe(const double* A, const double* B, double* D) {
  return guarded(nullptr, [&] {
    double *dA, *dB, *dD;
    KTH_HIP(hipMalloc(&dA, 64 * sizeof(double)));
    KTH_HIP(hipMalloc(&dB, 64 * sizeof(double)));
    KTH_HIP(hipMalloc(&dD, 256 * sizeof(double)));
    KTH_HIP(hipMemcpy(dA, A, 64 * sizeof(double), hipMemcpyHostToDevice));
    KTH_HIP(hipMemcpy(dB, B, 64 * sizeof(double), hipMemcpyHostToDevice));
    launch_mfma_probe(dA, dB, dD, nullptr);
    KTH_HIP(hipDeviceSynchronize());
    KTH_HIP(hipMemcpy(D, dD, 256 * sizeof(double), hipMemcpyDeviceToHost));
    (void)hipFree(dA);
    (void)hipFree(dB);
    (void)hipFree(dD);
  });
}

}  // extern "C"
