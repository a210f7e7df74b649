/*
 * kth.h -- C ABI of the MI355X k-th eigenpair library (libkth.so).
 *
 * Problem (eq. (1)): A x = lambda B x, A real symmetric, B symmetric positive
 * definite, n x n sparse; eigenvalues ascending lambda_1 <= ... <= lambda_n; k is
 * 1-based.  nu(sigma) = #{ i : lambda_i < sigma } (Section 2.1).
 *
 * Conventions for every call
 *   - Every call returns kth_status; nothing throws across the ABI.  On failure a
 *     message is kept per context (kth_last_error).
 *   - Matrices: CSR with BOTH triangles stored, 0-based, int64 row pointers,
 *     int32 column indices strictly increasing within each row, float64 values.
 *     A and B may have different patterns: the library analyses their union,
 *     which must hold every diagonal entry and be structurally symmetric.
 *   - Host pointers unless a flag says otherwise.  The library copies what it
 *     needs; the caller may free its arrays on return.  Output buffers are owned
 *     by the caller.  Handles are owned by the library and freed by *_destroy.
 *   - Device memory comes from the context's allocator (hipMalloc unless an
 *     allocator is injected); work runs on the context's HIP stream.  Calls
 *     returning host results synchronise that stream.
 *   - One context per host thread.
 */
#ifndef KTH_H
#define KTH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KTH_OK = 0,
  KTH_EINVAL = 1,      /* invalid argument or malformed pattern                       */
  KTH_ENOMEM = 2,      /* device or host allocation failed                             */
  KTH_EDEVICE = 3,     /* HIP runtime error, or no usable gfx950 device                */
  KTH_ENOTPD = 4,      /* B is not positive definite (its LDL^T has nonpositive pivots) */
  KTH_ESINGULAR = 5,   /* exactly zero pivot: sigma is an eigenvalue to working precision */
  KTH_ENOCONV = 6,     /* Lanczos iteration limit reached                              */
  KTH_ECLUSTER = 7,    /* error bounds never became disjoint (multiple / clustered eigenvalues) */
  KTH_ESTATE = 8       /* call not valid in the object's current state                  */
} kth_status;

typedef enum { KTH_FP64 = 0, KTH_FP32_IR = 1 } kth_precision;

typedef struct kth_ctx_s* kth_ctx;
typedef struct kth_pencil_s* kth_pencil;
typedef struct kth_factor_s* kth_factor_t;   /* kept numeric factor */

typedef void* (*kth_alloc_fn)(size_t bytes, void* user);
typedef void (*kth_free_fn)(void* ptr, void* user);

/* pencil flags */
#define KTH_DEVICE_PTRS    1u  /* arrays of kth_pencil_create / kth_pencil_set_values are device pointers */
#define KTH_CHECK_SYMMETRY 2u  /* verify structural symmetry of the union pattern (O(nnz log)) */
/* solve flags (with KTH_DEVICE_PTRS) */
#define KTH_SOLVE_UNREFINED 4u /* FP32 factor: one solve pass in the factor's precision, no refinement */

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t to run on,
 * or NULL for a stream owned by the context.  alloc/free: device allocator (both
 * NULL: hipMalloc / hipFree behind a stream-ordered block cache); `user` is passed
 * back to them.  alloc returns NULL on failure (the call then fails with
 * KTH_ENOMEM); free is called once the stream that used the block (the context's,
 * or a kth_eig_batch worker's) has finished with it, so the allocator may reuse it
 * at once.  Python: Context(torch_allocator=True) routes both to torch's caching
 * allocator on the context's stream.
 * Fails with KTH_EDEVICE if the device is not a gfx950 GPU. */
kth_status kth_ctx_create(int device, void* hip_stream, kth_alloc_fn alloc, kth_free_fn free_fn,
                          void* user, kth_ctx* out);
/* Releases the caller's handle.  Pencils hold their context and kept factors their
 * pencil: a destroyed parent is freed when its last child is destroyed. */
kth_status kth_ctx_destroy(kth_ctx ctx);
const char* kth_status_string(kth_status s);
const char* kth_last_error(kth_ctx ctx);   /* message of the last failing call on ctx ("" if none) */

/* Host-only analysis statistics of a pattern (no device needed): fill-reducing
 * order, symbolic factorization and the algorithmic flop count of one numeric
 * LDL^T (sum over columns j of c_j^2 + 2 c_j, c_j = structural nonzeros below the
 * diagonal of column j of L).  stats[0..15] receives
 *   n, nnz, n_supervariables, n_supernodes_fundamental, n_supernodes, max_front,
 *   max_pivot_block, levels, flops, flops_padded, nnz_l, nnz_l_padded,
 *   front_pool_bytes, factor_bytes, t_order_s, t_symbolic_s.
 * perm_out (may be NULL): n entries, elimination position -> original index. */
kth_status kth_analyze(int64_t n, const int64_t* rowptr, const int32_t* col, uint32_t flags,
                       double* stats, int64_t* perm_out);

/* Create a pencil from A (a_rowptr, a_col, a_val) and B (b_rowptr, b_col, b_val).
 * Ordering and symbolic analysis run here on the host, on the union of the two
 * patterns (Section 3.3: they depend on the pattern only and are reused for B and
 * every shift); values and maps are uploaded.  With KTH_DEVICE_PTRS all six arrays
 * are device pointers (they are copied to the host for the analysis).  The
 * library keeps its own copies. */
kth_status kth_pencil_create(kth_ctx ctx, int64_t n, const int64_t* a_rowptr, const int32_t* a_col,
                             const double* a_val, const int64_t* b_rowptr, const int32_t* b_col,
                             const double* b_val, uint32_t flags, kth_pencil* out);
/* Replace the values (same patterns; the analysis is kept): a_val on A's pattern,
 * b_val on B's.  flags: KTH_DEVICE_PTRS. */
kth_status kth_pencil_set_values(kth_pencil p, const double* a_val, const double* b_val,
                                 uint32_t flags);
kth_status kth_pencil_destroy(kth_pencil p);

/* nu(sigma) by Sylvester's law of inertia (Section 2.1, Alg. 1'): FP64 multifrontal
 * LDL^T of A - sigma B (entries formed as fma(-sigma, b, a)) with Bunch-Kaufman
 * pivots restricted to each front's fully-summed block; nu = number of negative
 * eigenvalues of D.  nzero (may be NULL) receives the number of exactly zero
 * pivots; if it is nonzero the call returns KTH_ESINGULAR (nu still written). */
kth_status kth_inertia(kth_pencil p, double sigma, int64_t* nu, int64_t* nzero);
/* nu at nsigma shifts (multisection): the factorizations advance together through
 * the level schedule, as many at a time as free device memory allows (at most
 * 64), batch index = grid dimension y.  nu: nsigma entries (always written);
 * returns KTH_ESINGULAR if any shift gives an exactly zero pivot. */
kth_status kth_inertia_batch(kth_pencil p, int32_t nsigma, const double* sigmas, int64_t* nu);

/* Numeric factor of A - sigma B kept for solves (the linear systems of Alg. 2 and
 * Alg. 3).  KTH_FP32_IR: the same factorization in FP32 storage and arithmetic
 * (entries fma(-sigma, b, a) formed in FP64, then rounded; pivots and 2x2 blocks
 * kept in FP64).  Every kth_solve on such a factor refines in FP64: with
 * M = A - sigma B and residual r = R - M X formed in FP64, corrections from GMRES
 * on M32^{-1} M (the FP32 factor as preconditioner, <= 20 steps each) are added
 * until ||r||_inf <= 4 eps64 (||M||_inf ||x||_inf + ||R||_inf), where ||M||_inf is
 * bounded by ||A||_inf + |sigma| ||B||_inf.  The solve returns KTH_ENOCONV (x: last
 * iterate) if ||r||_inf fails to halve on two consecutive corrections or 4
 * corrections do not reach the target. */
kth_status kth_factor(kth_pencil p, double sigma, kth_precision prec, kth_factor_t* out);
/* Inertia of a kept FP64 factor: counts of negative, zero and positive
 * eigenvalues of D (neg + zero + pos = n).  KTH_ESTATE for an FP32 factor. */
kth_status kth_factor_inertia(kth_factor_t f, int64_t* neg, int64_t* zero, int64_t* pos);
/* Solve (A - sigma B) X = R for nrhs columns (column-major, leading dims >= n).
 * r and x: host pointers, or device pointers with flags & KTH_DEVICE_PTRS.
 * flags & KTH_SOLVE_UNREFINED: an FP32 factor is applied once, unrefined. */
kth_status kth_solve(kth_factor_t f, int32_t nrhs, const double* r, int64_t ldr, double* x,
                     int64_t ldx, uint32_t flags);
kth_status kth_factor_destroy(kth_factor_t f);

/* Allocation-free solve, for callers that cannot allocate device memory (work
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same X = (A - sigma B)^{-1} R as kth_solve with KTH_DEVICE_PTRS, bit for bit,
 * for an FP64 factor, or one unrefined pass of an FP32 factor (flags must then hold
 * KTH_SOLVE_UNREFINED: refinement allocates).  r, x: DEVICE pointers, column-major,
 * leading dimensions >= n.  The solve's work vectors come from one fixed array of
 * KTH_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on (its
 * address is taken when a context is created on that GPU); a factor whose solve
 * needs more -- 8 (2 n + total front rows + backward partial sums) bytes; the
 * factors of the n = 524288 tight-binding workload fit -- is rejected with
 * KTH_EINVAL before anything is enqueued.
 * The call only enqueues kernels on the context's stream and returns (no
 * synchronisation): synchronise that stream before reading x.  It calls no
 * hipMalloc or hipFree.  All calls on one GPU share that GPU's array: calls that
 * overlap in time on one GPU (other streams, contexts or threads) race, calls on
 * one stream run in order.  Every part of the array a call reads is first written
 * by that call, so what an earlier call left there does not matter. */
#define KTH_NOALLOC_SCRATCH_BYTES (64u << 20)
kth_status kth_solve_noalloc(kth_factor_t f, int32_t nrhs, const double* r, int64_t ldr, double* x,
                             int64_t ldx, uint32_t flags);
/* Pivot statistics of a kept factor (FP64 or FP32): n2x2 = number of 2x2 blocks of
 * D; min_pivot_rel = smallest |eigenvalue of a D block| / (||A||_inf + |sigma|
 * ||B||_inf); max_abs_l = largest |L_ij| (element growth of the restricted
 * Bunch-Kaufman pivoting, Section 2.1).  Any pointer may be NULL. */
kth_status kth_factor_stats(kth_factor_t f, int64_t* n2x2, double* min_pivot_rel, double* max_abs_l);

typedef struct {
  int64_t m_max;          /* stage 2 stops at <= m_max eigenvalues in the interval (20, the
                             paper's value); 0: a cost model picks it (kth_info.m_max_used):
                             2 with root_finder = 1, whose last shifts land within about a
                             count of their targets; with bisection 2 t_f / (2.6 x 1.15 t_s)
                             clamped to [2, 20], from the measured time t_f of a stage-1
                             factorization and t_s of a stage-1 solve (Alg. 3 takes about
                             2.6 m + 8 steps of about 1.15 solves for m eigenvalues)       */
  double tau_res;         /* relative residual tolerance of Alg. 3 (1e-10)                    */
  double tau_diff;        /* relative difference tolerance of Alg. 3 (1e-10)                  */
  double tau_len;         /* bisection also stops below this interval length (0: off)        */
  int32_t max_lanczos;    /* shift-and-invert Lanczos iteration limit (500)                   */
  int32_t multisection;   /* shifts per stage-2 round (1: plain bisection)                    */
  uint64_t seed;          /* seed of the starting vectors, when start_vectors is NULL         */
  kth_precision si_precision;  /* precision of the shift-and-invert factor                   */
  const double* start_vectors; /* optional host array [n_start_vectors][n]: row 0 stage 1, row 1
                                  stage 3, rows 2-3 stage-1 restarts, rows 4.. further columns of a
                                  block shift-and-invert start; rows not given are drawn by the
                                  library's own generator                                      */
  const double* warm_interval; /* optional [2]: sigma_l, sigma_u (skip stages 1-2)             */
  const int64_t* warm_counts;  /* optional [2]: nu_l, nu_u matching warm_interval              */
  double ir_tol;          /* FP32 shift-and-invert solves: target backward error (0: 4 eps64) */
  int32_t batch_workers;  /* kth_eig_batch: pencils solved concurrently, each on its own
                             streams (0: 8; 1: one after another on the context stream) */
  int32_t root_finder;    /* stage 2: 0 bisection (Alg. 1'); 1 safeguarded interpolation of
                             the eigenvalue count (a bracketing root-finder, Section 2.1):
                             each shift aims, by linear interpolation of nu between the
                             bracket ends, at the count k - m_max/2 (lower end) or
                             k + m_max/2 - 1 (upper end), whichever end is farther from k,
                             at a fraction of the bracket within [1/64, 63/64]; after two
                             consecutive such steps that each failed to halve nu_u - nu_l
                             the next shift is the midpoint.  Same stopping rule.  Needs
                             multisection = 1.                                             */
  int32_t si_block;       /* shift-and-invert Lanczos: 1 single vector (Alg. 3); p > 1 block
                             method with block size p; 0 (automatic) Alg. 3 for at most
                             3 m + 30 steps, then the block method with p = m (a multiple
                             eigenvalue leaves Alg. 3 short of m Ritz values, Section 3.4),
                             and the block method at once when stage 2 stopped on tau_len
                             with more than m_max eigenvalues.  The block method validates
                             overlapping bounds as a cluster (see kth_info.si_block).       */
  int32_t n_start_vectors;  /* rows of start_vectors (0: 4)                                  */
  int32_t b_solver;       /* stage-1 B-solves: 0 the LDL^T factor of B (task (ii)); 1 when B is
                             strictly diagonally dominant with a positive diagonal (positive
                             definite by Gershgorin's theorem, no factor needed), Jacobi-
                             preconditioned conjugate gradients to a relative residual of
                             1e-14, else the factor                                        */
} kth_opts;

typedef struct {
  int64_t k_validated;    /* index certified by disjoint error bounds (Prop. 3)               */
  int64_t nu_lower, nu_upper;
  double sigma_lower, sigma_upper, sigma_si;
  int32_t stage1_steps, bisection_steps, si_steps, it_bound, it_residual, it_difference;
  double rel_residual;        /* ||A x - lambda B x||_2 / ||x||_2 (explicit products)         */
  double rel_residual_normA;  /* ||A x - lambda B x||_2 / (||A||_inf ||x||_2)                  */
  double eta;                 /* error bound of the returned eigenvalue (Prop. 3)              */
  double min_pivot_rel;       /* smallest |pivot| / ||A - sigma B||_inf over the factorizations */
  int64_t n_factorizations;
  double flops_factor;        /* algorithmic flops of one numeric factorization               */
  double t_task[7];           /* seconds in tasks (i)-(vii) of Section 4.3                    */
  double peak_device_bytes;
  int32_t n_sigmas;           /* shifts whose inertia was computed (stage 1 and 2)            */
  double sigmas[128];         /* those shifts, in order (first 128)                            */
  int64_t nus[128];           /* their counts                                                  */
  int32_t si_precision;       /* precision of the shift-and-invert factor in the end (kth_precision) */
  int32_t ir_steps;           /* FP32-factor applications spent on refinement (all SI solves)  */
  int32_t ir_fallback;        /* 1 if a stalled refinement switched the factor to FP64          */
  double ir_max_berr;         /* largest backward error at exit of a refined solve             */
  double max_abs_l;           /* largest |L_ij| over the counted FP64 factorizations           */
  int32_t weak_pivot_nudges;  /* shifts moved because a count was not trusted: a zero pivot, a
                                 pivot below 1e-13 (||A||_inf + |sigma| ||B||_inf), or a
                                 multiplier above 1e8 (restricted pivoting, Section 2.1)     */
  int32_t weak_pivot_kept;    /* counts accepted with a weak nonzero pivot after three moves   */
  int32_t stage1_restarts;    /* stage-1 Lanczos restarts after a breakdown (beta = 0)         */
  int32_t si_block;           /* block size of the shift-and-invert Lanczos that ran last (1:
                                 Alg. 3); si_steps counts the steps of both methods         */
  int64_t m_max_used;         /* stage-2 stopping count in effect (opts.m_max, or the model's) */
  int32_t b_cg_iterations;    /* conjugate-gradient steps of the B-solves (b_solver = 1)       */
  int32_t pad1;
} kth_info;

void kth_opts_default(kth_opts* o);
/* The k-th eigenpair by the three-stage algorithm (Alg. 4): Alg. 2 -> Alg. 1' -> Alg. 3.
 * lambda: the eigenvalue.  x (may be NULL): caller-owned n doubles, B-normalised
 * (x^T B x = 1) with its largest-|.| entry positive.  info (may be NULL). */
kth_status kth_eig(kth_pencil p, int64_t k, const kth_opts* opts, double* lambda, double* x,
                   kth_info* info);
/* Many pencils in one call (each with its own k), all from ctx.  Worker threads
 * (opts->batch_workers) take the pencils in turn, each on streams of its own that
 * first wait for the work queued on the context stream; the call returns when all
 * are done.  per_pencil: np statuses (the call itself returns KTH_OK unless its
 * arguments are invalid); kth_last_error(ctx) holds one failing pencil's message.
 * Each pencil handle may appear once: a pencil owns the workspace of its runs, so
 * a repeated handle is rejected with KTH_EINVAL before any work starts (run the
 * same pencil for several k with successive kth_eig calls). */
kth_status kth_eig_batch(kth_ctx ctx, int32_t np, const kth_pencil* p, const int64_t* k,
                         const kth_opts* opts, double* lambda, double* const* x, kth_info* info,
                         kth_status* per_pencil);
/* Hellmann-Feynman backward of a simple eigenvalue: for each STORED entry q
 * (row r, column c): grad_a[q] = g * x_r * x_c over A's pattern and
 * grad_b[q] = -g * lambda * x_r * x_c over B's, x B-normalised.  x, grad_a,
 * grad_b: host arrays (n, nnz of A, nnz of B). */
kth_status kth_eig_backward(kth_pencil p, double lambda, const double* x, double g,
                            double* grad_a, double* grad_b);

/* Measurement: one FP64 factorization of A - sigma B with a HIP event pair around
 * every kernel launch (on the context stream, or on the library's second stream
 * for the pivot tiles factored ahead).  out (nout >= 28 doubles) receives
 *   [0] elapsed seconds (first to last event), [1] algorithmic flops of one
 *   factorization (exact structure), [2] the same over the padded fronts,
 *   [3 + 4c .. 6 + 4c] for kernel class c = 0..5 (small fronts, large-front
 *   assembly, pivot tiles, panel solves, left-looking and contribution-block
 *   products k_gemm_lt, split-depth reductions): seconds, dense operation count,
 *   number of launches, algorithmic HBM bytes (class 4 only: each output entry read
 *   and written once, each operand row read once); [27] nu(sigma); with nout >= 32,
 *   [28 .. 31] the contribution-block launches' share of class 4 (seconds,
 *   operation count, launches, algorithmic bytes). */
kth_status kth_profile_factor(kth_pencil p, double sigma, double* out, int32_t nout);

/* Measurement of the bandwidth-bound steps with a kept factor f: HIP events on the
 * context stream around `reps` back-to-back solves (one pass: FP64, or an FP32
 * factor unrefined), `reps` products B x, and `reps` fused products A x and B x.
 * out (nout >= 6 doubles): [0] seconds per solve, [1] its algorithmic bytes
 * (every entry of L read in the forward and in the backward sweep, 2 * 8 * nnz(L)
 * for FP64, + 32 n for the vectors), [2] seconds per B x, [3] its bytes (12 nnz +
 * 24 n), [4] seconds per fused A x, B x, [5] its bytes (20 nnz + 32 n). */
kth_status kth_profile_solve(kth_factor_t f, int32_t reps, double* out, int32_t nout);

/* Diagnostics: one v_mfma_f64_16x16x4 on device 0, zero accumulator; lane l of
 * the wavefront supplies A[l] and B[l] (64 doubles each) and result register r
 * of lane l lands in D[4 l + r] (256 doubles).  Host pointers.  Used by the
 * tests to pin the operand layout the kernels assume. */
kth_status kth_debug_mfma_probe(const double* A, const double* B, double* D);
/* The same for one v_mfma_f32_16x16x4_f32 (float arrays of 64, 64 and 256). */
kth_status kth_debug_mfma_probe_f32(const float* A, const float* B, float* D);

#ifdef __cplusplus
}
#endif
#endif /* KTH_H */
