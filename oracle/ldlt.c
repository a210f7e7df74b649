/*
 * Oracle (test infrastructure only): plain, slow sparse LDL^T of C = A - sigma*B
 * and its inertia.  Not part of the product library; only the tests, the smoke
 * check and the benchmark's CPU-baseline leg use it.
 *
 * What it follows
 *   - Section 2.1 and Alg. 1: P (A - sigma B) P^T = L D L^T with P a Bunch-Kaufman
 *     permutation, L unit lower, D block diagonal (1x1 / 2x2); by Sylvester's law
 *     the number of negative eigenvalues of D equals nu_sigma(A, B).
 *   - Section 3.3, Alg. 1': a sigma-independent fill-reducing order Q is applied
 *     first, so the factor is of P Q (A - sigma B) Q^T P^T.
 *
 * Plain multifrontal over *fundamental* supernodes (columns whose structure
 * coincide), each front a dense nf x nf array, eliminated one pivot at a time
 * with the textbook Bunch-Kaufman rule (alpha = (1 + sqrt 17) / 8) whose
 * candidate rows are the front's fully-summed rows (so the sparsity structure
 * is static).  No blocking, no amalgamation.  C entries are formed with one
 * rounding, fma(-sigma, b, a).
 *
 * Everything here is independent of the GPU library: its own ordering input,
 * its own symbolic analysis, its own numeric kernels.
 */
#define _POSIX_C_SOURCE 199309L
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

typedef struct {
  int64_t neg, zero, pos;
  double min_abs_d;     /* smallest |eigenvalue| over all D blocks              */
  double max_abs_l;     /* largest |L_ij| (element growth diagnostic)           */
  double flops;         /* algorithmic count sum_j (c_j^2 + 2 c_j)              */
  double flops_done;    /* same count over the supernodes actually eliminated   */
  int64_t nnz_l;        /* structural nonzeros of L below the diagonal          */
  int64_t nsuper;
  int64_t max_front;
  int64_t n2x2;
  int32_t completed;    /* 0 if stopped early by the flop cap                   */
} orc_stats;

typedef struct {
  int64_t n;
  int64_t nsup;
  int64_t *perm;        /* elimination position k -> original index           */
  int64_t *sfirst;      /* [nsup+1] first column of each supernode              */
  int64_t *rptr;        /* [nsup+1] offsets into rows                           */
  int64_t *rows;        /* front row lists (global elimination indices)        */
  int64_t *lptr;        /* [nsup+1] offsets of L panels (nf*ns doubles each)    */
  double *L;            /* column-major nf x ns panels; unit diagonal implied  */
  double *D;            /* [n] diagonal of D (pivot order)                      */
  double *E;            /* [n] sub-diagonal of D (nonzero at 2x2 pivots)        */
  int64_t *lperm;       /* [n] local pivot order: position -> front-local row   */
} orc_factor;

static void *xmalloc(size_t b) {
  void *p = malloc(b ? b : 1);
  if (!p) { fprintf(stderr, "oracle: out of memory (%zu bytes)\n", b); abort(); }
  return p;
}
static void *xcalloc(size_t n, size_t s) {
  void *p = calloc(n ? n : 1, s ? s : 1);
  if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
  return p;
}
static int cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}
static int64_t find_pos(const int64_t *v, int64_t len, int64_t key) {
  int64_t lo = 0, hi = len - 1;
  while (lo <= hi) {
    int64_t mid = (lo + hi) / 2;
    if (v[mid] == key) return mid;
    if (v[mid] < key) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

/* symmetric interchange of rows/cols k and r (k < r) of a lower-stored
 * symmetric nf x nf column-major array (only i >= j entries are meaningful) */
static void sym_swap(double *F, int64_t nf, int64_t k, int64_t r) {
#define AT(i, j) F[(i) + (j) * nf]
  double t;
  if (k == r) return;
  for (int64_t c = 0; c < k; c++) { t = AT(k, c); AT(k, c) = AT(r, c); AT(r, c) = t; }
  t = AT(k, k); AT(k, k) = AT(r, r); AT(r, r) = t;
  for (int64_t i = k + 1; i < r; i++) { t = AT(i, k); AT(i, k) = AT(r, i); AT(r, i) = t; }
  for (int64_t i = r + 1; i < nf; i++) { t = AT(i, k); AT(i, k) = AT(i, r); AT(i, r) = t; }
#undef AT
}

/* Inertia of one D block.  1x1: sign of d.  2x2 [[a b][b c]]: the product of its
 * eigenvalues is det = ac - b^2 and their sum is a + c. */
static void count_1x1(double d, orc_stats *st) {
  if (d < 0) st->neg++; else if (d > 0) st->pos++; else st->zero++;
  double ad = fabs(d);
  if (ad < st->min_abs_d) st->min_abs_d = ad;
}
static void count_2x2(double a, double b, double c, orc_stats *st) {
  double det = a * c - b * b, tr = a + c;
  if (det < 0) { st->neg++; st->pos++; }
  else if (det > 0) { if (tr < 0) st->neg += 2; else st->pos += 2; }
  else { st->zero++; if (tr < 0) st->neg++; else if (tr > 0) st->pos++; else st->zero++; }
  /* eigenvalues of the symmetric 2x2 block */
  double m = 0.5 * tr, q = sqrt(0.25 * (a - c) * (a - c) + b * b);
  double e1 = fabs(m - q), e2 = fabs(m + q);
  double e = e1 < e2 ? e1 : e2;
  if (e < st->min_abs_d) st->min_abs_d = e;
}

/*
 * Partial factorization of the ns fully-summed columns of the nf x nf front F
 * (column-major, lower triangle used), Bunch-Kaufman pivoting with candidates
 * among the fully-summed rows (Section 2.1; alpha = (1 + sqrt 17) / 8); at most
 * cap pivot columns when cap > 0.  lp: pivot order within the block (ns entries,
 * initialised to the identity by the caller).  D, E (may be NULL): pivots and
 * 2x2 off-diagonals of the block.  Returns the number of columns eliminated.
 */
static int64_t partial_factor(double *F, int64_t nf, int64_t ns, int64_t cap, int64_t *lp,
                              orc_stats *st, double *D, double *E) {
  const double alpha = (1.0 + sqrt(17.0)) / 8.0;
#define FA(i, j) F[(i) + (j) * nf]
  int64_t k = 0;
  while (k < ns && (cap <= 0 || k < cap)) {
    double g1 = 0; int64_t r = k;
    for (int64_t i = k + 1; i < ns; i++) if (fabs(FA(i, k)) > g1) { g1 = fabs(FA(i, k)); r = i; }
    int two = 0;
    if (g1 == 0 || fabs(FA(k, k)) >= alpha * g1) {
      /* 1x1 at k */
    } else {
      double gr = 0;
      for (int64_t i = k; i < ns; i++) if (i != r) {
        double v = i < r ? fabs(FA(r, i)) : fabs(FA(i, r));
        if (v > gr) gr = v;
      }
      if (fabs(FA(k, k)) * gr >= alpha * g1 * g1) {
        /* 1x1 at k */
      } else if (fabs(FA(r, r)) >= alpha * gr) {
        sym_swap(F, nf, k, r);
        int64_t t = lp[k]; lp[k] = lp[r]; lp[r] = t;
      } else {
        two = 1;
        if (r != k + 1) {
          sym_swap(F, nf, k + 1, r);
          int64_t t = lp[k + 1]; lp[k + 1] = lp[r]; lp[r] = t;
        }
      }
    }
    if (!two) {
      double d = FA(k, k);
      count_1x1(d, st);
      if (D) { D[k] = d; E[k] = 0; }
      if (d != 0) {
        /* trailing -= F(:,k) F(:,k)^T / d  (lower triangle) */
        for (int64_t j = k + 1; j < nf; j++) {
          double wj = FA(j, k);
          if (wj == 0) continue;
          for (int64_t i = j; i < nf; i++) FA(i, j) -= FA(i, k) * (wj / d);
        }
        for (int64_t i = k + 1; i < nf; i++) {
          FA(i, k) /= d;
          if (fabs(FA(i, k)) > st->max_abs_l) st->max_abs_l = fabs(FA(i, k));
        }
      } else {
        for (int64_t i = k + 1; i < nf; i++) FA(i, k) = 0;   /* zero pivot: recorded, skipped */
      }
      FA(k, k) = 1.0;
      k += 1;
    } else {
      double a = FA(k, k), b = FA(k + 1, k), c = FA(k + 1, k + 1);
      double det = a * c - b * b;
      count_2x2(a, b, c, st);
      st->n2x2++;
      if (D) { D[k] = a; E[k] = b; D[k + 1] = c; E[k + 1] = 0; }
      /* W = [F(:,k) F(:,k+1)], L = W D^{-1}, trailing -= L W^T */
      for (int64_t j = k + 2; j < nf; j++) {
        double w1 = FA(j, k), w2 = FA(j, k + 1);
        for (int64_t i = j; i < nf; i++) {
          double l1 = (c * FA(i, k) - b * FA(i, k + 1)) / det;
          double l2 = (a * FA(i, k + 1) - b * FA(i, k)) / det;
          FA(i, j) -= l1 * w1 + l2 * w2;
        }
      }
      for (int64_t i = k + 2; i < nf; i++) {
        double w1 = FA(i, k), w2 = FA(i, k + 1);
        FA(i, k) = (c * w1 - b * w2) / det;
        FA(i, k + 1) = (a * w2 - b * w1) / det;
        if (fabs(FA(i, k)) > st->max_abs_l) st->max_abs_l = fabs(FA(i, k));
        if (fabs(FA(i, k + 1)) > st->max_abs_l) st->max_abs_l = fabs(FA(i, k + 1));
      }
      FA(k, k) = 1.0; FA(k + 1, k) = 0.0; FA(k + 1, k + 1) = 1.0;
      k += 2;
    }
  }
#undef FA
  return k;
}

/*
 * orc_ldlt: factor Q C Q^T, C = A - sigma B given as symmetric CSR (both
 * triangles, sorted columns).  perm[k] = original index eliminated k-th before
 * postordering (NULL: identity).  keep != 0 keeps L, D for orc_solve.
 * flop_cap > 0 stops after the supernode whose cumulative count passes it
 * (stats.completed = 0 then).  shapes (may be NULL; room for 2 n entries)
 * receives (nf, ns) of every supernode in elimination order (stats.nsuper of them).
 * Returns 0, or -1 on invalid input.
 */
int orc_ldlt(int64_t n, const int64_t *rowptr, const int32_t *col, const double *aval,
             const double *bval, double sigma, const int64_t *perm_in, int keep,
             double flop_cap, orc_stats *st, orc_factor **out, int64_t *shapes) {
  memset(st, 0, sizeof(*st));
  st->min_abs_d = INFINITY;
  st->completed = 1;
  if (out) *out = NULL;
  if (n <= 0) return -1;

  /* ---- permutation (new -> old) and its inverse ---- */
  int64_t *perm = xmalloc(sizeof(int64_t) * n), *iperm = xmalloc(sizeof(int64_t) * n);
  for (int64_t k = 0; k < n; k++) perm[k] = perm_in ? perm_in[k] : k;
  for (int64_t k = 0; k < n; k++) iperm[k] = -1;
  for (int64_t k = 0; k < n; k++) {
    if (perm[k] < 0 || perm[k] >= n || iperm[perm[k]] != -1) { free(perm); free(iperm); return -1; }
    iperm[perm[k]] = k;
  }

  /* ---- elimination tree of the permuted pattern (row-by-row with path compression) ---- */
  int64_t *parent = xmalloc(sizeof(int64_t) * n), *anc = xmalloc(sizeof(int64_t) * n);
  for (int64_t i = 0; i < n; i++) {
    parent[i] = -1; anc[i] = -1;
    int64_t oi = perm[i];
    for (int64_t p = rowptr[oi]; p < rowptr[oi + 1]; p++) {
      int64_t j = iperm[col[p]];
      while (j != -1 && j < i) {            /* climb from j towards the root */
        int64_t nx = anc[j];
        anc[j] = i;
        if (nx == -1) { parent[j] = i; break; }
        j = nx;
      }
    }
  }
  free(anc);

  /* ---- postorder ---- */
  int64_t *head = xmalloc(sizeof(int64_t) * n), *next = xmalloc(sizeof(int64_t) * n);
  for (int64_t i = 0; i < n; i++) head[i] = -1;
  for (int64_t i = n - 1; i >= 0; i--)
    if (parent[i] != -1) { next[i] = head[parent[i]]; head[parent[i]] = i; }
  int64_t *post = xmalloc(sizeof(int64_t) * n), *stack = xmalloc(sizeof(int64_t) * n);
  int64_t np = 0;
  for (int64_t r = 0; r < n; r++) {
    if (parent[r] != -1) continue;
    int64_t top = 0;
    stack[top++] = r;
    while (top) {
      int64_t v = stack[top - 1];
      int64_t c = head[v];
      if (c != -1) { head[v] = next[c]; stack[top++] = c; }
      else { post[np++] = v; top--; }
    }
  }
  free(stack); free(next); free(head);
  /* compose: elimination position k holds original index perm[post[k]] */
  int64_t *perm2 = xmalloc(sizeof(int64_t) * n), *pos = xmalloc(sizeof(int64_t) * n);
  for (int64_t k = 0; k < n; k++) { perm2[k] = perm[post[k]]; pos[post[k]] = k; }
  int64_t *par2 = xmalloc(sizeof(int64_t) * n);
  for (int64_t k = 0; k < n; k++) par2[k] = parent[post[k]] == -1 ? -1 : pos[parent[post[k]]];
  free(parent); free(post); free(pos);
  for (int64_t k = 0; k < n; k++) iperm[perm2[k]] = k;
  free(perm); perm = perm2; parent = par2;

  /* ---- column structures by merging children (children precede parents) ---- */
  int64_t *nchild = xcalloc(n, sizeof(int64_t));
  for (int64_t j = 0; j < n; j++) if (parent[j] != -1) nchild[parent[j]]++;
  int64_t **S = xcalloc(n, sizeof(int64_t *));
  int64_t *cnt = xcalloc(n, sizeof(int64_t));
  /* children lists */
  int64_t *chead = xmalloc(sizeof(int64_t) * n), *cnext = xmalloc(sizeof(int64_t) * n);
  for (int64_t j = 0; j < n; j++) chead[j] = -1;
  for (int64_t j = n - 1; j >= 0; j--)
    if (parent[j] != -1) { cnext[j] = chead[parent[j]]; chead[parent[j]] = j; }
  /* supernode bookkeeping (grown dynamically) */
  int64_t cap_s = 1024, cap_r = 1 << 20, nsup = 0, nrows = 0;
  int64_t *sfirst = xmalloc(sizeof(int64_t) * (cap_s + 1));
  int64_t *rptr = xmalloc(sizeof(int64_t) * (cap_s + 1));
  int64_t *rows = xmalloc(sizeof(int64_t) * cap_r);
  int64_t *mark = xmalloc(sizeof(int64_t) * n);
  for (int64_t j = 0; j < n; j++) mark[j] = -1;
  int64_t *tmp = xmalloc(sizeof(int64_t) * n);
  double nnzl = 0, flops = 0;
  for (int64_t j = 0; j < n; j++) {
    int64_t len = 0;
    int64_t oj = perm[j];
    for (int64_t p = rowptr[oj]; p < rowptr[oj + 1]; p++) {
      int64_t i = iperm[col[p]];
      if (i > j && mark[i] != j) { mark[i] = j; tmp[len++] = i; }
    }
    for (int64_t c = chead[j]; c != -1; c = cnext[c]) {
      for (int64_t q = 0; q < cnt[c]; q++) {
        int64_t i = S[c][q];
        if (i > j && mark[i] != j) { mark[i] = j; tmp[len++] = i; }
      }
      free(S[c]); S[c] = NULL;
    }
    qsort(tmp, (size_t)len, sizeof(int64_t), cmp_i64);
    S[j] = xmalloc(sizeof(int64_t) * (len ? len : 1));
    memcpy(S[j], tmp, sizeof(int64_t) * len);
    cnt[j] = len;
    nnzl += (double)len;
    flops += (double)len * len + 2.0 * len;
    int join = (j > 0 && parent[j - 1] == j && nchild[j] == 1 && cnt[j - 1] == cnt[j] + 1);
    if (!join) {
      if (nsup == cap_s) {
        cap_s *= 2;
        sfirst = realloc(sfirst, sizeof(int64_t) * (cap_s + 1));
        rptr = realloc(rptr, sizeof(int64_t) * (cap_s + 1));
        if (!sfirst || !rptr) abort();
      }
      while (nrows + len + 1 > cap_r) { cap_r *= 2; rows = realloc(rows, sizeof(int64_t) * cap_r); if (!rows) abort(); }
      sfirst[nsup] = j;
      rptr[nsup] = nrows;
      rows[nrows++] = j;
      memcpy(rows + nrows, tmp, sizeof(int64_t) * len);
      nrows += len;
      nsup++;
    }
    if (parent[j] == -1) { free(S[j]); S[j] = NULL; }
  }
  sfirst[nsup] = n;
  rptr[nsup] = nrows;
  for (int64_t j = 0; j < n; j++) if (S[j]) { free(S[j]); S[j] = NULL; }
  free(S); free(tmp); free(mark); free(chead); free(cnext);
  st->nnz_l = (int64_t)nnzl;
  st->flops = flops;
  st->nsuper = nsup;
  if (shapes)
    for (int64_t s = 0; s < nsup; s++) {
      shapes[2 * s] = rptr[s + 1] - rptr[s];
      shapes[2 * s + 1] = sfirst[s + 1] - sfirst[s];
    }

  /* supernode of each column, supernode parents and child lists */
  int64_t *snode = xmalloc(sizeof(int64_t) * n);
  for (int64_t s = 0; s < nsup; s++)
    for (int64_t j = sfirst[s]; j < sfirst[s + 1]; j++) snode[j] = s;
  int64_t *spar = xmalloc(sizeof(int64_t) * nsup);
  for (int64_t s = 0; s < nsup; s++) {
    int64_t last = sfirst[s + 1] - 1;
    spar[s] = parent[last] == -1 ? -1 : snode[parent[last]];
  }
  int64_t *shead = xmalloc(sizeof(int64_t) * nsup), *snext = xmalloc(sizeof(int64_t) * nsup);
  for (int64_t s = 0; s < nsup; s++) shead[s] = -1;
  for (int64_t s = nsup - 1; s >= 0; s--)
    if (spar[s] != -1) { snext[s] = shead[spar[s]]; shead[spar[s]] = s; }

  /* ---- factor storage ---- */
  orc_factor *fac = NULL;
  if (keep) {
    fac = xcalloc(1, sizeof(orc_factor));
    fac->n = n; fac->nsup = nsup;
    fac->perm = perm; fac->sfirst = sfirst; fac->rptr = rptr; fac->rows = rows;
    fac->lptr = xmalloc(sizeof(int64_t) * (nsup + 1));
    int64_t tot = 0;
    for (int64_t s = 0; s < nsup; s++) {
      fac->lptr[s] = tot;
      tot += (rptr[s + 1] - rptr[s]) * (sfirst[s + 1] - sfirst[s]);
    }
    fac->lptr[nsup] = tot;
    fac->L = xmalloc(sizeof(double) * tot);
    fac->D = xcalloc(n, sizeof(double));
    fac->E = xcalloc(n, sizeof(double));
    fac->lperm = xmalloc(sizeof(int64_t) * n);
  }

  /* ---- numeric multifrontal factorization ---- */
  double **U = xcalloc(nsup, sizeof(double *));   /* update matrices awaiting parents */
  double done = 0;
  int64_t maxf = 0;
  for (int64_t s = 0; s < nsup; s++) {
    int64_t f = sfirst[s], ns = sfirst[s + 1] - f;
    int64_t nf = rptr[s + 1] - rptr[s];
    const int64_t *R = rows + rptr[s];
    if (nf > maxf) maxf = nf;
    double *F = xcalloc((size_t)nf * nf, sizeof(double));
#define FA(i, j) F[(i) + (j) * nf]
    /* assemble entries of C in the supernode's columns: C_ij = fma(-sigma, b, a) */
    for (int64_t jj = 0; jj < ns; jj++) {
      int64_t oj = perm[f + jj];
      for (int64_t p = rowptr[oj]; p < rowptr[oj + 1]; p++) {
        int64_t i = iperm[col[p]];
        if (i < f + jj) continue;
        int64_t pi = find_pos(R, nf, i);
        FA(pi, jj) += fma(-sigma, bval[p], aval[p]);
      }
    }
    /* extend-add the children's update matrices */
    for (int64_t c = shead[s]; c != -1; c = snext[c]) {
      int64_t cnf = rptr[c + 1] - rptr[c], cns = sfirst[c + 1] - sfirst[c], cnu = cnf - cns;
      const int64_t *CR = rows + rptr[c] + cns;
      int64_t *map = xmalloc(sizeof(int64_t) * (cnu ? cnu : 1));
      for (int64_t a = 0; a < cnu; a++) map[a] = find_pos(R, nf, CR[a]);
      for (int64_t b = 0; b < cnu; b++)
        for (int64_t a = b; a < cnu; a++) FA(map[a], map[b]) += U[c][a + b * cnu];
      free(map);
      free(U[c]); U[c] = NULL;
    }
    /* partial factorization of the ns fully-summed columns, Bunch-Kaufman pivoting
       with candidates among the fully-summed rows */
    int64_t *lp = xmalloc(sizeof(int64_t) * (ns ? ns : 1));
    for (int64_t k = 0; k < ns; k++) lp[k] = k;
    partial_factor(F, nf, ns, 0, lp, st, fac ? fac->D + f : NULL, fac ? fac->E + f : NULL);
    /* keep L panel, hand the update matrix to the parent */
    if (fac) {
      memcpy(fac->L + fac->lptr[s], F, sizeof(double) * nf * ns);
      for (int64_t q = 0; q < ns; q++) fac->lperm[f + q] = lp[q];
    }
    free(lp);
    int64_t nu = nf - ns;
    if (spar[s] != -1 && nu > 0) {
      double *u = xmalloc(sizeof(double) * nu * nu);
      for (int64_t b = 0; b < nu; b++)
        for (int64_t a = b; a < nu; a++) u[a + b * nu] = FA(ns + a, ns + b);
      U[s] = u;
    }
#undef FA
    free(F);
    for (int64_t jj = 0; jj < ns; jj++) {
      double cj = (double)(nf - 1 - jj);
      done += cj * cj + 2 * cj;
    }
    if (flop_cap > 0 && done >= flop_cap && s + 1 < nsup) { st->completed = 0; break; }
  }
  for (int64_t s = 0; s < nsup; s++) free(U[s]);
  free(U);
  st->flops_done = done;
  st->max_front = maxf;
  free(snode); free(spar); free(shead); free(snext); free(nchild); free(cnt); free(iperm);
  free(parent);
  if (fac && st->completed) {
    *out = fac;
  } else {
    if (fac) { free(fac->lptr); free(fac->L); free(fac->D); free(fac->E); free(fac->lperm); free(fac); }
    free(perm); free(sfirst); free(rptr); free(rows);
  }
  return 0;
}

/*
 * Timing sample (CPU baseline, not part of the oracle's results): the partial
 * factorization above on one synthetic dense front of nf rows with ns
 * fully-summed columns, at most cap pivots (cap <= 0: all ns).  Entries of the
 * lower triangle are uniform in [-1, 1) from a fixed 64-bit linear congruential
 * sequence.  secs: wall time of the factorization alone; flops: its algorithmic
 * count, sum over the pivot columns taken of c^2 + 2c (c = rows below the pivot).
 */
int orc_front_sample(int64_t nf, int64_t ns, int64_t cap, double *secs, double *flops) {
  if (nf <= 0 || ns <= 0 || ns > nf) return -1;
  double *F = xmalloc(sizeof(double) * nf * nf);
  uint64_t x = 0x2545F4914F6CDD1Dull;
  for (int64_t j = 0; j < nf; j++)
    for (int64_t i = j; i < nf; i++) {
      x = x * 6364136223846793005ull + 1442695040888963407ull;
      F[i + j * nf] = (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
  int64_t *lp = xmalloc(sizeof(int64_t) * ns);
  for (int64_t k = 0; k < ns; k++) lp[k] = k;
  orc_stats st;
  memset(&st, 0, sizeof(st));
  st.min_abs_d = INFINITY;
  struct timespec t0, t1;
  clock_gettime(CLOCK_MONOTONIC, &t0);
  int64_t done = partial_factor(F, nf, ns, cap, lp, &st, NULL, NULL);
  clock_gettime(CLOCK_MONOTONIC, &t1);
  *secs = (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
  double fl = 0;
  for (int64_t jj = 0; jj < done; jj++) {
    double c = (double)(nf - 1 - jj);
    fl += c * c + 2 * c;
  }
  *flops = fl;
  free(lp);
  free(F);
  return 0;
}

/* x = C^{-1} b with the kept factor (b and x of length n, may alias) */
int orc_solve(const orc_factor *fac, const double *b, double *x) {
  int64_t n = fac->n;
  double *y = xmalloc(sizeof(double) * n);   /* eliminated-order work vector */
  double *z = xmalloc(sizeof(double) * n);   /* per-supernode pivot-order values */
  for (int64_t k = 0; k < n; k++) y[k] = b[fac->perm[k]];
  /* forward: L z = P y */
  for (int64_t s = 0; s < fac->nsup; s++) {
    int64_t f = fac->sfirst[s], ns = fac->sfirst[s + 1] - f;
    int64_t nf = fac->rptr[s + 1] - fac->rptr[s];
    const int64_t *R = fac->rows + fac->rptr[s];
    const double *L = fac->L + fac->lptr[s];
    for (int64_t q = 0; q < ns; q++) z[f + q] = y[f + fac->lperm[f + q]];
    for (int64_t c = 0; c < ns; c++) {
      double v = z[f + c];
      for (int64_t i = c + 1; i < ns; i++) z[f + i] -= L[i + c * nf] * v;
      for (int64_t i = ns; i < nf; i++) y[R[i]] -= L[i + c * nf] * v;
    }
  }
  /* diagonal: z <- D^{-1} z */
  for (int64_t s = 0; s < fac->nsup; s++) {
    int64_t f = fac->sfirst[s], l = fac->sfirst[s + 1];
    for (int64_t k = f; k < l;) {
      if (k + 1 < l && fac->E[k] != 0) {
        double a = fac->D[k], bb = fac->E[k], c = fac->D[k + 1], det = a * c - bb * bb;
        double u = z[k], v = z[k + 1];
        z[k] = (c * u - bb * v) / det;
        z[k + 1] = (a * v - bb * u) / det;
        k += 2;
      } else {
        z[k] = fac->D[k] != 0 ? z[k] / fac->D[k] : 0.0;
        k += 1;
      }
    }
  }
  /* backward: L^T w = z, x = P^T w */
  for (int64_t s = fac->nsup - 1; s >= 0; s--) {
    int64_t f = fac->sfirst[s], ns = fac->sfirst[s + 1] - f;
    int64_t nf = fac->rptr[s + 1] - fac->rptr[s];
    const int64_t *R = fac->rows + fac->rptr[s];
    const double *L = fac->L + fac->lptr[s];
    for (int64_t c = ns - 1; c >= 0; c--) {
      double v = z[f + c];
      for (int64_t i = c + 1; i < ns; i++) v -= L[i + c * nf] * z[f + i];
      for (int64_t i = ns; i < nf; i++) v -= L[i + c * nf] * y[R[i]];
      z[f + c] = v;
    }
    for (int64_t q = 0; q < ns; q++) y[f + fac->lperm[f + q]] = z[f + q];
  }
  for (int64_t k = 0; k < n; k++) x[fac->perm[k]] = y[k];
  free(y); free(z);
  return 0;
}

void orc_free(orc_factor *fac) {
  if (!fac) return;
  free(fac->perm); free(fac->sfirst); free(fac->rptr); free(fac->rows); free(fac->lptr);
  free(fac->L); free(fac->D); free(fac->E); free(fac->lperm);
  free(fac);
}

/* y = (A - sigma B) x computed entrywise with the same fused rounding */
void orc_shifted_matvec(int64_t n, const int64_t *rowptr, const int32_t *col, const double *a,
                        const double *b, double sigma, const double *x, double *y) {
  for (int64_t i = 0; i < n; i++) {
    double s = 0;
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) s += fma(-sigma, b[p], a[p]) * x[col[p]];
    y[i] = s;
  }
}
