// Vector kernels of the Lanczos processes (Alg. 2, Alg. 3) and of the
// Hellmann-Feynman backward: fused SpMV with A and B on their shared pattern,
// deterministic multi-dot (V^T w) and multi-axpy (w -= V h), Ritz-vector
// assembly, the tridiagonal eigen-step (bisection on Sturm counts + inverse
// iteration), and the entrywise gradient.  All reductions use a fixed order,
// so repeated runs give identical bits.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "blas.hpp"

namespace kth {

namespace {

constexpr int NT = 256;

inline int blocks_for(int64_t n, int per) {
  int64_t g = (n + per - 1) / per;
  return (int)(g < 1 ? 1 : (g > 1048576 ? 1048576 : g));
}

// y_a = A x and/or y_b = B x (either output may be null); 8 lanes per row.
__global__ __launch_bounds__(NT) void k_spmv2(int64_t n, const int64_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ col,
                                              const double* __restrict__ a,
                                              const double* __restrict__ b,
                                              const double* __restrict__ x, double* ya, double* yb) {
  const int64_t row = (blockIdx.x * (int64_t)NT + threadIdx.x) >> 3;
  const int sub = threadIdx.x & 7;
  double sa = 0.0, sb = 0.0;
  if (row < n) {
    const int64_t e = rowptr[row + 1];
    for (int64_t q = rowptr[row] + sub; q < e; q += 8) {
      const double xv = x[col[q]];
      if (ya) sa = fma(a[q], xv, sa);
      if (yb) sb = fma(b[q], xv, sb);
    }
  }
  for (int off = 4; off > 0; off >>= 1) {
    sa += __shfl_xor(sa, off, 8);
    sb += __shfl_xor(sb, off, 8);
  }
  if (row < n && sub == 0) {
    if (ya) ya[row] = sa;
    if (yb) yb[row] = sb;
  }
}

// partial[blk * m + c] = sum over this block's rows of V[i, c] * w[i + c*ldw]
// (ldw = 0: one vector w for every column)
constexpr int kDotRows = 2048;
__global__ __launch_bounds__(NT) void k_multidot_partial(int64_t n, int m, const double* __restrict__ V,
                                                         int64_t ldv, const double* __restrict__ w0,
                                                         int64_t ldw, double* partial) {
  __shared__ double red[NT / 64];
  const int64_t r0 = (int64_t)blockIdx.x * kDotRows;
  const int64_t r1 = r0 + kDotRows < n ? r0 + kDotRows : n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = 0; c < m; c++) {
    const double* v = V + (int64_t)c * ldv;
    const double* w = w0 + (int64_t)c * ldw;
    double acc = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) acc = fma(v[i], w[i], acc);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int q = 0; q < NT / 64; q++) t += red[q];
      partial[(int64_t)blockIdx.x * m + c] = t;
    }
    __syncthreads();
  }
}

__global__ void k_reduce_partials(int nblk, int m, const double* __restrict__ partial, double* out,
                                  double alpha) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  double t = 0.0;
  for (int q = 0; q < nblk; q++) t += partial[(int64_t)q * m + c];
  out[c] = alpha * t;
}

// w[i] -= sum_c V[i, c] h[c] (and the same for a second pair Vb, wb if given)
__global__ __launch_bounds__(NT) void k_multiaxpy(int64_t n, int m, const double* __restrict__ V,
                                                  int64_t ldv, const double* __restrict__ h, double* w,
                                                  const double* __restrict__ Vb, double* wb) {
  extern __shared__ double hs[];
  for (int c = threadIdx.x; c < m; c += NT) hs[c] = h[c];
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
    double acc = 0.0, accb = 0.0;
    for (int c = 0; c < m; c++) {
      acc = fma(V[i + (int64_t)c * ldv], hs[c], acc);
      if (Vb) accb = fma(Vb[i + (int64_t)c * ldv], hs[c], accb);
    }
    w[i] -= acc;
    if (Vb) wb[i] -= accb;
  }
}

// X[:, q] = sum_c V[:, c] C[c + q*j] + u * cu[q],   q < m  (C: j x m column-major)
__global__ __launch_bounds__(NT) void k_ritz(int64_t n, int j, int m, const double* __restrict__ V,
                                             int64_t ldv, const double* __restrict__ C,
                                             const double* __restrict__ u,
                                             const double* __restrict__ cu, double* X, int64_t ldx) {
  extern __shared__ double cs[];  // j*m + m
  for (int t = threadIdx.x; t < j * m; t += NT) cs[t] = C[t];
  for (int t = threadIdx.x; t < m; t += NT) cs[j * m + t] = cu[t];
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
    const double ui = u[i];
    for (int q0 = 0; q0 < m; q0 += 8) {
      double acc[8];
#pragma unroll
      for (int r = 0; r < 8; r++) acc[r] = 0.0;
      for (int c = 0; c < j; c++) {
        const double v = V[i + (int64_t)c * ldv];
#pragma unroll
        for (int r = 0; r < 8; r++)
          if (q0 + r < m) acc[r] = fma(v, cs[c + (q0 + r) * j], acc[r]);
      }
#pragma unroll
      for (int r = 0; r < 8; r++)
        if (q0 + r < m) X[i + (int64_t)(q0 + r) * ldx] = fma(ui, cs[j * m + q0 + r], acc[r]);
    }
  }
}

// P[:, q] = f[q] * X[:, perm[q]]
__global__ void k_gather_cols(int64_t n, int m, const double* __restrict__ X, int64_t ldx,
                              const int32_t* __restrict__ perm, const double* __restrict__ f,
                              double* P, int64_t ldp) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    for (int q = 0; q < m; q++) P[i + (int64_t)q * ldp] = f[q] * X[i + (int64_t)perm[q] * ldx];
}

// D[:, q] = f[q] * X[:, q] - P[:, q]
__global__ void k_diff_cols(int64_t n, int m, const double* __restrict__ X, int64_t ldx,
                            const double* __restrict__ f, const double* __restrict__ P, int64_t ldp,
                            double* D, int64_t ldd) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    for (int q = 0; q < m; q++)
      D[i + (int64_t)q * ldd] = f[q] * X[i + (int64_t)q * ldx] - P[i + (int64_t)q * ldp];
}

__global__ void k_scale_copy(int64_t n, double s, const double* __restrict__ x, double* y) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    y[i] = s * x[i];
}

__global__ void k_scale_inplace_dev(int64_t n, const double* __restrict__ s, int si, bool inv, double* y) {
  const double f = inv ? 1.0 / s[si] : s[si];
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    y[i] *= f;
}

// r = a_scale * ya - lam * yb  (residual (A - lam B) x from the two products)
__global__ void k_residual(int64_t n, double lam, const double* __restrict__ ya,
                           const double* __restrict__ yb, double* r) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    r[i] = ya[i] - lam * yb[i];
}

// r = rhs - (A - sigma B) x (rhs null: r = (A - sigma B) x), every entry formed as
// fma(-sigma, b, a) (8 lanes per row)
__global__ __launch_bounds__(NT) void k_shifted_residual(int64_t n, const int64_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ col,
                                                         const double* __restrict__ a,
                                                         const double* __restrict__ b, double sigma,
                                                         const double* __restrict__ x,
                                                         const double* __restrict__ rhs, double* r) {
  const int64_t row = (blockIdx.x * (int64_t)NT + threadIdx.x) >> 3;
  const int sub = threadIdx.x & 7;
  double s = 0.0;
  if (row < n) {
    const int64_t e = rowptr[row + 1];
    for (int64_t q = rowptr[row] + sub; q < e; q += 8) s = fma(fma(-sigma, b[q], a[q]), x[col[q]], s);
  }
  for (int off = 4; off > 0; off >>= 1) s += __shfl_xor(s, off, 8);
  if (row < n && sub == 0) r[row] = rhs ? rhs[row] - s : s;
}

// partial[blk] = max |x_i| over the block's rows; then out = max over blocks (fixed order)
__global__ __launch_bounds__(NT) void k_absmax_partial(int64_t n, const double* __restrict__ x,
                                                       double* partial) {
  __shared__ double red[NT / 64];
  const int64_t r0 = (int64_t)blockIdx.x * kDotRows;
  const int64_t r1 = r0 + kDotRows < n ? r0 + kDotRows : n;
  double m = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) m = fmax(m, fabs(x[i]));
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < NT / 64; q++) t = fmax(t, red[q]);
    partial[blockIdx.x] = t;
  }
}

__global__ void k_max_partials(int nblk, const double* __restrict__ partial, double* out) {
  if (threadIdx.x != 0) return;
  double t = 0.0;
  for (int q = 0; q < nblk; q++) t = fmax(t, partial[q]);
  *out = t;
}

__global__ void k_vmul(int64_t n, const double* __restrict__ d, const double* __restrict__ x,
                       double* __restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    y[i] = d[i] * x[i];
}

__global__ void k_axpy(int64_t n, double a, const double* __restrict__ x, double* y) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    y[i] = fma(a, x[i], y[i]);
}

// out[map[i]] = in[i]: values of one pattern placed into the union pattern
__global__ void k_scatter_values(int64_t m, const int64_t* __restrict__ map,
                                 const double* __restrict__ in, double* out) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < m; i += (int64_t)gridDim.x * NT)
    out[map[i]] = in[i];
}

// Hellmann-Feynman: per stored entry q of row r: ga = g x_r x_c, gb = -g lam x_r x_c
__global__ __launch_bounds__(NT) void k_hf(int64_t n, const int64_t* __restrict__ rowptr,
                                           const int32_t* __restrict__ col, const double* __restrict__ x,
                                           double g, double lam, double* ga, double* gb) {
  const int64_t row = (blockIdx.x * (int64_t)NT + threadIdx.x) >> 3;
  const int sub = threadIdx.x & 7;
  if (row >= n) return;
  const double xr = g * x[row];
  const int64_t e = rowptr[row + 1];
  for (int64_t q = rowptr[row] + sub; q < e; q += 8) {
    const double v = xr * x[col[q]];
    ga[q] = v;
    gb[q] = -lam * v;
  }
}

// Number of eigenvalues of the symmetric tridiagonal (alpha, beta) below x.
__device__ int sturm_count(int j, const double* alpha, const double* beta, double x, double tiny) {
  int cnt = 0;
  double d = 1.0;
  for (int i = 0; i < j; i++) {
    const double b2 = i > 0 ? beta[i - 1] * beta[i - 1] : 0.0;
    d = (alpha[i] - x) - (i > 0 ? b2 / d : 0.0);
    if (d == 0.0) d = -tiny;
    if (d < 0.0) cnt++;
  }
  return cnt;
}

// Thread i: eigenvalue i (ascending) by bisection and its eigenvector by
// inverse iteration with a pivoted tridiagonal LU; Y column-major j x j.
__global__ void k_tridiag_eig(int j, const double* __restrict__ alpha, const double* __restrict__ beta,
                              double* theta, double* Y, double* work) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= j) return;
  double lo = alpha[0], hi = alpha[0], nrm = 0.0;
  for (int q = 0; q < j; q++) {
    const double r = (q > 0 ? fabs(beta[q - 1]) : 0.0) + (q + 1 < j ? fabs(beta[q]) : 0.0);
    lo = fmin(lo, alpha[q] - r);
    hi = fmax(hi, alpha[q] + r);
    nrm = fmax(nrm, fabs(alpha[q]) + r);
  }
  const double eps = 2.220446049250313e-16;
  const double tiny = eps * (nrm > 0 ? nrm : 1.0) * 1e-3;
  lo -= eps * nrm + 1e-300;
  hi += eps * nrm + 1e-300;
  // lambda_i in [lo, hi): count(lo) <= i < count(hi)
  for (int it = 0; it < 200; it++) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(j, alpha, beta, mid, tiny) <= i) lo = mid; else hi = mid;
  }
  const double th = 0.5 * (lo + hi);
  theta[i] = th;
  // inverse iteration: (T - th I) y = b, Gaussian elimination with partial pivoting
  double* u0 = work + (int64_t)i * 4 * j;   // diagonal of U
  double* u1 = u0 + j;                      // first superdiagonal
  double* u2 = u1 + j;                      // second superdiagonal
  double* mul = u2 + j;                     // multipliers
  double* y = Y + (int64_t)i * j;
  // factor once
  {
    double d = alpha[0] - th, e = j > 1 ? beta[0] : 0.0, f = 0.0;
    for (int q = 0; q < j - 1; q++) {
      const double sub = beta[q];
      const double dn = alpha[q + 1] - th, en = q + 2 < j ? beta[q + 1] : 0.0;
      if (fabs(d) >= fabs(sub)) {
        const double l = d != 0.0 ? sub / d : 0.0;
        u0[q] = d; u1[q] = e; u2[q] = f; mul[q] = l;
        d = dn - l * e;
        e = en - l * f;
        f = 0.0;
        y[q] = 0.0;  // marker: no swap
      } else {
        const double l = d / sub;
        u0[q] = sub; u1[q] = dn; u2[q] = en; mul[q] = l;
        const double nd = e - l * dn, ne = f - l * en;
        d = nd;
        e = ne;
        f = 0.0;
        y[q] = 1.0;  // marker: swapped
      }
    }
    u0[j - 1] = d;
    u1[j - 1] = 0.0;
    u2[j - 1] = 0.0;
  }
  for (int q = 0; q < j; q++) if (u0[q] == 0.0) u0[q] = tiny;
  // row-interchange markers (kept in y during the factorization) move to the work tail
  double* mark = work + (int64_t)j * 4 * j + (int64_t)i * j;
  for (int q = 0; q < j; q++) mark[q] = q < j - 1 ? y[q] : 0.0;
  // start vector: a fixed pattern with no special symmetry
  for (int q = 0; q < j; q++) y[q] = 1.0 + 0.1 * (double)((q * 7 + i * 3) % 11);
  for (int iter = 0; iter < 3; iter++) {
    // forward: apply L^{-1} with the recorded row interchanges
    for (int q = 0; q < j - 1; q++) {
      if (mark[q] != 0.0) { const double t = y[q]; y[q] = y[q + 1]; y[q + 1] = t; }
      y[q + 1] -= mul[q] * y[q];
    }
    // back substitution with U (bandwidth 3)
    for (int q = j - 1; q >= 0; q--) {
      double s = y[q];
      if (q + 1 < j) s -= u1[q] * y[q + 1];
      if (q + 2 < j) s -= u2[q] * y[q + 2];
      y[q] = s / u0[q];
    }
    double nn = 0.0;
    for (int q = 0; q < j; q++) nn = fmax(nn, fabs(y[q]));
    if (nn == 0.0 || !isfinite(nn)) { for (int q = 0; q < j; q++) y[q] = q == i ? 1.0 : 0.0; break; }
    for (int q = 0; q < j; q++) y[q] /= nn;
  }
  double s2 = 0.0;
  for (int q = 0; q < j; q++) s2 += y[q] * y[q];
  const double inv = 1.0 / sqrt(s2);
  for (int q = 0; q < j; q++) y[q] *= inv;
}

// Re-orthogonalise eigenvectors of tightly clustered eigenvalues (modified
// Gram-Schmidt inside each cluster; one thread per cluster start).
__global__ void k_tridiag_cluster_mgs(int j, const double* __restrict__ theta, double* Y, double reltol) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= j) return;
  double nrm = 0.0;
  for (int q = 0; q < j; q++) nrm = fmax(nrm, fabs(theta[q]));
  const double tol = reltol * (nrm > 0 ? nrm : 1.0);
  if (i > 0 && theta[i] - theta[i - 1] <= tol) return;   // not a cluster start
  int e = i + 1;
  while (e < j && theta[e] - theta[e - 1] <= tol) e++;
  for (int a = i + 1; a < e; a++) {
    double* ya = Y + (int64_t)a * j;
    for (int b = i; b < a; b++) {
      const double* yb = Y + (int64_t)b * j;
      double d = 0.0;
      for (int q = 0; q < j; q++) d += ya[q] * yb[q];
      for (int q = 0; q < j; q++) ya[q] -= d * yb[q];
    }
    double s2 = 0.0;
    for (int q = 0; q < j; q++) s2 += ya[q] * ya[q];
    const double inv = 1.0 / sqrt(s2);
    for (int q = 0; q < j; q++) ya[q] *= inv;
  }
}

}  // namespace

void spmv2(int64_t n, const int64_t* rowptr, const int32_t* col, const double* a, const double* b,
           const double* x, double* ya, double* yb, hipStream_t s) {
  hipLaunchKernelGGL(k_spmv2, dim3(blocks_for(n * 8, NT)), dim3(NT), 0, s, n, rowptr, col, a, b, x,
                     ya, yb);
}

int multidot_blocks(int64_t n) { return blocks_for(n, kDotRows); }

void multidot(int64_t n, int m, const double* V, int64_t ldv, const double* w, double* partial,
              double* out, double alpha, hipStream_t s) {
  multidot2(n, m, V, ldv, w, 0, partial, out, alpha, s);
}

void multidot2(int64_t n, int m, const double* V, int64_t ldv, const double* W, int64_t ldw,
               double* partial, double* out, double alpha, hipStream_t s) {
  if (m <= 0) return;
  const int nb = multidot_blocks(n);
  hipLaunchKernelGGL(k_multidot_partial, dim3(nb), dim3(NT), 0, s, n, m, V, ldv, W, ldw, partial);
  hipLaunchKernelGGL(k_reduce_partials, dim3((m + 63) / 64), dim3(64), 0, s, nb, m, partial, out, alpha);
}

void multiaxpy(int64_t n, int m, const double* V, int64_t ldv, const double* h, double* w,
               const double* Vb, double* wb, hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_multiaxpy, dim3(blocks_for(n, NT * 4)), dim3(NT), m * sizeof(double), s, n, m,
                     V, ldv, h, w, Vb, wb);
}

void ritz_vectors(int64_t n, int j, int m, const double* V, int64_t ldv, const double* C,
                  const double* u, const double* cu, double* X, int64_t ldx, hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_ritz, dim3(blocks_for(n, NT * 2)), dim3(NT), (size_t)(j * m + m) * sizeof(double),
                     s, n, j, m, V, ldv, C, u, cu, X, ldx);
}

void gather_cols(int64_t n, int m, const double* X, int64_t ldx, const int32_t* perm, const double* f,
                 double* P, int64_t ldp, hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_gather_cols, dim3(blocks_for(n, NT * 4)), dim3(NT), 0, s, n, m, X, ldx, perm, f, P, ldp);
}

void diff_cols(int64_t n, int m, const double* X, int64_t ldx, const double* f, const double* P,
               int64_t ldp, double* D, int64_t ldd, hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_diff_cols, dim3(blocks_for(n, NT * 4)), dim3(NT), 0, s, n, m, X, ldx, f, P, ldp, D, ldd);
}

void scale_copy(int64_t n, double a, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_copy, dim3(blocks_for(n, NT * 4)), dim3(NT), 0, s, n, a, x, y);
}

void scale_by_dev(int64_t n, const double* sdev, int idx, bool inv, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_inplace_dev, dim3(blocks_for(n, NT * 4)), dim3(NT), 0, s, n, sdev, idx,
                     inv, y);
}

void residual(int64_t n, double lam, const double* ya, const double* yb, double* r, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(blocks_for(n, NT * 4)), dim3(NT), 0, s, n, lam, ya, yb, r);
}

void shifted_residual(int64_t n, const int64_t* rowptr, const int32_t* col, const double* a,
                      const double* b, double sigma, const double* x, const double* rhs, double* r,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_shifted_residual, dim3(blocks_for(n * 8, NT)), dim3(NT), 0, s, n, rowptr, col,
                     a, b, sigma, x, rhs, r);
}

void absmax(int64_t n, const double* x, double* partial, double* out, hipStream_t s) {
  const int nb = multidot_blocks(n);
  hipLaunchKernelGGL(k_absmax_partial, dim3(nb), dim3(NT), 0, s, n, x, partial);
  hipLaunchKernelGGL(k_max_partials, dim3(1), dim3(64), 0, s, nb, partial, out);
}

void vmul(int64_t n, const double* d, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_vmul, dim3(blocks_for(n, NT * 4)), dim3(NT), 0, s, n, d, x, y);
}

void axpy(int64_t n, double a, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3(blocks_for(n, NT * 4)), dim3(NT), 0, s, n, a, x, y);
}

void scatter_values(int64_t m, const int64_t* map, const double* in, double* out, hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_scatter_values, dim3(blocks_for(m, NT * 4)), dim3(NT), 0, s, m, map, in, out);
}

void hf_gradient(int64_t n, const int64_t* rowptr, const int32_t* col, const double* x, double g,
                 double lam, double* ga, double* gb, hipStream_t s) {
  hipLaunchKernelGGL(k_hf, dim3(blocks_for(n * 8, NT)), dim3(NT), 0, s, n, rowptr, col, x, g, lam, ga, gb);
}

void tridiag_eig(int j, const double* alpha, const double* beta, double* theta, double* Y,
                 double* work, hipStream_t s) {
  hipLaunchKernelGGL(k_tridiag_eig, dim3((j + 63) / 64), dim3(64), 0, s, j, alpha, beta, theta, Y, work);
  hipLaunchKernelGGL(k_tridiag_cluster_mgs, dim3((j + 63) / 64), dim3(64), 0, s, j, theta, Y, 1e-10);
}

}  // namespace kth
