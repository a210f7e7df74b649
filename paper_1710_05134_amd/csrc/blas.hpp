// Launchers of the vector kernels (blas.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace kth {

void spmv2(int64_t n, const int64_t* rowptr, const int32_t* col, const double* a, const double* b,
           const double* x, double* ya, double* yb, hipStream_t s);
int multidot_blocks(int64_t n);
// out[c] = alpha * sum_i V[i, c] w[i], c < m; partial: multidot_blocks(n) * m doubles
void multidot(int64_t n, int m, const double* V, int64_t ldv, const double* w, double* partial,
              double* out, double alpha, hipStream_t s);
// out[c] = alpha * sum_i V[i, c] W[i, c]  (ldw = 0: W is one vector)
void multidot2(int64_t n, int m, const double* V, int64_t ldv, const double* W, int64_t ldw,
               double* partial, double* out, double alpha, hipStream_t s);
// P[:, q] = f[q] X[:, perm[q]]   (perm, f: device arrays of m entries)
void gather_cols(int64_t n, int m, const double* X, int64_t ldx, const int32_t* perm, const double* f,
                 double* P, int64_t ldp, hipStream_t s);
// D[:, q] = f[q] X[:, q] - P[:, q]
void diff_cols(int64_t n, int m, const double* X, int64_t ldx, const double* f, const double* P,
               int64_t ldp, double* D, int64_t ldd, hipStream_t s);
// w -= V h  (and wb -= Vb h when Vb is given)
void multiaxpy(int64_t n, int m, const double* V, int64_t ldv, const double* h, double* w,
               const double* Vb, double* wb, hipStream_t s);
// X[:, q] = V C[:, q] + u cu[q]
void ritz_vectors(int64_t n, int j, int m, const double* V, int64_t ldv, const double* C,
                  const double* u, const double* cu, double* X, int64_t ldx, hipStream_t s);
void scale_copy(int64_t n, double a, const double* x, double* y, hipStream_t s);
void scale_by_dev(int64_t n, const double* sdev, int idx, bool inv, double* y, hipStream_t s);
void residual(int64_t n, double lam, const double* ya, const double* yb, double* r, hipStream_t s);
// r = rhs - (A - sigma B) x (rhs null: r = (A - sigma B) x), entries fma(-sigma, b, a)
// as in the factorization
void shifted_residual(int64_t n, const int64_t* rowptr, const int32_t* col, const double* a,
                      const double* b, double sigma, const double* x, const double* rhs, double* r,
                      hipStream_t s);
// *out = max_i |x_i| (partial: multidot_blocks(n) doubles)
void absmax(int64_t n, const double* x, double* partial, double* out, hipStream_t s);
void axpy(int64_t n, double a, const double* x, double* y, hipStream_t s);
// y = d .* x (elementwise)
void vmul(int64_t n, const double* d, const double* x, double* y, hipStream_t s);
// out[map[i]] = in[i], i < m (device arrays)
void scatter_values(int64_t m, const int64_t* map, const double* in, double* out, hipStream_t s);
void hf_gradient(int64_t n, const int64_t* rowptr, const int32_t* col, const double* x, double g,
                 double lam, double* ga, double* gb, hipStream_t s);
// eigenvalues (ascending) and eigenvectors (columns of Y, j x j) of the
// symmetric tridiagonal (alpha[j], beta[j-1]); work: 5 j^2 doubles
void tridiag_eig(int j, const double* alpha, const double* beta, double* theta, double* Y,
                 double* work, hipStream_t s);

}  // namespace kth
