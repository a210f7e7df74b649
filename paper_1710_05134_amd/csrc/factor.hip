// Numeric multifrontal LDL^T of A - sigma B on gfx950 (FP64), and the sign
// count of D (Sylvester's law of inertia, Section 2.1; Alg. 1').
//
// Per tree level, leaves first:
//   * fronts with nf <= kSmallMaxNf: one workgroup each, the whole front in LDS:
//     assemble originals fma(-sigma, b, a), add children's update blocks, then
//     unblocked Bunch-Kaufman over the fully-summed columns, write the panel,
//     D and the update block.
//   * larger fronts: k_front_init assembles pieces of 16 columns x 512 rows in
//     HBM (each entry written once: children's contributions gathered through
//     inverse maps, then the original entries added); then per pivot tile of kNB
//     columns: k_tile_factor (Bunch-Kaufman inside the tile), k_panel_trsm (rows
//     below the tile: L21 = S21 P^T L11^{-T} D^{-1}, and W = L21 D kept
//     panel-shaped); the column block of each tile is first brought up to date
//     left-looking, C -= L(:, <k0) W(tile rows, <k0)^T on FP64 MFMA (k_gemm_lt),
//     and once all tiles are done the contribution block receives
//     -L_u W_u^T with depth ns in one product.  The next tile's diagonal block
//     gets the columns before the current tile ahead, in the same launch as the
//     current column block's rows, and the current tile's columns in the panel
//     solve of the next tile's rows; the host then runs the next tile's
//     factorization on a second stream.
// Row interchanges stay inside a tile; rows of earlier panels are not swapped --
// the solve applies each tile's permutation when it reaches that tile.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device.hpp"

namespace kth {

namespace {

constexpr double kAlphaBK = 0.6403882032022076;  // (1 + sqrt(17)) / 8

__device__ inline unsigned long long dbits(double x) { return __double_as_longlong(x); }

// 64-bit lane exchange by DPP (CTRL: a quad_perm or row-mirror control word).
template <int CTRL>
__device__ inline unsigned long long dpp_u64(unsigned long long v) {
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)(v & 0xffffffffull), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(v >> 32), CTRL, 0xF, 0xF, false);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

__device__ inline unsigned long long readlane_u64(unsigned long long v, int l) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v & 0xffffffffull), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
  return ((unsigned long long)hi << 32) | lo;
}

// Maximum of v over the 64 lanes, returned to every lane: DPP swaps within quads
// (xor 1, xor 2), half rows and rows (mirrors), then the four row maxima.
__device__ inline unsigned long long wave_max_u64(unsigned long long v) {
  unsigned long long o;
  o = dpp_u64<0xB1>(v); v = o > v ? o : v;    // quad_perm [1,0,3,2]
  o = dpp_u64<0x4E>(v); v = o > v ? o : v;    // quad_perm [2,3,0,1]
  o = dpp_u64<0x141>(v); v = o > v ? o : v;   // row_half_mirror
  o = dpp_u64<0x140>(v); v = o > v ? o : v;   // row_mirror
  const unsigned long long a = readlane_u64(v, 0), b = readlane_u64(v, 16);
  const unsigned long long c = readlane_u64(v, 32), d = readlane_u64(v, 48);
  const unsigned long long ab = a > b ? a : b, cd = c > d ? c : d;
  return ab > cd ? ab : cd;
}

// Maximum of v over the 64 lanes, returned to every lane (the same DPP steps on
// 32 bits).
__device__ inline unsigned wave_max_u32(unsigned v) {
  unsigned o;
  o = (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false); v = o > v ? o : v;
  o = (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false); v = o > v ? o : v;
  o = (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false); v = o > v ? o : v;
  o = (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false); v = o > v ? o : v;
  const unsigned a = (unsigned)__builtin_amdgcn_readlane((int)v, 0);
  const unsigned b = (unsigned)__builtin_amdgcn_readlane((int)v, 16);
  const unsigned c = (unsigned)__builtin_amdgcn_readlane((int)v, 32);
  const unsigned d = (unsigned)__builtin_amdgcn_readlane((int)v, 48);
  const unsigned ab = a > b ? a : b, cd = c > d ? c : d;
  return ab > cd ? ab : cd;
}

// Value of v in lane p (p uniform) through v_readlane.
__device__ inline double lane_value(double v, int p) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), p);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), p);
  return __hiloint2double(hi, lo);
}
__device__ inline float lane_value(float v, int p) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), p));
}

// Block-wide argmax of (v, idx): larger v wins, ties -> smaller idx (idx -1 = none).
template <int NT>
__device__ inline void block_argmax(double& v, int& idx, double* sv, int* si) {
  for (int off = 32; off > 0; off >>= 1) {
    double ov = __shfl_xor(v, off);
    int oi = __shfl_xor(idx, off);
    if (ov > v || (ov == v && oi >= 0 && (idx < 0 || oi < idx))) { v = ov; idx = oi; }
  }
  if constexpr (NT == 64) return;   // one wavefront: every lane already holds the result
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { sv[wave] = v; si[wave] = idx; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < NT / 64; w++) {
      if (sv[w] > sv[0] || (sv[w] == sv[0] && si[w] >= 0 && (si[0] < 0 || si[w] < si[0]))) {
        sv[0] = sv[w]; si[0] = si[w];
      }
    }
  }
  __syncthreads();
  v = sv[0];
  idx = si[0];
  __syncthreads();
}

template <int NT>
__device__ inline double block_max(double v, double* sv) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  if constexpr (NT == 64) return v;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sv[wave] = v;
  __syncthreads();
  double r = sv[0];
  for (int w = 1; w < NT / 64; w++) r = fmax(r, sv[w]);
  __syncthreads();
  return r;
}

// Symmetric interchange of rows/columns k < r of a lower-stored LDS matrix.
template <int NT, typename T>
__device__ inline void lds_sym_swap(T* F, int ld, int nrows, int k, int r) {
  // tasks: [0,k): columns left of k;  k: diagonal;  (k,r): the band between;  (r,nrows): below r
  for (int x = threadIdx.x; x < nrows - 1; x += NT) {
    if (x < k) {
      T t = F[k + x * ld]; F[k + x * ld] = F[r + x * ld]; F[r + x * ld] = t;
    } else if (x == k) {
      T t = F[k + k * ld]; F[k + k * ld] = F[r + r * ld]; F[r + r * ld] = t;
    } else if (x < r) {
      T t = F[x + k * ld]; F[x + k * ld] = F[r + x * ld]; F[r + x * ld] = t;
    } else {
      int i = x + 1;
      T t = F[i + k * ld]; F[i + k * ld] = F[i + r * ld]; F[i + r * ld] = t;
    }
  }
}

struct BKCounts {
  unsigned long long neg, zero, pos, n2x2;
  double mind, maxl;
};

// Unblocked Bunch-Kaufman LDL^T of the leading `ncand` columns of the nrows x nrows
// lower-stored LDS matrix F; candidate pivot rows are the first ncand rows; all
// nrows rows are eliminated against them (rows >= ncand form L21 and the Schur
// complement).  lp[] receives the pivot order, d[]/e[] the blocks of D.
// On return F holds unit-lower L in the eliminated columns and the Schur
// complement in the trailing block.  Counts accumulate in thread 0's cnt.
template <int NT, typename T>
__device__ void bk_factor_lds(T* F, int ld, int nrows, int ncand, int* lp, T* d,
                              T* e, T* lcol, BKCounts& cnt, double* sv, int* si) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = NT / 64;
  double maxl = 0.0;
  for (int q = tid; q < ncand; q += NT) lp[q] = q;
  __syncthreads();
  int k = 0;
  while (k < ncand) {
    // gamma_1 = max_{k < i < ncand} |F(i,k)|, argmax r (ties: smallest row)
    int r;
    double g1;
    if constexpr (NT == 64) {
      // one wavefront: a single 64-bit max over keys |x| (low 8 mantissa bits replaced by
      // 128 - row, so ties go to the smaller row; key 0 = no candidate)
      unsigned long long key = 0;
      for (int i = k + 1 + tid; i < ncand; i += NT) {
        unsigned long long kk2 = (dbits(fabs((double)F[i + k * ld])) & ~0xFFull) | (unsigned long long)(128 - i);
        key = kk2 > key ? kk2 : key;
      }
      for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(key, off);
        key = o > key ? o : key;
      }
      if (key == 0) { r = k; g1 = 0.0; }
      else { r = 128 - (int)(key & 0xFFull); g1 = fabs((double)F[r + k * ld]); }
    } else {
      double v = -1.0;
      int idx = -1;
      for (int i = k + 1 + tid; i < ncand; i += NT) {
        double x = fabs((double)F[i + k * ld]);
        if (x > v) { v = x; idx = i; }
      }
      block_argmax<NT>(v, idx, sv, si);
      g1 = idx < 0 ? 0.0 : v;
      r = idx < 0 ? k : idx;
    }
    const double akk = fabs((double)F[k + k * ld]);
    int kind = 0;  // 0: 1x1 at k; 1: 1x1 at r (swap k,r); 2: 2x2 (k, r -> k+1)
    if (!(g1 == 0.0 || akk >= kAlphaBK * g1)) {
      double gv = 0.0;
      for (int i = k + tid; i < ncand; i += NT) {
        if (i == r) continue;
        double x = i < r ? fabs((double)F[r + i * ld]) : fabs((double)F[i + r * ld]);
        gv = fmax(gv, x);
      }
      const double gr = block_max<NT>(gv, sv);
      if (akk * gr >= kAlphaBK * g1 * g1) kind = 0;
      else if (fabs((double)F[r + r * ld]) >= kAlphaBK * gr) kind = 1;
      else kind = 2;
    }
    __syncthreads();  // every thread has read the pivot candidates before any swap
    if (kind == 1) {
      lds_sym_swap<NT, T>(F, ld, nrows, k, r);
      if (tid == 0) { int t = lp[k]; lp[k] = lp[r]; lp[r] = t; }
      __syncthreads();
    } else if (kind == 2 && r != k + 1) {
      lds_sym_swap<NT, T>(F, ld, nrows, k + 1, r);
      if (tid == 0) { int t = lp[k + 1]; lp[k + 1] = lp[r]; lp[r] = t; }
      __syncthreads();
    }
    if (kind < 2) {
      const T dk = F[k + k * ld];
      if (tid == 0) {
        d[k] = dk; e[k] = 0.0;
        if (dk < 0) cnt.neg++; else if (dk > 0) cnt.pos++; else cnt.zero++;
        cnt.mind = fmin(cnt.mind, fabs((double)dk));
      }
      if (dk != 0.0) {
        for (int i = k + 1 + tid; i < nrows; i += NT) lcol[i] = F[i + k * ld] / dk;
        __syncthreads();
        if constexpr (NT == 64) {
          // lane owns row i: F(i, j) -= l_i F(j, k) for k < j <= i; loads of the next
          // group are issued before the stores of the current one (no aliasing: other j)
          const int i = lane;
          if (i > k && i < nrows) {
            const T li = lcol[i];
            int j = k + 1;
            if (j + 3 <= i) {
              T c0 = F[j + k * ld], c1 = F[j + 1 + k * ld], c2 = F[j + 2 + k * ld], c3 = F[j + 3 + k * ld];
              T a0 = F[i + j * ld], a1 = F[i + (j + 1) * ld], a2 = F[i + (j + 2) * ld], a3 = F[i + (j + 3) * ld];
              for (;;) {
                const T r0 = a0 - li * c0, r1 = a1 - li * c1, r2 = a2 - li * c2, r3 = a3 - li * c3;
                const int jn = j + 4;
                const bool more = jn + 3 <= i;
                if (more) {
                  c0 = F[jn + k * ld]; c1 = F[jn + 1 + k * ld]; c2 = F[jn + 2 + k * ld]; c3 = F[jn + 3 + k * ld];
                  a0 = F[i + jn * ld]; a1 = F[i + (jn + 1) * ld]; a2 = F[i + (jn + 2) * ld]; a3 = F[i + (jn + 3) * ld];
                }
                F[i + j * ld] = r0;
                F[i + (j + 1) * ld] = r1;
                F[i + (j + 2) * ld] = r2;
                F[i + (j + 3) * ld] = r3;
                j = jn;
                if (!more) break;
              }
            }
            for (; j <= i; j++) F[i + j * ld] -= li * F[j + k * ld];
          }
        } else {
          for (int j = k + 1 + wave; j < nrows; j += NW) {
            const T fj = F[j + k * ld];
            for (int i = j + lane; i < nrows; i += 64) F[i + j * ld] -= lcol[i] * fj;
          }
        }
        __syncthreads();
        for (int i = k + 1 + tid; i < nrows; i += NT) {
          F[i + k * ld] = lcol[i];
          maxl = fmax(maxl, fabs((double)lcol[i]));
        }
      } else {
        for (int i = k + 1 + tid; i < nrows; i += NT) F[i + k * ld] = 0.0;
      }
      if (tid == 0) F[k + k * ld] = 1.0;
      __syncthreads();
      k += 1;
    } else {
      const T a = F[k + k * ld], b = F[(k + 1) + k * ld], c = F[(k + 1) + (k + 1) * ld];
      const T det = a * c - b * b;
      if (tid == 0) {
        d[k] = a; e[k] = b; d[k + 1] = c; e[k + 1] = 0.0;
        const T tr = a + c;
        if (det < 0) { cnt.neg++; cnt.pos++; }
        else if (det > 0) { if (tr < 0) cnt.neg += 2; else cnt.pos += 2; }
        else { cnt.zero++; if (tr < 0) cnt.neg++; else if (tr > 0) cnt.pos++; else cnt.zero++; }
        cnt.n2x2++;
        const T m = 0.5 * tr, q = sqrt(0.25 * (a - c) * (a - c) + b * b);
        cnt.mind = fmin(cnt.mind, fmin(fabs((double)m - q), fabs((double)m + q)));
      }
      T* lcol2 = lcol + ld;
      for (int i = k + 2 + tid; i < nrows; i += NT) {
        const T w1 = F[i + k * ld], w2 = F[i + (k + 1) * ld];
        lcol[i] = (c * w1 - b * w2) / det;
        lcol2[i] = (a * w2 - b * w1) / det;
      }
      __syncthreads();
      if constexpr (NT == 64) {
        const int i = lane;
        if (i > k + 1 && i < nrows) {
          const T l1 = lcol[i], l2 = lcol2[i];
          int j = k + 2;
          for (; j + 1 <= i; j += 2) {
            const T w10 = F[j + k * ld], w20 = F[j + (k + 1) * ld];
            const T w11 = F[j + 1 + k * ld], w21 = F[j + 1 + (k + 1) * ld];
            const T a0 = F[i + j * ld], a1 = F[i + (j + 1) * ld];
            F[i + j * ld] = a0 - (l1 * w10 + l2 * w20);
            F[i + (j + 1) * ld] = a1 - (l1 * w11 + l2 * w21);
          }
          for (; j <= i; j++) F[i + j * ld] -= l1 * F[j + k * ld] + l2 * F[j + (k + 1) * ld];
        }
      } else {
        for (int j = k + 2 + wave; j < nrows; j += NW) {
          const T w1 = F[j + k * ld], w2 = F[j + (k + 1) * ld];
          for (int i = j + lane; i < nrows; i += 64) F[i + j * ld] -= lcol[i] * w1 + lcol2[i] * w2;
        }
      }
      __syncthreads();
      for (int i = k + 2 + tid; i < nrows; i += NT) {
        F[i + k * ld] = lcol[i];
        F[i + (k + 1) * ld] = lcol2[i];
        maxl = fmax(maxl, fmax(fabs((double)lcol[i]), fabs((double)lcol2[i])));
      }
      if (tid == 0) { F[k + k * ld] = 1.0; F[(k + 1) + k * ld] = 0.0; F[(k + 1) + (k + 1) * ld] = 1.0; }
      __syncthreads();
      k += 2;
    }
  }
  maxl = block_max<NT>(maxl, sv);
  if (tid == 0) cnt.maxl = fmax(cnt.maxl, maxl);
}

// Symmetric interchange of indices a < r of a pivot tile in the middle of its
// factorization at step k: the trailing lower triangle (columns >= k) lives in F,
// the finished multiplier columns (< k) in Lo.
template <typename T>
__device__ inline void tile_sym_swap(T* F, T* Lo, int ld, int kb, int k, int a, int r) {
  for (int x = threadIdx.x; x < kb - 1; x += blockDim.x) {
    if (x < a) {
      T* M = x < k ? Lo : F;
      T t = M[a + x * ld]; M[a + x * ld] = M[r + x * ld]; M[r + x * ld] = t;
    } else if (x == a) {
      T t = F[a + a * ld]; F[a + a * ld] = F[r + r * ld]; F[r + r * ld] = t;
    } else if (x < r) {
      T t = F[x + a * ld]; F[x + a * ld] = F[r + x * ld]; F[r + x * ld] = t;
    } else {
      int i = x + 1;
      T t = F[i + a * ld]; F[i + a * ld] = F[i + r * ld]; F[i + r * ld] = t;
    }
  }
}

// Bunch-Kaufman LDL^T of one kb x kb pivot tile (kb <= kNB) by 4 wavefronts with
// the trailing matrix in registers: lane i of wave w holds row i's entries in the
// columns j = 4m + w, R[m] (m = 0..15, static indices; entries above the diagonal
// are not kept meaningful and never read).  Per pivot step the waves owning
// columns k and k + 1 publish them (rows below the pivot, zero elsewhere) to an
// LDS buffer of the step's parity; after one barrier every wave finds the pivot
// itself from that column (lanes = rows, DPP maxima) and updates its registers
// with 16 independent broadcast reads of it.  When the search must look at row r
// (gamma_r), the registers are written to F (the tile in LDS; only its lower
// triangle is read), searched and, for an interchange, permuted there and loaded
// back.  The pivot rule and the rounding are those of the plain
// column-by-column algorithm: every entry F(i, j), k < j <= i, receives one fused
// multiply-add per pivot step, in step order.  Multipliers go to Lo (strictly
// below the diagonal, 0 inside 2x2 blocks; zeroed here), interchanges to lp, the
// block diagonal to d, e.
// A row's kNB / 4 register entries as one vector: an element picked by a
// wave-uniform index is read through indirect register addressing.
template <typename T> struct RowRegs { typedef T type __attribute__((ext_vector_type(kNB / 4))); };

// Column k of the registers, published by the wave that owns it: yb[0][i] = F(i, k)
// for k < i < kb (zero elsewhere); pv[0] = F(k, k), pv[1] = F(k + 1, k).
template <typename T>
__device__ __forceinline__ void bk_publish(const typename RowRegs<T>::type& R, T (&yb)[2][kNB],
                                           T (&pv)[3], int k, int kb, int wave, int i) {
  if (wave == (k & 3)) {
    const T v = R[k >> 2];
    yb[0][i] = (i > k && i < kb) ? v : (T)0.0;
    if (i == k) pv[0] = v;
    if (i == k + 1) pv[1] = v;
  }
}
// Column k + 1 (for a 2x2 pivot): yb[1][i] = F(i, k + 1) for k + 1 < i < kb (zero
// elsewhere); pv[2] = F(k + 1, k + 1).
template <typename T>
__device__ __forceinline__ void bk_publish_next(const typename RowRegs<T>::type& R, T (&yb)[2][kNB],
                                                T (&pv)[3], int k, int kb, int wave, int i) {
  if (k + 1 < kb && wave == ((k + 1) & 3)) {
    const T v = R[(k + 1) >> 2];
    yb[1][i] = (i > k + 1 && i < kb) ? v : (T)0.0;
    if (i == k + 1) pv[2] = v;
  }
}

template <typename T>
__device__ void bk_tile_regs(T* F, T* Lo, int ld, int kb, int* lp, T* d, T* e, BKCounts& cnt) {
  constexpr int NM = kNB / 4;
  __shared__ T yb[2][2][kNB];   // [parity][column k, column k + 1][row]
  __shared__ T pv[2][3];        // [parity]: F(k, k), F(k + 1, k), F(k + 1, k + 1)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = lane;
  double maxl = 0.0;
  if (tid < kNB) lp[tid] = tid;
  for (int x = tid; x < kNB * kNB; x += blockDim.x) Lo[(x & 63) + (x >> 6) * ld] = 0.0;
  typename RowRegs<T>::type R;
#pragma unroll
  for (int m = 0; m < NM; m++) {
    const int j = 4 * m + wave;
    R[m] = (j <= i && i < kb) ? F[i + j * ld] : (T)0.0;
  }
  int k = 0, par = 0;
  while (k < kb) {
    bk_publish<T>(R, yb[par], pv[par], k, kb, wave, i);
    __syncthreads();
    // gamma_1 and its row r among the candidates k < i < kb (ties: smallest row)
    // (key: the upper 24 bits of |F(i, k)|, then 128 - i; rows whose magnitudes agree
    // in exponent and the leading 12 mantissa bits count as ties)
    const T ck = yb[par][0][i];
    unsigned key = 0;
    if (i > k && i < kb)
      key = ((unsigned)(dbits(fabs((double)ck)) >> 32) & ~0xFFu) | (unsigned)(128 - i);
    key = wave_max_u32(key);
    const int r = key == 0 ? k : 128 - (int)(key & 0xFFu);
    const double g1 = key == 0 ? 0.0 : fabs((double)yb[par][0][r]);
    const double akk = fabs((double)pv[par][0]);
    int kind = 0;
    if (!(g1 == 0.0 || akk >= kAlphaBK * g1)) {
      // row and column r: through the tile in LDS
#pragma unroll
      for (int m = 0; m < NM; m++) F[i + (4 * m + wave) * ld] = R[m];
      __syncthreads();
      unsigned long long gb = 0;   // |.| >= 0: bit patterns order as the values
      if (i >= k && i < kb && i != r)
        gb = dbits(i < r ? fabs((double)F[r + i * ld]) : fabs((double)F[i + r * ld]));
      const double gr = __longlong_as_double((long long)wave_max_u64(gb));
      if (akk * gr >= kAlphaBK * g1 * g1) kind = 0;
      else if (fabs((double)F[r + r * ld]) >= kAlphaBK * gr) kind = 1;
      else kind = 2;
      if (kind == 1 || (kind == 2 && r != k + 1)) {
        const int a = kind == 1 ? k : k + 1;
        __syncthreads();   // every wave has read row r
        tile_sym_swap<T>(F, Lo, ld, kb, k, a, r);
        if (tid == 0) { int t = lp[a]; lp[a] = lp[r]; lp[r] = t; }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < NM; m++) R[m] = F[i + (4 * m + wave) * ld];
        bk_publish<T>(R, yb[par ^ 1], pv[par ^ 1], k, kb, wave, i);   // interchanged, other buffer
        if (kind == 2) bk_publish_next<T>(R, yb[par ^ 1], pv[par ^ 1], k, kb, wave, i);
        __syncthreads();
        par ^= 1;
      } else if (kind == 2) {
        bk_publish_next<T>(R, yb[par], pv[par], k, kb, wave, i);
        __syncthreads();
      }
    }
    if (kind < 2) {
      const T dk = pv[par][0];
      // the 1x1 pivots' signs and magnitudes are counted after the loop, from d
      if (tid == 0) { d[k] = dk; e[k] = 0.0; }
      if (dk != 0.0) {
        const bool act = i > k && i < kb;
        const T li = act ? yb[par][0][i] / dk : (T)0.0;
        // rows k < i < kb, columns k < j <= i: column k is zero outside k < j < kb, li
        // outside k < i < kb; entries above the diagonal take values never read
#pragma unroll
        for (int m = 0; m < NM; m++) R[m] = R[m] - li * yb[par][0][4 * m + wave];
        // multipliers: by the wave that published column k (not the next column's)
        if (wave == (k & 3) && act) { Lo[i + k * ld] = li; maxl = fmax(maxl, fabs((double)li)); }
      }
      k += 1;
    } else {
      const T a = pv[par][0], b = pv[par][1], c = pv[par][2];
      const T det = a * c - b * b;
      if (tid == 0) {
        d[k] = a; e[k] = b; d[k + 1] = c; e[k + 1] = 0.0;
        const T tr = a + c;
        if (det < 0) { cnt.neg++; cnt.pos++; }
        else if (det > 0) { if (tr < 0) cnt.neg += 2; else cnt.pos += 2; }
        else { cnt.zero++; if (tr < 0) cnt.neg++; else if (tr > 0) cnt.pos++; else cnt.zero++; }
        cnt.n2x2++;
        const T m = 0.5 * tr, q = sqrt(0.25 * (a - c) * (a - c) + b * b);
        cnt.mind = fmin(cnt.mind, fmin(fabs((double)m - q), fabs((double)m + q)));
      }
      const bool act = i > k + 1 && i < kb;
      T l1 = 0.0, l2 = 0.0;
      if (act) {
        const T w1 = yb[par][0][i], w2 = yb[par][1][i];
        l1 = (c * w1 - b * w2) / det;
        l2 = (a * w2 - b * w1) / det;
      }
      // columns j > k + 1 only: column k's entry F(k + 1, k) is masked here
#pragma unroll
      for (int m = 0; m < NM; m++) {
        const int j = 4 * m + wave;
        const T u1 = j > k + 1 ? yb[par][0][j] : (T)0.0;
        R[m] = R[m] - (l1 * u1 + l2 * yb[par][1][j]);
      }
      if (wave == (k & 3) && act) {
        Lo[i + k * ld] = l1;
        Lo[i + (k + 1) * ld] = l2;
        maxl = fmax(maxl, fmax(fabs((double)l1), fabs((double)l2)));
      }
      k += 2;
    }
    par ^= 1;
  }
  // 1x1 pivots (e = 0 here and before): counts by sign and the least magnitude, the
  // same tallies the steps would have made; largest multiplier over all waves
  __shared__ double mx[4];
  for (int off = 32; off > 0; off >>= 1) maxl = fmax(maxl, __shfl_xor(maxl, off));
  if (lane == 0) mx[wave] = maxl;
  __syncthreads();   // d, e and mx complete
  if (wave == 0) {
    const bool one = i < kb && e[i] == 0.0 && (i == 0 || e[i - 1] == 0.0);
    const T di = one ? d[i] : (T)0.0;
    const unsigned long long neg = __ballot(one && di < 0), pos = __ballot(one && di > 0);
    const unsigned long long zer = __ballot(one && di == 0);
    double mn = one ? fabs((double)di) : (double)INFINITY;
    for (int off = 32; off > 0; off >>= 1) mn = fmin(mn, __shfl_xor(mn, off));
    if (lane == 0) {
      cnt.neg += __popcll(neg);
      cnt.pos += __popcll(pos);
      cnt.zero += __popcll(zer);
      cnt.mind = fmin(cnt.mind, mn);
      cnt.maxl = fmax(cnt.maxl, fmax(fmax(mx[0], mx[1]), fmax(mx[2], mx[3])));
    }
  }
}

__device__ inline void flush_counts(const BKCounts& c, FactStats* st) {
  if (c.neg) atomicAdd(&st->neg, c.neg);
  if (c.zero) atomicAdd(&st->zero, c.zero);
  if (c.pos) atomicAdd(&st->pos, c.pos);
  if (c.n2x2) atomicAdd(&st->n2x2, c.n2x2);
  atomicMin(&st->min_d_bits, dbits(c.mind));
  atomicMax(&st->max_l_bits, dbits(c.maxl));
}

__global__ void k_fill_stats(FactStats* st) {
  st += blockIdx.x;
  if (threadIdx.x == 0) {
    st->neg = st->zero = st->pos = st->n2x2 = 0;
    st->min_d_bits = dbits(INFINITY);
    st->max_l_bits = 0;
  }
}

// ---------------------------------------------------------------------------
// Small fronts: everything in LDS.
// ---------------------------------------------------------------------------
template <int NT, typename T>
__global__ __launch_bounds__(NT) void k_small_fronts(FrontMeta M, const int32_t* fronts,
                                                     const double* __restrict__ aval,
                                                     const double* __restrict__ bval,
                                                     Batch bt, T* L, T* U,
                                                     double* D, double* E, int32_t* tperm,
                                                     FactStats* st) {
  const int64_t bidx = blockIdx.y;
  L += bidx * bt.sL; U += bidx * bt.sU; D += bidx * bt.sN; E += bidx * bt.sN;
  tperm += bidx * bt.sN; st += bidx;
  const double* sigma_dev = bt.sig + bidx;
  extern __shared__ unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  __shared__ double sv[NT / 64];
  __shared__ int si[NT / 64];
  __shared__ int lp[kSmallMaxNf];
  __shared__ T dd[kSmallMaxNf], ee[kSmallMaxNf];
  __shared__ T lcol[2 * kSmallMaxNf];
  const int s = fronts[blockIdx.x];
  const int tid = threadIdx.x;
  const int64_t f0 = M.sfirst[s];
  const int ns = (int)(M.sfirst[s + 1] - f0);
  const int nf = (int)(M.rptr[s + 1] - M.rptr[s]);
  const int nu = nf - ns;
  const double sigma = *sigma_dev;
  T* F = smem;
  for (int q = tid; q < nf * nf; q += NT) F[q] = 0.0;
  __syncthreads();
  for (int64_t e = M.acptr[f0] + tid; e < M.acptr[f0 + ns]; e += NT) {
    const int64_t p = M.asrc[e];
    F[M.adst[e]] = fma(-sigma, bval[p], aval[p]);
  }
  __syncthreads();
  for (int64_t q = M.cptr[s]; q < M.cptr[s + 1]; q++) {
    const int c = M.clist[q];
    const int nuc = (int)(M.rptr[c + 1] - M.rptr[c] - (M.sfirst[c + 1] - M.sfirst[c]));
    const T* Uc = U + M.uptr[c];
    const int32_t* map = M.emap + M.eptr[c];
    for (int x = tid; x < nuc * nuc; x += NT) {
      const int a = x % nuc, b = x / nuc;
      if (a >= b) F[map[a] + map[b] * nf] += Uc[a + (int64_t)b * nuc];
    }
    __syncthreads();
  }
  BKCounts cnt{0, 0, 0, 0, INFINITY, 0.0};
  bk_factor_lds<NT, T>(F, nf, nf, ns, lp, dd, ee, lcol, cnt, sv, si);
  T* Lp = L + M.lptr[s];
  for (int q = tid; q < nf * ns; q += NT) Lp[q] = F[q];
  for (int q = tid; q < ns; q += NT) {
    D[f0 + q] = dd[q];
    E[f0 + q] = ee[q];
    tperm[f0 + q] = lp[q];
  }
  if (M.uptr[s] >= 0 && nu > 0) {
    T* Ub = U + M.uptr[s];
    for (int x = tid; x < nu * nu; x += NT) {
      const int a = x % nu, b = x / nu;
      if (a >= b) Ub[x] = F[(ns + a) + (ns + b) * nf];
    }
  }
  if (tid == 0) flush_counts(cnt, st);
}

// ---------------------------------------------------------------------------
// Large fronts: assembly of a column chunk.
// ---------------------------------------------------------------------------
template <typename T>
struct FrontRef {
  T* Lp;  // panel, ld nf
  T* Ub;  // update block, ld nu (may be null)
  int nf, ns, nu;
  __device__ inline T* at(int i, int j) const {
    return j < ns ? Lp + i + (int64_t)j * nf : Ub + (i - ns) + (int64_t)(j - ns) * nu;
  }
};

template <typename T>
__device__ inline FrontRef<T> front_ref(const FrontMeta& M, int s, T* L, T* U) {
  FrontRef<T> f;
  const int64_t f0 = M.sfirst[s];
  f.ns = (int)(M.sfirst[s + 1] - f0);
  f.nf = (int)(M.rptr[s + 1] - M.rptr[s]);
  f.nu = f.nf - f.ns;
  f.Lp = L + M.lptr[s];
  f.Ub = M.uptr[s] >= 0 ? U + M.uptr[s] : nullptr;
  return f;
}

template <int NT, typename T>
__global__ __launch_bounds__(NT) void k_front_init(FrontMeta M, const Int2* tasks,
                                                   const double* __restrict__ aval,
                                                   const double* __restrict__ bval,
                                                   Batch bt, T* L, T* U) {
  const int64_t bidx = blockIdx.y;
  L += bidx * bt.sL; U += bidx * bt.sU;
  const double* sigma_dev = bt.sig + bidx;
  const Int2 tk = tasks[blockIdx.x];
  const int s = tk.a;
  const FrontRef<T> f = front_ref<T>(M, s, L, U);
  // the task is column chunk c0 .. c1 - 1, rows r0 .. r1 - 1 (lower triangle only)
  const int nrb = (f.nf + kAsmRows - 1) / kAsmRows;
  const int chunk = tk.b / nrb, rb = tk.b - chunk * nrb;
  const int c0 = chunk * kAsmCols, c1 = min(c0 + kAsmCols, f.nf);
  const int r0 = rb * kAsmRows, r1 = min(r0 + kAsmRows, f.nf);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = NT / 64;
  const double sigma = *sigma_dev;
  // every entry (i >= j) of the piece is written once: the sum of the children's
  // update-block entries that map to it (through their inverse maps), children in
  // list order; a root's update block does not exist (nu == 0, no columns >= ns)
  const int64_t q0 = M.cptr[s], q1 = M.cptr[s + 1];
  constexpr int RU = kAsmRows / 64;   // row groups of 64 per lane: independent load chains
  for (int j = c0 + wave; j < c1; j += NW) {
    const int i0 = max(j, r0);
    if (i0 >= r1) continue;
    T v[RU];
#pragma unroll
    for (int u = 0; u < RU; u++) v[u] = 0.0;
    for (int64_t q = q0; q < q1; q++) {
      const int c = M.clist[q];
      const int32_t* inv = M.imap + M.iptr[c];
      const int bj = inv[j];
      if (bj < 0) continue;
      const int nuc = (int)(M.rptr[c + 1] - M.rptr[c] - (M.sfirst[c + 1] - M.sfirst[c]));
      const T* Uc = U + M.uptr[c] + (int64_t)bj * nuc;
      int ai[RU];
#pragma unroll
      for (int u = 0; u < RU; u++) ai[u] = inv[min(i0 + 64 * u + lane, r1 - 1)];
      T uv[RU];
#pragma unroll
      for (int u = 0; u < RU; u++) uv[u] = Uc[max(ai[u], 0)];   // clamped: a valid entry
#pragma unroll
      for (int u = 0; u < RU; u++)
        if (ai[u] >= 0) v[u] += uv[u];
    }
#pragma unroll
    for (int u = 0; u < RU; u++) {
      const int i = i0 + 64 * u + lane;
      if (i < r1) *f.at(i, j) = v[u];
    }
  }
  __syncthreads();
  // original entries of A - sigma B in the piece (fully-summed columns only): the
  // entries of column j sit at acptr[f0 + j] .. in the front at row + j * nf
  const int64_t f0 = M.sfirst[s];
  for (int j = c0 + wave; j < min(c1, f.ns); j += NW) {
    const int64_t e1 = M.acptr[f0 + j + 1], base = (int64_t)j * f.nf;
    for (int64_t e = M.acptr[f0 + j] + lane; e < e1; e += 64) {
      const int64_t dst = M.adst[e];
      const int64_t i = dst - base;
      if (i < r0 || i >= r1) continue;
      const int64_t p = M.asrc[e];
      f.Lp[dst] += fma(-sigma, bval[p], aval[p]);
    }
  }
}

// ---------------------------------------------------------------------------
// Large fronts: Bunch-Kaufman inside pivot tile t (kNB columns), in LDS.
// ---------------------------------------------------------------------------
template <int NT, typename T>
__global__ __launch_bounds__(NT) void k_tile_factor(FrontMeta M, const int32_t* fronts, int t,
                                                    Batch bt, T* L, double* D, double* E,
                                                    int32_t* tperm, T* tinv, FactStats* st) {
  {
    const int64_t bidx = blockIdx.y;
    L += bidx * bt.sL; D += bidx * bt.sN; E += bidx * bt.sN; tperm += bidx * bt.sN;
    tinv += bidx * bt.sT; st += bidx;
  }
  constexpr int LD = kNB + 1;   // padded: row walks across lanes hit distinct LDS banks
  __shared__ T Tl[kNB * LD];    // the tile; after the factorization, the inverse of L_tt
  __shared__ T Lo[kNB * LD];    // multipliers (strictly lower part of L_tt)
  __shared__ int lp[kNB];
  __shared__ T dd[kNB], ee[kNB];
  const int s = fronts[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t f0 = M.sfirst[s];
  const int ns = (int)(M.sfirst[s + 1] - f0);
  const int nf = (int)(M.rptr[s + 1] - M.rptr[s]);
  const int k0 = t * kNB;
  const int kb = min(kNB, ns - k0);
  T* Lp = L + M.lptr[s];
  constexpr int U = 16;   // independent global accesses in flight per thread
  for (int x0 = 0; x0 < kb * kb; x0 += NT * U) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int x = x0 + u * NT + tid;
      const int i = x % kb, j = x / kb;
      v[u] = (x < kb * kb && i >= j) ? Lp[(k0 + i) + (int64_t)(k0 + j) * nf] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int x = x0 + u * NT + tid;
      if (x < kb * kb) Tl[(x % kb) + (x / kb) * LD] = v[u];
    }
  }
  __syncthreads();
  BKCounts cnt{0, 0, 0, 0, INFINITY, 0.0};
  bk_tile_regs<T>(Tl, Lo, LD, kb, lp, dd, ee, cnt);
  // unit-lower L_tt back to the panel (ones on the diagonal, zeros inside 2x2 blocks)
  for (int x0 = 0; x0 < kb * kb; x0 += NT * U) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int x = x0 + u * NT + tid;
      v[u] = x < kb * kb ? Lo[(x % kb) + (x / kb) * LD] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int x = x0 + u * NT + tid;
      const int i = x % kb, j = x / kb;
      if (x < kb * kb && i >= j) Lp[(k0 + i) + (int64_t)(k0 + j) * nf] = i == j ? (T)1.0 : v[u];
    }
  }
  for (int q = tid; q < kb; q += NT) {
    D[f0 + k0 + q] = dd[q];
    E[f0 + k0 + q] = ee[q];
    tperm[f0 + k0 + q] = lp[q];
  }
  // inverse of the unit-lower tile factor (identity beyond kb): column c of
  // L_tt^{-1} by forward substitution, row r = lane holding L(r, p < r) in
  // registers; wave w takes the columns c = w (mod 4), four chains at a time
  {
    T Lv[kNB];
#pragma unroll
    for (int p = 0; p < kNB; p++) Lv[p] = Lo[lane + p * LD];
#pragma unroll 1
    for (int c0 = wave; c0 < kNB; c0 += 16) {
      T x0 = lane == c0, x1 = lane == c0 + 4, x2 = lane == c0 + 8, x3 = lane == c0 + 12;
#pragma unroll
      for (int p = 0; p < kNB; p++) {
        x0 = fma(-Lv[p], lane_value(x0, p), x0);
        x1 = fma(-Lv[p], lane_value(x1, p), x1);
        x2 = fma(-Lv[p], lane_value(x2, p), x2);
        x3 = fma(-Lv[p], lane_value(x3, p), x3);
      }
      Tl[lane + c0 * LD] = x0;
      Tl[lane + (c0 + 4) * LD] = x1;
      Tl[lane + (c0 + 8) * LD] = x2;
      Tl[lane + (c0 + 12) * LD] = x3;
    }
  }
  __syncthreads();
  T* Ti = tinv + M.tptr[s] + (t & 1) * (kNB * kNB);   // two slots: tile t+1 may be factored
                                                      // while tile t's panel solve runs
  for (int x0 = 0; x0 < kNB * kNB; x0 += NT * U) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int x = x0 + u * NT + tid;
      v[u] = Tl[(x % kNB) + (x / kNB) * LD];
    }
#pragma unroll
    for (int u = 0; u < U; u++) Ti[x0 + u * NT + tid] = v[u];
  }
  if (tid == 0) flush_counts(cnt, st);
}

typedef double double4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));

// One 16x16x4 matrix-core step per element type.  Inputs: lane l supplies
// A(m = l % 16, k = l / 16) and B(k = l / 16, n = l % 16).  Output register r of
// lane l holds column n = l % 16 and row mrow(r, l) -- the FP64 and FP32
// instructions differ here (pinned by the probe tests).
template <typename T> struct MF;
template <> struct MF<double> {
  typedef double4v acc;
  __device__ static inline acc zero() { return (double4v){0.0, 0.0, 0.0, 0.0}; }
  __device__ static inline acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int mrow(int r, int lane) { return 4 * r + (lane >> 4); }
};
template <> struct MF<float> {
  typedef float4v acc;
  __device__ static inline acc zero() { return (float4v){0.f, 0.f, 0.f, 0.f}; }
  __device__ static inline acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int mrow(int r, int lane) { return 4 * (lane >> 4) + r; }
};

// s_waitcnt immediate that waits for the vector-memory counter to reach n (the
// LDS and export counters are left alone): vmcnt bits [3:0] and [15:14].
__device__ constexpr int vmcnt_imm(int n) {
  return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8);
}

// The 16 operand values of one depth chunk of k_gemm_lt: av[s][a] at byte
// address ba + a * 16 rows + s * 4 columns, bv likewise from bb (LDS, column
// stride kTile).  One asm block issues the 16 reads and waits for them.
__device__ __forceinline__ void lds_read_chunk(uint32_t ba, uint32_t bb, double (&av)[4][2],
                                               double (&bv)[4][2]) {
  asm volatile(
      "ds_read_b64 %0, %16\n ds_read_b64 %1, %16 offset:128\n"
      "ds_read_b64 %2, %16 offset:2048\n ds_read_b64 %3, %16 offset:2176\n"
      "ds_read_b64 %4, %16 offset:4096\n ds_read_b64 %5, %16 offset:4224\n"
      "ds_read_b64 %6, %16 offset:6144\n ds_read_b64 %7, %16 offset:6272\n"
      "ds_read_b64 %8, %17\n ds_read_b64 %9, %17 offset:128\n"
      "ds_read_b64 %10, %17 offset:2048\n ds_read_b64 %11, %17 offset:2176\n"
      "ds_read_b64 %12, %17 offset:4096\n ds_read_b64 %13, %17 offset:4224\n"
      "ds_read_b64 %14, %17 offset:6144\n ds_read_b64 %15, %17 offset:6272\n"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(av[0][0]), "=&v"(av[0][1]), "=&v"(av[1][0]), "=&v"(av[1][1]), "=&v"(av[2][0]),
        "=&v"(av[2][1]), "=&v"(av[3][0]), "=&v"(av[3][1]), "=&v"(bv[0][0]), "=&v"(bv[0][1]),
        "=&v"(bv[1][0]), "=&v"(bv[1][1]), "=&v"(bv[2][0]), "=&v"(bv[2][1]), "=&v"(bv[3][0]),
        "=&v"(bv[3][1])
      : "v"(ba), "v"(bb)
      : "memory");
}
__device__ __forceinline__ void lds_read_chunk(uint32_t ba, uint32_t bb, float (&av)[4][2],
                                               float (&bv)[4][2]) {
  asm volatile(
      "ds_read_b32 %0, %16\n ds_read_b32 %1, %16 offset:64\n"
      "ds_read_b32 %2, %16 offset:1024\n ds_read_b32 %3, %16 offset:1088\n"
      "ds_read_b32 %4, %16 offset:2048\n ds_read_b32 %5, %16 offset:2112\n"
      "ds_read_b32 %6, %16 offset:3072\n ds_read_b32 %7, %16 offset:3136\n"
      "ds_read_b32 %8, %17\n ds_read_b32 %9, %17 offset:64\n"
      "ds_read_b32 %10, %17 offset:1024\n ds_read_b32 %11, %17 offset:1088\n"
      "ds_read_b32 %12, %17 offset:2048\n ds_read_b32 %13, %17 offset:2112\n"
      "ds_read_b32 %14, %17 offset:3072\n ds_read_b32 %15, %17 offset:3136\n"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(av[0][0]), "=&v"(av[0][1]), "=&v"(av[1][0]), "=&v"(av[1][1]), "=&v"(av[2][0]),
        "=&v"(av[2][1]), "=&v"(av[3][0]), "=&v"(av[3][1]), "=&v"(bv[0][0]), "=&v"(bv[0][1]),
        "=&v"(bv[1][0]), "=&v"(bv[1][1]), "=&v"(bv[2][0]), "=&v"(bv[2][1]), "=&v"(bv[3][0]),
        "=&v"(bv[3][1])
      : "v"(ba), "v"(bb)
      : "memory");
}

// ---------------------------------------------------------------------------
// Large fronts: rows below pivot tile t, 64 rows per workgroup.
//   W = S P^T L_tt^{-T}  (MFMA, with the tile inverse from k_tile_factor)
//   L21 = W D^{-1}       (1x1 / 2x2 blocks)
// The panel rows receive L21, the W panel (same layout) receives W (= L21 D).
// With upd, the task of the next tile's rows (r0 < ns) then also subtracts this
// tile's part of the next diagonal block's update, L W^T over kNB columns, from
// the values it holds in LDS.
// ---------------------------------------------------------------------------
template <int NT, typename T>
__global__ __launch_bounds__(NT) void k_panel_trsm(FrontMeta M, const Int2* tasks, int t,
                                                   Batch bt, T* L, T* W,
                                                   const double* __restrict__ D,
                                                   const double* __restrict__ E,
                                                   const int32_t* __restrict__ tperm,
                                                   const T* __restrict__ tinv,
                                                   FactStats* st, int upd) {
  {
    const int64_t bidx = blockIdx.y;
    L += bidx * bt.sL; W += bidx * bt.sW; D += bidx * bt.sN; E += bidx * bt.sN;
    tperm += bidx * bt.sN; tinv += bidx * bt.sT; st += bidx;
  }
  __shared__ T As[kTile * kNB];   // S' rows x k, ld kTile; reused for W
  __shared__ T Bs[kNB * kNB];     // Linv(q, p) at q + p*kNB
  __shared__ T dd[kNB], ee[kNB];
  __shared__ int pp[kNB];
  __shared__ double sv[NT / 64];
  const Int2 tk = tasks[blockIdx.x];
  const int s = tk.a, r0 = tk.b;
  const int tid = threadIdx.x;
  const int64_t f0 = M.sfirst[s];
  const int ns = (int)(M.sfirst[s + 1] - f0);
  const int nf = (int)(M.rptr[s + 1] - M.rptr[s]);
  const int k0 = t * kNB;
  const int kb = min(kNB, ns - k0);
  T* Lp = L + M.lptr[s];
  T* Wp = W + M.lptr[s];   // W = L D, panel-shaped
  const T* Ti = tinv + M.tptr[s] + (t & 1) * (kNB * kNB);
  for (int q = tid; q < kNB; q += NT) {
    dd[q] = q < kb ? D[f0 + k0 + q] : 1.0;
    ee[q] = q < kb ? E[f0 + k0 + q] : 0.0;
    pp[q] = q < kb ? tperm[f0 + k0 + q] : 0;
  }
  const int nr = min(kTile, nf - r0);
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  // with upd on the next tile's rows: that tile's diagonal block (kb2 columns), the
  // entries this thread updates at the end, loaded now (its earlier depth is in)
  const bool nxt = upd && r0 < ns;
  const int kb2 = nxt ? min(kNB, ns - r0) : 0;
  T* Cb = Lp + r0 + (int64_t)r0 * nf;
  T cpre[2][2][4];
  if (nxt) {
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
      for (int b = 0; b < 2; b++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int i = wr + a * 16 + MF<T>::mrow(r, lane), j = wc + b * 16 + (lane & 15);
          cpre[a][b][r] = (i < nr && j < kb2 && i >= j) ? Cb[i + (int64_t)j * nf] : (T)0.0;
        }
  }
  __syncthreads();   // pp[] visible
  {
    constexpr int U = kTile * kNB / NT;   // 16 loads of each operand per thread, all in flight
    T va[U], vb[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int x = u * NT + tid;
      const int r = x % kTile, q = x / kTile;
      vb[u] = Ti[x];
      va[u] = (r < nr && q < kb) ? Lp[(r0 + r) + (int64_t)(k0 + pp[q]) * nf] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      As[u * NT + tid] = va[u];
      Bs[u * NT + tid] = vb[u];
    }
  }
  __syncthreads();
  typename MF<T>::acc acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) acc[a][b] = MF<T>::zero();
  const int m = lane & 15, kk = lane >> 4;
  for (int q0 = 0; q0 < kNB; q0 += 4) {
    T av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; a++) av[a] = As[(wr + a * 16 + m) + (q0 + kk) * kTile];
#pragma unroll
    for (int b = 0; b < 2; b++) bv[b] = Bs[(wc + b * 16 + m) + (q0 + kk) * kNB];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
      for (int b = 0; b < 2; b++)
        acc[a][b] = MF<T>::step(av[a], bv[b], acc[a][b]);
  }
  __syncthreads();   // everyone is done reading As
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int r = 0; r < 4; r++)
        As[(wr + a * 16 + MF<T>::mrow(r, lane)) + (wc + b * 16 + (lane & 15)) * kTile] = acc[a][b][r];
  __syncthreads();
  double maxl = 0.0;
  for (int x = tid; x < kTile * kNB; x += NT) {
    const int r = x % kTile, q = x / kTile;
    if (r >= nr || q >= kb) {
      Bs[x] = 0.0;
      continue;
    }
    const T wq = As[r + q * kTile];
    T l;
    if (q + 1 < kb && ee[q] != 0.0) {            // first row of a 2x2 block
      const T a = dd[q], b = ee[q], c = dd[q + 1], det = a * c - b * b;
      l = (c * wq - b * As[r + (q + 1) * kTile]) / det;
    } else if (q > 0 && ee[q - 1] != 0.0) {      // second row of a 2x2 block
      const T a = dd[q - 1], b = ee[q - 1], c = dd[q], det = a * c - b * b;
      l = (a * wq - b * As[r + (q - 1) * kTile]) / det;
    } else {
      l = dd[q] != 0.0 ? wq / dd[q] : 0.0;
    }
    Lp[(r0 + r) + (int64_t)(k0 + q) * nf] = l;
    Wp[(r0 + r) + (int64_t)(k0 + q) * nf] = wq;
    Bs[x] = l;   // L(r0 + r, k0 + q) at r + q * kTile (the inverse is no longer read)
    maxl = fmax(maxl, fabs((double)l));
  }
  if (nxt) {
    // these rows are the next tile's: its diagonal block C (rows and columns r0 ..,
    // lower part, kb2 columns) receives this tile's columns, C -= L W^T over the
    // kb (= kNB) columns just solved; the depth before k0 reached it beforehand
    __syncthreads();   // Bs (L) and As (W) complete
    typename MF<T>::acc xc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
      for (int b = 0; b < 2; b++) xc[a][b] = MF<T>::zero();
    for (int q0 = 0; q0 < kNB; q0 += 4) {
      T av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; a++) av[a] = Bs[(wr + a * 16 + m) + (q0 + kk) * kTile];
#pragma unroll
      for (int b = 0; b < 2; b++) bv[b] = As[(wc + b * 16 + m) + (q0 + kk) * kTile];
#pragma unroll
      for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) xc[a][b] = MF<T>::step(av[a], bv[b], xc[a][b]);
    }
    // xc[a][b][r]: i = wr + a * 16 + mrow(r, lane) (row of L), j = wc + b * 16 + lane % 16
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
      for (int b = 0; b < 2; b++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int i = wr + a * 16 + MF<T>::mrow(r, lane), j = wc + b * 16 + (lane & 15);
          if (i < nr && j < kb2 && i >= j) Cb[i + (int64_t)j * nf] = cpre[a][b][r] - xc[a][b][r];
        }
  }
  maxl = block_max<NT>(maxl, sv);
  if (tid == 0) atomicMax(&st->max_l_bits, dbits(maxl));
}

// ---------------------------------------------------------------------------
// Large fronts: left-looking updates on FP64 MFMA (v_mfma_f64_16x16x4), C -= A B^T
//   mode 0 / 1, column block of pivot tile t, rows [i0, i0 + kTile) (mode 0: the
//     tile's own diagonal block, lower part; mode 1: rows below it):
//       C(i, j) -= sum_{q < k0} L(i, q) W(j, q),   j in [k0, k0 + kb)
//     (a mode-1 task (front, row | kLaFlag): the diagonal block of tile t + 1,
//     columns [k0 + kNB, ..), the same depth k0)
//   mode 2, the contribution block, lower 64 x 64 tile number b of it:
//       U(i, j) -= sum_{q < ns} L(ns + i, q) W(ns + j, q),   i >= j
// W = L D is kept panel-shaped (same offsets and ld as L) by k_panel_trsm.  The
// depth is walked in chunks of 16 columns loaded straight from global memory into
// three LDS buffers; the next two chunks' loads are in flight while the current
// one feeds the matrix cores.
// ---------------------------------------------------------------------------
// Split depth (modes 0 / 1, nseg > 1): workgroup g takes output tile g / nseg and
// the depth segment [seg * segk, (seg + 1) * segk) with seg = g % nseg, and
// stores its product in part[g] (kTile x kTile); k_gemm_reduce adds the segments
// in order and applies them.
template <int NT, typename T>
__global__ __launch_bounds__(NT) void k_gemm_lt(FrontMeta M, const Int2* tasks, int t, int mode,
                                                int nseg, int segk, Batch bt, T* L, T* U, const T* W,
                                                T* part) {
  {
    const int64_t bidx = blockIdx.y;
    L += bidx * bt.sL; U += bidx * bt.sU; W += bidx * bt.sW;
    part += bidx * bt.sP;
  }
  constexpr int KC = 16;         // depth chunk staged through LDS
  // three chunk buffers per operand (rows x q, ld kTile), filled by direct
  // global-to-LDS loads two chunks ahead of the one being multiplied
  __shared__ T A0[kTile * KC], A1[kTile * KC], A2[kTile * KC];
  __shared__ T B0[kTile * KC], B1[kTile * KC], B2[kTile * KC];
  const int g = blockIdx.x;
  const int seg = g % nseg;
  const Int2 tk = tasks[g / nseg];
  const int s = tk.a;
  const FrontRef<T> f = front_ref<T>(M, s, L, U);
  const T* Lp = f.Lp;
  const T* Wp = W + M.lptr[s];
  int ia, ie, ja, je, K;   // C rows [ia, ie), columns [ja, je) (front numbering), depth K
  bool tri;                // lower triangle only
  T* Cb;                   // C(i, j) at Cb[(i - ia) + (j - ja) * ldc]
  int64_t ldc;
  int Kb = 0;              // first depth column of this workgroup
  if (mode < 2) {
    // a flagged task: the diagonal block of tile t + 1, still at depth t * kNB
    const bool la = (tk.b & kLaFlag) != 0;
    const int k0 = (t + (la ? 1 : 0)) * kNB, kb = min(kNB, f.ns - k0);
    ia = tk.b & ~kLaFlag; ie = min(ia + kTile, f.nf); ja = k0; je = k0 + kb; K = t * kNB;
    if (nseg > 1) { Kb = seg * segk; K = min(K, Kb + segk); }
    tri = (ia == k0);
    Cb = f.Lp + ia + (int64_t)ja * f.nf; ldc = f.nf;
  } else {
    const int tl = tk.b;
    int bi = (int)((sqrt(8.0 * tl + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= tl) bi++;
    while (bi * (bi + 1) / 2 > tl) bi--;
    const int bj = tl - bi * (bi + 1) / 2;
    ia = f.ns + bi * kTile; ie = min(ia + kTile, f.nf);
    ja = f.ns + bj * kTile; je = min(ja + kTile, f.nf);
    K = f.ns; tri = (bi == bj);
    Cb = f.Ub + (ia - f.ns) + (int64_t)(ja - f.ns) * f.nu; ldc = f.nu;
  }
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;   // the wave's 32 x 32 sub-tile
  // Output layout with A = rows i and B = rows j: lane l holds i = l % 16 of its
  // block and j = mrow(r, l) for register r -> 16 consecutive rows per column.
  const int il = lane & 15;
  typename MF<T>::acc acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) acc[a][b] = MF<T>::zero();
  // operand staging: each wave moves 4-byte pieces of its share of the chunk's
  // columns straight into LDS (lane l: piece l % EPL of row h * RPI + l / EPL);
  // rows beyond the tile are clamped (they only feed outputs that are not
  // written), columns beyond the depth are clamped and then zeroed in LDS
  constexpr int EPL = sizeof(T) / 4;        // 4-byte pieces per element
  constexpr int RPI = kTile / EPL;          // rows per load instruction
  constexpr int IPW = KC * EPL / (NT / 64); // load instructions per operand and wave
  static_assert(NT == 256 && kTile == 64, "four waves, 64-row tiles");
  const int nch = (K - Kb + KC - 1) / KC;
  auto issue = [&](int ch, T* Ab, T* Bb) {
    const int q0 = Kb + ch * KC;
#pragma unroll
    for (int u = 0; u < IPW; u++) {
      const int idx = wave * IPW + u, c = idx / EPL, h = idx % EPL;
      const int64_t q = min(q0 + c, K - 1);
      const int row = h * RPI + lane / EPL;
      const char* sa = reinterpret_cast<const char*>(Lp + min(ia + row, ie - 1) + q * f.nf) + 4 * (lane % EPL);
      const char* sb = reinterpret_cast<const char*>(Wp + min(ja + row, je - 1) + q * f.nf) + 4 * (lane % EPL);
      __builtin_amdgcn_global_load_lds(sa, (__attribute__((address_space(3))) void*)(Ab + c * kTile + h * RPI), 4, 0, 0);
      __builtin_amdgcn_global_load_lds(sb, (__attribute__((address_space(3))) void*)(Bb + c * kTile + h * RPI), 4, 0, 0);
    }
  };
  const bool direct = nseg == 1;
  const int m = lane & 15, kk = lane >> 4;
  // 16 operand values of a chunk (4 depth steps x 2 row blocks of A and of B), read
  // in one block that waits for its own reads: the compiler does not see these
  // LDS reads, so it adds no wait for the loads still filling the other buffers
  const uint32_t offA = ((wr + m) + kk * kTile) * (uint32_t)sizeof(T);
  const uint32_t offB = ((wc + m) + kk * kTile) * (uint32_t)sizeof(T);
  auto mult = [&](const T* Ab, const T* Bb) {
    typedef __attribute__((address_space(3))) T* lds_ptr;   // 32-bit LDS addresses
    const uint32_t ba = (uint32_t)(uintptr_t)(lds_ptr)Ab + offA;
    const uint32_t bb = (uint32_t)(uintptr_t)(lds_ptr)Bb + offB;
    T av[4][2], bv[4][2];
    lds_read_chunk(ba, bb, av, bv);
#pragma unroll
    for (int s4 = 0; s4 < 4; s4++)
      // D(m = j, n = i) = sum_q B(j, q) A(i, q)
#pragma unroll
      for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) acc[a][b] = MF<T>::step(bv[s4][b], av[s4][a], acc[a][b]);
  };
  // columns q >= K of the last chunk hold clamped copies: zero them
  auto zero_tail = [&](int ch, T* Ab, T* Bb) {
    const int cv = K - (Kb + ch * KC);
    if (cv >= KC) return;
    __syncthreads();
    for (int x = tid; x < kTile * KC; x += NT)
      if (x / kTile >= cv) { Ab[x] = 0.0; Bb[x] = 0.0; }
    __syncthreads();
  };
  constexpr int W1 = IPW * 2;               // one chunk's loads per wave (A and B)
  if (nch > 0) issue(0, A0, B0);
  if (nch > 1) issue(1, A1, B1);
  for (int ch = 0; ch < nch; ch += 3) {
#pragma unroll
    for (int v = 0; v < 3; v++) {
      const int c = ch + v;
      if (c >= nch) break;
      T* Ab = v == 0 ? A0 : v == 1 ? A1 : A2;
      T* Bb = v == 0 ? B0 : v == 1 ? B1 : B2;
      // chunk c has landed in this wave's pieces (the next chunk's may still be in
      // flight); after the barrier every wave's pieces have, and every wave is
      // done with chunk c - 1, whose buffers chunk c + 2 refills
      if (c + 1 < nch) __builtin_amdgcn_s_waitcnt(vmcnt_imm(W1));
      else __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_sched_barrier(0);
      if (c == nch - 1) zero_tail(c, Ab, Bb);
      if (c + 2 < nch) issue(c + 2, v == 0 ? A2 : v == 1 ? A0 : A1, v == 0 ? B2 : v == 1 ? B0 : B1);
      mult(Ab, Bb);
    }
  }
  if (!direct) {
    T* P = part + (int64_t)g * (kTile * kTile);
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
      for (int b = 0; b < 2; b++)
#pragma unroll
        for (int r = 0; r < 4; r++)
          P[(wr + a * 16 + il) + (wc + b * 16 + MF<T>::mrow(r, lane)) * kTile] = acc[a][b][r];
    return;
  }
  // C -= product, read after the depth loop (keeps the loop's registers free): the
  // 16 entries of C in one batch (indices clamped into the block, so every read is
  // valid; only entries inside it are written), then the writes
  const int im = ie - ia - 1, jm = je - ja - 1;
  T cv[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int i = min(wr + a * 16 + il, im), j = min(wc + b * 16 + MF<T>::mrow(r, lane), jm);
        cv[a][b][r] = Cb[i + (int64_t)j * ldc];
      }
  // the new values are formed before any (masked) write, so no write waits on the
  // reads or on the writes before it
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        cv[a][b][r] = cv[a][b][r] - acc[a][b][r];
        asm volatile("" : "+v"(cv[a][b][r]));
      }
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int i = wr + a * 16 + il, j = wc + b * 16 + MF<T>::mrow(r, lane);
        const bool ok = (ia + i < ie) && (ja + j < je) && (!tri || ia + i >= ja + j);
        if (ok) Cb[i + (int64_t)j * ldc] = cv[a][b][r];
      }
}

// C -= sum of the nseg depth segments of each output tile (in segment order) for
// the split left-looking column-block updates; one entry per thread, workgroup
// g covers entries [256 (g % 16), 256 (g % 16 + 1)) of output tile g / 16.
template <int NT, typename T>
__global__ __launch_bounds__(NT) void k_gemm_reduce(FrontMeta M, const Int2* tasks, int t,
                                                    int nseg, Batch bt, T* L, const T* part) {
  static_assert(NT * 16 == kTile * kTile, "one entry per thread");
  {
    const int64_t bidx = blockIdx.y;
    L += bidx * bt.sL;
    part += bidx * bt.sP;
  }
  const int o = blockIdx.x >> 4;
  const int x = (blockIdx.x & 15) * NT + threadIdx.x;
  const Int2 tk = tasks[o];
  const int s = tk.a;
  const int64_t f0 = M.sfirst[s];
  const int ns = (int)(M.sfirst[s + 1] - f0);
  const int nf = (int)(M.rptr[s + 1] - M.rptr[s]);
  const bool la = (tk.b & kLaFlag) != 0;   // the diagonal block of tile t + 1
  const int k0 = (t + (la ? 1 : 0)) * kNB, kb = min(kNB, ns - k0);
  const int ia = tk.b & ~kLaFlag, ie = min(ia + kTile, nf);
  const bool tri = (ia == k0);
  const int i = x % kTile, j = x / kTile;
  if (ia + i >= ie || j >= kb || (tri && i < j)) return;
  const T* P = part + (int64_t)o * nseg * (kTile * kTile) + x;
  T sum = 0.0;
  for (int q0 = 0; q0 < nseg; q0 += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; u++) v[u] = P[(int64_t)min(q0 + u, nseg - 1) * (kTile * kTile)];
#pragma unroll
    for (int u = 0; u < 8; u++)
      if (q0 + u < nseg) sum += v[u];
  }
  T* Cb = L + M.lptr[s] + ia + (int64_t)k0 * nf;
  Cb[i + (int64_t)j * nf] -= sum;
}

// The operand values of one 8-deep chunk of k_gemm_cb128: av[s][a] at byte address
// ba + a * 16 rows + s * 4 columns, bv likewise from bb, in LDS with a column
// stride of 144 elements (128 rows + 16 of padding: consecutive columns start on
// different banks).  One asm block issues the 16 reads and waits for them.
__device__ __forceinline__ void lds_read_cb128(uint32_t ba, uint32_t bb, double (&av)[2][4],
                                               double (&bv)[2][4]) {
  asm volatile(
      "ds_read_b64 %0, %16\n ds_read_b64 %1, %16 offset:128\n"
      "ds_read_b64 %2, %16 offset:256\n ds_read_b64 %3, %16 offset:384\n"
      "ds_read_b64 %4, %16 offset:4608\n ds_read_b64 %5, %16 offset:4736\n"
      "ds_read_b64 %6, %16 offset:4864\n ds_read_b64 %7, %16 offset:4992\n"
      "ds_read_b64 %8, %17\n ds_read_b64 %9, %17 offset:128\n"
      "ds_read_b64 %10, %17 offset:256\n ds_read_b64 %11, %17 offset:384\n"
      "ds_read_b64 %12, %17 offset:4608\n ds_read_b64 %13, %17 offset:4736\n"
      "ds_read_b64 %14, %17 offset:4864\n ds_read_b64 %15, %17 offset:4992\n"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(av[0][0]), "=&v"(av[0][1]), "=&v"(av[0][2]), "=&v"(av[0][3]), "=&v"(av[1][0]),
        "=&v"(av[1][1]), "=&v"(av[1][2]), "=&v"(av[1][3]), "=&v"(bv[0][0]), "=&v"(bv[0][1]),
        "=&v"(bv[0][2]), "=&v"(bv[0][3]), "=&v"(bv[1][0]), "=&v"(bv[1][1]), "=&v"(bv[1][2]),
        "=&v"(bv[1][3])
      : "v"(ba), "v"(bb)
      : "memory");
}
__device__ __forceinline__ void lds_read_cb128(uint32_t ba, uint32_t bb, float (&av)[2][4],
                                               float (&bv)[2][4]) {
  asm volatile(
      "ds_read_b32 %0, %16\n ds_read_b32 %1, %16 offset:64\n"
      "ds_read_b32 %2, %16 offset:128\n ds_read_b32 %3, %16 offset:192\n"
      "ds_read_b32 %4, %16 offset:2304\n ds_read_b32 %5, %16 offset:2368\n"
      "ds_read_b32 %6, %16 offset:2432\n ds_read_b32 %7, %16 offset:2496\n"
      "ds_read_b32 %8, %17\n ds_read_b32 %9, %17 offset:64\n"
      "ds_read_b32 %10, %17 offset:128\n ds_read_b32 %11, %17 offset:192\n"
      "ds_read_b32 %12, %17 offset:2304\n ds_read_b32 %13, %17 offset:2368\n"
      "ds_read_b32 %14, %17 offset:2432\n ds_read_b32 %15, %17 offset:2496\n"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(av[0][0]), "=&v"(av[0][1]), "=&v"(av[0][2]), "=&v"(av[0][3]), "=&v"(av[1][0]),
        "=&v"(av[1][1]), "=&v"(av[1][2]), "=&v"(av[1][3]), "=&v"(bv[0][0]), "=&v"(bv[0][1]),
        "=&v"(bv[0][2]), "=&v"(bv[0][3]), "=&v"(bv[1][0]), "=&v"(bv[1][1]), "=&v"(bv[1][2]),
        "=&v"(bv[1][3])
      : "v"(ba), "v"(bb)
      : "memory");
}

// ---------------------------------------------------------------------------
// Large fronts with big contribution blocks: the update
//   U(i, j) -= sum_{q < ns} L(ns + i, q) W(ns + j, q),   i >= j,
// on lower 128 x 128 tiles (tile tl = bi (bi + 1) / 2 + bj), twice the operand
// reuse of the 64 x 64 tiles of k_gemm_lt.  Four waves as 2 x 2 blocks of 64 x 64
// (4 x 4 MFMA blocks of 16 x 16 each).  The depth is walked in chunks of 8 columns
// loaded straight from global memory into a ring of four LDS buffers per operand
// (18 KB per chunk for FP64), three chunks in flight while one feeds the matrix
// cores; two workgroups fit one CU.  Each output entry receives the same products
// in the same order as in k_gemm_lt (4-deep MFMA steps in increasing depth).
// ---------------------------------------------------------------------------
template <int NT, typename T>
__global__ __launch_bounds__(NT, 2) void k_gemm_cb128(FrontMeta M, const Int2* tasks, Batch bt,
                                                      T* L, T* U, const T* W) {
  {
    const int64_t bidx = blockIdx.y;
    L += bidx * bt.sL; U += bidx * bt.sU; W += bidx * bt.sW;
  }
  constexpr int TB = 128;        // output tile edge
  constexpr int CS = TB + 16;    // LDS column stride (elements)
  constexpr int KC = 8;          // depth chunk staged through LDS
  constexpr int NS = 4;          // ring of chunk buffers
  __shared__ T As[NS][CS * KC];
  __shared__ T Bs[NS][CS * KC];
  const Int2 tk = tasks[blockIdx.x];
  const int s = tk.a, tl = tk.b;
  const FrontRef<T> f = front_ref<T>(M, s, L, U);
  const T* Lp = f.Lp;
  const T* Wp = W + M.lptr[s];
  int bi = (int)((sqrt(8.0 * tl + 1.0) - 1.0) * 0.5);
  while ((bi + 1) * (bi + 2) / 2 <= tl) bi++;
  while (bi * (bi + 1) / 2 > tl) bi--;
  const int bj = tl - bi * (bi + 1) / 2;
  const int ia = f.ns + bi * TB, ie = min(ia + TB, f.nf);
  const int ja = f.ns + bj * TB, je = min(ja + TB, f.nf);
  const int K = f.ns;
  const bool tri = bi == bj;
  T* Cb = f.Ub + (ia - f.ns) + (int64_t)(ja - f.ns) * f.nu;
  const int64_t ldc = f.nu;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;   // the wave's 64 x 64 sub-tile
  const int il = lane & 15;
  typename MF<T>::acc acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 4; b++) acc[a][b] = MF<T>::zero();
  // staging: a chunk column of 128 rows is TB * sizeof(T) / 256 load instructions
  // of 4-byte pieces (lane l: piece l % EPL of row h * RPI + l / EPL); rows past the
  // tile are clamped (they feed outputs that are not written), columns past the
  // depth clamped and then zeroed in LDS
  constexpr int EPL = sizeof(T) / 4;        // 4-byte pieces per element
  constexpr int RPI = 64 / EPL;             // rows per load instruction
  constexpr int IPC = TB / RPI;             // load instructions per column
  constexpr int IPW = KC * IPC / (NT / 64); // load instructions per operand and wave
  constexpr int W1 = 2 * IPW;               // one chunk's loads per wave (A and B)
  static_assert(NT == 256, "four waves");
  static_assert(W1 * (NS - 2) <= 63, "vmcnt range");
  const int nch = (K + KC - 1) / KC;
  auto issue = [&](int ch, T* Ab, T* Bb) {
    const int q0 = ch * KC;
#pragma unroll
    for (int u = 0; u < IPW; u++) {
      const int idx = wave * IPW + u, c = idx / IPC, h = idx % IPC;
      const int64_t q = min(q0 + c, K - 1);
      const int row = h * RPI + lane / EPL;
      const char* sa = reinterpret_cast<const char*>(Lp + min(ia + row, ie - 1) + q * f.nf) + 4 * (lane % EPL);
      const char* sb = reinterpret_cast<const char*>(Wp + min(ja + row, je - 1) + q * f.nf) + 4 * (lane % EPL);
      __builtin_amdgcn_global_load_lds(sa, (__attribute__((address_space(3))) void*)(Ab + c * CS + h * RPI), 4, 0, 0);
      __builtin_amdgcn_global_load_lds(sb, (__attribute__((address_space(3))) void*)(Bb + c * CS + h * RPI), 4, 0, 0);
    }
  };
  const int m = lane & 15, kk = lane >> 4;
  const uint32_t offA = ((wr + m) + kk * CS) * (uint32_t)sizeof(T);
  const uint32_t offB = ((wc + m) + kk * CS) * (uint32_t)sizeof(T);
  auto mult = [&](const T* Ab, const T* Bb) {
    typedef __attribute__((address_space(3))) T* lds_ptr;   // 32-bit LDS addresses
    const uint32_t ba = (uint32_t)(uintptr_t)(lds_ptr)Ab + offA;
    const uint32_t bb = (uint32_t)(uintptr_t)(lds_ptr)Bb + offB;
    T av[2][4], bv[2][4];
    lds_read_cb128(ba, bb, av, bv);
#pragma unroll
    for (int s2 = 0; s2 < 2; s2++)
#pragma unroll
      for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) acc[a][b] = MF<T>::step(bv[s2][b], av[s2][a], acc[a][b]);
  };
  auto zero_tail = [&](int ch, T* Ab, T* Bb) {
    const int cv = K - ch * KC;
    if (cv >= KC) return;
    __syncthreads();
    for (int x = tid; x < CS * KC; x += NT)
      if (x / CS >= cv) { Ab[x] = 0.0; Bb[x] = 0.0; }
    __syncthreads();
  };
#pragma unroll
  for (int v = 0; v < NS - 1; v++)
    if (v < nch) issue(v, As[v], Bs[v]);
  for (int ch = 0; ch < nch; ch += NS) {
#pragma unroll
    for (int v = 0; v < NS; v++) {
      const int c = ch + v;
      if (c >= nch) break;
      // chunk c has landed in this wave's pieces (up to NS - 2 later chunks may be
      // in flight); after the barrier every wave's pieces have, and every wave is
      // done with chunk c - 1, whose buffers chunk c + NS - 1 refills
      const int later = min(NS - 2, nch - 1 - c);
      if (later >= 2) __builtin_amdgcn_s_waitcnt(vmcnt_imm(2 * W1));
      else if (later == 1) __builtin_amdgcn_s_waitcnt(vmcnt_imm(W1));
      else __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_sched_barrier(0);
      if (c == nch - 1) zero_tail(c, As[v], Bs[v]);
      if (c + NS - 1 < nch) issue(c + NS - 1, As[(v + NS - 1) % NS], Bs[(v + NS - 1) % NS]);
      mult(As[v], Bs[v]);
    }
  }
  // C -= product, in two halves of the wave's rows: each half's 32 entries of C are
  // read in one batch (indices clamped into the block, so every read is valid; only
  // entries inside it are written), then written -- two waits for reads per tile
  // instead of one per 16 x 16 block
  const int im = ie - ia - 1, jm = je - ja - 1;
#pragma unroll
  for (int h = 0; h < 2; h++) {
    T cv[2][4][4];
#pragma unroll
    for (int a2 = 0; a2 < 2; a2++)
#pragma unroll
      for (int b = 0; b < 4; b++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int i = min(wr + (2 * h + a2) * 16 + il, im), j = min(wc + b * 16 + MF<T>::mrow(r, lane), jm);
          cv[a2][b][r] = Cb[i + (int64_t)j * ldc];
        }
    // the new values are formed before any (masked) write, so no write waits on
    // the reads or on the writes before it
#pragma unroll
    for (int a2 = 0; a2 < 2; a2++)
#pragma unroll
      for (int b = 0; b < 4; b++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          cv[a2][b][r] = cv[a2][b][r] - acc[2 * h + a2][b][r];
          asm volatile("" : "+v"(cv[a2][b][r]));
        }
#pragma unroll
    for (int a2 = 0; a2 < 2; a2++)
#pragma unroll
      for (int b = 0; b < 4; b++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int a = 2 * h + a2;
          const int i = wr + a * 16 + il, j = wc + b * 16 + MF<T>::mrow(r, lane);
          const bool ok = (ia + i < ie) && (ja + j < je) && (!tri || i >= j);
          if (ok) Cb[i + (int64_t)j * ldc] = cv[a2][b][r];
        }
  }
}

__global__ void k_set_scalar(double* p, double v) {
  if (threadIdx.x == 0) *p = v;
}

__global__ void k_set_scalars(double* p, int n, SigmaPack pk) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = pk.v[threadIdx.x];
}

// Raw probe of the FP32 instruction (same convention as the FP64 probe below).
__global__ void k_mfma_probe_f32(const float* A, const float* B, float* Dout) {
  const int lane = threadIdx.x;
  float4v c = {0.f, 0.f, 0.f, 0.f};
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(A[lane], B[lane], c, 0, 0, 0);
  for (int r = 0; r < 4; r++) Dout[4 * lane + r] = c[r];
}

// Raw probe: lane l feeds a[l] and b[l]; c[4 l + r] receives result register r.
__global__ void k_mfma_probe(const double* A, const double* B, double* Dout) {
  const int lane = threadIdx.x;
  double4v c = {0.0, 0.0, 0.0, 0.0};
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(A[lane], B[lane], c, 0, 0, 0);
  for (int r = 0; r < 4; r++) Dout[4 * lane + r] = c[r];
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_fill_stats(FactStats* st, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_stats, dim3(nb), dim3(64), 0, s, st);
}

template <typename T>
void launch_small_fronts(const FrontMeta& M, const int32_t* fronts, int32_t count, int32_t max_nf,
                         const double* aval, const double* bval, const Batch& bt, int nb,
                         T* L, T* U, double* D, double* E, int32_t* tperm,
                         FactStats* st, hipStream_t s) {
  if (count <= 0) return;
  const size_t lds = (size_t)max_nf * max_nf * sizeof(T);
  static const bool attr = [] {   // once per type, thread-safe
    (void)hipFuncSetAttribute((const void*)k_small_fronts<256, T>,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              kSmallMaxNf * kSmallMaxNf * (int)sizeof(T));
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL((k_small_fronts<256, T>), dim3(count, nb), dim3(256), lds, s, M, fronts, aval,
                     bval, bt, L, U, D, E, tperm, st);
}

template <typename T>
void launch_front_init(const FrontMeta& M, const Int2* tasks, int32_t count, const double* aval,
                       const double* bval, const Batch& bt, int nb, T* L, T* U, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL((k_front_init<256, T>), dim3(count, nb), dim3(256), 0, s, M, tasks, aval, bval,
                     bt, L, U);
}

template <typename T>
void launch_tile_factor(const FrontMeta& M, const int32_t* fronts, int32_t count, int32_t t,
                        const Batch& bt, int nb, T* L, double* D, double* E, int32_t* tperm,
                        T* tinv, FactStats* st, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL((k_tile_factor<256, T>), dim3(count, nb), dim3(256), 0, s, M, fronts, t, bt, L,
                     D, E, tperm, tinv, st);
}

template <typename T>
void launch_panel_trsm(const FrontMeta& M, const Int2* tasks, int32_t count, int32_t t,
                       const Batch& bt, int nb, T* L, T* W, const double* D, const double* E,
                       const int32_t* tperm, const T* tinv, FactStats* st, int upd, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL((k_panel_trsm<256, T>), dim3(count, nb), dim3(256), 0, s, M, tasks, t, bt, L, W,
                     D, E, tperm, tinv, st, upd);
}

template <typename T>
void launch_gemm_lt(const FrontMeta& M, const Int2* tasks, int32_t count, int32_t t, int mode,
                    int nseg, int segk, const Batch& bt, int nb, T* L, T* U, const T* W, T* part,
                    hipStream_t s) {
  if (count <= 0) return;
  if (mode == 2) nseg = 1;
  hipLaunchKernelGGL((k_gemm_lt<256, T>), dim3(count * nseg, nb), dim3(256), 0, s, M, tasks, t, mode,
                     nseg, segk, bt, L, U, W, part);
}

template <typename T>
void launch_gemm_cb128(const FrontMeta& M, const Int2* tasks, int32_t count, const Batch& bt, int nb,
                       T* L, T* U, const T* W, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL((k_gemm_cb128<256, T>), dim3(count, nb), dim3(256), 0, s, M, tasks, bt, L, U, W);
}

template <typename T>
void launch_gemm_reduce(const FrontMeta& M, const Int2* tasks, int32_t count, int32_t t, int nseg,
                        const Batch& bt, int nb, T* L, const T* part, hipStream_t s) {
  if (count <= 0 || nseg <= 1) return;
  hipLaunchKernelGGL((k_gemm_reduce<256, T>), dim3(count * 16, nb), dim3(256), 0, s, M, tasks, t,
                     nseg, bt, L, part);
}

#define KTH_INSTANTIATE_FACTOR(T)                                                                   \
  template void launch_small_fronts<T>(const FrontMeta&, const int32_t*, int32_t, int32_t,         \
                                       const double*, const double*, const Batch&, int, T*, T*,     \
                                       double*, double*, int32_t*, FactStats*, hipStream_t);        \
  template void launch_front_init<T>(const FrontMeta&, const Int2*, int32_t, const double*,        \
                                     const double*, const Batch&, int, T*, T*, hipStream_t);        \
  template void launch_tile_factor<T>(const FrontMeta&, const int32_t*, int32_t, int32_t,          \
                                      const Batch&, int, T*, double*, double*, int32_t*, T*,        \
                                      FactStats*, hipStream_t);                                     \
  template void launch_panel_trsm<T>(const FrontMeta&, const Int2*, int32_t, int32_t, const Batch&, \
                                     int, T*, T*, const double*, const double*, const int32_t*,     \
                                     const T*, FactStats*, int, hipStream_t);                       \
  template void launch_gemm_lt<T>(const FrontMeta&, const Int2*, int32_t, int32_t, int, int, int,    \
                                  const Batch&, int, T*, T*, const T*, T*, hipStream_t);            \
  template void launch_gemm_cb128<T>(const FrontMeta&, const Int2*, int32_t, const Batch&, int, T*,  \
                                     T*, const T*, hipStream_t);                                   \
  template void launch_gemm_reduce<T>(const FrontMeta&, const Int2*, int32_t, int32_t, int,         \
                                      const Batch&, int, T*, const T*, hipStream_t);
KTH_INSTANTIATE_FACTOR(double)
KTH_INSTANTIATE_FACTOR(float)
#undef KTH_INSTANTIATE_FACTOR

void launch_set_scalar(double* p, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(64), 0, s, p, v);
}

void launch_set_scalars(double* p, int n, const double* v8, hipStream_t s) {
  // up to kMaxBatch values passed by value (no host-memory lifetime issues, graph-safe)
  SigmaPack pk;
  for (int i = 0; i < n && i < kMaxBatch; i++) pk.v[i] = v8[i];
  hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, s, p, n, pk);
}

void launch_mfma_probe_f32(const float* A, const float* B, float* D, hipStream_t s) {
  hipLaunchKernelGGL(k_mfma_probe_f32, dim3(1), dim3(64), 0, s, A, B, D);
}

void launch_mfma_probe(const double* A, const double* B, double* D, hipStream_t s) {
  hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(64), 0, s, A, B, D);
}

}  // namespace kth
