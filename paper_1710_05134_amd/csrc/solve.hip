// Triangular solves with a kept multifrontal factor: (A - sigma B) x = b as
// L z = P b (forward, leaves to root), y = D^{-1} z, L^T w = y with x = P^T w
// (backward, root to leaves).  The forward pass is itself multifrontal: each
// front gathers its right-hand side, adds its children's update vectors (the
// tails of their work vectors) and hands its own tail to its parent, so no two
// fronts ever write the same entry.  Tile permutations are applied when the
// solve reaches each tile (the factor keeps earlier panels' rows unswapped).
// For a large front the chain of tile steps touches only its pivot block L11;
// the rows below it (L21, most of the factor) take two wide launches per level
// and pass: forward r2 -= L21 z, backward y1 -= L21^T x2, each as partial sums
// over fixed pieces added in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <vector>

#include "device.hpp"
#include "solve.hpp"

namespace kth {

namespace {

constexpr int NT = 256;

// Value of v in lane p (p uniform across the wavefront) through two v_readlane.
__device__ inline double lane_value(double v, int p) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), p);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), p);
  return __hiloint2double(hi, lo);
}

__device__ inline void tile_bounds(int t, int tw, int ns, int& k0, int& kb) {
  k0 = t * tw;
  kb = min(tw, ns - k0);
}

// Forward pass + diagonal for the fronts of one level.  xe: right-hand side in
// elimination order; R: work vectors (front s at rptr[s], nf entries);
// ye: output D^{-1} z in pivot order.
template <typename T>
__global__ __launch_bounds__(NT) void k_solve_fwd(FrontMeta M, const int32_t* fronts, const T* L,
                                                  const double* __restrict__ D,
                                                  const double* __restrict__ E,
                                                  const int32_t* __restrict__ tperm,
                                                  const double* __restrict__ xe, double* R,
                                                  double* ye) {
  __shared__ double z[kSmallMaxNf];
  const int s = fronts[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t f0 = M.sfirst[s];
  const int ns = (int)(M.sfirst[s + 1] - f0);
  const int nf = (int)(M.rptr[s + 1] - M.rptr[s]);
  const int tw = M.tilew[s];
  double* Rs = R + M.rptr[s];
  const T* Lp = L + M.lptr[s];
  for (int i = tid; i < nf; i += NT) Rs[i] = i < ns ? xe[f0 + i] : 0.0;
  __syncthreads();
  for (int64_t q = M.cptr[s]; q < M.cptr[s + 1]; q++) {
    const int c = M.clist[q];
    const int nsc = (int)(M.sfirst[c + 1] - M.sfirst[c]);
    const int nuc = (int)(M.rptr[c + 1] - M.rptr[c]) - nsc;
    const double* Rc = R + M.rptr[c] + nsc;
    const int32_t* map = M.emap + M.eptr[c];
    for (int a = tid; a < nuc; a += NT) Rs[map[a]] += Rc[a];
    __syncthreads();
  }
  const int ntiles = (ns + tw - 1) / tw;
  for (int t = 0; t < ntiles; t++) {
    int k0, kb;
    tile_bounds(t, tw, ns, k0, kb);
    // z = P_t r_t, then L_tt z = P_t r_t by one wave; lane holds z_lane, z_{lane+64}
    if (wave == 0) {
      double z0 = lane < kb ? Rs[k0 + tperm[f0 + k0 + lane]] : 0.0;
      double z1 = lane + 64 < kb ? Rs[k0 + tperm[f0 + k0 + lane + 64]] : 0.0;
      for (int p = 0; p < kb; p++) {
        const double zp = p < 64 ? __shfl(z0, p) : __shfl(z1, p - 64);
        if (lane > p && lane < kb) z0 -= (double)Lp[(k0 + lane) + (int64_t)(k0 + p) * nf] * zp;
        if (lane + 64 > p && lane + 64 < kb)
          z1 -= (double)Lp[(k0 + lane + 64) + (int64_t)(k0 + p) * nf] * zp;
      }
      if (lane < kb) z[lane] = z0;
      if (lane + 64 < kb) z[lane + 64] = z1;
    }
    __syncthreads();
    // rows below the tile
    for (int i = k0 + kb + tid; i < nf; i += NT) {
      double acc = 0.0;
      for (int q = 0; q < kb; q++) acc += (double)Lp[i + (int64_t)(k0 + q) * nf] * z[q];
      Rs[i] -= acc;
    }
    for (int q = tid; q < kb; q += NT) Rs[k0 + q] = z[q];
    __syncthreads();
  }
  // y = D^{-1} z (pivot order)
  for (int q = tid; q < ns; q += NT) {
    const int64_t k = f0 + q;
    double y;
    if (E[k] != 0.0) {
      const double a = D[k], b = E[k], c = D[k + 1], det = a * c - b * b;
      y = (c * Rs[q] - b * Rs[q + 1]) / det;
    } else if (q > 0 && E[k - 1] != 0.0 && ((q % tw) != 0)) {
      const double a = D[k - 1], b = E[k - 1], c = D[k], det = a * c - b * b;
      y = (a * Rs[q] - b * Rs[q - 1]) / det;
    } else {
      y = D[k] != 0.0 ? Rs[q] / D[k] : 0.0;
    }
    ye[k] = y;
  }
}

// Backward pass for the fronts of one level (root side first).  ye: D^{-1} z in
// pivot order; xe: solution in elimination order (ancestors already final).
template <typename T>
__global__ __launch_bounds__(NT) void k_solve_bwd(FrontMeta M, const int32_t* fronts, const T* L,
                                                  const int32_t* __restrict__ tperm,
                                                  const double* __restrict__ ye, double* xe) {
  __shared__ double g[kSmallMaxNf];
  const int s = fronts[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t f0 = M.sfirst[s];
  const int ns = (int)(M.sfirst[s + 1] - f0);
  const int nf = (int)(M.rptr[s + 1] - M.rptr[s]);
  const int tw = M.tilew[s];
  const int32_t* rows = M.rows + M.rptr[s];
  const T* Lp = L + M.lptr[s];
  const int ntiles = (ns + tw - 1) / tw;
  for (int t = ntiles - 1; t >= 0; t--) {
    int k0, kb;
    tile_bounds(t, tw, ns, k0, kb);
    // g_q = y_q - sum_{i >= k0+kb} L(i, k0+q) x(rows[i])  -- one column per lane group
    for (int q = wave; q < kb; q += NT / 64) {
      double acc = 0.0;
      for (int i = k0 + kb + lane; i < nf; i += 64)
        acc += (double)Lp[i + (int64_t)(k0 + q) * nf] * xe[rows[i]];
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
      if (lane == 0) g[q] = ye[f0 + k0 + q] - acc;
    }
    __syncthreads();
    // L_tt^T w = g, backward, by one wave; lane holds g_lane, g_{lane+64}
    if (wave == 0) {
      double g0 = lane < kb ? g[lane] : 0.0;
      double g1 = lane + 64 < kb ? g[lane + 64] : 0.0;
      for (int p = kb - 1; p >= 0; p--) {
        const double wp = p < 64 ? __shfl(g0, p) : __shfl(g1, p - 64);
        if (lane < p) g0 -= (double)Lp[(k0 + p) + (int64_t)(k0 + lane) * nf] * wp;
        if (lane + 64 < p) g1 -= (double)Lp[(k0 + p) + (int64_t)(k0 + lane + 64) * nf] * wp;
      }
      if (lane < kb) g[lane] = g0;
      if (lane + 64 < kb) g[lane + 64] = g1;
    }
    __syncthreads();
    for (int q = tid; q < kb; q += NT) xe[f0 + k0 + tperm[f0 + k0 + q]] = g[q];
    __syncthreads();
  }
}

// ---- large fronts (tile width kNB), level-batched tile steps ----------------

// R_s <- [xe(cols); 0] + children's update vectors, rows [r0, r0 + kSolveChunk)
template <typename T>
__global__ __launch_bounds__(NT) void k_lfwd_init(FrontMeta M, const Int2* tasks,
                                                  const double* __restrict__ xe, double* R) {
  const Int2 tk = tasks[blockIdx.x];
  const int s = tk.a, r0 = tk.b;
  const int64_t f0 = M.sfirst[s];
  const int ns = (int)(M.sfirst[s + 1] - f0);
  const int nf = (int)(M.rptr[s + 1] - M.rptr[s]);
  const int r1 = min(r0 + kSolveChunk, nf);
  double* Rs = R + M.rptr[s];
  for (int i = r0 + (int)threadIdx.x; i < r1; i += NT) Rs[i] = i < ns ? xe[f0 + i] : 0.0;
  __syncthreads();
  for (int64_t q = M.cptr[s]; q < M.cptr[s + 1]; q++) {
    const int c = M.clist[q];
    const int nsc = (int)(M.sfirst[c + 1] - M.sfirst[c]);
    const int nuc = (int)(M.rptr[c + 1] - M.rptr[c]) - nsc;
    const double* Rc = R + M.rptr[c] + nsc;
    const int32_t* map = M.emap + M.eptr[c];
    int lo = 0, hi = nuc;
    while (lo < hi) { int mid = (lo + hi) >> 1; if (map[mid] < r0) lo = mid + 1; else hi = mid; }
    const int a0 = lo;
    hi = nuc;
    while (lo < hi) { int mid = (lo + hi) >> 1; if (map[mid] < r1) lo = mid + 1; else hi = mid; }
    for (int a = a0 + (int)threadIdx.x; a < lo; a += NT) Rs[map[a]] += Rc[a];
    __syncthreads();
  }
}

// y = D^{-1} z for pivot q of a tile (2x2 blocks never straddle a tile edge);
// z: the tile's values, k = f0 + k0 + q
__device__ inline double apply_dinv(const double* __restrict__ D, const double* __restrict__ E,
                                    const double* z, int64_t k, int q, int kb) {
  if (q + 1 < kb && E[k] != 0.0) {
    const double a = D[k], b = E[k], c = D[k + 1], det = a * c - b * b;
    return (c * z[q] - b * z[q + 1]) / det;
  }
  if (q > 0 && E[k - 1] != 0.0) {
    const double a = D[k - 1], b = E[k - 1], c = D[k], det = a * c - b * b;
    return (a * z[q] - b * z[q - 1]) / det;
  }
  return D[k] != 0.0 ? z[q] / D[k] : 0.0;
}

// The entries apply_dinv reads for pivot q of a tile (k = its index), loaded ahead
// without depending on each other: d_k, e_k, d_{k+1}, e_{k-1}, d_{k-1} (zero where
// apply_dinv does not read them).
__device__ inline void dinv_load(const double* __restrict__ D, const double* __restrict__ E,
                                 int64_t k, int q, int kb, double (&v)[5]) {
  const bool in = q < kb;
  v[0] = in ? D[k] : 1.0;
  v[1] = in && q + 1 < kb ? E[k] : 0.0;
  v[2] = in && q + 1 < kb ? D[k + 1] : 0.0;
  v[3] = in && q > 0 ? E[k - 1] : 0.0;
  v[4] = in && q > 0 ? D[k - 1] : 0.0;
}
// apply_dinv on values from dinv_load: the same cases and arithmetic.
__device__ inline double dinv_apply(const double (&v)[5], const double* z, int q) {
  if (v[1] != 0.0) {
    const double a = v[0], b = v[1], c = v[2], det = a * c - b * b;
    return (c * z[q] - b * z[q + 1]) / det;
  }
  if (v[3] != 0.0) {
    const double a = v[4], b = v[3], c = v[0], det = a * c - b * b;
    return (a * z[q] - b * z[q - 1]) / det;
  }
  return v[0] != 0.0 ? z[q] / v[0] : 0.0;
}

// Sum over the 64 lanes of a wavefront of v[0..63] (lane l holds row l's products
// with 64 columns), by recursive halving: at offset h every lane keeps one half of
// its block of columns and adds its partner's copy of that half.  On return lane l
// holds in v[0] the total of column l.  63 exchanges instead of 64 x 6.
template <int H>
__device__ inline void column_sums_step(double (&v)[kNB], int lane) {
  const bool up = (lane & H) != 0;
#pragma unroll
  for (int j = 0; j < H; j++) {
    const double keep = up ? v[j + H] : v[j];
    const double send = up ? v[j] : v[j + H];
    v[j] = keep + __shfl_xor(send, H);
  }
  if constexpr (H > 1) column_sums_step<H / 2>(v, lane);
}

__device__ inline void wave_column_sums(double (&v)[kNB], int lane) {
  column_sums_step<kNB / 2>(v, lane);
}

constexpr int kChainBlk = 64;                      // rows / columns of a chain-step task
constexpr int kChainThreads = 64 + 4 * kChainBlk;  // wave 0: the tile; then four threads per row

// Forward tile steps t and t + 1 of the large fronts of a level, one launch.
// Every workgroup solves L_tt z = P_t r_t itself (wave 0, the tile in registers,
// row = lane), brings tile t+1's right-hand side up to date with it (four threads
// per row of tile t+1), solves L_{t+1,t+1} z' = P_{t+1} r'_{t+1} (wave 0, tile t+1
// staged in LDS by the other threads while tile t was solved), then updates its
// kChainBlk rows of the pivot block below both tiles with z and z' (four threads
// per row, 16 columns of each tile).  The workgroup of a front's first row chunk
// writes y = D^{-1} z and z itself (for the rows below the pivot block) of both
// tiles.  Without a tile t + 1 (the front's last tile) only tile t is done.  A
// front without pivot-block rows below the two tiles has one task with an empty
// row range.
template <typename T>
__global__ __launch_bounds__(kChainThreads) void k_lfwd_step(FrontMeta M, const Int2* tasks, int t,
                                                             const T* L, const double* __restrict__ D,
                                                             const double* __restrict__ E,
                                                             const int32_t* __restrict__ tperm,
                                                             double* R, double* ye, double* xe) {
  __shared__ double z0[kNB], z1[kNB], r1[kNB];
  __shared__ double tl1[kNB][kNB + 1];   // tile t + 1, [row][column]
  const Int2 tk = tasks[blockIdx.x];
  const int s = tk.a, r0 = tk.b;
  const int tid = threadIdx.x, lane = tid & 63;
  const int64_t f0 = M.sfirst[s];
  const int ns = (int)(M.sfirst[s + 1] - f0);
  const int nf = (int)(M.rptr[s + 1] - M.rptr[s]);
  const int k0 = t * kNB, kb0 = min(kNB, ns - k0);
  const int k1 = k0 + kb0, kb1 = min(kNB, ns - k1);
  const bool two = kb1 > 0;
  const T* Lp = L + M.lptr[s];
  double* Rs = R + M.rptr[s];
  const int u = tid - 64, qr = u & 3, rr = u >> 2;
  const int i = r0 + rr;
  double va[16], vb[16], vc[16];
  double ra = 0.0, ri = 0.0;
  // the workgroup that writes y = D^{-1} z for the two tiles at the end loads their
  // D and E entries now, with everything else
  const bool writer = r0 == (two ? k1 + kb1 : k1);
  double dv0[5] = {1.0, 0.0, 0.0, 0.0, 0.0}, dv1[5] = {1.0, 0.0, 0.0, 0.0, 0.0};
  if (writer && tid < 64) {
    dinv_load(D, E, f0 + k0 + lane, lane, kb0, dv0);
    if (two) dinv_load(D, E, f0 + k1 + lane, lane, kb1, dv1);
  }
  // unconditional loads from clamped (valid) addresses, masked afterwards, so that
  // they are all in flight together
  // the two tiles' interchanges and tile t's rows of R in stored order, loaded with
  // the tile (the interchange is then applied by a lane shuffle, not a second load)
  int tp1 = 0;
  if (tid < 64) {
    const int tp0 = lane < kb0 ? tperm[f0 + k0 + lane] : 0;
    const double rv0 = lane < kb0 ? Rs[k0 + lane] : 0.0;
    tp1 = two && lane < kb1 ? tperm[f0 + k1 + lane] : 0;
    const int lc = min(lane, kb0 - 1);
    double Lv[kNB];
#pragma unroll
    for (int p = 0; p < kNB; p++) Lv[p] = (double)Lp[(k0 + lc) + (int64_t)(k0 + min(p, kb0 - 1)) * nf];
    // strictly lower part of the tile only, so that every step updates all lanes
#pragma unroll
    for (int p = 0; p < kNB; p++) Lv[p] = (lane < kb0 && p < lane) ? Lv[p] : 0.0;
    const double rp = __shfl(rv0, tp0);   // R(k0 + tperm(lane)), from lane tperm(lane)
    double zl = lane < kb0 ? rp : 0.0;
#pragma unroll
    for (int p = 0; p < kNB; p++) zl = fma(-Lv[p], lane_value(zl, p), zl);
    z0[lane] = zl;   // zero beyond kb0
  } else {
    const int ic = min(i, ns - 1);
#pragma unroll
    for (int c = 0; c < 16; c++) vb[c] = (double)Lp[ic + (int64_t)(k0 + min(qr * 16 + c, kb0 - 1)) * nf];
    if (two) {
      const int ia = k1 + min(rr, kb1 - 1);
#pragma unroll
      for (int c = 0; c < 16; c++) va[c] = (double)Lp[ia + (int64_t)(k0 + min(qr * 16 + c, kb0 - 1)) * nf];
#pragma unroll
      for (int c = 0; c < 16; c++) vc[c] = (double)Lp[ic + (int64_t)(k1 + min(qr * 16 + c, kb1 - 1)) * nf];
      // tile t + 1 into LDS: row u mod 64, 16 columns from 16 (u / 64)
      const int tr = u & 63, tc0 = (u >> 6) * 16;
      double w[16];
#pragma unroll
      for (int c = 0; c < 16; c++)
        w[c] = (double)Lp[(k1 + min(tr, kb1 - 1)) + (int64_t)(k1 + min(tc0 + c, kb1 - 1)) * nf];
#pragma unroll
      for (int c = 0; c < 16; c++) tl1[tr][tc0 + c] = w[c];
      if (qr == 0 && rr < kb1) ra = Rs[k1 + rr];
    }
    // the row's right-hand side, read before the barrier: rows below the tiles are
    // written by their own workgroup only
    if (qr == 0 && i < ns) ri = Rs[i];
  }
  __syncthreads();
  if (two) {
    if (tid >= 64) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < 16; c++) acc = fma(va[c], z0[qr * 16 + c], acc);
      acc += __shfl_xor(acc, 1);
      acc += __shfl_xor(acc, 2);
      if (qr == 0) r1[rr] = ra - acc;   // stored (unswapped) row order of tile t + 1
    }
    __syncthreads();
    if (tid < 64) {
      double Lw[kNB];
#pragma unroll
      for (int p = 0; p < kNB; p++) Lw[p] = (lane < kb1 && p < lane) ? tl1[lane][p] : 0.0;
      double zl = lane < kb1 ? r1[tp1] : 0.0;
#pragma unroll
      for (int p = 0; p < kNB; p++) zl = fma(-Lw[p], lane_value(zl, p), zl);
      z1[lane] = zl;
    }
    __syncthreads();
  }
  if (tid >= 64) {
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 16; c++) acc = fma(vb[c], z0[qr * 16 + c], acc);
    if (two) {
#pragma unroll
      for (int c = 0; c < 16; c++) acc = fma(vc[c], z1[qr * 16 + c], acc);
    }
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    if (qr == 0 && i < ns) Rs[i] = ri - acc;
  }
  // the first chunk's workgroup: y = D^{-1} z and z itself (xe of the pivots is free
  // once the level's gather has read it)
  if (writer) {
    if (tid < kb0) {
      ye[f0 + k0 + tid] = dinv_apply(dv0, z0, tid);
      xe[f0 + k0 + tid] = z0[tid];
    }
    if (two && tid < kb1) {
      ye[f0 + k1 + tid] = dinv_apply(dv1, z1, tid);
      xe[f0 + k1 + tid] = z1[tid];
    }
  }
}

// Forward, rows below the pivot block: workgroup (task, seg) stores for its
// kL21Rows rows the products with column segment seg,
//   P[(task nseg + seg) kL21Rows + r] = sum_{q in seg} L(r0 + r, q) z_q,
// z_q = xe[f0 + q]; segments past the front's columns store nothing.
template <typename T>
__global__ __launch_bounds__(kL21Rows) void k_lfwd_l21(FrontMeta M, const Int2* tasks, int nseg,
                                                       const T* L, const double* __restrict__ xe,
                                                       double* P) {
  __shared__ double z[kL21Cols];
  const Int2 tk = tasks[blockIdx.x];
  const int s = tk.a, r0 = tk.b, seg = blockIdx.y;
  const int64_t f0 = M.sfirst[s];
  const int ns = (int)(M.sfirst[s + 1] - f0);
  const int nf = (int)(M.rptr[s + 1] - M.rptr[s]);
  const int c0 = seg * kL21Cols;
  if (c0 >= ns) return;
  const int c1 = min(c0 + kL21Cols, ns);
  const int tid = threadIdx.x;
  for (int q = tid; q < c1 - c0; q += kL21Rows) z[q] = xe[f0 + c0 + q];
  __syncthreads();
  const int i = r0 + tid;
  if (i >= nf) return;
  const T* Lp = L + M.lptr[s] + i;
  double acc = 0.0;
  int q = c0;
  // 32 loads in flight per pass (8 passes for a full segment), the products
  // accumulated in column order
  for (; q + 32 <= c1; q += 32) {
    double v[32];
#pragma unroll
    for (int u = 0; u < 32; u++) v[u] = (double)Lp[(int64_t)(q + u) * nf];
#pragma unroll
    for (int u = 0; u < 32; u++) acc = fma(v[u], z[q - c0 + u], acc);
  }
  for (; q + 8 <= c1; q += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; u++) v[u] = (double)Lp[(int64_t)(q + u) * nf];
#pragma unroll
    for (int u = 0; u < 8; u++) acc = fma(v[u], z[q - c0 + u], acc);
  }
  for (; q < c1; q++) acc = fma((double)Lp[(int64_t)q * nf], z[q - c0], acc);
  P[((int64_t)blockIdx.x * nseg + seg) * kL21Rows + tid] = acc;
}

// R_i -= the segments' products of row i, in segment order.
__global__ __launch_bounds__(kL21Rows) void k_lfwd_l21_reduce(FrontMeta M, const Int2* tasks,
                                                              int nseg, const double* P, double* R) {
  const Int2 tk = tasks[blockIdx.x];
  const int s = tk.a, r0 = tk.b;
  const int ns = (int)(M.sfirst[s + 1] - M.sfirst[s]);
  const int nf = (int)(M.rptr[s + 1] - M.rptr[s]);
  const int i = r0 + (int)threadIdx.x;
  if (i >= nf) return;
  const int used = (ns + kL21Cols - 1) / kL21Cols;
  const double* p = P + (int64_t)blockIdx.x * nseg * kL21Rows + threadIdx.x;
  double sum = 0.0;
  for (int g = 0; g < used; g++) sum += p[(int64_t)g * kL21Rows];
  R[M.rptr[s] + i] -= sum;
}

// Backward tile steps t + 1 and t (pairs in reverse), one launch, in the form that
// pushes each finished tile into the columns before it.  Every workgroup solves
// L_{t+1,t+1}^T w' = y_{t+1} itself (wave 0: the tile through LDS, column = lane),
// y_{t+1} having received the contributions of all later tiles and of the rows
// below the pivot block; its other threads push w' into tile t's y (four threads
// per column), wave 0 solves L_tt^T w = y_t (tile t staged in LDS meanwhile), and
// the other threads subtract, for kChainBlk columns j < k0 of the pivot block,
// y_j -= sum_i L(k0 + i, j) x_i + sum_i L(k1 + i, j) x'_i, the rows of each tile
// in their stored (unswapped) order.  The workgroup of the first column chunk
// writes x(f0 + k + perm[q]) = w_q of both tiles.  Without a tile t + 1 only tile t
// is done; tile 0 has one task with an empty column range.
template <typename T>
__global__ __launch_bounds__(kChainThreads) void k_lbwd_push(FrontMeta M, const Int2* tasks, int t,
                                                             const T* L,
                                                             const int32_t* __restrict__ tperm,
                                                             double* ye, double* xe) {
  __shared__ double tl[kNB][kNB + 1];    // tile t + 1 (wave 0's transposition buffer)
  __shared__ double tl0[kNB][kNB + 1];   // tile t, [row][column]
  __shared__ double xs0[kNB], xs1[kNB], yt[kNB];
  const Int2 tk = tasks[blockIdx.x];
  const int s = tk.a, c0 = tk.b;
  const int tid = threadIdx.x, lane = tid & 63;
  const int64_t f0 = M.sfirst[s];
  const int ns = (int)(M.sfirst[s + 1] - f0);
  const int nf = (int)(M.rptr[s + 1] - M.rptr[s]);
  const int k0 = t * kNB, kb0 = min(kNB, ns - k0);
  const int k1 = k0 + kb0, kb1 = min(kNB, ns - k1);
  const bool two = kb1 > 0;
  const T* Lp = L + M.lptr[s];
  const int u = tid - 64, qr = u & 3, jj = u >> 2;
  const int j = c0 + jj;
  double va[16], vb[16], vc[16];
  double yv = 0.0, yj = 0.0;
  int tp0 = 0;   // tile t's interchanges (used after its chain), loaded early
  if (tid < 64) {
    tp0 = lane < kb0 ? tperm[f0 + k0 + lane] : 0;
    if (two) {
      // row lane of tile t + 1 into LDS (coalesced loads), then column lane from it;
      // one wave: its LDS writes and reads complete in order
      const int lc = min(lane, kb1 - 1);
      double Lr[kNB];
#pragma unroll
      for (int p = 0; p < kNB; p++) Lr[p] = (double)Lp[(k1 + lc) + (int64_t)(k1 + min(p, kb1 - 1)) * nf];
      double g = lane < kb1 ? ye[f0 + k1 + lane] : 0.0;
      const int tp = lane < kb1 ? tperm[f0 + k1 + lane] : 0;
#pragma unroll
      for (int p = 0; p < kNB; p++) tl[lane][p] = Lr[p];
      double Lc[kNB];
#pragma unroll
      for (int p = 0; p < kNB; p++) Lc[p] = (p > lane && p < kb1) ? tl[p][lane] : 0.0;
      // w_q = g_q - sum_{p > q} L(p, q) w_p, p descending (zero beyond kb1)
#pragma unroll
      for (int p = kNB - 1; p >= 0; p--) g = fma(-Lc[p], lane_value(g, p), g);
      xs1[lane] = 0.0;
      if (lane < kb1) xs1[tp] = g;
      if (c0 == 0 && lane < kb1) xe[f0 + k1 + tp] = g;
    }
  } else {
    // tile t + 1's push into tile t's columns: column jj of tile t, 16 rows of t + 1
    if (two) {
#pragma unroll
      for (int c = 0; c < 16; c++)
        va[c] = (double)Lp[(k1 + min(qr * 16 + c, kb1 - 1)) + (int64_t)(k0 + min(jj, kb0 - 1)) * nf];
    }
    if (qr == 0 && jj < kb0) yv = ye[f0 + k0 + jj];
    // the entry of y this thread updates at the end (no other access here touches it)
    if (qr == 0 && j < k0) yj = ye[f0 + j];
    // this chunk's columns j < k0: 16 rows of each tile
    const int jc = min(j, max(k0 - 1, 0));
#pragma unroll
    for (int c = 0; c < 16; c++) vb[c] = (double)Lp[(k0 + min(qr * 16 + c, kb0 - 1)) + (int64_t)jc * nf];
    if (two) {
#pragma unroll
      for (int c = 0; c < 16; c++) vc[c] = (double)Lp[(k1 + min(qr * 16 + c, kb1 - 1)) + (int64_t)jc * nf];
    }
    // tile t into LDS: row u mod 64, 16 columns from 16 (u / 64)
    const int tr = u & 63, tc0 = (u >> 6) * 16;
    double w[16];
#pragma unroll
    for (int c = 0; c < 16; c++)
      w[c] = (double)Lp[(k0 + min(tr, kb0 - 1)) + (int64_t)(k0 + min(tc0 + c, kb0 - 1)) * nf];
#pragma unroll
    for (int c = 0; c < 16; c++) tl0[tr][tc0 + c] = w[c];
  }
  __syncthreads();
  if (tid >= 64) {
    double acc = 0.0;
    if (two) {
#pragma unroll
      for (int c = 0; c < 16; c++) acc = fma(va[c], xs1[qr * 16 + c], acc);
    }
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    if (qr == 0) yt[jj] = yv - acc;   // pivot order of tile t; zero-based garbage beyond kb0
  }
  __syncthreads();
  if (tid < 64) {
    double Lc[kNB];
#pragma unroll
    for (int p = 0; p < kNB; p++) Lc[p] = (p > lane && p < kb0) ? tl0[p][lane] : 0.0;
    double g = lane < kb0 ? yt[lane] : 0.0;
#pragma unroll
    for (int p = kNB - 1; p >= 0; p--) g = fma(-Lc[p], lane_value(g, p), g);
    xs0[lane] = 0.0;
    if (lane < kb0) xs0[tp0] = g;
    if (c0 == 0 && lane < kb0) xe[f0 + k0 + tp0] = g;
  }
  __syncthreads();
  if (tid >= 64) {
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 16; c++) acc = fma(vb[c], xs0[qr * 16 + c], acc);
    if (two) {
#pragma unroll
      for (int c = 0; c < 16; c++) acc = fma(vc[c], xs1[qr * 16 + c], acc);
    }
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    if (qr == 0 && j < k0) ye[f0 + j] = yj - acc;
  }
}

// Backward, rows below the pivot block: workgroup (task, t) stores the column sums
// of its kL21Rows rows over pivot tile t,
//   P[(task ntile + t) kNB + q] = sum_i L(i, k0 + q) x(rows[i]),
// row = thread (coalesced loads), wave_column_sums; tiles past the front's columns
// store nothing.
template <typename T>
__global__ __launch_bounds__(kL21Rows) void k_lbwd_l21(FrontMeta M, const Int2* tasks, int ntile,
                                                       const T* L, const double* __restrict__ xe,
                                                       double* P) {
  __shared__ double wsum[kL21Rows / 64][kNB];
  const Int2 tk = tasks[blockIdx.x];
  const int s = tk.a, r0 = tk.b, t = blockIdx.y;
  const int64_t f0 = M.sfirst[s];
  const int ns = (int)(M.sfirst[s + 1] - f0);
  const int nf = (int)(M.rptr[s + 1] - M.rptr[s]);
  const int k0 = t * kNB;
  if (k0 >= ns) return;
  const int kb = min(kNB, ns - k0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = r0 + tid;
  const int ic = min(i, nf - 1);
  const double xi = i < nf ? xe[M.rows[M.rptr[s] + ic]] : 0.0;
  const T* Lp = L + M.lptr[s];
  double v[kNB];
#pragma unroll
  for (int q = 0; q < kNB; q++) v[q] = (double)Lp[ic + (int64_t)(k0 + min(q, kb - 1)) * nf];
#pragma unroll
  for (int q = 0; q < kNB; q++) v[q] = q < kb ? v[q] * xi : 0.0;
  wave_column_sums(v, lane);
  wsum[wave][lane] = v[0];
  __syncthreads();
  if (tid < 64) {
    double acc = 0.0;
#pragma unroll
    for (int w = 0; w < kL21Rows / 64; w++) acc += wsum[w][lane];
    P[((int64_t)blockIdx.x * ntile + t) * kNB + lane] = acc;
  }
}

// y(f0 + k0 + q) -= the row chunks' column sums of tile t, in chunk order
// (workgroup (front, t), one lane per column).
__global__ __launch_bounds__(64) void k_lbwd_l21_reduce(FrontMeta M, const int32_t* fronts,
                                                        const int32_t* __restrict__ l21base,
                                                        int ntile, const double* P, double* ye) {
  const int s = fronts[blockIdx.x], t = blockIdx.y, lane = threadIdx.x;
  const int64_t f0 = M.sfirst[s];
  const int ns = (int)(M.sfirst[s + 1] - f0);
  const int nf = (int)(M.rptr[s + 1] - M.rptr[s]);
  const int k0 = t * kNB;
  if (k0 >= ns || nf <= ns) return;
  const int kb = min(kNB, ns - k0);
  const int nrb = (nf - ns + kL21Rows - 1) / kL21Rows;
  const double* p = P + ((int64_t)l21base[s] * ntile + t) * kNB + lane;
  double sum = 0.0;
  for (int j = 0; j < nrb; j++) sum += p[(int64_t)j * ntile * kNB];
  if (lane < kb) ye[f0 + k0 + lane] -= sum;
}

__global__ void k_gather(int64_t n, const int64_t* __restrict__ perm, const double* __restrict__ x,
                         double* __restrict__ xe) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    xe[k] = x[perm[k]];
}

__global__ void k_scatter(int64_t n, const int64_t* __restrict__ perm, const double* __restrict__ xe,
                          double* __restrict__ x) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    x[perm[k]] = xe[k];
}

inline int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (int)(g < 65536 ? (g > 0 ? g : 1) : 65536);
}

}  // namespace

template <typename T>
void solve_enqueue(const SolvePlan& P, const FrontMeta& M, const T* L, const double* D,
                   const double* E, const int32_t* tperm, const int64_t* perm, int64_t n,
                   const double* b, double* x, double* xe, double* ye, double* R, double* partial,
                   hipStream_t s) {
  const int32_t* sc = P.sched;
  double* p21 = partial + P.l21_part_off;
  hipLaunchKernelGGL(k_gather, dim3(grid_for(n)), dim3(256), 0, s, n, perm, b, xe);
  for (const SolveLevel& lv : P.levels) {
    if (lv.small_cnt > 0)
      hipLaunchKernelGGL((k_solve_fwd<T>), dim3(lv.small_cnt), dim3(NT), 0, s, M, sc + lv.small_off,
                         L, D, E, tperm, xe, R, ye);
    if (lv.large_cnt == 0) continue;
    hipLaunchKernelGGL((k_lfwd_init<T>), dim3(lv.init_cnt), dim3(NT), 0, s, M,
                       reinterpret_cast<const Int2*>(sc + lv.init_off), xe, R);
    for (const SolveStep& st : lv.steps)
      hipLaunchKernelGGL((k_lfwd_step<T>), dim3(st.fwd_cnt), dim3(kChainThreads), 0, s, M,
                         reinterpret_cast<const Int2*>(sc + st.fwd_off), st.t, L, D, E, tperm, R, ye,
                         xe);
    if (lv.l21_cnt > 0) {
      const Int2* tk = reinterpret_cast<const Int2*>(sc + lv.l21_off);
      hipLaunchKernelGGL((k_lfwd_l21<T>), dim3(lv.l21_cnt, lv.l21_nseg), dim3(kL21Rows), 0, s, M, tk,
                         lv.l21_nseg, L, xe, p21);
      hipLaunchKernelGGL(k_lfwd_l21_reduce, dim3(lv.l21_cnt), dim3(kL21Rows), 0, s, M, tk,
                         lv.l21_nseg, p21, R);
    }
  }
  for (size_t l = P.levels.size(); l-- > 0;) {
    const SolveLevel& lv = P.levels[l];
    if (lv.small_cnt > 0)
      hipLaunchKernelGGL((k_solve_bwd<T>), dim3(lv.small_cnt), dim3(NT), 0, s, M, sc + lv.small_off,
                         L, tperm, ye, xe);
    if (lv.l21_cnt > 0) {
      const Int2* tk = reinterpret_cast<const Int2*>(sc + lv.l21_off);
      hipLaunchKernelGGL((k_lbwd_l21<T>), dim3(lv.l21_cnt, lv.l21_ntile), dim3(kL21Rows), 0, s, M, tk,
                         lv.l21_ntile, L, xe, p21);
      hipLaunchKernelGGL(k_lbwd_l21_reduce, dim3(lv.large_cnt, lv.l21_ntile), dim3(64), 0, s, M,
                         sc + lv.large_off, P.l21base, lv.l21_ntile, p21, ye);
    }
    for (size_t q = lv.steps.size(); q-- > 0;) {
      const SolveStep& st = lv.steps[q];
      hipLaunchKernelGGL((k_lbwd_push<T>), dim3(st.bwd_cnt), dim3(kChainThreads), 0, s, M,
                         reinterpret_cast<const Int2*>(sc + st.bwd_off), st.t, L, tperm, ye, xe);
    }
  }
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(n)), dim3(256), 0, s, n, perm, xe, x);
}

// ---- work array of the allocation-free solve (kth_solve_noalloc) -----------
// A __device__ object has one instance on every GPU the code object is loaded on.
// Its name is only a host-side stand-in: host code uses the per-device address
// that hipGetSymbolAddress returns (taken once per device, with that device
// current, when a context is created) and passes it to the kernels.
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace {
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;   // indexed by device
}  // namespace

hipError_t noalloc_scratch_init(int device) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (device < 0) return hipErrorInvalidDevice;
  if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = static_cast<double*>(p);
  return hipSuccess;
}

double* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return device >= 0 && device < (int)g_scratch_ptr.size() ? g_scratch_ptr[device] : nullptr;
}

template void solve_enqueue<double>(const SolvePlan&, const FrontMeta&, const double*, const double*,
                                    const double*, const int32_t*, const int64_t*, int64_t,
                                    const double*, double*, double*, double*, double*, double*,
                                    hipStream_t);
template void solve_enqueue<float>(const SolvePlan&, const FrontMeta&, const float*, const double*,
                                   const double*, const int32_t*, const int64_t*, int64_t,
                                   const double*, double*, double*, double*, double*, double*,
                                   hipStream_t);

}  // namespace kth
