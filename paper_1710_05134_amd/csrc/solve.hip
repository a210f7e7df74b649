// Triangular solves with a kept multifrontal factor: (A - sigma B) x = b as
// L z = P b (forward, leaves to root), y = D^{-1} z, L^T w = y with x = P^T w
// (backward, root to leaves).  The forward pass is itself multifrontal: each
// front gathers its right-hand side, adds its children's update vectors (the
// tails of their work vectors) and hands its own tail to its parent, so no two
// fronts ever write the same entry.  Tile permutations are applied when the
// solve reaches each tile (the factor keeps earlier panels' rows unswapped).
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

constexpr int kFwdThreads = 64 + kSolveRows;   // wave 0: tile solve; the rest: one row each
constexpr int kBwdThreads = kSolveRows;        // one row each (four waves)

// Forward tile step t of the large fronts of a level, one launch.  Every
// workgroup solves L_tt z = P_t r_t itself (wave 0, the 64x64 tile in registers,
// row = lane) while its other waves load their rows' 64 entries of L below the
// tile; then R_i -= L(i, tile) z for its kSolveRows rows.  The workgroup of a
// front's first row chunk also writes y = D^{-1} z.  A front without rows below
// the tile has one task with an empty row range.
template <typename T>
__global__ __launch_bounds__(kFwdThreads) void k_lfwd_step(FrontMeta M, const Int2* tasks, int t,
                                                           const T* L, const double* __restrict__ D,
                                                           const double* __restrict__ E,
                                                           const int32_t* __restrict__ tperm,
                                                           double* R, double* ye) {
  __shared__ double z[kNB];
  const Int2 tk = tasks[blockIdx.x];
  const int s = tk.a, r0 = tk.b;
  const int tid = threadIdx.x, lane = tid & 63;
  const int64_t f0 = M.sfirst[s];
  const int ns = (int)(M.sfirst[s + 1] - f0);
  const int nf = (int)(M.rptr[s + 1] - M.rptr[s]);
  const int k0 = t * kNB, kb = min(kNB, ns - k0);
  const T* Lp = L + M.lptr[s];
  double* Rs = R + M.rptr[s];
  double Lv[kNB];
  const int i = r0 + tid - 64;
  // unconditional loads from clamped (valid) addresses, masked afterwards, so that
  // all 64 are in flight together
  if (tid < 64) {
    const int lc = min(lane, kb - 1);
#pragma unroll
    for (int p = 0; p < kNB; p++) Lv[p] = (double)Lp[(k0 + lc) + (int64_t)(k0 + min(p, kb - 1)) * nf];
    // strictly lower part of the tile only, so that every step updates all lanes
#pragma unroll
    for (int p = 0; p < kNB; p++) Lv[p] = (lane < kb && p < lane) ? Lv[p] : 0.0;
    double zl = lane < kb ? Rs[k0 + tperm[f0 + k0 + lane]] : 0.0;
#pragma unroll
    for (int p = 0; p < kNB; p++) zl = fma(-Lv[p], lane_value(zl, p), zl);
    z[lane] = zl;
  } else {
    const int ic = min(i, nf - 1);
#pragma unroll
    for (int q = 0; q < kNB; q++) Lv[q] = (double)Lp[ic + (int64_t)(k0 + min(q, kb - 1)) * nf];
#pragma unroll
    for (int q = 0; q < kNB; q++) Lv[q] = q < kb ? Lv[q] : 0.0;
  }
  // this row's right-hand side, read before the barrier: rows below the tile are
  // written by their own workgroup only
  const double ri = (tid >= 64 && i < nf) ? Rs[i] : 0.0;
  __syncthreads();
  if (tid >= 64 && i < nf) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < kNB; q++) acc = fma(Lv[q], z[q], acc);
    Rs[i] = ri - acc;
  }
  if (r0 == k0 + kb && tid < kb) ye[f0 + k0 + tid] = apply_dinv(D, E, z, f0 + k0 + tid, tid, kb);
}

// Backward, tile t of front s: w = L_tt^{-T} (y_t - sum of the front's partial
// column sums of step t, in chunk order), x(f0 + k0 + perm[q]) = w_q.  Called by
// all threads of a workgroup; tl: LDS staging of the tile (row-major, padded).
template <typename T>
__device__ inline void bwd_finish_tile(const FrontMeta& M, int s, int t, const T* L,
                                       const int32_t* __restrict__ tperm,
                                       const double* __restrict__ ye, const double* partial,
                                       double* xe, double (&tl)[kNB][kNB + 1]) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int64_t f0 = M.sfirst[s];
  const int ns = (int)(M.sfirst[s + 1] - f0);
  const int nf = (int)(M.rptr[s + 1] - M.rptr[s]);
  const int k0 = t * kNB, kb = min(kNB, ns - k0), rb = k0 + kb;
  const int ntask = nf > rb ? (nf - rb + kSolveRows - 1) / kSolveRows : 1;
  const T* Lp = L + M.lptr[s];
  for (int e = tid; e < kNB * kNB; e += blockDim.x) {
    const int r = e & 63, c = e >> 6;
    tl[r][c] = (r < kb && c < kb) ? (double)Lp[(k0 + r) + (int64_t)(k0 + c) * nf] : 0.0;
  }
  __syncthreads();
  if (tid < 64) {
    // partial sums in chunk order, loaded eight at a time
    double acc = 0.0;
    for (int j0 = 0; j0 < ntask; j0 += 8) {
      double pv[8];
#pragma unroll
      for (int u = 0; u < 8; u++) pv[u] = partial[(int64_t)min(j0 + u, ntask - 1) * kNB + lane];
#pragma unroll
      for (int u = 0; u < 8; u++)
        if (j0 + u < ntask) acc += pv[u];
    }
    double g = lane < kb ? ye[f0 + k0 + lane] - acc : 0.0;
    // column lane of the tile, strictly below the diagonal
    double Lc[kNB];
#pragma unroll
    for (int p = 0; p < kNB; p++) Lc[p] = p > lane ? tl[p][lane] : 0.0;
#pragma unroll
    for (int p = kNB - 1; p >= 0; p--) g = fma(-Lc[p], lane_value(g, p), g);
    if (lane < kb) xe[f0 + k0 + tperm[f0 + k0 + lane]] = g;
  }
  __syncthreads();
}

// Backward tile step t (tiles in reverse), one launch, no inter-workgroup
// synchronisation: the workgroup of a front's first row chunk first finishes tile
// t+1 (whose rows open its chunk) from the partial sums the previous launch left;
// then every workgroup stores the column sums sum_i L(i, k0+q) x(rows[i]) of its
// kSolveRows rows (row = thread, coalesced loads, wave_column_sums) in the front's
// slot for this step's parity.  Tile 0 is finished by k_lbwd_finish.
// partial: [2][slots][kNB]; pbase[s]: the front's first slot (its chunk j at +j).
template <typename T>
__global__ __launch_bounds__(kBwdThreads) void k_lbwd_step(FrontMeta M, const Int2* tasks, int t,
                                                           const T* L,
                                                           const int32_t* __restrict__ tperm,
                                                           const double* __restrict__ ye,
                                                           const int64_t* __restrict__ pbase,
                                                           int64_t half, double* partial,
                                                           double* xe) {
  __shared__ double wsum[kBwdThreads / 64][kNB];
  __shared__ double tl[kNB][kNB + 1];
  const Int2 tk = tasks[blockIdx.x];
  const int s = tk.a, r0 = tk.b;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t f0 = M.sfirst[s];
  const int ns = (int)(M.sfirst[s + 1] - f0);
  const int nf = (int)(M.rptr[s + 1] - M.rptr[s]);
  const int k0 = t * kNB, kb = min(kNB, ns - k0);
  const int rb = k0 + kb;                      // first row below the tile
  const int64_t pb = pbase[s];
  const int i = r0 + tid;
  const int ic = min(i, nf - 1);
  const int64_t gi = M.rows[M.rptr[s] + ic];
  // tile t+1 exists and opens this chunk: this workgroup finishes it first; x of
  // its rows is ready after that, x of every other row already
  const bool fin = r0 == rb && rb < ns;
  const bool late = fin && i < min(rb + kNB, ns);
  double xi = (!late && i < nf) ? xe[gi] : 0.0;
  if (fin) bwd_finish_tile(M, s, t + 1, L, tperm, ye, partial + (((t + 1) & 1) * half + pb) * kNB, xe, tl);
  if (late) xi = xe[gi];
  const T* Lp = L + M.lptr[s];
  {
    // unconditional loads from clamped (valid) addresses, masked afterwards, so
    // that all 64 are in flight together
    double v[kNB];
#pragma unroll
    for (int q = 0; q < kNB; q++) v[q] = (double)Lp[ic + (int64_t)(k0 + min(q, kb - 1)) * nf];
#pragma unroll
    for (int q = 0; q < kNB; q++) v[q] = q < kb ? v[q] * xi : 0.0;
    wave_column_sums(v, lane);
    wsum[wave][lane] = v[0];
  }
  __syncthreads();
  if (tid < 64) {
    double acc = 0.0;
#pragma unroll
    for (int w = 0; w < kBwdThreads / 64; w++) acc += wsum[w][lane];
    const int j = (r0 - rb) / kSolveRows;
    partial[((t & 1) * half + pb + j) * kNB + lane] = acc;
  }
}

// Backward: tile 0 of every large front of a level (one workgroup per front).
template <typename T>
__global__ __launch_bounds__(kBwdThreads) void k_lbwd_finish(FrontMeta M, const int32_t* fronts,
                                                             const T* L,
                                                             const int32_t* __restrict__ tperm,
                                                             const double* __restrict__ ye,
                                                             const int64_t* __restrict__ pbase,
                                                             const double* partial, double* xe) {
  __shared__ double tl[kNB][kNB + 1];
  const int s = fronts[blockIdx.x];
  bwd_finish_tile(M, s, 0, L, tperm, ye, partial + pbase[s] * kNB, xe, tl);
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
  hipLaunchKernelGGL(k_gather, dim3(grid_for(n)), dim3(256), 0, s, n, perm, b, xe);
  for (const SolveLevel& lv : P.levels) {
    if (lv.small_cnt > 0)
      hipLaunchKernelGGL((k_solve_fwd<T>), dim3(lv.small_cnt), dim3(NT), 0, s, M, sc + lv.small_off,
                         L, D, E, tperm, xe, R, ye);
    if (lv.large_cnt == 0) continue;
    hipLaunchKernelGGL((k_lfwd_init<T>), dim3(lv.init_cnt), dim3(NT), 0, s, M,
                       reinterpret_cast<const Int2*>(sc + lv.init_off), xe, R);
    for (const SolveStep& st : lv.steps)
      hipLaunchKernelGGL((k_lfwd_step<T>), dim3(st.task_cnt), dim3(kFwdThreads), 0, s, M,
                         reinterpret_cast<const Int2*>(sc + st.task_off), st.t, L, D, E, tperm, R, ye);
  }
  for (size_t l = P.levels.size(); l-- > 0;) {
    const SolveLevel& lv = P.levels[l];
    if (lv.small_cnt > 0)
      hipLaunchKernelGGL((k_solve_bwd<T>), dim3(lv.small_cnt), dim3(NT), 0, s, M, sc + lv.small_off,
                         L, tperm, ye, xe);
    for (size_t q = lv.steps.size(); q-- > 0;) {
      const SolveStep& st = lv.steps[q];
      hipLaunchKernelGGL((k_lbwd_step<T>), dim3(st.task_cnt), dim3(kBwdThreads), 0, s, M,
                         reinterpret_cast<const Int2*>(sc + st.task_off), st.t, L, tperm, ye,
                         P.pbase, P.partial_half, partial, xe);
    }
    if (lv.large_cnt > 0)
      hipLaunchKernelGGL((k_lbwd_finish<T>), dim3(lv.large_cnt), dim3(kBwdThreads), 0, s, M,
                         sc + lv.large_off, L, tperm, ye, P.pbase, partial, xe);
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
