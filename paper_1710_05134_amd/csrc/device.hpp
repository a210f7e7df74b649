// Device-side data layout shared by the numeric kernels and their host launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace kth {

// Tree / front metadata (device pointers, built once per pattern).
struct FrontMeta {
  const int64_t* sfirst;  // [nsup+1] first elimination column of each supernode
  const int64_t* rptr;    // [nsup+1] offsets into rows
  const int32_t* rows;    // front row lists (elimination indices)
  const int64_t* lptr;    // [nsup+1] panel offsets (nf*ns, ld nf)
  const int64_t* uptr;    // [nsup]   update-block offsets in the pool (-1: none)
  const int64_t* eptr;    // [nsup+1] extend-add map offsets
  const int32_t* emap;
  const int64_t* cptr;    // [nsup+1] children
  const int32_t* clist;
  const int64_t* acptr;   // [n+1] original entries per elimination column
  const int64_t* asrc;
  const int64_t* adst;
  const int32_t* tilew;   // [nsup] pivot-tile width (ns for fronts factored in one piece)
  const int64_t* tptr;    // [nsup]   tile-inverse offsets (kNB*kNB per large front; -1 otherwise)
  const int64_t* iptr;    // [nsup]   child c of a large front: offset of its inverse map (-1: none)
  const int32_t* imap;    // inverse maps: imap[iptr[c] + i] = child row of parent row i, or -1
};

// Results of one numeric factorization that the host reads back.
struct FactStats {
  unsigned long long neg, zero, pos, n2x2;
  unsigned long long min_d_bits;   // bit pattern of min |eigenvalue of a D block| (>= 0)
  unsigned long long max_l_bits;   // bit pattern of max |L_ij|
  unsigned long long pad[2];
};

// Largest front factored wholly in LDS by one workgroup.
constexpr int kSmallMaxNf = 128;
// Pivot-tile width (and panel width) of large fronts.
constexpr int kNB = 64;
// Column chunk and row block of one large-front assembly task (the row block is
// the 64 x 8 rows one wavefront gathers per column in one pass).
constexpr int kAsmCols = 16;
constexpr int kAsmRows = 512;
// Rows per workgroup of the panel triangular solve.
constexpr int kTrsmRows = 64;
// Rows per gather task of the large-front solve.
constexpr int kSolveChunk = 256;
// solve: rows below a front's pivot block (L21) per task, and the forward pass's
// column segment width there
constexpr int kL21Rows = 256;
constexpr int kL21Cols = 256;
// Schur-update output tile.
constexpr int kTile = 64;
// Task flag of a left-looking rows-below launch (mode 1) for pivot tile t: the
// task (front, row | kLaFlag) is the diagonal block of tile t + 1 at the same depth
// t * kNB (its update without tile t's columns, applied ahead).
constexpr int kLaFlag = 1 << 30;
// fronts whose contribution block has at least this many rows update it on
// 128 x 128 tiles (k_gemm_cb128)
constexpr int kCb128MinNu = 384;
// depth segment of a split left-looking update of the rows below a pivot tile
constexpr int kSegK = 256;
// workgroups a split-depth left-looking launch aims at (four per CU)
constexpr int kLLTargetWgs = 1024;

struct Int2 { int32_t a, b; };

// Several factorizations of one pencil advance together (multisection): the
// batch index is blockIdx.y, and every per-factorization array is offset by
// its stride (in elements).
constexpr int kMaxBatch = 64;
struct Batch {
  int64_t sL = 0;   // factor panels
  int64_t sU = 0;   // update-block pool
  int64_t sW = 0;   // panel workspace
  int64_t sT = 0;   // tile inverses
  int64_t sP = 0;   // split-depth partial products
  int64_t sN = 0;   // n-vectors (D, E, pivot order)
  const double* sig = nullptr;   // [batch] shifts
};
struct SigmaPack { double v[kMaxBatch]; };

// ---- launchers (factor.hip); nb = number of batched factorizations ---------
void launch_fill_stats(FactStats* st, int nb, hipStream_t s);
// T = double (inertia-deciding factors) or float (shift-and-invert factor).
template <typename T>
void launch_small_fronts(const FrontMeta& M, const int32_t* fronts, int32_t count, int32_t max_nf,
                         const double* aval, const double* bval, const Batch& bt, int nb,
                         T* L, T* U, double* D, double* E, int32_t* tperm,
                         FactStats* st, hipStream_t s);
template <typename T>
void launch_front_init(const FrontMeta& M, const Int2* tasks, int32_t count, const double* aval,
                       const double* bval, const Batch& bt, int nb, T* L, T* U, hipStream_t s);
template <typename T>
void launch_tile_factor(const FrontMeta& M, const int32_t* fronts, int32_t count, int32_t t,
                        const Batch& bt, int nb, T* L, double* D, double* E, int32_t* tperm,
                        T* tinv, FactStats* st, hipStream_t s);
// Panel solve of the rows below pivot tile t, tasks (front, first row).  With upd,
// a task whose rows are the next tile's (first row < ns) also applies this tile's
// columns to the next tile's diagonal block: C -= L W^T over the tile's depth.
template <typename T>
void launch_panel_trsm(const FrontMeta& M, const Int2* tasks, int32_t count, int32_t t,
                       const Batch& bt, int nb, T* L, T* W, const double* D, const double* E,
                       const int32_t* tperm, const T* tinv, FactStats* st, int upd, hipStream_t s);
// Left-looking updates C -= L W^T (W = L D panel-shaped): mode 0/1, column block of
// pivot tile t for tasks (front, first row) -- mode 0 the tile's diagonal block,
// mode 1 rows below it; mode 2, tasks (front, lower tile number) of the
// contribution block with depth ns.
// Modes 0 / 1 with nseg > 1 split the depth into segments of segk columns (a
// multiple of 16) whose partial products go to part (bt.sP elements per batch:
// count * nseg * kTile^2 needed); launch_gemm_reduce then applies them.  A mode-1
// task (front, row | kLaFlag) is the diagonal block of tile t + 1 at depth t * kNB.
template <typename T>
void launch_gemm_lt(const FrontMeta& M, const Int2* tasks, int32_t count, int32_t t, int mode,
                    int nseg, int segk, const Batch& bt, int nb, T* L, T* U, const T* W, T* part,
                    hipStream_t s);
// Contribution-block update on lower 128 x 128 tiles, tasks (front, tile number).
template <typename T>
void launch_gemm_cb128(const FrontMeta& M, const Int2* tasks, int32_t count, const Batch& bt, int nb,
                       T* L, T* U, const T* W, hipStream_t s);
template <typename T>
void launch_gemm_reduce(const FrontMeta& M, const Int2* tasks, int32_t count, int32_t t, int nseg,
                        const Batch& bt, int nb, T* L, const T* part, hipStream_t s);
void launch_set_scalar(double* p, double v, hipStream_t s);
void launch_set_scalars(double* p, int n, const double* values, hipStream_t s);
// MFMA operand-layout probe (tests only): D = A(16x4) * B(4x16) via one instruction.
void launch_mfma_probe(const double* A, const double* B, double* D, hipStream_t s);
void launch_mfma_probe_f32(const float* A, const float* B, float* D, hipStream_t s);

}  // namespace kth
