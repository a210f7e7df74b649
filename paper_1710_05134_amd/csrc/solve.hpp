// Host-side plan of the level-scheduled triangular solves.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "device.hpp"

namespace kth {

struct SolveStep {               // tiles t and t + 1 (t even) of the level's large fronts
  int32_t t;
  int32_t nfronts;               // active large fronts (prefix of the level's list)
  int32_t fwd_off, fwd_cnt;      // Int2 (front, first row) tasks of 64 pivot-block rows below
                                 // the two tiles, in row order per front; (front, ns) if none
  int32_t bwd_off, bwd_cnt;      // Int2 (front, first column) tasks of 64 columns before
                                 // tile t, first chunk first; (front, 0) for tile 0
};

struct SolveLevel {
  int32_t small_off = 0, small_cnt = 0;   // fronts solved by one workgroup each
  int32_t large_off = 0, large_cnt = 0;   // large fronts (sorted by ns, descending)
  int32_t init_off = 0, init_cnt = 0;     // Int2 (front, row) tasks of the gather step
  std::vector<SolveStep> steps;
  // rows below each large front's pivot block (L21): Int2 (front, first row) tasks of
  // kL21Rows rows, in row order per front; the forward pass splits the columns into
  // l21_nseg segments of kL21Cols, the backward pass into l21_ntile tiles of kNB
  int32_t l21_off = 0, l21_cnt = 0;
  int32_t l21_nseg = 0, l21_ntile = 0;
};

struct SolvePlan {
  const int32_t* sched = nullptr;    // device int32 schedule array
  std::vector<SolveLevel> levels;
  int64_t partial_size = 1;          // doubles for the L21 partial sums (max over levels)
  const int32_t* l21base = nullptr;  // device [nsup]: a large front's first L21 task in its level
  int64_t l21_part_off = 0;          // doubles: the L21 partial sums' place within partial
};

// Size of the fixed per-GPU work array of the allocation-free solve.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
// Takes the address of that array on `device` (which must be current) once per
// device; returns the HIP error of hipGetSymbolAddress (hipSuccess when known).
hipError_t noalloc_scratch_init(int device);
// The array's device address on `device` (nullptr before noalloc_scratch_init).
double* noalloc_scratch(int device);

// x = (A - sigma B)^{-1} b with a kept factor (T = double or float panels).
// xe, ye: n-vectors of scratch; R: work vectors (rows.size() doubles);
// partial: P.partial_size doubles.
template <typename T>
void solve_enqueue(const SolvePlan& P, const FrontMeta& M, const T* L, const double* D,
                   const double* E, const int32_t* tperm, const int64_t* perm, int64_t n,
                   const double* b, double* x, double* xe, double* ye, double* R, double* partial,
                   hipStream_t s);

}  // namespace kth
