// Host-side plan of the level-scheduled triangular solves.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "device.hpp"

namespace kth {

struct SolveStep {
  int32_t t;
  int32_t nfronts;               // active large fronts (prefix of the level's list)
  int32_t task_off, task_cnt;    // Int2 (front, first row) tasks of kSolveRows rows below the
                                 // tile, in row order per front; (front, nf) if none
};

struct SolveLevel {
  int32_t small_off = 0, small_cnt = 0;   // fronts solved by one workgroup each
  int32_t large_off = 0, large_cnt = 0;   // large fronts (sorted by ns, descending)
  int32_t init_off = 0, init_cnt = 0;     // Int2 (front, row) tasks of the gather step
  std::vector<SolveStep> steps;
};

struct SolvePlan {
  const int32_t* sched = nullptr;    // device int32 schedule array
  std::vector<SolveLevel> levels;
  int64_t partial_size = 1;          // doubles for the backward partial sums: 2 * half * kNB
  int64_t partial_half = 0;          // slots per step parity (max over levels)
  const int64_t* pbase = nullptr;    // device [nsup]: a large front's first slot in its level
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
