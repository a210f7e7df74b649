// Host-side plan of the level-scheduled triangular solves.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "device.hpp"

namespace kth {

struct SolvePlan {
  const int32_t* fronts = nullptr;   // device: all fronts grouped by level
  std::vector<int32_t> level_off;    // offset of each level's group
  std::vector<int32_t> level_cnt;
};

// x = (A - sigma B)^{-1} b with a kept factor (T = double or float panels).
// xe, ye: n-vectors of scratch; R: work vectors (rows.size() doubles).
template <typename T>
void solve_enqueue(const SolvePlan& P, const FrontMeta& M, const T* L, const double* D,
                   const double* E, const int32_t* tperm, const int64_t* perm, int64_t n,
                   const double* b, double* x, double* xe, double* ye, double* R, hipStream_t s);

}  // namespace kth
