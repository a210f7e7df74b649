// Algorithm drivers on top of the device engine: kept factors and solves,
// batched inertia, the three-stage k-th eigenpair algorithm (Alg. 4), batched
// pencils and the Hellmann-Feynman backward.
#pragma once
#include <vector>

#include "../../include/kth.h"
#include "engine.hpp"

namespace kth {

void numeric_factor(Pencil& P, NumFactor& F, double sigma, kth_precision prec);

// Outcome of one solve with a kept factor.  FP64 factors: one pass, steps = 0.
// FP32 factors (GMRES-based iterative refinement): x0 = M32^{-1} b; then, while the
// normwise backward error ||b - M x||_inf / (||M||_inf ||x||_inf + ||b||_inf)
// (M = A - sigma B, residual in FP64) exceeds kIrTol, a correction d solves
// M d = r by GMRES on M32^{-1} M (FP64 vectors, the FP32 factor as left
// preconditioner, at most kGmresMax steps, stopped at a kGmresTol reduction of the
// preconditioned residual) and x += d.  It gives up after kIrMaxOuter corrections
// or when the residual fails to halve on two consecutive corrections.
constexpr double kIrTol = 4.0 * 2.220446049250313e-16;
constexpr int kIrMaxOuter = 4;
constexpr int kGmresMax = 20;
constexpr double kGmresTol = 1e-12;
struct SolveOutcome {
  int steps = 0;          // applications of the FP32 factor after the first
  bool converged = true;
  double berr = 0;        // backward error at exit (FP32 factors)
};
SolveOutcome solve_refined(Pencil& P, NumFactor& F, const double* b, double* x,
                           double tol = kIrTol);
// nrhs solves (column-major); unrefined: FP32 factors skip the refinement.
void solve_many(Pencil& P, NumFactor& F, int32_t nrhs, const double* r, int64_t ldr, double* x,
                int64_t ldx, bool device_ptrs, bool unrefined = false);
void inertia_batch(Pencil& P, int32_t nsigma, const double* sigmas, int64_t* nu);
kth_status three_stage(Pencil& P, int64_t k, const kth_opts& o, double* lambda, double* x,
                       kth_info* info);
void eig_batch(Ctx& c, const std::vector<Pencil*>& ps, const int64_t* k, const kth_opts& o,
               double* lambda, double* const* x, kth_info* info, kth_status* per);
void hf_backward(Pencil& P, double lambda, const double* x, double g, double* ga, double* gb);

}  // namespace kth
