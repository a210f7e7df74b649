// Algorithm drivers on top of the device engine: kept factors and solves,
// batched inertia, the three-stage k-th eigenpair algorithm (Alg. 4), batched
// pencils and the Hellmann-Feynman backward.
#pragma once
#include <vector>

#include "../../include/kth.h"
#include "engine.hpp"

namespace kth {

void numeric_factor(Pencil& P, NumFactor& F, double sigma, kth_precision prec);
void solve_many(Pencil& P, NumFactor& F, int32_t nrhs, const double* r, int64_t ldr, double* x,
                int64_t ldx, bool device_ptrs);
void inertia_batch(Pencil& P, int32_t nsigma, const double* sigmas, int64_t* nu);
kth_status three_stage(Pencil& P, int64_t k, const kth_opts& o, double* lambda, double* x,
                       kth_info* info);
void eig_batch(Ctx& c, const std::vector<Pencil*>& ps, const int64_t* k, const kth_opts& o,
               double* lambda, double* const* x, kth_info* info, kth_status* per);
void hf_backward(Pencil& P, double lambda, const double* x, double g, double* ga, double* gb);

}  // namespace kth
