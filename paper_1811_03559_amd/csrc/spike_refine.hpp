// Iterative refinement in FP64 around the SPIKE solve (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "spike_launch.hpp"
#include "spike_plan.hpp"

namespace spike {

// After the factorisation: ||A||_inf and ||A||_1 of the caller's FP64 band,
// and whether refinement is needed (FP32 factors, or boosted pivots).
int prepare_refine(const KParams& k, const Plan& pl, char* ws, hipStream_t st);

// Solve op(A) X = F in place on B (nrhs <= nrhs_max) with refinement:
// X0 = SPIKE solve; then up to max_refine times r = F - op(A) X (FP64, from
// the caller's band), stop once max_c ||r_c|| / (||op(A)|| ||X_c||) <= tol,
// else X += SPIKE solve(r).  The stopping decision is taken on the device;
// later iterations' kernels idle, so no host synchronisation is needed.
int refined_solve(const KParams& k, const LaunchCfg& c, const Plan& pl, char* ws, hipStream_t st,
                  double* B, int64_t ldb, int nrhs, bool trans);

// ||A||_inf and ||A||_1 of the caller's FP64 band into the status block
// (atomic maxima: the fields must hold 0 or smaller values before).
int launch_anorm(const KParams& k, int64_t n, int kl, int ku, hipStream_t st);

// R = F - op(A) X from the caller's FP64 band (F and R share leading
// dimension ld), with per-column max |R| and max |X| into colred[2q],
// colred[2q+1] (atomic maxima over zeroed slots); idles while *skip != 0.
int launch_residual(const KParams& k, int64_t n, int kl, int ku, const double* F, const double* X, int64_t ldx,
                    double* R, int64_t ld, int nrhs, bool trans, unsigned long long* colred, const int32_t* skip,
                    hipStream_t st);

}  // namespace spike
