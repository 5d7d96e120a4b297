// Restarted GMRES around the SPIKE solve (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "spike_launch.hpp"
#include "spike_plan.hpp"

namespace spike {

struct GmresResult {
  int iters, restarts, converged;
  double berr;
};

// Device bytes of the Krylov workspace for n x nrhs right-hand sides and a
// basis of `restart` vectors.
size_t gmres_workspace_bytes(int64_t n, int nrhs, int restart);

// Solve op(A) X = B in place (nrhs <= the plan's nrhs_max) by restarted
// GMRES(restart) preconditioned on the right by the factorisation in k,
// until the backward error is <= tol for every column or max_iters Arnoldi
// steps were taken.  Blocks the host (it reads every Hessenberg column).
// Returns 0, 1 when the factorisation failed (B untouched), or an error.
int gmres_solve(const KParams& k, const LaunchCfg& c, const Plan& pl, char* ws, hipStream_t st, double* B,
                int64_t ldb, int nrhs, bool trans, int restart, int max_iters, double tol, GmresResult* res);

}  // namespace spike
