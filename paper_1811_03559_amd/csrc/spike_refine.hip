// FP64 residual, backward error and iterative-refinement driver.
//
// The residual R = F - op(A) X reads the caller's FP64 band directly.  For
// op(A) = A a workgroup owns 256 consecutive rows and walks the band columns
// that touch them, so each band column segment is read once with coalesced
// accesses; for op(A) = A^T a wavefront owns an output row (a band column).
#include <hip/hip_runtime.h>

#include <climits>

#include "spike_device.hpp"
#include "spike_refine.hpp"

namespace spike {

namespace {

constexpr int RT = 256;

__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* p, double v) {
  atomicMax(p, dbits(v));
}

__device__ __forceinline__ double from_bits(unsigned long long b) { return __longlong_as_double((long long)b); }

// ||A||_inf (row abs-sums) and ||A||_1 (column abs-sums) of the FP64 band.
__global__ __launch_bounds__(RT) void k_anorm(const double* ab, int64_t ldab, int64_t n, int kl, int ku,
                                               DevStatus* st) {
  const int64_t i0 = (int64_t)blockIdx.x * RT;
  const int64_t i = i0 + threadIdx.x;
  double rs = 0.0;
  const int64_t jlo = i0 - kl > 0 ? i0 - kl : 0;
  const int64_t jhi = i0 + RT + ku < n ? i0 + RT + ku : n;   // exclusive
  for (int64_t j = jlo; j < jhi; ++j) {
    int64_t d = i - j;
    if (i < n && d <= kl && -d <= ku) rs += fabs(ab[(ku + d) + j * ldab]);
  }
  // column sums of columns [i0, i0 + RT): wave per column
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  double cmax = 0.0;
  for (int64_t c = i0 + wave; c < i0 + RT && c < n; c += RT / 64) {
    double cs = 0.0;
    for (int s = lane; s < kl + ku + 1; s += 64) {
      int64_t r = c + s - ku;
      if (r >= 0 && r < n) cs += fabs(ab[s + c * ldab]);
    }
    for (int off = 32; off > 0; off >>= 1) cs += __shfl_xor(cs, off);
    cmax = fmax(cmax, cs);
  }
  for (int off = 32; off > 0; off >>= 1) rs = fmax(rs, __shfl_xor(rs, off));
  if (lane == 0) {
    atomic_max_nonneg(&st->anorm_inf_bits, rs);
    atomic_max_nonneg(&st->anorm_one_bits, cmax);
  }
}

__global__ void k_refine_activate(DevStatus* st) {
  if (threadIdx.x == 0) st->refine_active = 1;
}

__global__ void k_refine_begin(DevStatus* st, unsigned long long* colred, int nrhs) {
  if (threadIdx.x == 0) {
    st->refine_iters = 0;
    st->berr = -1.0;
    st->skip = st->refine_active ? 0 : 1;
  }
  for (int q = threadIdx.x; q < 2 * nrhs; q += blockDim.x) colred[q] = 0ull;
}

__global__ __launch_bounds__(RT) void k_copy_cols(const double* S, int64_t lds, double* D, int64_t ldd,
                                                   int64_t n, int nrhs, const int32_t* skip) {
  if (*skip) return;
  for (int64_t idx = (int64_t)blockIdx.x * RT + threadIdx.x; idx < n * nrhs; idx += (int64_t)gridDim.x * RT) {
    int64_t r = idx % n, q = idx / n;
    D[r + q * ldd] = S[r + q * lds];
  }
}

// Right-hand sides handled per pass over the band (accumulators per thread)
// and band columns staged per LDS round.
constexpr int RQ = 16;
constexpr int RJ = 64;

// R = F - A X, plus per-column max |R| and max |X| (colred[2q], colred[2q+1]).
// A workgroup owns RT consecutive rows; for every group of RQ right-hand
// sides it walks the band columns touching those rows once (coalesced along
// each column), with the matching RJ x RQ slice of X staged in LDS.  Each
// row's sum runs over the columns in ascending order.
__global__ __launch_bounds__(RT) void k_residual_n(const double* ab, int64_t ldab, int64_t n, int kl, int ku,
                                                    const double* F, const double* X, int64_t ldx, double* R,
                                                    int64_t ld, int nrhs, unsigned long long* colred,
                                                    const int32_t* skip) {
  if (*skip) return;
  __shared__ double xs[RJ][RQ + 1];
  const int64_t i0 = (int64_t)blockIdx.x * RT;
  const int64_t i = i0 + threadIdx.x;
  const int64_t jlo = i0 - kl > 0 ? i0 - kl : 0;
  const int64_t jhi = i0 + RT + ku < n ? i0 + RT + ku : n;
  const int lane = threadIdx.x % 64;
  for (int q0 = 0; q0 < nrhs; q0 += RQ) {
    const int nq = nrhs - q0 < RQ ? nrhs - q0 : RQ;
    double acc[RQ];
#pragma unroll
    for (int t = 0; t < RQ; ++t) acc[t] = 0.0;
    for (int64_t jb = jlo; jb < jhi; jb += RJ) {
      const int nj = jhi - jb < RJ ? (int)(jhi - jb) : RJ;
      __syncthreads();
      for (int e = threadIdx.x; e < RJ * RQ; e += RT) {
        const int jj = e % RJ, t = e / RJ;
        xs[jj][t] = (jj < nj && t < nq) ? X[(jb + jj) + (int64_t)(q0 + t) * ldx] : 0.0;
      }
      __syncthreads();
      for (int jj = 0; jj < nj; ++jj) {
        const int64_t j = jb + jj;
        const int64_t d = i - j;
        if (i < n && d <= kl && -d <= ku) {
          const double a = ab[(ku + d) + j * ldab];
#pragma unroll
          for (int t = 0; t < RQ; ++t) acc[t] = fma(a, xs[jj][t], acc[t]);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < RQ; ++t) {
      if (t >= nq) break;
      const int q = q0 + t;
      double r = 0.0, xa = 0.0;
      if (i < n) {
        r = F[i + (int64_t)q * ld] - acc[t];
        R[i + (int64_t)q * ld] = r;
        xa = fabs(X[i + (int64_t)q * ldx]);
      }
      double ra = fabs(r);
      for (int off = 32; off > 0; off >>= 1) {
        ra = fmax(ra, __shfl_xor(ra, off));
        xa = fmax(xa, __shfl_xor(xa, off));
      }
      if (lane == 0) {
        atomic_max_nonneg(&colred[2 * q], ra);
        atomic_max_nonneg(&colred[2 * q + 1], xa);
      }
    }
  }
}

// R = F - A^T X: wavefront per output row i (band column i of A).  The
// column is read once per group of RQ right-hand sides; lanes keep partial
// sums that are reduced across the wavefront at the end.
__global__ __launch_bounds__(RT) void k_residual_t(const double* ab, int64_t ldab, int64_t n, int kl, int ku,
                                                    const double* F, const double* X, int64_t ldx, double* R,
                                                    int64_t ld, int nrhs, unsigned long long* colred,
                                                    const int32_t* skip) {
  if (*skip) return;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t i = (int64_t)blockIdx.x * (RT / 64) + wave;
  if (i >= n) return;
  const int w = kl + ku + 1;
  for (int q0 = 0; q0 < nrhs; q0 += RQ) {
    const int nq = nrhs - q0 < RQ ? nrhs - q0 : RQ;
    double acc[RQ];
#pragma unroll
    for (int t = 0; t < RQ; ++t) acc[t] = 0.0;
    for (int s = lane; s < w; s += 64) {
      const int64_t j = i + s - ku;   // A(j, i) at ab[s + i*ldab]
      if (j < 0 || j >= n) continue;
      const double a = ab[s + i * ldab];
#pragma unroll
      for (int t = 0; t < RQ; ++t)
        if (t < nq) acc[t] = fma(a, X[j + (int64_t)(q0 + t) * ldx], acc[t]);
    }
#pragma unroll
    for (int t = 0; t < RQ; ++t) {
      if (t >= nq) break;
      double v = acc[t];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0) {
        const int q = q0 + t;
        double r = F[i + (int64_t)q * ld] - v;
        R[i + (int64_t)q * ld] = r;
        atomic_max_nonneg(&colred[2 * q], fabs(r));
        atomic_max_nonneg(&colred[2 * q + 1], fabs(X[i + (int64_t)q * ldx]));
      }
    }
  }
}

// Backward error and the stopping decision of iteration `it`.
__global__ void k_berr(DevStatus* st, unsigned long long* colred, int nrhs, int trans, double tol, int it,
                       int max_refine) {
  if (threadIdx.x != 0 || st->skip) return;
  const double an = from_bits(trans ? st->anorm_one_bits : st->anorm_inf_bits);
  double berr = 0.0;
  bool finite = true;
  for (int q = 0; q < nrhs; ++q) {
    double rm = from_bits(colred[2 * q]), xm = from_bits(colred[2 * q + 1]);
    double b = (an * xm) > 0.0 ? rm / (an * xm) : (rm > 0.0 ? __builtin_huge_val() : 0.0);
    if (!__builtin_isfinite(rm) || !__builtin_isfinite(xm)) finite = false;
    berr = fmax(berr, b);
    colred[2 * q] = 0ull;
    colred[2 * q + 1] = 0ull;
  }
  // a non-finite residual or solution is reported as NaN and ends the loop
  if (!finite) berr = __builtin_nan("");
  st->berr = berr;
  if (!finite || berr <= tol || it >= max_refine) st->skip = 1;
  else st->refine_iters = it + 1;
}

__global__ __launch_bounds__(RT) void k_axpy_cols(double* B, int64_t ldb, const double* R, int64_t ldr, int64_t n,
                                                   int nrhs, const int32_t* skip) {
  if (*skip) return;
  for (int64_t idx = (int64_t)blockIdx.x * RT + threadIdx.x; idx < n * nrhs; idx += (int64_t)gridDim.x * RT) {
    int64_t r = idx % n, q = idx / n;
    B[r + q * ldb] += R[r + q * ldr];
  }
}

int chk() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : SPIKE_ERR_HIP - (int)e;
}

}  // namespace

int prepare_refine(const KParams& k, const Plan& pl, char*, hipStream_t st) {
  int64_t blocks = (pl.n + RT - 1) / RT;
  hipLaunchKernelGGL(k_anorm, dim3((unsigned)blocks), dim3(RT), 0, st, k.dAB, k.ldab, pl.n, pl.kl, pl.ku, k.status);
  if (int e = chk()) return e;
  hipLaunchKernelGGL(k_refine_activate, dim3(1), dim3(64), 0, st, k.status);
  return chk();
}

int refined_solve(const KParams& k, const LaunchCfg& c, const Plan& pl, char* ws, hipStream_t st, double* B,
                  int64_t ldb, int nrhs, bool trans) {
  const int64_t n = pl.n;
  double* Fc = reinterpret_cast<double*>(ws + pl.off_xacc);
  double* Rr = reinterpret_cast<double*>(ws + pl.off_res);
  auto* colred = reinterpret_cast<unsigned long long*>(ws + pl.off_colred);
  const int32_t* skip = &k.status->skip;
  unsigned grid = (unsigned)((n * nrhs + RT - 1) / RT);
  if (grid > 65535u * 4u) grid = 65535u * 4u;
  hipLaunchKernelGGL(k_refine_begin, dim3(1), dim3(64), 0, st, k.status, colred, nrhs);
  if (int e = chk()) return e;
  hipLaunchKernelGGL(k_copy_cols, dim3(grid), dim3(RT), 0, st, B, ldb, Fc, n, n, nrhs, skip);
  if (int e = chk()) return e;
  if (int e = launch_solve(k, c, st, B, ldb, nrhs, trans)) return e;
  KParams kr = k;
  kr.skip = skip;
  const unsigned rblocks_n = (unsigned)((n + RT - 1) / RT);
  const unsigned rblocks_t = (unsigned)((n + RT / 64 - 1) / (RT / 64));
  for (int it = 0; it <= pl.max_refine; ++it) {
    if (!trans)
      hipLaunchKernelGGL(k_residual_n, dim3(rblocks_n), dim3(RT), 0, st, k.dAB, k.ldab, n, pl.kl, pl.ku, Fc, B,
                         ldb, Rr, n, nrhs, colred, skip);
    else
      hipLaunchKernelGGL(k_residual_t, dim3(rblocks_t), dim3(RT), 0, st, k.dAB, k.ldab, n, pl.kl, pl.ku, Fc, B,
                         ldb, Rr, n, nrhs, colred, skip);
    if (int e = chk()) return e;
    hipLaunchKernelGGL(k_berr, dim3(1), dim3(64), 0, st, k.status, colred, nrhs, trans ? 1 : 0, pl.refine_tol, it,
                       pl.max_refine);
    if (int e = chk()) return e;
    if (it == pl.max_refine) break;
    if (int e = launch_solve(kr, c, st, Rr, n, nrhs, trans)) return e;
    hipLaunchKernelGGL(k_axpy_cols, dim3(grid), dim3(RT), 0, st, B, ldb, Rr, n, n, nrhs, skip);
    if (int e = chk()) return e;
  }
  return 0;
}

}  // namespace spike
