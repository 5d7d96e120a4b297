// FP64 residual, backward error and iterative-refinement driver.
//
// The residual R = F - op(A) X reads the caller's FP64 band directly; a
// wavefront owns 64 consecutive output rows for both operations.
#include <hip/hip_runtime.h>

#include <climits>

#include "spike_device.hpp"
#include "spike_profile.hpp"
#include "spike_refine.hpp"

namespace spike {

namespace {

constexpr int RT = 256;

__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* p, double v) {
  atomicMax(p, dbits(v));
}

__device__ __forceinline__ double from_bits(unsigned long long b) { return __longlong_as_double((long long)b); }

// Band entries loaded ahead of their use, per thread and round.  A load
// whose entry lies outside the band reads a stored entry of the same band
// column instead and its value is replaced by zero, so the RU loads of a
// round have no branches between them and are in flight together.
constexpr int RU = 8;

// Stored position of row i in band column j, clamped into the band.
__device__ __forceinline__ int64_t band_pos(int64_t i, int64_t j, int64_t ldab, int kl, int ku) {
  int64_t d = i - j;
  d = d < -ku ? -ku : (d > kl ? kl : d);
  return (ku + d) + j * ldab;
}

__device__ __forceinline__ double max_over_wave(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// ||A||_inf (row abs-sums) and ||A||_1 (column abs-sums) of the FP64 band.
// Thread t of a workgroup sums row i0 + t over the band columns that touch
// the workgroup's rows (the same column for all threads at a time, so the
// loads are coalesced along it; a wavefront skips the columns that hold none
// of its rows' entries) and column i0 + t over its band entries (one
// contiguous run per thread).
__global__ __launch_bounds__(RT) void k_anorm(const double* ab, int64_t ldab, int64_t n, int kl, int ku,
                                               DevStatus* st) {
  const int64_t i0 = (int64_t)blockIdx.x * RT;
  const int64_t i = i0 + threadIdx.x;
  const bool live = i < n;
  double rs = 0.0, cs = 0.0;
  const int64_t w0 = i0 + (threadIdx.x & ~63);
  const int64_t jlo = w0 - kl > 0 ? w0 - kl : 0;
  const int64_t jhi = w0 + 64 + ku < n ? w0 + 64 + ku : n;   // exclusive
  for (int64_t j0 = jlo; j0 < jhi; j0 += RU) {
    double a[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int64_t j = j0 + u < jhi ? j0 + u : jhi - 1;
      const int64_t d = i - j;
      const bool in = live && j0 + u < jhi && d <= kl && -d <= ku;
      a[u] = gld(ab + band_pos(i, j, ldab, kl, ku));
      a[u] = in ? a[u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < RU; ++u) rs += fabs(a[u]);
  }
  // column sums of the wavefront's 64 columns w0 .. w0 + 63, lanes over the
  // stored rows s of a column (coalesced), CB columns' loads in flight
  // together; each lane sums its rows in ascending order, then the
  // wavefront's tree sum
  constexpr int CB = 16;
  const int wl = kl + ku + 1, lane = threadIdx.x & 63;
  for (int c0 = 0; c0 < 64; c0 += CB) {
    double part[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) part[cb] = 0.0;
    for (int s0 = 0; s0 < wl; s0 += 64) {
      const int sl = s0 + lane;
      double a[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const int64_t c = w0 + c0 + cb, r = c + sl - ku;
        const bool in = c < n && sl < wl && r >= 0 && r < n;
        const int64_t cc = c < n ? c : n - 1;
        a[cb] = gld(ab + (sl < wl ? sl : wl - 1) + cc * ldab);
        a[cb] = in ? a[cb] : 0.0;
      }
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) part[cb] += fabs(a[cb]);
    }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      double v = part[cb];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      cs = fmax(cs, v);
    }
  }
  rs = max_over_wave(rs);
  if ((threadIdx.x & 63) == 0) {
    atomic_max_nonneg(&st->anorm_inf_bits, rs);
    atomic_max_nonneg(&st->anorm_one_bits, cs);
  }
}

__global__ void k_refine_activate(DevStatus* st) {
  if (threadIdx.x == 0) st->refine_active = 1;
}

__global__ void k_refine_begin(DevStatus* st, unsigned long long* colred, int nrhs) {
  if (threadIdx.x == 0) {
    st->refine_iters = 0;
    st->berr = -1.0;
    // a failed factorisation (zero pivot, singular interface) leaves every
    // solve kernel idle; the refinement kernels idle with them, so B stays F
    const bool failed = st->zero_row != ULLONG_MAX || st->iface != ULLONG_MAX;
    st->skip = (st->refine_active && !failed) ? 0 : 1;
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


// Lane `src` (wave-uniform) of v, for every lane: the value lands in scalar
// registers, so the products that use it read no LDS.
__device__ __forceinline__ double lane_value(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

// R = F - op(A) X, plus per-column max |R| and max |X| (colred[2q],
// colred[2q+1]).  A wavefront owns 64 consecutive output rows i, a lane each;
// for every group of NQ right-hand sides it walks the j that couple to its
// rows in rounds of 64, lane l holding row jb + l of the NQ columns of X,
// which the products take lane by lane through scalar registers.  The entry
// is A(i, j) for op(A) = A (band column j: the lanes' loads are coalesced)
// and A(j, i) for A^T (band column i: each lane streams its own column,
// which its cache lines then serve for the following j).  RU entries per
// lane are loaded before their products (an entry outside the band reads
// the row's diagonal entry and enters as zero).  Each row's sum runs over j
// in ascending order.
template <int NQ, bool TRANS>
__global__ __launch_bounds__(RT) void k_residual(const double* ab, int64_t ldab, int64_t n, int kl, int ku,
                                                  const double* F, const double* X, int64_t ldx, double* R,
                                                  int64_t ld, int nrhs, unsigned long long* colred,
                                                  const int32_t* skip) {
  if (*skip) return;
  __shared__ double red[2][RT / 64][NQ];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t w0 = (int64_t)blockIdx.x * RT + 64 * wave;
  const int64_t i = w0 + lane;
  const bool live = i < n;
  const int64_t home = live ? ku + i * ldab : 0;   // stand-in address: the row's diagonal entry
  // j couples to row i when i - j lies in [-lo_r, hi_r]: [-ku, kl] for A,
  // [-kl, ku] for A^T; [jlo, jhi) covers the wavefront's rows
  const int hi_r = TRANS ? ku : kl, lo_r = TRANS ? kl : ku;
  const int64_t jlo = w0 - hi_r > 0 ? w0 - hi_r : 0;
  const int64_t jhi = w0 + 64 + lo_r < n ? w0 + 64 + lo_r : n;
  for (int q0 = 0; q0 < nrhs; q0 += NQ) {
    const int nq = nrhs - q0 < NQ ? nrhs - q0 : NQ;
    double acc[NQ];
#pragma unroll
    for (int t = 0; t < NQ; ++t) acc[t] = 0.0;
    for (int64_t jb = jlo; jb < jhi; jb += 64) {
      const int nj = jhi - jb < 64 ? (int)(jhi - jb) : 64;
      double xv[NQ];
#pragma unroll
      for (int t = 0; t < NQ; ++t) {
        const bool ok = lane < nj && t < nq;
        xv[t] = gld(X + (ok ? (jb + lane) + (int64_t)(q0 + t) * ldx : 0));
        xv[t] = ok ? xv[t] : 0.0;
      }
      for (int jj0 = 0; jj0 < nj; jj0 += RU) {
        double a[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
          const int64_t j = jb + jj0 + u;
          const int64_t d = i - j;
          const bool in = live && jj0 + u < nj && d <= hi_r && -d <= lo_r;
          a[u] = gld(ab + (in ? (TRANS ? (ku - d) + i * ldab : (ku + d) + j * ldab) : home));
          a[u] = in ? a[u] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
#pragma unroll
          for (int t = 0; t < NQ; ++t) acc[t] = fma(a[u], lane_value(xv[t], jj0 + u), acc[t]);
        }
      }
    }
    // R = F - A X and the per-column maxima, reduced over the workgroup
#pragma unroll
    for (int t0 = 0; t0 < NQ; t0 += 8) {
      constexpr int G = NQ < 8 ? NQ : 8;
      double f[G], x[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int t = t0 + g;
        const bool ok = live && t < nq;
        const int64_t q = q0 + (ok ? t : 0);
        f[g] = gld(F + (ok ? i + q * ld : 0));
        x[g] = gld(X + (ok ? i + q * ldx : 0));
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int t = t0 + g;
        double ra = 0.0, xa = 0.0;
        if (live && t < nq) {
          const double r = f[g] - acc[t];
          gst(R + i + (int64_t)(q0 + t) * ld, r);
          ra = fabs(r);
          xa = fabs(x[g]);
        }
        ra = max_over_wave(ra);
        xa = max_over_wave(xa);
        if (lane == 0) {
          red[0][wave][t] = ra;
          red[1][wave][t] = xa;
        }
      }
    }
    __syncthreads();
    if (tid < 2 * nq) {
      const int which = tid / nq, t = tid % nq;
      double m = red[which][0][t];
#pragma unroll
      for (int w = 1; w < RT / 64; ++w) m = fmax(m, red[which][w][t]);
      atomic_max_nonneg(&colred[2 * (q0 + t) + which], m);
    }
    __syncthreads();   // red is rewritten by the next group
  }
}

// Backward error and the stopping decision of iteration `it`: stop at the
// target, at the cap, on a non-finite residual, or when the backward error
// failed to halve since the previous iteration (the stopping rule of
// LAPACK's refinement routines: further corrections no longer pay, and on
// factors far from A, such as heavily boosted ones, they diverge).
__global__ void k_berr(DevStatus* st, unsigned long long* colred, int nrhs, int trans, double tol, int it,
                       int max_refine) {
  if (threadIdx.x != 0 || st->skip) return;
  const double prev = st->berr;   // previous iteration's, or -1
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
  const bool stalled = it > 0 && prev >= 0.0 && !(berr <= 0.5 * prev);
  if (!finite || berr <= tol || it >= max_refine || stalled) st->skip = 1;
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
  {
    ProfScope ps("k_anorm", st);
    hipLaunchKernelGGL(k_anorm, dim3((unsigned)blocks), dim3(RT), 0, st, k.dAB, k.ldab, pl.n, pl.kl, pl.ku,
                       k.status);
  }
  if (int e = chk()) return e;
  hipLaunchKernelGGL(k_refine_activate, dim3(1), dim3(64), 0, st, k.status);
  return chk();
}

int launch_anorm(const KParams& k, int64_t n, int kl, int ku, hipStream_t st) {
  const int64_t blocks = (n + RT - 1) / RT;
  ProfScope ps("k_anorm", st);
  hipLaunchKernelGGL(k_anorm, dim3((unsigned)blocks), dim3(RT), 0, st, k.dAB, k.ldab, n, kl, ku, k.status);
  return chk();
}

int launch_residual(const KParams& k, int64_t n, int kl, int ku, const double* F, const double* X, int64_t ldx,
                    double* R, int64_t ld, int nrhs, bool trans, unsigned long long* colred, const int32_t* skip,
                    hipStream_t st) {
  const unsigned rblocks = (unsigned)((n + RT - 1) / RT);
  ProfScope ps(trans ? "k_residual_t" : "k_residual_n", st);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(rblocks), dim3(RT), 0, st, k.dAB, k.ldab, n, kl, ku, F, X, ldx, R, ld, nrhs,
                       colred, skip);
  };
  if (nrhs == 1) trans ? go(k_residual<1, true>) : go(k_residual<1, false>);
  else if (nrhs <= 8) trans ? go(k_residual<8, true>) : go(k_residual<8, false>);
  else if (nrhs <= 16) trans ? go(k_residual<16, true>) : go(k_residual<16, false>);
  else trans ? go(k_residual<32, true>) : go(k_residual<32, false>);
  return chk();
}

int refined_solve(const KParams& k, const LaunchCfg& c, const Plan& pl, char* ws, hipStream_t st, double* B,
                  int64_t ldb, int nrhs, bool trans) {
  const int64_t n = pl.n;
  double* Fc = reinterpret_cast<double*>(ws + pl.off_xacc);
  double* Rr = reinterpret_cast<double*>(ws + pl.off_res);
  auto* colred = reinterpret_cast<unsigned long long*>(ws + pl.off_colred);
  const int32_t* skip = &k.status->skip;
  // the elementwise kernels stride over the grid; 4096 workgroups keep HBM
  // busy and keep the launches that find the loop finished short
  unsigned grid = (unsigned)((n * nrhs + RT - 1) / RT);
  if (grid > 4096u) grid = 4096u;
  hipLaunchKernelGGL(k_refine_begin, dim3(1), dim3(64), 0, st, k.status, colred, nrhs);
  if (int e = chk()) return e;
  {
    ProfScope ps("k_copy_cols", st);
    hipLaunchKernelGGL(k_copy_cols, dim3(grid), dim3(RT), 0, st, B, ldb, Fc, n, n, nrhs, skip);
  }
  if (int e = chk()) return e;
  if (int e = launch_solve(k, c, st, B, ldb, nrhs, trans)) return e;
  KParams kr = k;
  kr.skip = skip;
  const unsigned rblocks = (unsigned)((n + RT - 1) / RT);
  for (int it = 0; it <= pl.max_refine; ++it) {
    {
      ProfScope ps(trans ? "k_residual_t" : "k_residual_n", st);
      auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(rblocks), dim3(RT), 0, st, k.dAB, k.ldab, n, pl.kl, pl.ku, Fc, B, ldb, Rr,
                           n, nrhs, colred, skip);
      };
      if (nrhs == 1) trans ? go(k_residual<1, true>) : go(k_residual<1, false>);
      else if (nrhs <= 8) trans ? go(k_residual<8, true>) : go(k_residual<8, false>);
      else if (nrhs <= 16) trans ? go(k_residual<16, true>) : go(k_residual<16, false>);
      else trans ? go(k_residual<32, true>) : go(k_residual<32, false>);
    }
    if (int e = chk()) return e;
    hipLaunchKernelGGL(k_berr, dim3(1), dim3(64), 0, st, k.status, colred, nrhs, trans ? 1 : 0, pl.refine_tol, it,
                       pl.max_refine);
    if (int e = chk()) return e;
    if (it == pl.max_refine) break;
    if (int e = launch_solve(kr, c, st, Rr, n, nrhs, trans)) return e;
    {
      ProfScope ps("k_axpy_cols", st);
      hipLaunchKernelGGL(k_axpy_cols, dim3(grid), dim3(RT), 0, st, B, ldb, Rr, n, n, nrhs, skip);
    }
    if (int e = chk()) return e;
  }
  return 0;
}

}  // namespace spike
