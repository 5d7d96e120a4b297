// Complex banded systems on the real SPIKE path.
//
// A complex n x n band A (kl, ku) with entries a = ar + i ai acts on
// z = x + i y like the real 2n x 2n matrix whose 2 x 2 block (j, c) is
// [[ar, -ai], [ai, ar]] when the unknowns are interleaved (x_0, y_0, x_1,
// y_1, ...), which is exactly the memory order of an interleaved complex
// vector.  That real matrix is banded with 2 kl + 1 subdiagonals and
// 2 ku + 1 superdiagonals, so the complex factorisation is the real one of
// the embedding, whose dense contractions run on the FP64 (or FP32) matrix
// cores.  Its transpose is the embedding of the conjugate transpose A^H;
// A^T z = f is A^H conj(z) = conj(f).
//
// Row j is first multiplied by d_j = conj(a_jj) / |a_jj| (a unitary
// diagonal D), so the embedded system is D A: its diagonal entries are real
// and positive, and so, for a diagonally dominant A, are the leading
// entries of the 2 x 2 diagonal blocks met during the non-pivoting
// elimination (without the rotation a diagonal entry close to the imaginary
// axis makes a tiny real pivot).  Solves then use D A z = D f,
// (D A)^H = A^H D^H, so A^H z = f is (D A)^H w = f with z = conj(D) w, and
// A^T z = f is (D A)^T w = f with z = D w.
#include <hip/hip_runtime.h>

#include "spike_device.hpp"
#include "spike_profile.hpp"

namespace spike {

namespace {

constexpr int ZT = 256;

// The factorisation failed: the solves leave the right-hand sides untouched.
__device__ __forceinline__ bool failed(const DevStatus* s) {
  return s->zero_row != ~0ull || s->iface != ~0ull;
}

// Real band R (ldr = 2 kl + 2 ku + 3 rows, 2n columns) of D A for the
// complex band zab (interleaved re/im doubles, element (i, j) at
// 2 ((ku + i - j) + j ldab)), with d_j = conj(a_jj) / |a_jj| (1 when
// a_jj = 0) written to Dv (interleaved complex).
__global__ __launch_bounds__(ZT) void k_zembed(const double* zab, int64_t ldab, int64_t n, int kl, int ku,
                                               double* R, int64_t ldr, double* Dv) {
  for (int64_t j = (int64_t)blockIdx.x * ZT + threadIdx.x; j < n; j += (int64_t)gridDim.x * ZT) {
    const double* a = zab + 2 * (ku + j * ldab);
    const double re = gld(a), im = gld(a + 1);
    const double m = hypot(re, im);
    Dv[2 * j] = m > 0.0 ? re / m : 1.0;
    Dv[2 * j + 1] = m > 0.0 ? -im / m : 0.0;
  }
  const int klr = 2 * kl + 1, kur = 2 * ku + 1;
  const int64_t total = 2 * n * ldr;
  for (int64_t idx = (int64_t)blockIdx.x * ZT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * ZT) {
    const int64_t cr = idx / ldr;                  // real column
    const int sr = (int)(idx % ldr);               // band row: real row = cr + sr - kur
    const int64_t rr = cr + sr - kur;
    double v = 0.0;
    if (rr >= 0 && rr < 2 * n && sr <= kur + klr) {
      const int64_t j = rr >> 1, c = cr >> 1;      // complex row and column
      const int s = (int)(rr & 1), t = (int)(cr & 1);
      if (j - c <= kl && c - j <= ku) {
        const double* a = zab + 2 * ((ku + j - c) + c * ldab);
        const double* ad = zab + 2 * (ku + j * ldab);
        const double are = gld(a), aim = gld(a + 1), dre0 = gld(ad), dim0 = gld(ad + 1);
        const double m = hypot(dre0, dim0);
        const double dre = m > 0.0 ? dre0 / m : 1.0, dim = m > 0.0 ? -dim0 / m : 0.0;
        const double re = dre * are - dim * aim, im = dre * aim + dim * are;   // d_j a
        v = (s == t) ? re : (s == 0 ? -im : im);
      }
    }
    R[sr + cr * ldr] = v;
  }
}

// B(r, :) *= d_r (conj_d: conj(d_r)) for an interleaved complex n x nrhs block
// (idle after a failed factorisation).
__global__ __launch_bounds__(ZT) void k_zrowscale(double* B, int64_t ldb2, int64_t n, int nrhs, const double* Dv,
                                                  int conj_d, const DevStatus* status) {
  if (failed(status)) return;
  for (int64_t idx = (int64_t)blockIdx.x * ZT + threadIdx.x; idx < n * nrhs; idx += (int64_t)gridDim.x * ZT) {
    const int64_t r = idx % n;
    const int q = (int)(idx / n);
    double* p = B + 2 * r + q * ldb2;
    const double dre = Dv[2 * r], dim = conj_d ? -Dv[2 * r + 1] : Dv[2 * r + 1];
    const double bre = p[0], bim = p[1];
    p[0] = dre * bre - dim * bim;
    p[1] = dre * bim + dim * bre;
  }
}

// Negate the imaginary parts of an interleaved complex n x nrhs block (idle
// after a failed factorisation).
__global__ __launch_bounds__(ZT) void k_zconj(double* B, int64_t ldb2, int64_t n, int nrhs, const DevStatus* status) {
  if (failed(status)) return;
  for (int64_t idx = (int64_t)blockIdx.x * ZT + threadIdx.x; idx < n * nrhs; idx += (int64_t)gridDim.x * ZT) {
    const int64_t r = idx % n;
    const int q = (int)(idx / n);
    double* p = B + 2 * r + 1 + q * ldb2;
    *p = -*p;
  }
}

unsigned grid_of(int64_t total) {
  const int64_t g = (total + ZT - 1) / ZT;
  return (unsigned)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

int chk() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : -1000 - (int)e;
}

}  // namespace

int launch_zembed(const double* zab, int64_t ldab, int64_t n, int kl, int ku, double* R, int64_t ldr, double* Dv,
                  hipStream_t st) {
  if (n == 0) return 0;
  ProfScope ps("k_zembed", st);
  hipLaunchKernelGGL(k_zembed, dim3(grid_of(2 * n * ldr)), dim3(ZT), 0, st, zab, ldab, n, kl, ku, R, ldr, Dv);
  return chk();
}

int launch_zrowscale(double* B, int64_t ldb2, int64_t n, int nrhs, const double* Dv, bool conj_d,
                     const DevStatus* status, hipStream_t st) {
  if (n == 0 || nrhs == 0) return 0;
  hipLaunchKernelGGL(k_zrowscale, dim3(grid_of(n * nrhs)), dim3(ZT), 0, st, B, ldb2, n, nrhs, Dv, conj_d ? 1 : 0,
                     status);
  return chk();
}

int launch_zconj(double* B, int64_t ldb2, int64_t n, int nrhs, const DevStatus* status, hipStream_t st) {
  if (n == 0 || nrhs == 0) return 0;
  hipLaunchKernelGGL(k_zconj, dim3(grid_of(n * nrhs)), dim3(ZT), 0, st, B, ldb2, n, nrhs, status);
  return chk();
}

}  // namespace spike
