// Restarted GMRES in FP64 with a SPIKE factorisation as the right
// preconditioner (a project addition around the paper's remark that
// boosted, non-pivoting factors need an outer correction, section "An
// efficient pivoting scheme"): op(A) M^{-1} u = F, X = M^{-1} u, where
// M^{-1} is the handle's solve (boosted or pivoting factors, FP64 or FP32)
// and op(A) the caller's FP64 band.
//
// All vectors stay on the device; the right-hand sides are independent
// GMRES runs that share every launch (the preconditioner solve takes all
// columns at once).  Per Arnoldi step the host reads the Hessenberg column
// (classical Gram-Schmidt with one reorthogonalisation pass) and applies
// the Givens rotations; the restart test is the backward error
// ||F - op(A) X||_inf / (||op(A)||_inf ||X||_inf) of the true residual.
// Dot products are two-stage sums in a fixed order, so results repeat
// bitwise.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "spike_device.hpp"
#include "spike_krylov.hpp"
#include "spike_profile.hpp"
#include "spike_refine.hpp"

namespace spike {

namespace {

constexpr int KT = 256;
constexpr int64_t kChunk = 16384;   // rows per block of a dot product

int chk() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : SPIKE_ERR_HIP - (int)e;
}

unsigned grid_for(int64_t total) {
  int64_t g = (total + KT - 1) / KT;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 4096));
}

// partial[pair * nchunk + chunk] = sign * sum over the chunk's rows of
// V_i(r, q) W(r, q), pair = i * nrhs + q; vectors are n x nrhs blocks with
// leading dimension ld, basis vector i at V + i * vstride.
__global__ __launch_bounds__(KT) void k_dots(const double* V, int64_t vstride, const double* W, int64_t ld,
                                              int64_t n, int nrhs, double sign, double* partial, int nchunk) {
  __shared__ double red[KT];
  const int pair = blockIdx.y, chunk = blockIdx.x;
  const int i = pair / nrhs, q = pair % nrhs;
  const double* v = V + (int64_t)i * vstride + (int64_t)q * ld;
  const double* w = W + (int64_t)q * ld;
  const int64_t r0 = (int64_t)chunk * kChunk, r1 = std::min<int64_t>(n, r0 + kChunk);
  double s = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += KT) s = fma(gld(v + r), gld(w + r), s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = KT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)pair * nchunk + chunk] = sign * red[0];
}

// out[pair] = sum over chunks of partial[pair * nchunk + chunk], in order.
__global__ void k_sum_partials(const double* partial, int nchunk, int npairs, double* out) {
  const int pair = blockIdx.x * blockDim.x + threadIdx.x;
  if (pair >= npairs) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += partial[(int64_t)pair * nchunk + c];
  out[pair] = s;
}

// W(:, q) = sign W(:, q) - sum_{i < nvec} V_i(:, q) h[i nrhs + q]
__global__ __launch_bounds__(KT) void k_vupdate(double* W, const double* V, int64_t vstride, int64_t ld, int64_t n,
                                                 int nrhs, int nvec, double sign, const double* h) {
  for (int64_t idx = (int64_t)blockIdx.x * KT + threadIdx.x; idx < n * nrhs; idx += (int64_t)gridDim.x * KT) {
    const int64_t r = idx % n;
    const int q = (int)(idx / n);
    double acc = sign * W[r + (int64_t)q * ld];
    for (int i = 0; i < nvec; ++i) acc = fma(-gld(V + (int64_t)i * vstride + (int64_t)q * ld + r), h[i * nrhs + q], acc);
    W[r + (int64_t)q * ld] = acc;
  }
}

// s[q] = 1 / sqrt(nrm2[q]) (0 for a zero vector)
__global__ void k_inv_norm(const double* nrm2, double* s, int nrhs) {
  const int q = threadIdx.x;
  if (q < nrhs) s[q] = nrm2[q] > 0.0 ? 1.0 / sqrt(nrm2[q]) : 0.0;
}

// D(:, q) = S(:, q) * s[q]
__global__ __launch_bounds__(KT) void k_scale_into(double* D, const double* S, int64_t ld, int64_t n, int nrhs,
                                                    const double* s) {
  for (int64_t idx = (int64_t)blockIdx.x * KT + threadIdx.x; idx < n * nrhs; idx += (int64_t)gridDim.x * KT) {
    const int64_t r = idx % n;
    const int q = (int)(idx / n);
    D[r + (int64_t)q * ld] = S[r + (int64_t)q * ld] * s[q];
  }
}

// U(:, q) = sum_{i < nvec} V_i(:, q) y[i nrhs + q]
__global__ __launch_bounds__(KT) void k_lincomb(double* U, const double* V, int64_t vstride, int64_t ld, int64_t n,
                                                 int nrhs, int nvec, const double* y) {
  for (int64_t idx = (int64_t)blockIdx.x * KT + threadIdx.x; idx < n * nrhs; idx += (int64_t)gridDim.x * KT) {
    const int64_t r = idx % n;
    const int q = (int)(idx / n);
    double acc = 0.0;
    for (int i = 0; i < nvec; ++i) acc = fma(gld(V + (int64_t)i * vstride + (int64_t)q * ld + r), y[i * nrhs + q], acc);
    U[r + (int64_t)q * ld] = acc;
  }
}

// D = S (n x nrhs blocks of leading dimensions ldd, lds); with add: D += S
__global__ __launch_bounds__(KT) void k_copy_add(double* D, int64_t ldd, const double* S, int64_t lds, int64_t n,
                                                  int nrhs, int add) {
  for (int64_t idx = (int64_t)blockIdx.x * KT + threadIdx.x; idx < n * nrhs; idx += (int64_t)gridDim.x * KT) {
    const int64_t r = idx % n;
    const int q = (int)(idx / n);
    const double v = S[r + (int64_t)q * lds];
    D[r + (int64_t)q * ldd] = add ? D[r + (int64_t)q * ldd] + v : v;
  }
}

__global__ __launch_bounds__(KT) void k_fill(double* D, int64_t count, double v) {
  for (int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x; i < count; i += (int64_t)gridDim.x * KT) D[i] = v;
}

__global__ void k_zero_u64(unsigned long long* c, int count, int32_t* flag) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) c[i] = 0ull;
  if (threadIdx.x == 0) *flag = 0;
}

struct Layout {
  int64_t blk;        // doubles of one n x nrhs block
  int nchunk;
  size_t off_V, off_Z, off_W, off_X, off_F, off_R, off_zero, off_partial, off_h, off_s, off_colred, off_flag, total;
};

Layout layout(int64_t n, int nrhs, int m) {
  Layout L;
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  L.blk = n * nrhs;
  L.nchunk = (int)std::max<int64_t>(1, (n + kChunk - 1) / kChunk);
  const size_t b = (size_t)L.blk * 8;
  size_t off = 0;
  L.off_V = off; off = al(off + b * (m + 1));
  L.off_Z = off; off = al(off + b);
  L.off_W = off; off = al(off + b);
  L.off_X = off; off = al(off + b);
  L.off_F = off; off = al(off + b);
  L.off_R = off; off = al(off + b);
  L.off_zero = off; off = al(off + b);
  L.off_partial = off; off = al(off + 8 * (size_t)(m + 1) * nrhs * L.nchunk);
  L.off_h = off; off = al(off + 8 * 3 * (size_t)(m + 1) * nrhs + 8 * (size_t)nrhs * (m + 1));
  L.off_s = off; off = al(off + 8 * (size_t)nrhs);
  L.off_colred = off; off = al(off + 8 * 2 * (size_t)nrhs);
  L.off_flag = off; off = al(off + 8);
  L.total = off;
  return L;
}

}  // namespace

size_t gmres_workspace_bytes(int64_t n, int nrhs, int restart) { return layout(n, nrhs, restart).total; }

int gmres_solve(const KParams& k, const LaunchCfg& c, const Plan& pl, char* ws, hipStream_t st, double* B,
                int64_t ldb, int nrhs, bool trans, int m, int max_iters, double tol, GmresResult* res) {
  const int64_t n = pl.n;
  const Layout L = layout(n, nrhs, m);
  auto D = [&](size_t off) { return reinterpret_cast<double*>(ws + off); };
  double* V = D(L.off_V);
  double* Z = D(L.off_Z);
  double* W = D(L.off_W);
  double* X = D(L.off_X);
  double* F = D(L.off_F);
  double* R = D(L.off_R);
  double* Zero = D(L.off_zero);
  double* partial = D(L.off_partial);
  double* h1 = D(L.off_h);
  double* h2 = h1 + (m + 1) * nrhs;
  double* hn = h2 + (m + 1) * nrhs;
  double* ydev = hn + (m + 1) * nrhs;
  double* sdev = D(L.off_s);
  auto* colred = reinterpret_cast<unsigned long long*>(ws + L.off_colred);
  auto* flag = reinterpret_cast<int32_t*>(ws + L.off_flag);
  const int64_t ld = n;
  const int64_t vstride = L.blk;
  const unsigned grid = grid_for(L.blk);
  int e = 0;
  // the status (zero pivots, interface failures) and the norms of op(A)
  DevStatus hs;
  if ((e = (hipMemcpyAsync(&hs, k.status, sizeof(hs), hipMemcpyDeviceToHost, st) == hipSuccess ? 0 : chk()))) return e;
  if (hipStreamSynchronize(st) != hipSuccess) return chk();
  if (hs.zero_row != ~0ull || hs.iface != ~0ull) return 1;   // failed factorisation: dB untouched
  if (hs.anorm_inf_bits == 0ull && hs.anorm_one_bits == 0ull) {
    if ((e = launch_anorm(k, n, pl.kl, pl.ku, st))) return e;
    if (hipMemcpyAsync(&hs, k.status, sizeof(hs), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return chk();
  }
  double anorm;
  {
    const unsigned long long bits = trans ? hs.anorm_one_bits : hs.anorm_inf_bits;
    std::memcpy(&anorm, &bits, sizeof(anorm));
  }

  auto precond = [&](double* Y) { return launch_solve(k, c, st, Y, ld, nrhs, trans); };
  auto dots = [&](const double* Vb, int nvec, const double* Wv, double sign, double* out) -> int {
    if (nvec <= 0) return 0;
    hipLaunchKernelGGL(k_dots, dim3(L.nchunk, nvec * nrhs), dim3(KT), 0, st, Vb, vstride, Wv, ld, n, nrhs, sign,
                       partial, L.nchunk);
    if (int e2 = chk()) return e2;
    const int np = nvec * nrhs;
    hipLaunchKernelGGL(k_sum_partials, dim3((np + 63) / 64), dim3(64), 0, st, partial, L.nchunk, np, out);
    return chk();
  };
  auto residual = [&](std::vector<double>& berr, std::vector<double>& xinf) -> int {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, colred, 2 * nrhs, flag);
    if (int e2 = chk()) return e2;
    if (int e2 = launch_residual(k, n, pl.kl, pl.ku, F, X, ld, R, ld, nrhs, trans, colred, flag, st)) return e2;
    std::vector<unsigned long long> cr(2 * nrhs);
    if (hipMemcpyAsync(cr.data(), colred, 8 * 2 * nrhs, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return chk();
    for (int q = 0; q < nrhs; ++q) {
      double rm, xm;
      std::memcpy(&rm, &cr[2 * q], 8);
      std::memcpy(&xm, &cr[2 * q + 1], 8);
      xinf[q] = xm;
      berr[q] = (anorm * xm) > 0.0 ? rm / (anorm * xm) : (rm > 0.0 ? INFINITY : 0.0);
      if (!std::isfinite(rm) || !std::isfinite(xm)) berr[q] = NAN;
    }
    return 0;
  };

  // F = B, X = M^{-1} F, a zero block for the products
  hipLaunchKernelGGL(k_copy_add, dim3(grid), dim3(KT), 0, st, F, ld, B, ldb, n, nrhs, 0);
  hipLaunchKernelGGL(k_copy_add, dim3(grid), dim3(KT), 0, st, X, ld, B, ldb, n, nrhs, 0);
  hipLaunchKernelGGL(k_fill, dim3(grid), dim3(KT), 0, st, Zero, L.blk, 0.0);
  if ((e = chk())) return e;
  if ((e = precond(X))) return e;

  std::vector<double> berr(nrhs), xinf(nrhs), beta(nrhs);
  std::vector<double> H((size_t)nrhs * (m + 1) * m), g((size_t)nrhs * (m + 1)), cs((size_t)nrhs * m),
      sn((size_t)nrhs * m), hh(3 * (size_t)(m + 1) * nrhs), y((size_t)(m + 1) * nrhs);
  int iters = 0, restarts = 0;
  bool converged = false;
  double worst = 0.0;
  for (;;) {
    if ((e = residual(berr, xinf))) return e;
    worst = 0.0;
    bool bad = false;
    for (int q = 0; q < nrhs; ++q) {
      if (!(berr[q] == berr[q])) bad = true;
      worst = std::max(worst, berr[q]);
    }
    if (bad) {
      worst = NAN;
      break;
    }
    if (worst <= tol) {
      converged = true;
      break;
    }
    if (iters >= max_iters) break;
    // V_0 = R / ||R||_2
    if ((e = dots(R, 1, R, 1.0, hn))) return e;
    hipLaunchKernelGGL(k_inv_norm, dim3(1), dim3(64), 0, st, hn, sdev, nrhs);
    hipLaunchKernelGGL(k_scale_into, dim3(grid), dim3(KT), 0, st, V, R, ld, n, nrhs, sdev);
    if ((e = chk())) return e;
    if (hipMemcpyAsync(hh.data(), hn, 8 * nrhs, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return chk();
    for (int q = 0; q < nrhs; ++q) {
      beta[q] = std::sqrt(hh[q]);
      std::fill(g.begin() + (size_t)q * (m + 1), g.begin() + (size_t)(q + 1) * (m + 1), 0.0);
      g[(size_t)q * (m + 1)] = beta[q];
    }
    int jend = 0;
    for (int j = 0; j < m && iters < max_iters; ++j) {
      // W = op(A) M^{-1} V_j, orthogonalised against V_0 .. V_j twice
      hipLaunchKernelGGL(k_copy_add, dim3(grid), dim3(KT), 0, st, Z, ld, V + (int64_t)j * vstride, ld, n, nrhs, 0);
      if ((e = chk())) return e;
      if ((e = precond(Z))) return e;
      hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, colred, 2 * nrhs, flag);
      if ((e = launch_residual(k, n, pl.kl, pl.ku, Zero, Z, ld, W, ld, nrhs, trans, colred, flag, st))) return e;
      // W holds -op(A) Z: the first pass flips its sign
      if ((e = dots(V, j + 1, W, -1.0, h1))) return e;
      hipLaunchKernelGGL(k_vupdate, dim3(grid), dim3(KT), 0, st, W, V, vstride, ld, n, nrhs, j + 1, -1.0, h1);
      if ((e = chk())) return e;
      if ((e = dots(V, j + 1, W, 1.0, h2))) return e;
      hipLaunchKernelGGL(k_vupdate, dim3(grid), dim3(KT), 0, st, W, V, vstride, ld, n, nrhs, j + 1, 1.0, h2);
      if ((e = chk())) return e;
      if ((e = dots(W, 1, W, 1.0, hn))) return e;
      hipLaunchKernelGGL(k_inv_norm, dim3(1), dim3(64), 0, st, hn, sdev, nrhs);
      hipLaunchKernelGGL(k_scale_into, dim3(grid), dim3(KT), 0, st, V + (int64_t)(j + 1) * vstride, W, ld, n, nrhs,
                         sdev);
      if ((e = chk())) return e;
      if (hipMemcpyAsync(hh.data(), h1, 8 * 3 * (size_t)(m + 1) * nrhs, hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return chk();
      ++iters;
      jend = j + 1;
      bool all_done = true;
      for (int q = 0; q < nrhs; ++q) {
        double* Hq = &H[(size_t)q * (m + 1) * m];   // column-major (m + 1) x m
        double* gq = &g[(size_t)q * (m + 1)];
        for (int i = 0; i <= j; ++i)
          Hq[i + (size_t)j * (m + 1)] = hh[(size_t)i * nrhs + q] + hh[(size_t)(m + 1) * nrhs + (size_t)i * nrhs + q];
        Hq[(j + 1) + (size_t)j * (m + 1)] = std::sqrt(hh[2 * (size_t)(m + 1) * nrhs + q]);
        // previous rotations, then a new one annihilating H(j+1, j)
        for (int i = 0; i < j; ++i) {
          const double a = Hq[i + (size_t)j * (m + 1)], b = Hq[i + 1 + (size_t)j * (m + 1)];
          Hq[i + (size_t)j * (m + 1)] = cs[(size_t)q * m + i] * a + sn[(size_t)q * m + i] * b;
          Hq[i + 1 + (size_t)j * (m + 1)] = -sn[(size_t)q * m + i] * a + cs[(size_t)q * m + i] * b;
        }
        const double a = Hq[j + (size_t)j * (m + 1)], b = Hq[j + 1 + (size_t)j * (m + 1)];
        const double r = std::hypot(a, b);
        const double cj = r > 0.0 ? a / r : 1.0, sj = r > 0.0 ? b / r : 0.0;
        cs[(size_t)q * m + j] = cj;
        sn[(size_t)q * m + j] = sj;
        Hq[j + (size_t)j * (m + 1)] = r;
        Hq[j + 1 + (size_t)j * (m + 1)] = 0.0;
        gq[j + 1] = -sj * gq[j];
        gq[j] = cj * gq[j];
        // the 2-norm residual estimate against the backward-error target
        const double target = tol * anorm * xinf[q];
        if (!(std::fabs(gq[j + 1]) <= target) && beta[q] > 0.0 && b != 0.0) all_done = false;
      }
      if (all_done) break;
    }
    // y = H^{-1} g per column, U = V y, X += M^{-1} U
    for (int q = 0; q < nrhs; ++q) {
      const double* Hq = &H[(size_t)q * (m + 1) * m];
      const double* gq = &g[(size_t)q * (m + 1)];
      for (int i = jend - 1; i >= 0; --i) {
        double s = gq[i];
        for (int t = i + 1; t < jend; ++t) s -= Hq[i + (size_t)t * (m + 1)] * y[(size_t)t * nrhs + q];
        const double d = Hq[i + (size_t)i * (m + 1)];
        y[(size_t)i * nrhs + q] = (beta[q] > 0.0 && d != 0.0) ? s / d : 0.0;
      }
    }
    if (hipMemcpyAsync(ydev, y.data(), 8 * (size_t)jend * nrhs, hipMemcpyHostToDevice, st) != hipSuccess)
      return chk();
    hipLaunchKernelGGL(k_lincomb, dim3(grid), dim3(KT), 0, st, Z, V, vstride, ld, n, nrhs, jend, ydev);
    if ((e = chk())) return e;
    if ((e = precond(Z))) return e;
    hipLaunchKernelGGL(k_copy_add, dim3(grid), dim3(KT), 0, st, X, ld, Z, ld, n, nrhs, 1);
    if ((e = chk())) return e;
    ++restarts;
  }
  hipLaunchKernelGGL(k_copy_add, dim3(grid), dim3(KT), 0, st, B, ldb, X, ld, n, nrhs, 0);
  if ((e = chk())) return e;
  if (hipStreamSynchronize(st) != hipSuccess) return chk();
  res->iters = iters;
  res->restarts = restarts;
  res->converged = converged ? 1 : 0;
  res->berr = worst;
  return 0;
}

}  // namespace spike
