// Leaf kernels built on the MFMA tile engine (non-pivoting factors).
//
// Factor stage, middle partitions (the three full sweeps of Table tab:sweeps):
//   k_ftip_w : G_W = L^{-1} [C^_i; 0]            (forward, kl columns)
//   k_ftip_u : [V W] = U^{-1} [L^{-1}[0; B^_i]  G_W], keeping only the top ku
//              and bottom kl rows (the spike tips), written straight to the
//              node tips.
// Solve stage (one workgroup per partition, up to 64 right-hand sides): the
// same stages as k_leaf_dstage / k_leaf_retrieve / k_leaf_zsweep /
// k_leaf_dtstage with every full sweep on the tile engine; the truncated
// pieces use the workgroup routines with 16-wide panels.
#pragma once
#include "spike_kernels.hpp"
#include "spike_gemv.hpp"
#include "spike_tile.hpp"

namespace spike {

constexpr int FNB = 16;   // panel width of the small truncated sweeps in the fast kernels

template <typename T>
__device__ __forceinline__ int is_f64() { return sizeof(T) == 8 ? 1 : 0; }

__device__ __forceinline__ TSrc tsrc(const void* p, int f64, int64_t rs, int64_t ld, int lo1, int hi1,
                                     int lo2 = 0, int hi2 = 0, int csplit = 0, int clo = 0) {
  TSrc s;
  s.p = p;
  s.f64 = f64;
  s.rs = rs;
  s.ld = ld;
  s.lo1 = lo1;
  s.hi1 = hi1;
  s.lo2 = lo2;
  s.hi2 = hi2;
  s.csplit = csplit;
  s.clo = clo;
  return s;
}

__device__ __forceinline__ TDst tdst(void* p1, void* p2, int f64, int64_t rs, int64_t ld, int top, int bot, int m,
                                     int sub = 0) {
  TDst d;
  d.p1 = p1;
  d.p2 = p2;
  d.f64 = f64;
  d.rs = rs;
  d.ld = ld;
  d.top = top;
  d.bot = bot;
  d.m = m;
  d.sub = sub;
  return d;
}

template <typename T>
__device__ __forceinline__ const T* leaf_dinv(const KParams& k, const LeafDesc& L) {
  return reinterpret_cast<const T*>(k.dinv) + L.dinv_off;
}

// Full read/write view of a leaf's right-hand side (frame aware).
__device__ __forceinline__ TSrc rhs_src(const Mat<double>& X, int m, int lo = 0, int hi = -1) {
  return tsrc(X.p, 1, X.rs, X.ld, lo, hi < 0 ? m : hi);
}
__device__ __forceinline__ TDst rhs_dst(const Mat<double>& X, int m, int sub = 0) {
  return tdst(X.p, nullptr, 1, X.rs, X.ld, m, m, m, sub);
}

// ---------------------------------------------------------------- factor stage
// 16 x 16 diagonal-block inverses of every partition's L and U.
template <typename T>
__global__ __launch_bounds__(NT) void k_diag_inv(KParams k) {
  const LeafDesc L = k.leaves[blockIdx.x];
  BandAcc<T> A = leaf_band<T>(k, L);
  T* dv = reinterpret_cast<T*>(k.dinv) + L.dinv_off;
  diag_inverses<T>(A, dv, blockIdx.y * NT + threadIdx.x, gridDim.y * NT);
}

// Truncated spike sweeps of every partition (after the MFMA block LU), on
// the tile engine.  L^{-1}[0; B'] is zero above row m - h (h = the coupling
// block's height), and its rows from there on depend only on the trailing
// block of L: the sweep runs on the trailing principal block from the
// 16-aligned row jv <= m - h.  Middle partitions stop there (k_ftip_u takes
// the V columns from row m - ku on).  The first partition (normal frame) and
// the last (reversed frame) also keep the side block (the bottom h rows) for
// the retrieval stage and take their single tip, the bottom klf rows of
// U^{-1} L^{-1}[0; B'], from the trailing block of U from the 16-aligned row
// ju <= m - klf.
template <typename T, int HT>
__device__ __forceinline__ void ftip_v_body(const KParams& k, const int bx_, const int gx_, int ncg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int b = xcd_grouped(bx_, gx_);
  const int li = b / ncg, cg = b % ncg;
  const LeafDesc L = k.leaves[li];
  if (L.type == LEAF_SINGLE) return;
  const bool rev = L.type == LEAF_LAST;
  const BandAcc<T> A = leaf_band<T>(k, L);
  const int m = L.m, kl = k.kl, ku = k.ku, kw = k.kw;
  const int klf = A.kl, kuf = rev ? kl : ku, h = kuf;
  if (64 * cg >= kuf) return;
  const T* dv = leaf_dinv<T>(k, L);
  T* fs = reinterpret_cast<T*>(k.fscr) + L.fscr_off;   // m x kw, ld m
  // 1. L sweep of [0; B'] on rows [jv, m)
  const int jv = ((m - h) / 16) * 16, r0 = m - h - jv;
  BandAcc<T> As = A;
  As.a += (int64_t)jv * A.ldw;
  As.m = m - jv;
  TSrc src;
  if (!rev) {
    const double* bh = k.bhat + (int64_t)li * ku * ku;   // B^_i, lower part
    src = tsrc(bh - r0, 1, 1, ku, r0, r0 + ku);
  } else {
    const double* ch = k.chat + (int64_t)(k.p - 2) * kl * kl;   // C^_p, rows reversed
    src = tsrc(ch + (kl - 1 + r0), 1, -1, kl, r0, r0 + kl);
  }
  tile_sweep<T, HT, OP_L_FWD>(As, dv + (int64_t)(jv / 16) * dinv_stride(), src,
                              tdst(fs + jv, nullptr, is_f64<T>(), 1, m, m - jv, m - jv, m - jv), 64 * cg, kuf, lds);
  if (cg == 0) note_sweep(k, 0, L.type, As.m, m);
  if (L.type == LEAF_MIDDLE) return;
  __syncthreads();
  // 2. side block: the bottom h rows of L^{-1}[0; B'], columns of this group
  T* sd = reinterpret_cast<T*>(k.side) + (rev ? (int64_t)k.side_ld * k.kmax : 0);
  const int c0 = 64 * cg, nc = min(64, kuf - c0);
  for (int idx = threadIdx.x; idx < h * nc; idx += NT) {
    const int r = idx % h, c = c0 + idx / h;
    sd[r + (int64_t)c * k.side_ld] = fs[(m - h + r) + (int64_t)c * m];
  }
  // 3. the tip: bottom klf rows of U^{-1} (L^{-1}[0; B']), rows [ju, m)
  const int ju = ((m - klf) / 16) * 16, mu = m - ju, bot = m - klf - ju;
  BandAcc<T> Au = A;
  Au.a += (int64_t)ju * A.ldw;
  Au.m = mu;
  const TSrc su = tsrc(fs + ju, is_f64<T>(), 1, m, jv > ju ? jv - ju : 0, mu);
  Tips tips{k.tips, kw, ku};
  TDst du = rev ? tdst(nullptr, tips.Wt(k.p - 1) + (ku - 1), 1, -1, kw, 0, bot, mu)
                : tdst(nullptr, tips.Vb(0), 1, 1, kw, 0, bot, mu);
  tile_sweep<T, HT, OP_U_BWD>(Au, dv + (int64_t)(ju / 16) * dinv_stride(), su, du, 64 * cg, kuf, lds);
  if (cg == 0) note_sweep(k, 0, L.type, Au.m, m);
}
template <typename T, int HT>
__global__ __launch_bounds__(NT) void k_ftip_v(KParams k, int ncg) {
  ftip_v_body<T, HT>(k, blockIdx.x, gridDim.x, ncg);
}
// the same for up to kMaxBatch systems: workgroup i belongs to system s
// with off[s] <= i < off[s + 1] (its parameter block at kp[s])
template <typename T, int HT>
__global__ __launch_bounds__(NT) void k_ftip_v_b(BatchArgs ba, int ncg) {
  const int s = batch_sys(ba, blockIdx.x);
  ftip_v_body<T, HT>(*ba.kp[s], blockIdx.x - ba.off[s], ba.off[s + 1] - ba.off[s], ncg);
}

template <typename T, int HT>
__device__ __forceinline__ void ftip_w_body(const KParams& k, const int bx_, const int gx_, int ncg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int b = xcd_grouped(bx_, gx_);
  const int li = 1 + b / ncg, cg = b % ncg;
  const LeafDesc L = k.leaves[li];
  BandAcc<T> A = leaf_band<T>(k, L);
  const T* dv = leaf_dinv<T>(k, L);
  const int m = L.m, kl = k.kl, ku = k.ku;
  T* fs = reinterpret_cast<T*>(k.fscr) + L.fscr_off;
  const double* ch = k.chat + (int64_t)(li - 1) * kl * kl;
  TSrc src = tsrc(ch, 1, 1, kl, 0, kl);
  TDst dst = tdst(fs + (int64_t)ku * m, nullptr, is_f64<T>(), 1, m, m, m, m);
  tile_sweep<T, HT, OP_L_FWD>(A, dv, src, dst, 64 * cg, kl, lds);
  if (cg == 0) note_sweep(k, 0, L.type, A.m, m);   // W: L sweep
}
template <typename T, int HT>
__global__ __launch_bounds__(NT) void k_ftip_w(KParams k, int ncg) {
  ftip_w_body<T, HT>(k, blockIdx.x, gridDim.x, ncg);
}
// the same for up to kMaxBatch systems: workgroup i belongs to system s
// with off[s] <= i < off[s + 1] (its parameter block at kp[s])
template <typename T, int HT>
__global__ __launch_bounds__(NT) void k_ftip_w_b(BatchArgs ba, int ncg) {
  const int s = batch_sys(ba, blockIdx.x);
  ftip_w_body<T, HT>(*ba.kp[s], blockIdx.x - ba.off[s], ba.off[s + 1] - ba.off[s], ncg);
}

template <typename T, int HT>
__device__ __forceinline__ void ftip_u_body(const KParams& k, const int bx_, const int gx_, int ncg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int b = xcd_grouped(bx_, gx_);
  const int li = 1 + b / ncg, cg = b % ncg;
  const LeafDesc L = k.leaves[li];
  BandAcc<T> A = leaf_band<T>(k, L);
  const T* dv = leaf_dinv<T>(k, L);
  const int m = L.m, kl = k.kl, ku = k.ku, kw = k.kw;
  const T* fs = reinterpret_cast<const T*>(k.fscr) + L.fscr_off;
  // V columns hold L^{-1}[0; B^] only from row m - ku on (zero above)
  TSrc src = tsrc(fs, is_f64<T>(), 1, m, 0, m, 0, 0, ku, m - ku);
  double* tp = k.tips + (int64_t)li * kw * kw;
  TDst dst = tdst(tp, tp + ku, 1, 1, kw, ku, m - kl, m);
  tile_sweep<T, HT, OP_U_BWD>(A, dv, src, dst, 64 * cg, kw, lds);
  if (cg == 0) note_sweep(k, 0, L.type, A.m, m, 2);   // V and W: one U pass
}
template <typename T, int HT>
__global__ __launch_bounds__(NT) void k_ftip_u(KParams k, int ncg) {
  ftip_u_body<T, HT>(k, blockIdx.x, gridDim.x, ncg);
}
// the same for up to kMaxBatch systems: workgroup i belongs to system s
// with off[s] <= i < off[s + 1] (its parameter block at kp[s])
template <typename T, int HT>
__global__ __launch_bounds__(NT) void k_ftip_u_b(BatchArgs ba, int ncg) {
  const int s = batch_sys(ba, blockIdx.x);
  ftip_u_body<T, HT>(*ba.kp[s], blockIdx.x - ba.off[s], ba.off[s + 1] - ba.off[s], ncg);
}

// ---------------------------------------------------------------- solve stage
template <typename T, int HT>
__device__ void fdstage_body(const KParams& k, int li, double* B, int64_t ldb, int nrhs, T* lds) {
  if (solve_idle(k)) return;
  const LeafDesc L = k.leaves[li];
  const int m = L.m, kl = k.kl, ku = k.ku, kw = k.kw;
  BandAcc<T> A = leaf_band<T>(k, L);
  const T* dv = leaf_dinv<T>(k, L);
  Mat<double> X = leaf_rhs(L, B, ldb);
  double* nv = k.nodeval + (int64_t)li * kw * k.R;
  leaf_sweep<T, HT, OP_L_FWD>(A, dv, rhs_src(X, m), rhs_dst(X, m), 0, nrhs, lds);
  note_sweep(k, 1, L.type, A.m, m);
  if (L.type == LEAF_SINGLE) {
    leaf_sweep<T, HT, OP_U_BWD>(A, dv, rhs_src(X, m), rhs_dst(X, m), 0, nrhs, lds);
    note_sweep(k, 1, L.type, A.m, m);
    return;
  }
  if (L.type == LEAF_MIDDLE) {
    // U sweep over G (left in place for the retrieval); keep only the tips
    leaf_sweep<T, HT, OP_U_BWD>(A, dv, rhs_src(X, m), tdst(nv, nv + ku, 1, 1, kw, ku, m - kl, m), 0, nrhs, lds);
    note_sweep(k, 1, L.type, A.m, m);
    return;
  }
  const int klf = A.kl, r0 = m - klf;
  double* scr = k.sscr + L.sscr_off;
  Mat<double> Tm = make_mat(scr + m, (int64_t)1, k.sscr_ld, r0);
  for (int idx = threadIdx.x; idx < klf * nrhs; idx += NT) {
    int r = r0 + idx % klf, q = idx / klf;
    Tm.at(r, q) = X.at(r, q);
  }
  __syncthreads();
  wg_usweep<FNB, T>(A, Tm, nrhs, r0, lds);
  note_sweep(k, 1, L.type, klf, m);
  for (int idx = threadIdx.x; idx < klf * nrhs; idx += NT) {
    int r = r0 + idx % klf, q = idx / klf;
    if (L.type == LEAF_FIRST) nv[(ku + (r - r0)) + (int64_t)q * kw] = Tm.at(r, q);
    else nv[(m - 1 - r) + (int64_t)q * kw] = Tm.at(r, q);
  }
}

template <typename T, int HT>
__device__ void fretrieve_body(const KParams& k, int li, double* B, int64_t ldb, int nrhs, T* lds) {
  if (solve_idle(k)) return;
  const LeafDesc L = k.leaves[li];
  if (L.type == LEAF_SINGLE) return;
  const int m = L.m, kl = k.kl, ku = k.ku, kw = k.kw, R = k.R;
  BandAcc<T> A = leaf_band<T>(k, L);
  const T* dv = leaf_dinv<T>(k, L);
  Mat<double> X = leaf_rhs(L, B, ldb);
  if (L.type == LEAF_MIDDLE) {
    double* scr = k.sscr + L.sscr_off;
    Mat<double> S = make_mat(scr, (int64_t)1, k.sscr_ld);
    const double* ch = k.chat + (int64_t)(li - 1) * kl * kl;
    const double* bh = k.bhat + (int64_t)li * ku * ku;
    const double* xb = k.xint + (int64_t)(li - 1) * kw * R;
    const double* xt = k.xint + (int64_t)li * kw * R + kl;
    if (nrhs == 1) {
      for (int idx = threadIdx.x; idx < kl; idx += NT) {
        double acc = 0.0;
        for (int c = 0; c < kl; ++c) acc += ch[idx + (int64_t)c * kl] * xb[c];
        S.at(idx, 0) = acc;
      }
      for (int idx = threadIdx.x; idx < ku; idx += NT) {
        double acc = 0.0;
        for (int c = 0; c < ku; ++c) acc += bh[idx + (int64_t)c * ku] * xt[c];
        S.at(m - ku + idx, 0) = acc;
      }
      __syncthreads();
    } else {
      wg_gemm_cols<double>(kl, nrhs, kl, 1.0, ch, 1, kl, xb, 1, kw, 0.0, &S.at(0, 0), 1, k.sscr_ld);
      wg_gemm_cols<double>(ku, nrhs, ku, 1.0, bh, 1, ku, xt, 1, kw, 0.0, &S.at(m - ku, 0), 1, k.sscr_ld);
    }
    // G_i -= L^{-1} [C^ X_{i-1,b}; 0; B^ X_{i+1,t}], then one full U sweep
    leaf_sweep<T, HT, OP_L_FWD>(A, dv, tsrc(scr, 1, 1, k.sscr_ld, 0, kl, m - ku, m), rhs_dst(X, m, 1), 0, nrhs, lds);
    leaf_sweep<T, HT, OP_U_BWD>(A, dv, rhs_src(X, m), rhs_dst(X, m), 0, nrhs, lds);
    note_sweep(k, 1, L.type, A.m, m, 2);
    return;
  }
  const bool rev = L.type == LEAF_LAST;
  const int klf = A.kl, kuf = rev ? kl : ku;
  const int h = kuf;
  const T* sd = reinterpret_cast<const T*>(k.side) + (rev ? (int64_t)k.side_ld * k.kmax : 0);
  const double* xn = rev ? k.xint + (int64_t)(k.p - 2) * kw * R : k.xint + kl;
  if (nrhs == 1) {
    for (int r = threadIdx.x; r < h; r += NT) {
      double acc = 0.0;
      for (int c = 0; c < kuf; ++c) acc += (double)sd[r + (int64_t)c * k.side_ld] * xn[c];
      X.at(m - h + r, 0) -= acc;
    }
    __syncthreads();
  } else {
    wg_gemm_cols<T>(h, nrhs, kuf, -1.0, sd, 1, k.side_ld, xn, 1, kw, 1.0, &X.at(m - h, 0), X.rs, X.ld);
  }
  (void)klf;
  leaf_sweep<T, HT, OP_U_BWD>(A, dv, rhs_src(X, m), rhs_dst(X, m), 0, nrhs, lds);
  note_sweep(k, 1, L.type, A.m, m);
}

template <typename T, int HT>
__device__ void fzsweep_body(const KParams& k, int li, double* B, int64_t ldb, int nrhs, T* lds) {
  if (solve_idle(k)) return;
  const LeafDesc L = k.leaves[li];
  const int m = L.m, kl = k.kl, ku = k.ku, kw = k.kw, R = k.R;
  BandAcc<T> A = leaf_band<T>(k, L);
  const T* dv = leaf_dinv<T>(k, L);
  Mat<double> X = leaf_rhs(L, B, ldb);
  if (L.type == LEAF_SINGLE) {
    leaf_sweep<T, HT, OP_UT_FWD>(A, dv, rhs_src(X, m), rhs_dst(X, m), 0, nrhs, lds);
    leaf_sweep<T, HT, OP_LT_BWD>(A, dv, rhs_src(X, m), rhs_dst(X, m), 0, nrhs, lds);
    note_sweep(k, 2, L.type, A.m, m, 2);
    return;
  }
  double* scr = k.sscr + L.sscr_off;
  Mat<double> S = make_mat(scr, (int64_t)1, k.sscr_ld);
  const bool rev = L.type == LEAF_LAST;
  const int klf = A.kl, kuf = rev ? kl : ku;
  const int top0 = L.type == LEAF_MIDDLE ? ku : 0;
  // H = U^{-T} [0; F~; 0] into scratch
  leaf_sweep<T, HT, OP_UT_FWD>(A, dv, rhs_src(X, m, top0, m - klf), tdst(scr, nullptr, 1, 1, k.sscr_ld, m, m, m), 0,
                               nrhs, lds);
  note_sweep(k, 2, L.type, A.m, m);
  if (L.type == LEAF_MIDDLE) {
    double* zprev = k.ztip + (int64_t)(li - 1) * kw * R;       // top_kl(Z_i)
    double* znext = k.ztip + (int64_t)li * kw * R + kl;        // bottom_ku(Z_i)
    leaf_sweep<T, HT, OP_LT_BWD>(A, dv, tsrc(scr, 1, 1, k.sscr_ld, 0, m), tdst(zprev, znext, 1, 1, kw, kl, m - ku, m),
                                 0, nrhs, lds);
    note_sweep(k, 2, L.type, A.m, m);
    return;
  }
  const int rmin = m - kuf;
  const int r0 = (max(rmin, 0) / FNB) * FNB;
  Mat<double> Tm = make_mat(scr + m, (int64_t)1, k.sscr_ld, r0);
  for (int idx = threadIdx.x; idx < (m - r0) * nrhs; idx += NT) {
    int r = r0 + idx % (m - r0), q = idx / (m - r0);
    Tm.at(r, q) = S.at(r, q);
  }
  __syncthreads();
  wg_ltsweep<FNB, T>(A, Tm, nrhs, rmin, lds);
  note_sweep(k, 2, L.type, m - r0, m);
  if (!rev) {
    double* z = k.ztip + kl;
    for (int idx = threadIdx.x; idx < ku * nrhs; idx += NT) {
      int r = idx % ku, q = idx / ku;
      z[r + (int64_t)q * kw] = Tm.at(m - ku + r, q);
    }
  } else {
    double* z = k.ztip + (int64_t)(k.p - 2) * kw * R;
    for (int idx = threadIdx.x; idx < kl * nrhs; idx += NT) {
      int r = idx % kl, q = idx / kl;
      z[r + (int64_t)q * kw] = Tm.at(m - 1 - r, q);
    }
  }
}

template <typename T, int HT>
__device__ void fdtstage_body(const KParams& k, int li, double* B, int64_t ldb, int nrhs, T* lds) {
  if (solve_idle(k)) return;
  const LeafDesc L = k.leaves[li];
  if (L.type == LEAF_SINGLE) return;
  const int m = L.m, kl = k.kl, ku = k.ku, kw = k.kw, R = k.R;
  BandAcc<T> A = leaf_band<T>(k, L);
  const T* dv = leaf_dinv<T>(k, L);
  Mat<double> X = leaf_rhs(L, B, ldb);
  const double* nv = k.nodeval + (int64_t)li * kw * R;
  if (L.type == LEAF_MIDDLE) {
    for (int idx = threadIdx.x; idx < ku * nrhs; idx += NT) {
      int r = idx % ku, q = idx / ku;
      X.at(r, q) = nv[r + (int64_t)q * kw];
    }
    for (int idx = threadIdx.x; idx < kl * nrhs; idx += NT) {
      int r = idx % kl, q = idx / kl;
      X.at(m - kl + r, q) = nv[ku + r + (int64_t)q * kw];
    }
    __syncthreads();
    leaf_sweep<T, HT, OP_UT_FWD>(A, dv, rhs_src(X, m), rhs_dst(X, m), 0, nrhs, lds);
    leaf_sweep<T, HT, OP_LT_BWD>(A, dv, rhs_src(X, m), rhs_dst(X, m), 0, nrhs, lds);
    note_sweep(k, 2, L.type, A.m, m, 2);
    return;
  }
  const bool rev = L.type == LEAF_LAST;
  const int klf = A.kl;
  double* scr = k.sscr + L.sscr_off;
  Mat<double> S = make_mat(scr, (int64_t)1, k.sscr_ld);
  const int r0 = m - klf;
  Mat<double> Tm = make_mat(scr + m, (int64_t)1, k.sscr_ld, r0);
  for (int idx = threadIdx.x; idx < klf * nrhs; idx += NT) {
    int r = r0 + idx % klf, q = idx / klf;
    Tm.at(r, q) = rev ? nv[(m - 1 - r) + (int64_t)q * kw] : nv[ku + (r - r0) + (int64_t)q * kw];
  }
  __syncthreads();
  wg_utsweep<FNB, T>(A, Tm, nrhs, r0, lds);
  note_sweep(k, 2, L.type, klf, m);
  for (int idx = threadIdx.x; idx < m * nrhs; idx += NT) {
    int r = idx % m, q = idx / m;
    double v = S.at(r, q);
    if (r >= r0) v += Tm.at(r, q);
    X.at(r, q) = v;
  }
  __syncthreads();
  leaf_sweep<T, HT, OP_LT_BWD>(A, dv, rhs_src(X, m), rhs_dst(X, m), 0, nrhs, lds);
  note_sweep(k, 2, L.type, A.m, m);
}

// ---------------------------------------------------------------- runners
template <typename K>
inline void allow_lds_f(K kernel, size_t lds) {
  hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// Single-system and batched launches of the solve-stage partition kernels.
template <typename T, int HT>
__global__ __launch_bounds__(NT) void k_fdstage(KParams k, double* B, int64_t ldb, int nrhs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  fdstage_body<T, HT>(k, blockIdx.x, B, ldb, nrhs, reinterpret_cast<T*>(smem_raw));
}
template <typename T, int HT>
__global__ __launch_bounds__(NT) void k_fdstage_b(BatchArgs ba) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int s = batch_sys(ba, blockIdx.x);
  fdstage_body<T, HT>(*ba.kp[s], blockIdx.x - ba.off[s], ba.B[s], ba.ldb[s], ba.nrhs[s], reinterpret_cast<T*>(smem_raw));
}

template <typename T, int HT>
__global__ __launch_bounds__(NT) void k_fretrieve(KParams k, double* B, int64_t ldb, int nrhs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  fretrieve_body<T, HT>(k, blockIdx.x, B, ldb, nrhs, reinterpret_cast<T*>(smem_raw));
}
template <typename T, int HT>
__global__ __launch_bounds__(NT) void k_fretrieve_b(BatchArgs ba) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int s = batch_sys(ba, blockIdx.x);
  fretrieve_body<T, HT>(*ba.kp[s], blockIdx.x - ba.off[s], ba.B[s], ba.ldb[s], ba.nrhs[s], reinterpret_cast<T*>(smem_raw));
}

template <typename T, int HT>
__global__ __launch_bounds__(NT) void k_fzsweep(KParams k, double* B, int64_t ldb, int nrhs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  fzsweep_body<T, HT>(k, blockIdx.x, B, ldb, nrhs, reinterpret_cast<T*>(smem_raw));
}
template <typename T, int HT>
__global__ __launch_bounds__(NT) void k_fzsweep_b(BatchArgs ba) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int s = batch_sys(ba, blockIdx.x);
  fzsweep_body<T, HT>(*ba.kp[s], blockIdx.x - ba.off[s], ba.B[s], ba.ldb[s], ba.nrhs[s], reinterpret_cast<T*>(smem_raw));
}

template <typename T, int HT>
__global__ __launch_bounds__(NT) void k_fdtstage(KParams k, double* B, int64_t ldb, int nrhs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  fdtstage_body<T, HT>(k, blockIdx.x, B, ldb, nrhs, reinterpret_cast<T*>(smem_raw));
}
template <typename T, int HT>
__global__ __launch_bounds__(NT) void k_fdtstage_b(BatchArgs ba) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int s = batch_sys(ba, blockIdx.x);
  fdtstage_body<T, HT>(*ba.kp[s], blockIdx.x - ba.off[s], ba.B[s], ba.ldb[s], ba.nrhs[s], reinterpret_cast<T*>(smem_raw));
}

template <typename T, int HT>
int run_fast_factor(const KParams& k, const LaunchCfg& c, hipStream_t st) {
  if (!c.flu) {   // the MFMA block LU writes the inverses itself
    ProfScope ps("k_diag_inv", st);
    hipLaunchKernelGGL((k_diag_inv<T>), dim3(k.p, c.dinv_chunks), dim3(NT), 0, st, k);
    SPIKE_CHECK_LAUNCH();
  }
  if (c.flu && k.p > 1) {   // truncated tip sweeps (k_leaf_factor's work after the block LU)
    const int ncg_v = (k.kmax + 63) / 64;
    allow_lds_f(k_ftip_v<T, HT>, c.fast_lds);
    ProfScope ps("k_ftip_v", st);
    hipLaunchKernelGGL((k_ftip_v<T, HT>), dim3(k.p * ncg_v), dim3(NT), c.fast_lds, st, k, ncg_v);
    SPIKE_CHECK_LAUNCH();
  }
  if (!k.fast_tips) return 0;
  const int nmid = k.p - 2;
  const int ncg_w = (k.kl + 63) / 64, ncg_u = (k.kw + 63) / 64;
  allow_lds_f(k_ftip_w<T, HT>, c.fast_lds);
  allow_lds_f(k_ftip_u<T, HT>, c.fast_lds);
  if (ncg_w > 0) {
    ProfScope ps("k_ftip_w", st);
    hipLaunchKernelGGL((k_ftip_w<T, HT>), dim3(nmid * ncg_w), dim3(NT), c.fast_lds, st, k, ncg_w);
    SPIKE_CHECK_LAUNCH();
  }
  {
    ProfScope ps("k_ftip_u", st);
    hipLaunchKernelGGL((k_ftip_u<T, HT>), dim3(nmid * ncg_u), dim3(NT), c.fast_lds, st, k, ncg_u);
    SPIKE_CHECK_LAUNCH();
  }
  return 0;
}

template <typename T, int HT>
int run_fast_phase(const KParams& k, const LaunchCfg& c, hipStream_t st, double* B, int64_t ldb, int nrhs,
                   int phase) {
  switch (phase) {
    case 0: {
      allow_lds_f(k_fdstage<T, HT>, c.fast_lds);
      ProfScope ps("k_fdstage", st);
      hipLaunchKernelGGL((k_fdstage<T, HT>), dim3(k.p), dim3(NT), c.fast_lds, st, k, B, ldb, nrhs);
      break;
    }
    case 1: {
      allow_lds_f(k_fretrieve<T, HT>, c.fast_lds);
      ProfScope ps("k_fretrieve", st);
      hipLaunchKernelGGL((k_fretrieve<T, HT>), dim3(k.p), dim3(NT), c.fast_lds, st, k, B, ldb, nrhs);
      break;
    }
    case 2: {
      allow_lds_f(k_fzsweep<T, HT>, c.fast_lds);
      ProfScope ps("k_fzsweep", st);
      hipLaunchKernelGGL((k_fzsweep<T, HT>), dim3(k.p), dim3(NT), c.fast_lds, st, k, B, ldb, nrhs);
      break;
    }
    default: {
      allow_lds_f(k_fdtstage<T, HT>, c.fast_lds);
      ProfScope ps("k_fdtstage", st);
      hipLaunchKernelGGL((k_fdtstage<T, HT>), dim3(k.p), dim3(NT), c.fast_lds, st, k, B, ldb, nrhs);
      break;
    }
  }
  SPIKE_CHECK_LAUNCH();
  return 0;
}

// the tip kernels for several systems (which: 0 V tips of every partition,
// 1 W L-sweep and 2 [V W] U-sweep of the middle partitions); cnt[s] counts
// the system's partitions for which the kernel runs
template <typename T, int HT>
int run_ftip_batch(BatchArgs ba, const int* cnt, int which, int kl, int ku, size_t lds, hipStream_t st) {
  const int kmax = kl > ku ? kl : ku;
  const int ncg = which == 0 ? (kmax + 63) / 64 : (which == 1 ? (kl + 63) / 64 : (kl + ku + 63) / 64);
  int tot = 0;
  for (int s = 0; s < ba.nsys; ++s) {
    ba.off[s] = tot;
    tot += cnt[s] * ncg;
  }
  ba.off[ba.nsys] = tot;
  if (tot <= 0) return 0;
  switch (which) {
    case 0: {
      allow_lds_f(k_ftip_v_b<T, HT>, lds);
      ProfScope ps("k_ftip_v", st);
      hipLaunchKernelGGL((k_ftip_v_b<T, HT>), dim3(tot), dim3(NT), lds, st, ba, ncg);
      break;
    }
    case 1: {
      allow_lds_f(k_ftip_w_b<T, HT>, lds);
      ProfScope ps("k_ftip_w", st);
      hipLaunchKernelGGL((k_ftip_w_b<T, HT>), dim3(tot), dim3(NT), lds, st, ba, ncg);
      break;
    }
    default: {
      allow_lds_f(k_ftip_u_b<T, HT>, lds);
      ProfScope ps("k_ftip_u", st);
      hipLaunchKernelGGL((k_ftip_u_b<T, HT>), dim3(tot), dim3(NT), lds, st, ba, ncg);
      break;
    }
  }
  SPIKE_CHECK_LAUNCH();
  return 0;
}

template <typename T, int HT>
int run_fast_phase_batch(const BatchArgs& ba, size_t lds, hipStream_t st, int phase, int nitems) {
  if (nitems <= 0) return 0;
  switch (phase) {
    case 0: {
      allow_lds_f(k_fdstage_b<T, HT>, lds);
      ProfScope ps("k_fdstage", st);
      hipLaunchKernelGGL((k_fdstage_b<T, HT>), dim3(nitems), dim3(NT), lds, st, ba);
      break;
    }
    case 1: {
      allow_lds_f(k_fretrieve_b<T, HT>, lds);
      ProfScope ps("k_fretrieve", st);
      hipLaunchKernelGGL((k_fretrieve_b<T, HT>), dim3(nitems), dim3(NT), lds, st, ba);
      break;
    }
    case 2: {
      allow_lds_f(k_fzsweep_b<T, HT>, lds);
      ProfScope ps("k_fzsweep", st);
      hipLaunchKernelGGL((k_fzsweep_b<T, HT>), dim3(nitems), dim3(NT), lds, st, ba);
      break;
    }
    default: {
      allow_lds_f(k_fdtstage_b<T, HT>, lds);
      ProfScope ps("k_fdtstage", st);
      hipLaunchKernelGGL((k_fdtstage_b<T, HT>), dim3(nitems), dim3(NT), lds, st, ba);
      break;
    }
  }
  SPIKE_CHECK_LAUNCH();
  return 0;
}

}  // namespace spike
