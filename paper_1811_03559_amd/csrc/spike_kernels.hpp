// HIP kernels of the recursive SPIKE solver for gfx950 (templates; the
// instantiations live in separate translation units, see spike_inst.hip).
//
// Stages (one launch each; merge stages once per tree level):
//   factor : k_leaf_factor  - copy A_i (reversed frame for the last block),
//                             LU with boosting or partial pivoting, spike tips
//            k_merge_factor - interface system E_J (Schur form), its
//                             coefficients and the merged node's tips
//   solve  : k_leaf_dstage  - D stage (G = L^{-1}P F kept in place, Y tips)
//            k_merge_up     - reduced system, bottom-up (D^[l] solves)
//            k_merge_down   - reduced system, top-down (interface values)
//            k_leaf_retrieve- retrieval X_i = Y_i - A_i^{-1}(B_i X + C_i X)
//   transpose: k_leaf_zsweep, k_gform, k_merge_tup, k_merge_tdown,
//            k_leaf_dtstage (transpose S stage, transposed reduced system,
//            transpose D stage).
#pragma once
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>

#include "spike_device.hpp"
#include "spike_tile.hpp"
#include "spike_launch.hpp"
#include "spike_profile.hpp"

namespace spike {

// Node tips: a kw x kw block per node (ld kw): rows [0, ku) top tip, rows
// [ku, kw) bottom tip; columns [0, ku) V, columns [ku, kw) W.
struct Tips {
  double* base;
  int kw, ku;
  __device__ double* node(int id) const { return base + (int64_t)id * kw * kw; }
  __device__ double* Vt(int id) const { return node(id); }
  __device__ double* Vb(int id) const { return node(id) + ku; }
  __device__ double* Wt(int id) const { return node(id) + (int64_t)ku * kw; }
  __device__ double* Wb(int id) const { return node(id) + ku + (int64_t)ku * kw; }
};

__device__ __forceinline__ bool status_bad(const DevStatus* s) {
  return s->zero_row != ULLONG_MAX || s->iface != ULLONG_MAX;
}

// Solve kernels idle when the factorisation failed, or inside a refinement
// loop that has converged.
__device__ __forceinline__ bool solve_idle(const KParams& k) {
  return status_bad(k.status) || (k.skip != nullptr && *k.skip != 0);
}

// Counts one triangular sweep of one column set over `rows` of a partition
// of m rows (stage and counter layout as KParams::sweeps).  Called by one
// thread of one workgroup per partition.
__device__ __forceinline__ void note_sweep(const KParams& k, int stage, int type, int rows, int m, int sets = 1) {
  if (k.sweeps != nullptr && threadIdx.x == 0)
    atomicAdd(&k.sweeps[(stage * 4 + type) * 2 + (rows >= m ? 1 : 0)], (unsigned long long)sets);
}

static __global__ void k_zero_counters(unsigned long long* c, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) c[i] = 0ull;
}

__device__ inline void init_status_fields(DevStatus* s) {
  s->zero_row = ULLONG_MAX;
  s->iface = ULLONG_MAX;
  s->n_boosts = 0;
  s->refine_iters = 0;
  s->min_pivot_bits = dbits(__builtin_huge_val());
  s->berr = -1.0;
  s->refine_active = 0;
  s->skip = 1;
  s->anorm_inf_bits = 0ull;
  s->anorm_one_bits = 0ull;
}

static __global__ void k_init_status(DevStatus* s) {
  if (threadIdx.x == 0 && blockIdx.x == 0) init_status_fields(s);
}

template <typename T>
__device__ __forceinline__ BandAcc<T> leaf_band(const KParams& k, const LeafDesc& L) {
  const bool rev = L.type == LEAF_LAST;
  BandAcc<T> A;
  A.a = reinterpret_cast<T*>(k.band) + L.band_off;
  A.m = L.m;
  A.kl = rev ? k.ku : k.kl;
  A.kuw = k.pivot ? k.kl + k.ku : (rev ? k.kl : k.ku);
  A.ldw = k.ldw;
  A.ipiv = k.pivot ? k.ipiv + L.ipiv_off : nullptr;
  A.lp = k.pivot ? reinterpret_cast<T*>(k.lpan) + L.lp_off : nullptr;
  A.lpld = k.lpld;
  return A;
}

// Right-hand side of a leaf in its own frame.
__device__ __forceinline__ Mat<double> leaf_rhs(const LeafDesc& L, double* B, int64_t ldb) {
  if (L.type == LEAF_LAST) return make_mat(B + L.start + L.m - 1, (int64_t)-1, ldb);
  return make_mat(B + L.start, (int64_t)1, ldb);
}

// ===========================================================================
// Factorisation stage
// ===========================================================================
template <int NB, typename T>
__global__ __launch_bounds__(NT) void k_leaf_factor(KParams k) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  __shared__ double sred[NWAVE];
  const int li = blockIdx.x;
  const LeafDesc L = k.leaves[li];
  const int m = L.m;
  const bool rev = L.type == LEAF_LAST;
  BandAcc<T> A = leaf_band<T>(k, L);
  int* ipiv_w = k.pivot ? k.ipiv + L.ipiv_off : nullptr;
  const int klf = A.kl, kuf = rev ? k.kl : k.ku, kuwf = A.kuw;
  const int64_t s = L.start;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;

  if (!k.lu_done) {
    // 1. copy the block into its frame (wave per column) and take ||A_i||_1.
    double cmax = 0.0;
    for (int c = wave; c < m; c += NWAVE) {
      const int64_t gc = rev ? s + m - 1 - c : s + c;
      double csum = 0.0;
      for (int sr = lane; sr < k.ldw; sr += 64) {
        const int i = c + sr - kuwf;
        T v = T(0);
        if (i >= 0 && i < m && i - c <= klf && c - i <= kuf) {
          const int64_t gi = rev ? s + m - 1 - i : s + i;
          const double a = k.dAB[(k.ku + gi - gc) + gc * k.ldab];
          v = (T)a;
          csum += fabs(a);
        }
        A.a[sr + (int64_t)c * k.ldw] = v;
      }
      for (int off = 32; off > 0; off >>= 1) csum += __shfl_xor(csum, off);
      cmax = fmax(cmax, csum);
    }
    if (lane == 0) sred[wave] = cmax;

    // 2. coupling blocks: B^_i (rows s_{i+1}-ku.., cols s_{i+1}..) and
    //    C^_i (rows s_i.., cols s_i-kl..), in the normal frame.
    if (li < k.p - 1) {
      double* bh = k.bhat + (int64_t)li * k.ku * k.ku;
      const int64_t s1 = s + m;
      for (int idx = threadIdx.x; idx < k.ku * k.ku; idx += NT) {
        int r = idx % k.ku, c = idx / k.ku;
        int64_t gi = s1 - k.ku + r, gc = s1 + c;
        bh[idx] = (r >= c) ? k.dAB[(k.ku + gi - gc) + gc * k.ldab] : 0.0;
      }
    }
    if (li > 0) {
      double* ch = k.chat + (int64_t)(li - 1) * k.kl * k.kl;
      for (int idx = threadIdx.x; idx < k.kl * k.kl; idx += NT) {
        int r = idx % k.kl, c = idx / k.kl;
        int64_t gi = s + r, gc = s - k.kl + c;
        ch[idx] = (r <= c) ? k.dAB[(k.ku + gi - gc) + gc * k.ldab] : 0.0;
      }
    }
    __syncthreads();
    double anorm1 = 0.0;
    for (int w = 0; w < NWAVE; ++w) anorm1 = fmax(anorm1, sred[w]);

    // 3. block factorisation
    T boost = T(0);
    if (!k.pivot && k.boost_tau > 0.0) boost = (T)(k.boost_tau * anorm1);
    LuStats st;
    wg_lu<NB, T>(A, ipiv_w, boost, lds, st);
    if (threadIdx.x == 0) {
      if (st.first_zero >= 0) {
        int64_t grow = rev ? s + m - 1 - st.first_zero : s + st.first_zero;
        atomicMin(&k.status->zero_row, (unsigned long long)(grow + 1));
      }
      if (st.boosts) atomicAdd(&k.status->n_boosts, st.boosts);
      atomicMin(&k.status->min_pivot_bits, dbits(st.min_piv));
    }
  }
  if (L.type == LEAF_SINGLE) return;
  __syncthreads();

  // 4. spike tips (section "Optimizing per-partition costs", Table tab:sweeps)
  const int kl = k.kl, ku = k.ku, kw = k.kw;
  T* fs = reinterpret_cast<T*>(k.fscr) + L.fscr_off;   // m x kw, ld m
  Tips tips{k.tips, kw, ku};
  if (L.type == LEAF_MIDDLE && k.fast_tips) {
    // Only the truncated L sweep of V here; the full sweeps run on the tile
    // engine afterwards.  L^{-1}[0; B^] is zero above row m - ku.
    const int jv = (max(m - ku, 0) / NB) * NB;
    for (int64_t idx = threadIdx.x; idx < (int64_t)(m - jv) * ku; idx += NT) {
      int r = jv + (int)(idx % (m - jv)), c = (int)(idx / (m - jv));
      fs[r + (int64_t)c * m] = T(0);
    }
    __syncthreads();
    const double* bh = k.bhat + (int64_t)li * ku * ku;
    for (int idx = threadIdx.x; idx < ku * ku; idx += NT) {
      int r = idx % ku, c = idx / ku;
      fs[(m - ku + r) + (int64_t)c * m] = (T)bh[idx];
    }
    __syncthreads();
    wg_lsweep<NB, T>(A, make_mat(fs, (int64_t)1, (int64_t)m), ku, jv, lds);
    note_sweep(k, 0, L.type, m - jv, m);
    return;
  }
  if (L.type == LEAF_MIDDLE) {
    // V RHS [0; B^_i] in columns [0, ku), W RHS [C^_i; 0] in columns [ku, kw).
    for (int64_t idx = threadIdx.x; idx < (int64_t)m * kw; idx += NT) fs[idx] = T(0);
    __syncthreads();
    const double* bh = k.bhat + (int64_t)li * ku * ku;
    const double* ch = k.chat + (int64_t)(li - 1) * kl * kl;
    for (int idx = threadIdx.x; idx < ku * ku; idx += NT) {
      int r = idx % ku, c = idx / ku;
      fs[(m - ku + r) + (int64_t)c * m] = (T)bh[idx];
    }
    for (int idx = threadIdx.x; idx < kl * kl; idx += NT) {
      int r = idx % kl, c = idx / kl;
      fs[r + (int64_t)(ku + c) * m] = (T)ch[idx];
    }
    __syncthreads();
    // W: full L sweep; V: L sweep truncated to where B^ (moved by at most kl
    // rows under pivoting) becomes nonzero; then one full U sweep over [V W].
    wg_lsweep<NB, T>(A, make_mat(fs + (int64_t)ku * m, (int64_t)1, (int64_t)m), kl, 0, lds);
    const int vstart = m - ku - (k.pivot ? kl : 0);
    wg_lsweep<NB, T>(A, make_mat(fs, (int64_t)1, (int64_t)m), ku, vstart, lds);
    wg_usweep<NB, T>(A, make_mat(fs, (int64_t)1, (int64_t)m), kw, 0, lds);
    note_sweep(k, 0, L.type, m, m);                                   // W: L sweep
    note_sweep(k, 0, L.type, m - (max(vstart, 0) / NB) * NB, m);      // V: truncated L sweep
    note_sweep(k, 0, L.type, m, m, 2);                                // V and W: one U pass
    double* tp = tips.node(li);
    for (int idx = threadIdx.x; idx < kw * kw; idx += NT) {
      int r = idx % kw, c = idx / kw;
      int fr = r < ku ? r : m - kl + (r - ku);
      tp[r + (int64_t)c * kw] = (double)fs[fr + (int64_t)c * m];
    }
  } else {
    // First block (normal frame) / last block (reversed frame): only the
    // bottom tip of L^{-1} P [0; B'] is needed, via truncated sweeps; the
    // nonzero part of L^{-1} P [0; B'] is kept for the retrieval stage.
    const int h = kuf + (k.pivot ? klf : 0);
    const int jstart = ((m - h) / NB) * NB;
    // rows [zstart, m) take part in the L sweep (from jstart) or in the tip
    // solve (the bottom klf rows); all of them start from the RHS [0; B']
    const int zstart = min(jstart, m - klf);
    for (int64_t idx = threadIdx.x; idx < (int64_t)(m - zstart) * kuf; idx += NT) {
      int r = zstart + (int)(idx % (m - zstart)), c = (int)(idx / (m - zstart));
      fs[r + (int64_t)c * m] = T(0);
    }
    __syncthreads();
    if (!rev) {
      const double* bh = k.bhat;   // B^_1
      for (int idx = threadIdx.x; idx < ku * ku; idx += NT) {
        int r = idx % ku, c = idx / ku;
        fs[(m - ku + r) + (int64_t)c * m] = (T)bh[idx];
      }
    } else {
      const double* ch = k.chat + (int64_t)(k.p - 2) * kl * kl;   // C^_p, rows reversed
      for (int idx = threadIdx.x; idx < kl * kl; idx += NT) {
        int r = idx % kl, c = idx / kl;
        fs[(m - kl + r) + (int64_t)c * m] = (T)ch[(kl - 1 - r) + (int64_t)c * kl];
      }
    }
    __syncthreads();
    wg_lsweep<NB, T>(A, make_mat(fs, (int64_t)1, (int64_t)m), kuf, jstart, lds);
    note_sweep(k, 0, L.type, m - jstart, m);
    T* sd = reinterpret_cast<T*>(k.side) + (rev ? (int64_t)k.side_ld * k.kmax : 0);
    for (int idx = threadIdx.x; idx < h * kuf; idx += NT) {
      int r = idx % h, c = idx / h;
      sd[r + (int64_t)c * k.side_ld] = fs[(m - h + r) + (int64_t)c * m];
    }
    __syncthreads();
    wg_usweep<NB, T>(A, make_mat(fs, (int64_t)1, (int64_t)m), kuf, m - klf, lds);
    note_sweep(k, 0, L.type, klf, m);
    if (!rev) {
      double* vb = tips.Vb(0);
      for (int idx = threadIdx.x; idx < kl * ku; idx += NT) {
        int r = idx % kl, c = idx / kl;
        vb[r + (int64_t)c * kw] = (double)fs[(m - kl + r) + (int64_t)c * m];
      }
    } else {
      double* wt = tips.Wt(k.p - 1);
      for (int idx = threadIdx.x; idx < ku * kl; idx += NT) {
        int r = idx % ku, c = idx / ku;
        wt[r + (int64_t)c * kw] = (double)fs[(m - 1 - r) + (int64_t)c * m];
      }
    }
  }
}

// Interface system of merge J = (L, R) at interface mi:
//   E_J = [[I, Vb_L], [Wt_R, I]],  S = I - Wt_R Vb_L  (Schur complement, LU
//   with partial pivoting), and the coefficients
//   [alpha; beta] = E^{-1}[0; Vt_R],  [gamma; delta] = E^{-1}[Wb_L; 0],
//   then the tips of the merged node (boundary rows of V_J, W_J).
template <int NBD>
__global__ __launch_bounds__(NT) void k_merge_factor(KParams k, int mbeg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  const MergeDesc J = k.merges[mbeg + blockIdx.x];
  const int kl = k.kl, ku = k.ku, kw = k.kw, mi = J.mif;
  const int l = J.left, r = J.right;
  Tips tp{k.tips, kw, ku};
  const bool nv = J.b < k.p - 1, nw = J.a > 0;
  double* S = k.sfac + (int64_t)mi * ku * ku;
  int* sp = k.spiv + (int64_t)mi * ku;
  double* C = k.coef + (int64_t)mi * kw * kw;
  double* alpha = C;
  double* beta = C + kl;
  double* gamma = C + (int64_t)ku * kw;
  double* delta = C + kl + (int64_t)ku * kw;

  for (int idx = threadIdx.x; idx < ku * ku; idx += NT) S[idx] = (idx % ku == idx / ku) ? 1.0 : 0.0;
  for (int idx = threadIdx.x; idx < kw * kw; idx += NT) C[idx] = 0.0;
  __syncthreads();
  wg_gemm(ku, ku, kl, -1.0, gm(tp.Wt(r), 1, kw), gm(tp.Vb(l), 1, kw), 1.0, S, ku, lds);
  DenseAcc<double> D{S, ku, ku - 1, ku - 1, ku, sp};
  LuStats st;
  wg_lu<NBD, double>(D, sp, 0.0, lds, st);
  if (threadIdx.x == 0 && st.first_zero >= 0)
    atomicMin(&k.status->iface, (unsigned long long)(mi + 1));
  __syncthreads();
  if (nv) {
    wg_copy(ku, ku, tp.Vt(r), kw, beta, kw);
    __syncthreads();
    wg_lsweep<NBD, double>(D, make_mat(beta, (int64_t)1, (int64_t)kw), ku, 0, lds);
    wg_usweep<NBD, double>(D, make_mat(beta, (int64_t)1, (int64_t)kw), ku, 0, lds);
    wg_gemm(kl, ku, ku, -1.0, gm(tp.Vb(l), 1, kw), gm(beta, 1, kw), 0.0, alpha, kw, lds);
  }
  if (nw) {
    wg_gemm(ku, kl, kl, -1.0, gm(tp.Wt(r), 1, kw), gm(tp.Wb(l), 1, kw), 0.0, delta, kw, lds);
    wg_lsweep<NBD, double>(D, make_mat(delta, (int64_t)1, (int64_t)kw), kl, 0, lds);
    wg_usweep<NBD, double>(D, make_mat(delta, (int64_t)1, (int64_t)kw), kl, 0, lds);
    wg_copy(kl, kl, tp.Wb(l), kw, gamma, kw);
    __syncthreads();
    wg_gemm(kl, kl, ku, -1.0, gm(tp.Vb(l), 1, kw), gm(delta, 1, kw), 1.0, gamma, kw, lds);
  }
  if (J.a == 0 && J.b == k.p - 1) return;   // root: no tips needed
  const int jid = k.p + mi;
  if (nv && nw) {
    wg_gemm(ku, ku, ku, -1.0, gm(tp.Vt(l), 1, kw), gm(beta, 1, kw), 0.0, tp.Vt(jid), kw, lds);
    wg_gemm(kl, kl, kl, -1.0, gm(tp.Wb(r), 1, kw), gm(gamma, 1, kw), 0.0, tp.Wb(jid), kw, lds);
  }
  if (nv) {
    wg_copy(kl, ku, tp.Vb(r), kw, tp.Vb(jid), kw);
    __syncthreads();
    wg_gemm(kl, ku, kl, -1.0, gm(tp.Wb(r), 1, kw), gm(alpha, 1, kw), 1.0, tp.Vb(jid), kw, lds);
  }
  if (nw) {
    wg_copy(ku, kl, tp.Wt(l), kw, tp.Wt(jid), kw);
    __syncthreads();
    wg_gemm(ku, kl, ku, -1.0, gm(tp.Vt(l), 1, kw), gm(delta, 1, kw), 1.0, tp.Wt(jid), kw, lds);
  }
}

// ===========================================================================
// Solve stage, A X = F
// ===========================================================================
template <int NB, typename T>
__global__ __launch_bounds__(NT) void k_leaf_dstage(KParams k, double* B, int64_t ldb, int nrhs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  if (solve_idle(k)) return;
  const int li = blockIdx.x;
  const LeafDesc L = k.leaves[li];
  const int m = L.m, kl = k.kl, ku = k.ku, kw = k.kw;
  BandAcc<T> A = leaf_band<T>(k, L);
  Mat<double> X = leaf_rhs(L, B, ldb);
  double* scr = k.sscr + L.sscr_off;
  const int64_t sld = k.sscr_ld;
  double* nv = k.nodeval + (int64_t)li * kw * k.R;
  wg_lsweep<NB, T>(A, X, nrhs, 0, lds);
  note_sweep(k, 1, L.type, m, m);
  if (L.type == LEAF_SINGLE) {
    wg_usweep<NB, T>(A, X, nrhs, 0, lds);
    note_sweep(k, 1, L.type, m, m);
    return;
  }
  if (L.type == LEAF_MIDDLE) {
    Mat<double> S = make_mat(scr, (int64_t)1, sld);
    for (int idx = threadIdx.x; idx < m * nrhs; idx += NT) {
      int r = idx % m, q = idx / m;
      S.at(r, q) = X.at(r, q);
    }
    __syncthreads();
    wg_usweep<NB, T>(A, S, nrhs, 0, lds);
    note_sweep(k, 1, L.type, m, m);
    for (int idx = threadIdx.x; idx < kw * nrhs; idx += NT) {
      int r = idx % kw, q = idx / kw;
      int fr = r < ku ? r : m - kl + (r - ku);
      nv[r + (int64_t)q * kw] = S.at(fr, q);
    }
    return;
  }
  // first / last: Y_b = U_bb^{-1} G_b on a copy of the bottom rows.
  const int klf = A.kl;
  const int r0 = m - klf;
  Mat<double> Tm = make_mat(scr + m, (int64_t)1, sld, r0);
  for (int idx = threadIdx.x; idx < klf * nrhs; idx += NT) {
    int r = r0 + idx % klf, q = idx / klf;
    Tm.at(r, q) = X.at(r, q);
  }
  __syncthreads();
  wg_usweep<NB, T>(A, Tm, nrhs, r0, lds);
  note_sweep(k, 1, L.type, klf, m);
  for (int idx = threadIdx.x; idx < klf * nrhs; idx += NT) {
    int r = r0 + idx % klf, q = idx / klf;
    if (L.type == LEAF_FIRST) nv[(ku + (r - r0)) + (int64_t)q * kw] = Tm.at(r, q);
    else nv[(m - 1 - r) + (int64_t)q * kw] = Tm.at(r, q);
  }
}

template <int NBD>
__global__ __launch_bounds__(NT) void k_merge_up(KParams k, int mbeg, int nrhs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  if (solve_idle(k)) return;
  const MergeDesc J = k.merges[mbeg + blockIdx.x];
  const int kl = k.kl, ku = k.ku, kw = k.kw, mi = J.mif, R = k.R;
  Tips tp{k.tips, kw, ku};
  double* nvl = k.nodeval + (int64_t)J.left * kw * R;
  double* nvr = k.nodeval + (int64_t)J.right * kw * R;
  double* nvj = k.nodeval + (int64_t)(k.p + mi) * kw * R;
  double* s = k.st + (int64_t)mi * kw * R;
  double* t = s + kl;
  DenseAcc<double> D{k.sfac + (int64_t)mi * ku * ku, ku, ku - 1, ku - 1, ku, k.spiv + (int64_t)mi * ku};
  wg_copy(ku, nrhs, nvr, kw, t, kw);
  wg_copy(kl, nrhs, nvl + ku, kw, s, kw);
  __syncthreads();
  wg_gemm(ku, nrhs, kl, -1.0, gm(tp.Wt(J.right), 1, kw), gm(s, 1, kw), 1.0, t, kw, lds);
  wg_lsweep<NBD, double>(D, make_mat(t, (int64_t)1, (int64_t)kw), nrhs, 0, lds);
  wg_usweep<NBD, double>(D, make_mat(t, (int64_t)1, (int64_t)kw), nrhs, 0, lds);
  wg_gemm(kl, nrhs, ku, -1.0, gm(tp.Vb(J.left), 1, kw), gm(t, 1, kw), 1.0, s, kw, lds);
  if (J.a > 0) {
    wg_copy(ku, nrhs, nvl, kw, nvj, kw);
    __syncthreads();
    wg_gemm(ku, nrhs, ku, -1.0, gm(tp.Vt(J.left), 1, kw), gm(t, 1, kw), 1.0, nvj, kw, lds);
  }
  if (J.b < k.p - 1) {
    wg_copy(kl, nrhs, nvr + ku, kw, nvj + ku, kw);
    __syncthreads();
    wg_gemm(kl, nrhs, kl, -1.0, gm(tp.Wb(J.right), 1, kw), gm(s, 1, kw), 1.0, nvj + ku, kw, lds);
  }
}

static __global__ __launch_bounds__(NT) void k_merge_down(KParams k, int mbeg, int nrhs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  if (solve_idle(k)) return;
  const MergeDesc J = k.merges[mbeg + blockIdx.x];
  const int kl = k.kl, ku = k.ku, kw = k.kw, mi = J.mif, R = k.R;
  double* x = k.xint + (int64_t)mi * kw * R;
  const double* C = k.coef + (int64_t)mi * kw * kw;
  wg_copy(kw, nrhs, k.st + (int64_t)mi * kw * R, kw, x, kw);
  __syncthreads();
  if (J.b < k.p - 1)
    wg_gemm(kw, nrhs, ku, -1.0, gm(C, 1, kw), gm(k.xint + (int64_t)J.b * kw * R + kl, 1, kw), 1.0, x,
            kw, lds);
  if (J.a > 0)
    wg_gemm(kw, nrhs, kl, -1.0, gm(C + (int64_t)ku * kw, 1, kw),
            gm(k.xint + (int64_t)(J.a - 1) * kw * R, 1, kw), 1.0, x, kw, lds);
}

template <int NB, typename T>
__global__ __launch_bounds__(NT) void k_leaf_retrieve(KParams k, double* B, int64_t ldb, int nrhs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  if (solve_idle(k)) return;
  const int li = blockIdx.x;
  const LeafDesc L = k.leaves[li];
  if (L.type == LEAF_SINGLE) return;
  const int m = L.m, kl = k.kl, ku = k.ku, kw = k.kw, R = k.R;
  BandAcc<T> A = leaf_band<T>(k, L);
  Mat<double> X = leaf_rhs(L, B, ldb);
  if (L.type == LEAF_MIDDLE) {
    // X_i = U^{-1}(G_i - L^{-1} P [C^ X_{i-1,b}; 0; B^ X_{i+1,t}])
    double* scr = k.sscr + L.sscr_off;
    const int64_t sld = k.sscr_ld;
    Mat<double> S = make_mat(scr, (int64_t)1, sld);
    for (int idx = threadIdx.x; idx < m * nrhs; idx += NT) scr[idx % m + (int64_t)(idx / m) * sld] = 0.0;
    __syncthreads();
    const double* ch = k.chat + (int64_t)(li - 1) * kl * kl;
    const double* bh = k.bhat + (int64_t)li * ku * ku;
    const double* xb = k.xint + (int64_t)(li - 1) * kw * R;        // X_{i-1,b}: rows [0, kl)
    const double* xt = k.xint + (int64_t)li * kw * R + kl;         // X_{i+1,t}: rows [kl, kw)
    if (nrhs == 1) {
      for (int r = threadIdx.x; r < kl; r += NT) {
        double acc = 0.0;
        for (int c = 0; c < kl; ++c) acc += ch[r + (int64_t)c * kl] * xb[c];
        S.at(r, 0) = acc;
      }
      for (int r = threadIdx.x; r < ku; r += NT) {
        double acc = 0.0;
        for (int c = 0; c < ku; ++c) acc += bh[r + (int64_t)c * ku] * xt[c];
        S.at(m - ku + r, 0) = acc;
      }
      __syncthreads();
    } else {
      wg_gemm_cols<double>(kl, nrhs, kl, 1.0, ch, 1, kl, xb, 1, kw, 0.0, &S.at(0, 0), 1, sld);
      wg_gemm_cols<double>(ku, nrhs, ku, 1.0, bh, 1, ku, xt, 1, kw, 0.0, &S.at(m - ku, 0), 1, sld);
    }
    wg_lsweep<NB, T>(A, S, nrhs, 0, lds);
    for (int idx = threadIdx.x; idx < m * nrhs; idx += NT) {
      int r = idx % m, q = idx / m;
      X.at(r, q) -= S.at(r, q);
    }
    __syncthreads();
    wg_usweep<NB, T>(A, X, nrhs, 0, lds);
    note_sweep(k, 1, L.type, m, m, 2);
    return;
  }
  // first / last: subtract the stored side block times the neighbour value.
  const bool rev = L.type == LEAF_LAST;
  const int klf = A.kl, kuf = rev ? kl : ku;
  const int h = kuf + (k.pivot ? klf : 0);
  const T* sd = reinterpret_cast<const T*>(k.side) + (rev ? (int64_t)k.side_ld * k.kmax : 0);
  const double* xn = rev ? k.xint + (int64_t)(k.p - 2) * kw * R            // X_{p-1,b}
                         : k.xint + kl;                                      // X_{2,t}
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
  wg_usweep<NB, T>(A, X, nrhs, 0, lds);
  note_sweep(k, 1, L.type, m, m);
}

// ===========================================================================
// Transpose solve, A^T X = F
// ===========================================================================
template <int NB, typename T>
__global__ __launch_bounds__(NT) void k_leaf_zsweep(KParams k, double* B, int64_t ldb, int nrhs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  if (solve_idle(k)) return;
  const int li = blockIdx.x;
  const LeafDesc L = k.leaves[li];
  const int m = L.m, kl = k.kl, ku = k.ku, kw = k.kw, R = k.R;
  BandAcc<T> A = leaf_band<T>(k, L);
  Mat<double> X = leaf_rhs(L, B, ldb);
  if (L.type == LEAF_SINGLE) {
    wg_utsweep<NB, T>(A, X, nrhs, 0, lds);
    wg_ltsweep<NB, T>(A, X, nrhs, 0, lds);
    note_sweep(k, 2, L.type, m, m, 2);
    return;
  }
  double* scr = k.sscr + L.sscr_off;
  const int64_t sld = k.sscr_ld;
  Mat<double> S = make_mat(scr, (int64_t)1, sld);
  const bool rev = L.type == LEAF_LAST;
  const int klf = A.kl, kuf = rev ? kl : ku;
  // Z_i = A_i^{-T} [0; F~_i; 0] (first block keeps its top rows, last block
  // its bottom rows, eq. ATF with the first/last convention).
  const int top0 = L.type == LEAF_MIDDLE ? ku : 0;   // zero rows [0, top0)
  const int bot0 = m - klf;                            // zero rows [bot0, m)
  for (int idx = threadIdx.x; idx < m * nrhs; idx += NT) {
    int r = idx % m, q = idx / m;
    S.at(r, q) = (r < top0 || r >= bot0) ? 0.0 : X.at(r, q);
  }
  __syncthreads();
  wg_utsweep<NB, T>(A, S, nrhs, 0, lds);
  note_sweep(k, 2, L.type, m, m);
  if (L.type == LEAF_MIDDLE) {
    wg_ltsweep<NB, T>(A, S, nrhs, 0, lds);
    note_sweep(k, 2, L.type, m, m);
    double* zprev = k.ztip + (int64_t)(li - 1) * kw * R;   // b part: top_kl(Z_i)
    double* znext = k.ztip + (int64_t)li * kw * R + kl;    // t part: bottom_ku(Z_i)
    for (int idx = threadIdx.x; idx < kl * nrhs; idx += NT) {
      int r = idx % kl, q = idx / kl;
      zprev[r + (int64_t)q * kw] = S.at(r, q);
    }
    for (int idx = threadIdx.x; idx < ku * nrhs; idx += NT) {
      int r = idx % ku, q = idx / ku;
      znext[r + (int64_t)q * kw] = S.at(m - ku + r, q);
    }
    return;
  }
  // first / last: keep H = U^{-T}[.] in scratch; bottom kuf rows of Z from a
  // truncated L^T sweep on a copy.
  const int rmin = m - kuf - (k.pivot ? klf : 0);
  const int r0 = (max(rmin, 0) / NB) * NB;
  Mat<double> Tm = make_mat(scr + m, (int64_t)1, sld, r0);
  for (int idx = threadIdx.x; idx < (m - r0) * nrhs; idx += NT) {
    int r = r0 + idx % (m - r0), q = idx / (m - r0);
    Tm.at(r, q) = S.at(r, q);
  }
  __syncthreads();
  wg_ltsweep<NB, T>(A, Tm, nrhs, rmin, lds);
  note_sweep(k, 2, L.type, m - r0, m);
  if (!rev) {
    double* z = k.ztip + kl;   // interface 0, t part: bottom_ku(Z_1)
    for (int idx = threadIdx.x; idx < ku * nrhs; idx += NT) {
      int r = idx % ku, q = idx / ku;
      z[r + (int64_t)q * kw] = Tm.at(m - ku + r, q);
    }
  } else {
    double* z = k.ztip + (int64_t)(k.p - 2) * kw * R;   // interface p-2, b part: top_kl(Z_p)
    for (int idx = threadIdx.x; idx < kl * nrhs; idx += NT) {
      int r = idx % kl, q = idx / kl;
      z[r + (int64_t)q * kw] = Tm.at(m - 1 - r, q);
    }
  }
}

// G tips of the transpose S stage (eqs. gform1/gform2 with the spikes
// replaced by B^/C^ times A^{-T} solves):
//   G_{i,b}   = F_{i,b}   - C^_{i+1}^T top_kl(Z_{i+1})
//   G_{i+1,t} = F_{i+1,t} - B^_i^T     bottom_ku(Z_i)
__device__ inline void gform_body(const KParams& k, int mi, const double* B, int64_t ldb, int nrhs) {
  if (solve_idle(k)) return;
  const int kl = k.kl, ku = k.ku, kw = k.kw, R = k.R;
  const LeafDesc Lm = k.leaves[mi], Lr = k.leaves[mi + 1];
  double* x = k.xint + (int64_t)mi * kw * R;
  const double* z = k.ztip + (int64_t)mi * kw * R;
  const double* ch = k.chat + (int64_t)mi * kl * kl;
  const double* bh = k.bhat + (int64_t)mi * ku * ku;
  if (nrhs == 1) {
    for (int r = threadIdx.x; r < kl; r += NT) {
      double acc = B[Lm.start + Lm.m - kl + r];
      for (int c = 0; c < kl; ++c) acc -= ch[c + (int64_t)r * kl] * z[c];
      x[r] = acc;
    }
    for (int r = threadIdx.x; r < ku; r += NT) {
      double acc = B[Lr.start + r];
      for (int c = 0; c < ku; ++c) acc -= bh[c + (int64_t)r * ku] * z[kl + c];
      x[kl + r] = acc;
    }
    return;
  }
  for (int idx = threadIdx.x; idx < kl * nrhs; idx += NT) {
    const int r = idx % kl, q = idx / kl;
    x[r + (int64_t)q * kw] = B[(Lm.start + Lm.m - kl + r) + (int64_t)q * ldb];
  }
  for (int idx = threadIdx.x; idx < ku * nrhs; idx += NT) {
    const int r = idx % ku, q = idx / ku;
    x[kl + r + (int64_t)q * kw] = B[(Lr.start + r) + (int64_t)q * ldb];
  }
  __syncthreads();
  // x_top -= C^^T z_top, x_bottom -= B^^T z_bottom (transposed coupling blocks)
  wg_gemm_cols<double>(kl, nrhs, kl, -1.0, ch, kl, 1, z, 1, kw, 1.0, x, 1, kw);
  wg_gemm_cols<double>(ku, nrhs, ku, -1.0, bh, ku, 1, z + kl, 1, kw, 1.0, x + kl, 1, kw);
}
static __global__ __launch_bounds__(NT) void k_gform(KParams k, const double* B, int64_t ldb, int nrhs) {
  gform_body(k, blockIdx.x, B, ldb, nrhs);
}
static __global__ __launch_bounds__(NT) void k_gform_b(BatchArgs ba) {
  const int s = batch_sys(ba, blockIdx.x);
  gform_body(*ba.kp[s], blockIdx.x - ba.off[s], ba.B[s], ba.ldb[s], ba.nrhs[s]);
}

// Transposed reduced solve, first pass (adjoint of the top-down pass), run
// bottom-up: collect the neighbour contributions of the descendants, keep
// (s-bar, t-bar), and emit this merge's contributions coef^T x-bar.
static __global__ __launch_bounds__(NT) void k_merge_tup(KParams k, int mbeg, int nrhs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  if (solve_idle(k)) return;
  const int d = mbeg + blockIdx.x;
  const MergeDesc J = k.merges[d];
  const int kl = k.kl, ku = k.ku, kw = k.kw, mi = J.mif, R = k.R;
  double* x = k.xint + (int64_t)mi * kw * R;
  for (int ci = k.cptr[mi]; ci < k.cptr[mi + 1]; ++ci) {
    const Contrib c = k.contrib[ci];
    const double* cr = k.crl + (int64_t)c.merge * kw * R;
    if (c.kind == 0) {
      for (int idx = threadIdx.x; idx < ku * nrhs; idx += NT) {
        int r = idx % ku, q = idx / ku;
        x[kl + r + (int64_t)q * kw] -= cr[r + (int64_t)q * kw];
      }
    } else {
      for (int idx = threadIdx.x; idx < kl * nrhs; idx += NT) {
        int r = idx % kl, q = idx / kl;
        x[r + (int64_t)q * kw] -= cr[ku + r + (int64_t)q * kw];
      }
    }
    __syncthreads();
  }
  wg_copy(kw, nrhs, x, kw, k.st + (int64_t)mi * kw * R, kw);
  const double* C = k.coef + (int64_t)mi * kw * kw;
  double* out = k.crl + (int64_t)d * kw * R;
  if (J.b < k.p - 1) wg_gemm(ku, nrhs, kw, 1.0, gm(C, kw, 1), gm(x, 1, kw), 0.0, out, kw, lds);
  if (J.a > 0)
    wg_gemm(kl, nrhs, kw, 1.0, gm(C + (int64_t)ku * kw, kw, 1), gm(x, 1, kw), 0.0, out + ku, kw, lds);
}

// Transposed reduced solve, second pass (adjoint of the bottom-up pass), run
// top-down: E_J^{-T} through S^{-T}, and hand the adjoints to the children.
template <int NBD>
__global__ __launch_bounds__(NT) void k_merge_tdown(KParams k, int mbeg, int nrhs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  if (solve_idle(k)) return;
  const MergeDesc J = k.merges[mbeg + blockIdx.x];
  const int kl = k.kl, ku = k.ku, kw = k.kw, mi = J.mif, R = k.R;
  Tips tp{k.tips, kw, ku};
  double* sb = k.st + (int64_t)mi * kw * R;
  double* tb = sb + kl;
  double* nvl = k.nodeval + (int64_t)J.left * kw * R;
  double* nvr = k.nodeval + (int64_t)J.right * kw * R;
  double* nvj = k.nodeval + (int64_t)(k.p + mi) * kw * R;
  DenseAcc<double> D{k.sfac + (int64_t)mi * ku * ku, ku, ku - 1, ku - 1, ku, k.spiv + (int64_t)mi * ku};
  if (J.a > 0) wg_gemm(ku, nrhs, ku, -1.0, gm(tp.Vt(J.left), kw, 1), gm(nvj, 1, kw), 1.0, tb, kw, lds);
  if (J.b < k.p - 1)
    wg_gemm(kl, nrhs, kl, -1.0, gm(tp.Wb(J.right), kw, 1), gm(nvj + ku, 1, kw), 1.0, sb, kw, lds);
  wg_gemm(ku, nrhs, kl, -1.0, gm(tp.Vb(J.left), kw, 1), gm(sb, 1, kw), 1.0, tb, kw, lds);
  wg_utsweep<NBD, double>(D, make_mat(tb, (int64_t)1, (int64_t)kw), nrhs, 0, lds);
  wg_ltsweep<NBD, double>(D, make_mat(tb, (int64_t)1, (int64_t)kw), nrhs, 0, lds);
  wg_gemm(kl, nrhs, ku, -1.0, gm(tp.Wt(J.right), kw, 1), gm(tb, 1, kw), 1.0, sb, kw, lds);
  wg_copy(kl, nrhs, sb, kw, nvl + ku, kw);
  wg_copy(ku, nrhs, tb, kw, nvr, kw);
  if (J.a > 0) wg_copy(ku, nrhs, nvj, kw, nvl, kw);
  if (J.b < k.p - 1) wg_copy(kl, nrhs, nvj + ku, kw, nvr + ku, kw);
}

template <int NB, typename T>
__global__ __launch_bounds__(NT) void k_leaf_dtstage(KParams k, double* B, int64_t ldb, int nrhs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  if (solve_idle(k)) return;
  const int li = blockIdx.x;
  const LeafDesc L = k.leaves[li];
  if (L.type == LEAF_SINGLE) return;
  const int m = L.m, kl = k.kl, ku = k.ku, kw = k.kw, R = k.R;
  BandAcc<T> A = leaf_band<T>(k, L);
  Mat<double> X = leaf_rhs(L, B, ldb);
  const double* nv = k.nodeval + (int64_t)li * kw * R;
  if (L.type == LEAF_MIDDLE) {
    // X_i = A_i^{-T} [Y_it; F~_i; Y_ib]  (eq. sweeps_in_D)
    for (int idx = threadIdx.x; idx < ku * nrhs; idx += NT) {
      int r = idx % ku, q = idx / ku;
      X.at(r, q) = nv[r + (int64_t)q * kw];
    }
    for (int idx = threadIdx.x; idx < kl * nrhs; idx += NT) {
      int r = idx % kl, q = idx / kl;
      X.at(m - kl + r, q) = nv[ku + r + (int64_t)q * kw];
    }
    __syncthreads();
    wg_utsweep<NB, T>(A, X, nrhs, 0, lds);
    wg_ltsweep<NB, T>(A, X, nrhs, 0, lds);
    note_sweep(k, 2, L.type, m, m, 2);
    return;
  }
  // first / last: X = P^T L^{-T} (H + [0; U_bb^{-T} Y_b]), H kept in scratch.
  const bool rev = L.type == LEAF_LAST;
  const int klf = A.kl;
  double* scr = k.sscr + L.sscr_off;
  const int64_t sld = k.sscr_ld;
  Mat<double> S = make_mat(scr, (int64_t)1, sld);
  const int r0 = m - klf;
  Mat<double> Tm = make_mat(scr + m, (int64_t)1, sld, r0);
  for (int idx = threadIdx.x; idx < klf * nrhs; idx += NT) {
    int r = r0 + idx % klf, q = idx / klf;
    Tm.at(r, q) = rev ? nv[(m - 1 - r) + (int64_t)q * kw] : nv[ku + (r - r0) + (int64_t)q * kw];
  }
  __syncthreads();
  wg_utsweep<NB, T>(A, Tm, nrhs, r0, lds);
  for (int idx = threadIdx.x; idx < m * nrhs; idx += NT) {
    int r = idx % m, q = idx / m;
    double v = S.at(r, q);
    if (r >= r0) v += Tm.at(r, q);
    X.at(r, q) = v;
  }
  __syncthreads();
  wg_ltsweep<NB, T>(A, X, nrhs, 0, lds);
  note_sweep(k, 2, L.type, klf, m);
  note_sweep(k, 2, L.type, m, m);
}

// ===========================================================================
// Host-side runners (one explicit instantiation per translation unit)
// ===========================================================================
#define SPIKE_CHECK_LAUNCH()                              \
  do {                                                    \
    hipError_t e_ = hipGetLastError();                    \
    if (e_ != hipSuccess) return SPIKE_ERR_HIP - (int)e_; \
  } while (0)

template <typename K>
inline void allow_lds(K kernel, size_t lds) {
  hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int NB, typename T>
int run_leaf_factor(const KParams& k, const LaunchCfg& c, hipStream_t st) {
  allow_lds(k_leaf_factor<NB, T>, c.leaf_lds);
  ProfScope ps("k_leaf_factor", st);
  hipLaunchKernelGGL((k_leaf_factor<NB, T>), dim3(k.p), dim3(NT), c.leaf_lds, st, k);
  SPIKE_CHECK_LAUNCH();
  return 0;
}

template <int NB, typename T>
int run_leaf_phase(const KParams& k, const LaunchCfg& c, hipStream_t st, double* B, int64_t ldb, int nrhs,
                   int phase) {
  switch (phase) {
    case 0: {
      allow_lds(k_leaf_dstage<NB, T>, c.leaf_lds);
      ProfScope ps("k_leaf_dstage", st);
      hipLaunchKernelGGL((k_leaf_dstage<NB, T>), dim3(k.p), dim3(NT), c.leaf_lds, st, k, B, ldb, nrhs);
      break;
    }
    case 1: {
      allow_lds(k_leaf_retrieve<NB, T>, c.leaf_lds);
      ProfScope ps("k_leaf_retrieve", st);
      hipLaunchKernelGGL((k_leaf_retrieve<NB, T>), dim3(k.p), dim3(NT), c.leaf_lds, st, k, B, ldb, nrhs);
      break;
    }
    case 2: {
      allow_lds(k_leaf_zsweep<NB, T>, c.leaf_lds);
      ProfScope ps("k_leaf_zsweep", st);
      hipLaunchKernelGGL((k_leaf_zsweep<NB, T>), dim3(k.p), dim3(NT), c.leaf_lds, st, k, B, ldb, nrhs);
      break;
    }
    default: {
      allow_lds(k_leaf_dtstage<NB, T>, c.leaf_lds);
      ProfScope ps("k_leaf_dtstage", st);
      hipLaunchKernelGGL((k_leaf_dtstage<NB, T>), dim3(k.p), dim3(NT), c.leaf_lds, st, k, B, ldb, nrhs);
      break;
    }
  }
  SPIKE_CHECK_LAUNCH();
  return 0;
}

template <int NBD>
int run_merge_factor(const KParams& k, const LaunchCfg& c, hipStream_t st) {
  allow_lds(k_merge_factor<NBD>, c.merge_lds);
  for (int l = 0; l + 1 < (int)c.level_off.size(); ++l) {
    int beg = c.level_off[l], cnt = c.level_off[l + 1] - beg;
    if (cnt <= 0) continue;
    ProfScope ps("k_merge_factor", st);
    hipLaunchKernelGGL((k_merge_factor<NBD>), dim3(cnt), dim3(NT), c.merge_lds, st, k, beg);
    SPIKE_CHECK_LAUNCH();
  }
  return 0;
}

template <int NBD>
int run_merge_solve(const KParams& k, const LaunchCfg& c, hipStream_t st, int nrhs, bool trans) {
  allow_lds(k_merge_up<NBD>, c.merge_lds);
  allow_lds(k_merge_tdown<NBD>, c.merge_lds);
  allow_lds(k_merge_down, c.merge_lds);
  allow_lds(k_merge_tup, c.merge_lds);
  const int L = (int)c.level_off.size() - 1;
  if (!trans) {
    for (int l = 0; l < L; ++l) {
      int beg = c.level_off[l], cnt = c.level_off[l + 1] - beg;
      ProfScope ps("k_merge_up", st);
      hipLaunchKernelGGL((k_merge_up<NBD>), dim3(cnt), dim3(NT), c.merge_lds, st, k, beg, nrhs);
      SPIKE_CHECK_LAUNCH();
    }
    for (int l = L - 1; l >= 0; --l) {
      int beg = c.level_off[l], cnt = c.level_off[l + 1] - beg;
      ProfScope ps("k_merge_down", st);
      hipLaunchKernelGGL(k_merge_down, dim3(cnt), dim3(NT), c.merge_lds, st, k, beg, nrhs);
      SPIKE_CHECK_LAUNCH();
    }
  } else {
    for (int l = 0; l < L; ++l) {
      int beg = c.level_off[l], cnt = c.level_off[l + 1] - beg;
      ProfScope ps("k_merge_tup", st);
      hipLaunchKernelGGL(k_merge_tup, dim3(cnt), dim3(NT), c.merge_lds, st, k, beg, nrhs);
      SPIKE_CHECK_LAUNCH();
    }
    for (int l = L - 1; l >= 0; --l) {
      int beg = c.level_off[l], cnt = c.level_off[l + 1] - beg;
      ProfScope ps("k_merge_tdown", st);
      hipLaunchKernelGGL((k_merge_tdown<NBD>), dim3(cnt), dim3(NT), c.merge_lds, st, k, beg, nrhs);
      SPIKE_CHECK_LAUNCH();
    }
  }
  return 0;
}

}  // namespace spike
