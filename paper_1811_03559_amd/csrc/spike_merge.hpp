// Recursive reduced system on MFMA tiles (bandwidths up to 256).
//
// Every merge J = (L, R) of the tree owns the interface system
// E_J = [[I, V_b(L)], [W_t(R), I]] (recursive-reduced-system subsection),
// solved through its Schur complement S = I - W_t(R) V_b(L).  A level of the
// tree is factored in five launches, each spread over all merges of the
// level and over 64 x 64 output tiles (or 64-column groups):
//   1. S = I - W_t(R) V_b(L)   and   Dm = -W_t(R) W_b(L)
//   2. P S = L U (partial pivoting, one workgroup per merge), the 16 x 16
//      diagonal-block inverses of L and U and the row permutation
//   3. beta = S^{-1} V_t(R),  delta = S^{-1} Dm   (blocked substitution)
//   4. alpha = -V_b(L) beta,  gamma = W_b(L) - V_b(L) delta, and the top
//      tips of J: V_t = -V_t(L) beta, W_t = W_t(L) - V_t(L) delta
//   5. the bottom tips of J: V_b = V_b(R) - W_b(R) alpha, W_b = -W_b(R) gamma.
// The solve stage uses the same factors: right-hand sides are permuted, then
// swept with L and U (or U^T, L^T and the inverse permutation).
#pragma once
#include "spike_gemv.hpp"
#include "spike_kernels.hpp"
#include "spike_rowlu.hpp"

namespace spike {

// Element-wise copy idx -> (load(idx), store(idx, v)) for idx in [0, total),
// NL loads in flight per thread before their stores (global memory latency
// is paid once per batch, not once per element).
template <int NL, typename LD, typename ST>
__device__ __forceinline__ void batched_copy(int total, LD load, ST store) {
  for (int base = threadIdx.x; base < total; base += NT * NL) {
    double v[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int idx = base + u * NT;
      v[u] = idx < total ? load(idx) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int idx = base + u * NT;
      if (idx < total) store(idx, v[u]);
    }
  }
}

// ------------------------------------------------- fused merge products
// The GEMMs of a merge that share their left operand are one product with
// kw = kl + ku output columns, split into a low part (columns [0, ku)) and a
// high part (columns [ku, kw)) with their own destinations:
//   phase 1:  [S | Dm]            = [I | 0]       - W_t(R) [V_b(L) | W_b(L)]
//   phase 4:  [alpha | gamma]     = [0 | W_b(L)]  - V_b(L) [beta | delta]
//   phase 5a: [V_t(J) | W_t(J)]   = [0 | W_t(L)]  - V_t(L) [beta | delta]
//   phase 5b: [V_b(J) | W_b(J)]   = [V_b(R) | 0]  - W_b(R) [alpha | gamma]
// (phases 4 and 5a need only beta and delta and share one launch).
struct FJob {
  int M, K, on_lo, on_hi, addI;
  const double* A;   // A(i, kk) = A[i + kk lda]
  int64_t lda;
  const double* B;   // B(kk, j) = B[kk + j ldb], j < kw
  int64_t ldb;
  const double* cin_lo;
  const double* cin_hi;
  int64_t ldcin;
  double* c_lo;
  double* c_hi;
  int64_t ldc;
};

__host__ __device__ constexpr int fjobs(int ph) { return ph == 45 ? 2 : 1; }

__device__ inline FJob fused_job(const KParams& k, const MergeDesc& J, int ph, int job) {
  const int kl = k.kl, ku = k.ku, kw = k.kw, mi = J.mif;
  const Tips tp{k.tips, kw, ku};
  const bool nv = J.b < k.p - 1, nw = J.a > 0, root = J.a == 0 && J.b == k.p - 1;
  double* coef = k.coef + (int64_t)mi * kw * kw;
  const int jid = k.p + mi;
  FJob g;
  g.addI = 0;
  g.cin_lo = nullptr;
  g.cin_hi = nullptr;
  g.ldcin = kw;
  g.lda = kw;
  g.ldb = kw;
  g.ldc = kw;
  if (ph == 1) {
    g.M = ku;
    g.K = kl;
    g.A = tp.Wt(J.right);
    g.B = tp.Vb(J.left);   // [V_b(L) | W_b(L)]
    g.c_lo = k.sfac + (int64_t)mi * ku * ku;
    g.c_hi = k.qw + (int64_t)mi * kw * kw;
    g.ldc = ku;
    g.addI = 1;
    g.on_lo = 1;
    g.on_hi = nw;
  } else if (ph == 4 || (ph == 45 && job == 0)) {
    g.M = kl;
    g.K = ku;
    g.A = tp.Vb(J.left);
    g.B = coef + kl;       // [beta | delta]
    g.c_lo = coef;         // alpha
    g.c_hi = coef + (int64_t)ku * kw;   // gamma
    g.cin_hi = tp.Wb(J.left);
    g.on_lo = nv;
    g.on_hi = nw;
  } else if (ph == 45) {
    g.M = ku;
    g.K = ku;
    g.A = tp.Vt(J.left);
    g.B = coef + kl;       // [beta | delta]
    g.c_lo = tp.Vt(jid);
    g.c_hi = tp.Wt(jid);
    g.cin_hi = tp.Wt(J.left);
    g.on_lo = nv && nw && !root;
    g.on_hi = nw && !root;
  } else {   // 5b
    g.M = kl;
    g.K = kl;
    g.A = tp.Wb(J.right);
    g.B = coef;            // [alpha | gamma]
    g.c_lo = tp.Vb(jid);
    g.c_hi = tp.Wb(jid);
    g.cin_lo = tp.Vb(J.right);
    g.on_lo = nv && !root;
    g.on_hi = nv && nw && !root;
  }
  return g;
}

// One 64 x 64 output tile per workgroup; wavefront (wi, wj) owns a 32 x 32
// quarter as 2 x 2 MFMA tiles; K runs in chunks of 16 through double-
// buffered LDS, the next chunk loaded into registers during the current one.
constexpr int FG_T = 64, FG_KC = 16, FG_PAD = FG_T + 1;
template <int PH>
__device__ __forceinline__ void mgemm_body(const KParams& k, const int bx_, const int gx_, int mbeg, int tpj, int tn) {
  using M = Mf<double>;
  __shared__ double As[2][FG_KC * FG_PAD];   // As[kk][i]
  __shared__ double Bs[2][FG_KC * FG_PAD];   // Bs[kk][j]
  constexpr int NJ = fjobs(PH);
  const int b = xcd_grouped(bx_, gx_);
  const int tile = b % tpj, rest = b / tpj;
  const int job = rest % NJ, mm = rest / NJ;
  const MergeDesc J = k.merges[mbeg + mm];
  const FJob g = fused_job(k, J, PH, job);
  const int kw = k.kw, ku = k.ku;
  const int i0 = (tile / tn) * FG_T, j0 = (tile % tn) * FG_T;
  if (i0 >= g.M) return;
  const bool any_lo = g.on_lo && j0 < ku, any_hi = g.on_hi && j0 + FG_T > ku;
  if (!any_lo && !any_hi) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave & 1, wj = wave >> 1, cl = lane & 15, kq = lane >> 4;
  // staging: thread tid loads A(i0 + (e % 64), kc + e / 64) and
  // B(kc + e % 16, j0 + e / 16) for e = tid + 256 u, u < 4
  double ra[4], rb[4];
  auto load = [&](int kc) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + NT * u;
      const int ai = i0 + (e % FG_T), ak = kc + e / FG_T;
      ra[u] = (ai < g.M && ak < g.K) ? g.A[ai + (int64_t)ak * g.lda] : 0.0;
      const int bk = kc + (e % FG_KC), bj = j0 + e / FG_KC;
      rb[u] = (bk < g.K && bj < kw) ? g.B[bk + (int64_t)bj * g.ldb] : 0.0;
    }
  };
  auto store = [&](int b) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + NT * u;
      As[b][(e / FG_T) * FG_PAD + (e % FG_T)] = ra[u];
      Bs[b][(e % FG_KC) * FG_PAD + e / FG_KC] = rb[u];
    }
  };
  M::v4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = M::v4{0.0, 0.0, 0.0, 0.0};
  const int nch = (g.K + FG_KC - 1) / FG_KC;
  if (nch > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int b = ch & 1;
    if (ch + 1 < nch) load((ch + 1) * FG_KC);
#pragma unroll
    for (int k4 = 0; k4 < FG_KC; k4 += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[b][(k4 + kq) * FG_PAD + wi * 32 + a * 16 + cl];
#pragma unroll
      for (int c = 0; c < 2; ++c) bv[c] = Bs[b][(k4 + kq) * FG_PAD + wj * 32 + c * 16 + cl];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][c] = M::mma(av[a], bv[c], acc[a][c]);
    }
    if (ch + 1 < nch) store(b ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + wi * 32 + a * 16 + M::row(lane, q), j = j0 + wj * 32 + c * 16 + cl;
        if (i >= g.M || j >= kw) continue;
        const bool lo = j < ku;
        if (lo ? !g.on_lo : !g.on_hi) continue;
        const int jj = lo ? j : j - ku;
        double v = -acc[a][c][q];
        const double* cin = lo ? g.cin_lo : g.cin_hi;
        if (cin) v += cin[i + (int64_t)jj * g.ldcin];
        if (g.addI && lo && i == jj) v += 1.0;
        (lo ? g.c_lo : g.c_hi)[i + (int64_t)jj * g.ldc] = v;
      }
}
template <int PH>
__global__ __launch_bounds__(NT) void k_mgemm(KParams k, int mbeg, int tpj, int tn) {
  mgemm_body<PH>(k, blockIdx.x, gridDim.x, mbeg, tpj, tn);
}
// the same for up to kMaxBatch systems: workgroup i belongs to system s
// with off[s] <= i < off[s + 1] (its parameter block at kp[s])
template <int PH>
__global__ __launch_bounds__(NT) void k_mgemm_b(BatchArgs ba, int tpj, int tn) {
  const int s = batch_sys(ba, blockIdx.x);
  mgemm_body<PH>(*ba.kp[s], blockIdx.x - ba.off[s], ba.off[s + 1] - ba.off[s], ba.mbeg[s], tpj, tn);
}

// ---------------------------------------------------------------- LU of S
// LDS doubles of k_mlu for order n.
__host__ __device__ constexpr int mlu_lds_elems(int n) { return n * 17 + n * 17 + 16; }

// P S = L U with partial pivoting (ties to the smallest row), interchanges
// applied to whole rows; then the row permutation perm (row i of P S is row
// perm[i] of S) and the 16 x 16 diagonal-block inverses of L and U.
static __global__ __launch_bounds__(NT) void k_mlu(KParams k, int mbeg) {
  using Mq = Mf<double>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  __shared__ int s_pl[256];     // panel-local row permutation
  __shared__ int s_perm[256];   // row permutation of the whole factorisation
  __shared__ int s_mv[64];      // rows that move: destination, then source
  __shared__ int s_nmv;
  __shared__ int s_zero;
  const MergeDesc J = k.merges[mbeg + blockIdx.x];
  const int n = k.ku, mi = J.mif;
  double* S = k.sfac + (int64_t)mi * n * n;
  int* ipiv = k.spiv + (int64_t)mi * n;
  constexpr int PW = 17;
  double* P = lds;                  // panel rows J0..n-1: P[r * PW + c]
  double* Ub = P + (size_t)n * PW;  // U12 columns: Ub[c * PW + t]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_zero = 0;
  for (int i = tid; i < n; i += NT) s_perm[i] = i;

  for (int J0 = 0; J0 < n; J0 += 16) {
    const int jb = min(16, n - J0), rows = n - J0;
    batched_copy<16>(
        rows * 16,
        [&](int idx) {
          const int r = idx % rows, c = idx / rows;
          return c < jb ? S[(J0 + r) + (int64_t)(J0 + c) * n] : 0.0;
        },
        [&](int idx, double v) { P[(idx % rows) * PW + idx / rows] = v; });
    for (int r = tid; r < rows; r += NT) s_pl[r] = r;
    __syncthreads();
    if (wave == 0) {
      for (int t = 0; t < jb; ++t) {
        double best = -1.0;
        int bi = 0x7fffffff;
        for (int r = t + lane; r < rows; r += 64) {
          const double v = fabs(P[r * PW + t]);
          if (v > best) {
            best = v;
            bi = r;
          }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          const double ob = __shfl_xor(best, off);
          const int oi = __shfl_xor(bi, off);
          if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
          }
        }
        if (bi == 0x7fffffff) bi = t;
        if (lane == 0) {
          ipiv[J0 + t] = J0 + bi;
          int a = s_pl[t];
          s_pl[t] = s_pl[bi];
          s_pl[bi] = a;
          a = s_perm[J0 + t];
          s_perm[J0 + t] = s_perm[J0 + bi];
          s_perm[J0 + bi] = a;
        }
        if (bi != t && lane < 16) {
          const double a = P[t * PW + lane];
          P[t * PW + lane] = P[bi * PW + lane];
          P[bi * PW + lane] = a;
        }
        wave_lds_sync();
        const double piv = P[t * PW + t];
        if (piv == 0.0 && lane == 0) s_zero = 1;
        const double rp = piv != 0.0 ? 1.0 / piv : 0.0;
        for (int r = t + 1 + lane; r < rows; r += 64) P[r * PW + t] *= rp;
        wave_lds_sync();
        double urow[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) urow[c] = P[t * PW + c];
        for (int r = t + 1 + lane; r < rows; r += 64) {
          const double l = P[r * PW + t];
#pragma unroll
          for (int c = 0; c < 16; ++c)
            if (c > t && c < jb) P[r * PW + c] -= l * urow[c];
        }
        wave_lds_sync();
      }
      // rows that moved in this panel (at most 2 jb): compact with a ballot
      int base = 0;
      for (int r0 = 0; r0 < rows; r0 += 64) {
        const int r = r0 + lane;
        const bool mv = r < rows && s_pl[r] != r;
        const unsigned long long bal = __ballot(mv);
        if (mv) {
          const int pos = base + __popcll(bal & ((1ull << lane) - 1ull));
          s_mv[pos] = r;
          s_mv[32 + pos] = s_pl[r];
        }
        base += __popcll(bal);
      }
      if (lane == 0) s_nmv = base;
    }
    __syncthreads();
    // the panel back to S; interchanges on the other columns (only the rows
    // that move, at most 32 per column)
    for (int idx = tid; idx < rows * jb; idx += NT) {
      const int r = idx % rows, c = idx / rows;
      S[(J0 + r) + (int64_t)(J0 + c) * n] = P[r * PW + c];
    }
    const int nmv = s_nmv, nother = n - jb;
    constexpr int MAXV = (32 * 256 + NT - 1) / NT;
    double mv[MAXV];
#pragma unroll
    for (int u = 0; u < MAXV; ++u) {
      const int idx = tid + u * NT;
      mv[u] = 0.0;
      if (idx < nmv * nother) {
        const int j = idx % nmv, co = idx / nmv;
        const int c = co < J0 ? co : co + jb;
        mv[u] = S[(J0 + s_mv[32 + j]) + (int64_t)c * n];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MAXV; ++u) {
      const int idx = tid + u * NT;
      if (idx < nmv * nother) {
        const int j = idx % nmv, co = idx / nmv;
        const int c = co < J0 ? co : co + jb;
        S[(J0 + s_mv[j]) + (int64_t)c * n] = mv[u];
      }
    }
    __syncthreads();
    // U12 = L11^{-1} A12 (columns right of the panel), kept in LDS too
    const int ncr = n - J0 - jb;
    for (int cc = tid; cc < ncr; cc += NT) {
      const int c = J0 + jb + cc;
      double x[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) x[t] = t < jb ? S[(J0 + t) + (int64_t)c * n] : 0.0;
#pragma unroll
      for (int t = 1; t < 16; ++t) {
        double sacc = x[t];
#pragma unroll
        for (int q = 0; q < t; ++q) sacc -= P[t * PW + q] * x[q];
        x[t] = sacc;
      }
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        if (t < jb) S[(J0 + t) + (int64_t)c * n] = x[t];
        Ub[cc * PW + t] = t < jb ? x[t] : 0.0;
      }
    }
    __syncthreads();
    // trailing update A22 -= L21 U12 on 16 x 16 tiles
    const int nrt = (rows - jb + 15) / 16, nct = (ncr + 15) / 16;
    constexpr int TB = 6;   // tiles per wavefront whose loads are in flight together
    const int cl = lane & 15, kq = lane >> 4;
    for (int t0 = wave * TB; t0 < nrt * nct; t0 += (NT / 64) * TB) {
      Mq::v4 acc[TB];
#pragma unroll
      for (int u = 0; u < TB; ++u) {
        const int tt = t0 + u, tr = tt % nrt, tc = tt / nrt;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = jb + tr * 16 + Mq::row(lane, q), c = tc * 16 + cl;
          acc[u][q] = (tt < nrt * nct && r < rows && c < ncr) ? S[(J0 + r) + (int64_t)(J0 + jb + c) * n] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < TB; ++u) {
        const int tt = t0 + u, tr = tt % nrt, tc = tt / nrt;
        if (tt >= nrt * nct) continue;
#pragma unroll
        for (int k4 = 0; k4 < 16; k4 += 4) {
          const int ra = jb + tr * 16 + cl;
          const double a = ra < rows ? -P[ra * PW + k4 + kq] : 0.0;
          const int cb = tc * 16 + cl;
          const double b = cb < ncr ? Ub[cb * PW + k4 + kq] : 0.0;
          acc[u] = Mq::mma(a, b, acc[u]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = jb + tr * 16 + Mq::row(lane, q), c = tc * 16 + cl;
          if (r < rows && c < ncr) S[(J0 + r) + (int64_t)(J0 + jb + c) * n] = acc[u][q];
        }
      }
    }
    __syncthreads();
  }
  // permutation: row i of P S is row perm[i] of S
  int* perm = k.sperm + (int64_t)mi * n;
  if (tid == 0 && s_zero) atomicMin(&k.status->iface, (unsigned long long)(mi + 1));
  for (int i = tid; i < n; i += NT) perm[i] = s_perm[i];
  const int nbs = (n + 15) / 16;
  const DenseAcc<double> D{S, n, n - 1, n - 1, n, nullptr};
  diag_inverses<double>(D, k.sdinv + (int64_t)mi * nbs * dinv_stride(), tid, NT);
}

// Register-resident variant for order n <= 64 RS, NWR wavefronts: S lives in
// registers for the whole factorisation (wavefront w holds the columns
// c = w + NWR cs, lane l the rows l + 64 s), so a column step costs one
// workgroup barrier and no global traffic.  Rows are not interchanged while
// eliminating: the pivot of step j is the largest |entry| of column j among
// the rows not yet chosen (ties to the smallest row index), it is marked
// chosen, and every other unchosen row is eliminated against it.  Row r
// chosen at step i becomes row i of P S, so the packed L \ U written out is
// the same as with interchanges.  The wavefront owning column j + 1 updates
// that column first and publishes its pivot and multipliers (double-buffered
// in LDS) before updating its other columns.
constexpr int NWR = 8;
struct MluDiagAcc {   // 16 x 16 diagonal blocks of P S, kept in LDS
  const double* d;
  int m;
  __device__ __forceinline__ double at(int i, int c) const { return d[(i >> 4) * 272 + (i & 15) * 17 + (c & 15)]; }
  __device__ __forceinline__ bool in(int, int) const { return true; }
};

template <int CS, int RS>
__global__ __launch_bounds__(NWR * 64) void k_mlu_reg(KParams k, int mbeg) {
  __shared__ double s_l[2][RS * 64];      // multipliers of the current / next step
  __shared__ int s_p[2];                  // pivot rows
  __shared__ double s_dg[RS * 4 * 272];   // diagonal 16 x 16 blocks of P S
  __shared__ int s_zero;
  const MergeDesc J = k.merges[mbeg + blockIdx.x];
  const int n = k.ku, mi = J.mif;
  double* S = k.sfac + (int64_t)mi * n * n;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
  if (tid == 0) s_zero = 0;

  double a[CS][RS];
  int rstep[RS];        // step at which the row was chosen
  unsigned done = 0;    // bit s: row lane + 64 s chosen, or outside [0, n)
#pragma unroll
  for (int s = 0; s < RS; ++s) {
    rstep[s] = 0;
    if (lane + 64 * s >= n) done |= 1u << s;
  }
#pragma unroll
  for (int cs = 0; cs < CS; ++cs) {
    const int c = w + NWR * cs;
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      const int r = lane + 64 * s;
      a[cs][s] = (c < n && r < n) ? S[r + (int64_t)c * n] : 0.0;
    }
  }

  // pivot and multipliers of this wavefront's column slot CS0 into buffer b
  auto pivot_col = [&](auto CSI, int b) __attribute__((always_inline)) {
    constexpr int cs = decltype(CSI)::value;
    // candidates: |a| of unchosen rows (NaN as -0.5), chosen rows -1; the
    // maximum over the wavefront, then the smallest row holding it
    double v[RS];
    double best = -2.0;
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      double x = fabs(a[cs][s]);
      if (x != x) x = -0.5;
      if (done & (1u << s)) x = -1.0;
      v[s] = x;
      best = fmax(best, x);
    }
    const double vmax = wave_max_f64(best);
    int p = 0;
#pragma unroll
    for (int s = RS - 1; s >= 0; --s) {
      const unsigned long long hit = __ballot(v[s] == vmax);
      if (hit) p = 64 * s + (int)__builtin_ctzll(hit);
    }
    p = __builtin_amdgcn_readfirstlane(p);
    const int sp = p >> 6, lp = p & 63;
    double piv = 0.0;
#pragma unroll
    for (int s = 0; s < RS; ++s)
      if (s == sp) piv = lane_read(a[cs][s], lp);
    if (piv == 0.0 && lane == 0) s_zero = 1;
    const double rp = piv != 0.0 ? 1.0 / piv : 0.0;
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      const int r = lane + 64 * s;
      const bool elim = !(done & (1u << s)) && r != p;
      const double l = elim ? a[cs][s] * rp : 0.0;
      if (elim) a[cs][s] = l;
      s_l[b][r] = l;
    }
    if (lane == 0) s_p[b] = p;
  };
  // rank-1 update of column slot CSI with pivot row (sp, lp) and multipliers l
  auto update = [&](auto CSI, int sp, int lp, const double(&l)[RS]) __attribute__((always_inline)) {
    constexpr int cs = decltype(CSI)::value;
    double u = 0.0;
#pragma unroll
    for (int s = 0; s < RS; ++s)
      if (s == sp) u = lane_read(a[cs][s], lp);
#pragma unroll
    for (int s = 0; s < RS; ++s) a[cs][s] = fma(-l[s], u, a[cs][s]);
  };

  if (w == 0 && n > 0) pivot_col(std::integral_constant<int, 0>{}, 0);   // order 0 (ku = 0): nothing to do
  __syncthreads();
  // step j = NWR cs + t eliminates column j (slot cs of wavefront t)
  static_for<0, CS>([&](auto CSI) __attribute__((always_inline)) {
    constexpr int cs = decltype(CSI)::value;
    for (int t = 0; t < NWR; ++t) {
      const int j = NWR * cs + t;
      if (j >= n) break;
      const int b = j & 1;
      const int p = __builtin_amdgcn_readfirstlane(s_p[b]);
      const int sp = p >> 6, lp = p & 63;
      double l[RS];
#pragma unroll
      for (int s = 0; s < RS; ++s) l[s] = s_l[b][lane + 64 * s];
      if (lane == lp) {
#pragma unroll
        for (int s = 0; s < RS; ++s)
          if (s == sp) {
            done |= 1u << s;
            rstep[s] = j;
          }
      }
      // the owner of column j + 1 updates it and publishes its pivot first
      const bool ahead = j + 1 < n && w == (t + 1) % NWR;
      const bool ahead_here = ahead && t + 1 < NWR;   // column j + 1 in slot cs
      if (ahead_here) {
        update(CSI, sp, lp, l);
        pivot_col(CSI, b ^ 1);
      }
      if constexpr (cs + 1 < CS) {
        if (ahead && !ahead_here) {
          update(std::integral_constant<int, cs + 1>{}, sp, lp, l);
          pivot_col(std::integral_constant<int, cs + 1>{}, b ^ 1);
        }
      }
      // the other columns right of j
      if (w > t && !ahead_here && w + NWR * cs < n) update(CSI, sp, lp, l);
      static_for<cs + 1, CS>([&](auto C2) __attribute__((always_inline)) {
        constexpr int c2 = decltype(C2)::value;
        if (w + NWR * c2 < n && !(ahead && !ahead_here && c2 == cs + 1)) update(C2, sp, lp, l);
      });
      __syncthreads();
    }
  });

  // write P S = L U packed, the permutation and the diagonal blocks
  int* perm = k.sperm + (int64_t)mi * n;
#pragma unroll
  for (int s = 0; s < RS; ++s) {
    const int r = lane + 64 * s;
    if (r < n) perm[rstep[s]] = r;
  }
#pragma unroll
  for (int cs = 0; cs < CS; ++cs) {
    const int c = w + NWR * cs;
    if (c >= n) continue;
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      const int r = lane + 64 * s, i = rstep[s];
      if (r < n) {
        S[i + (int64_t)c * n] = a[cs][s];
        if ((i >> 4) == (c >> 4)) s_dg[(i >> 4) * 272 + (i & 15) * 17 + (c & 15)] = a[cs][s];
      }
    }
  }
  __syncthreads();
  if (tid == 0 && s_zero) atomicMin(&k.status->iface, (unsigned long long)(mi + 1));
  const int nbs = (n + 15) / 16;
  diag_inverses<double>(MluDiagAcc{s_dg, n}, k.sdinv + (int64_t)mi * nbs * dinv_stride(), tid, NWR * 64);
}

// Blocked variant for order n <= 16 NBT: the same pivot rule as k_mlu_reg
// (the pivot of step j is the largest |entry| of column j among the rows not
// yet chosen, ties to the smallest row index; no rows move, and the row
// chosen at step i becomes row i of P S), with the rank-1 updates gathered
// into rank-16 products on the matrix cores.  Wavefront w < nb (nb = the
// number of 16-column blocks) holds column block w of S as 16 x 16 MFMA
// tiles; one more wavefront factors the blocks, one at a time, with one row
// per lane and slot in registers (no workgroup barrier inside a block).  For
// block J it publishes the multipliers of every row, masked so that rows
// chosen in earlier blocks get none and the row chosen at step t of the
// block keeps only those of steps < t, and the inverse of the unit lower
// triangle L11 of the block's pivot rows.  Every wavefront right of the
// block then forms U12 = L11^{-1} (its pivot rows) and subtracts
// (multipliers) x U12 from all its tiles, which leaves U12 in the pivot rows
// and the Schur complement elsewhere; tiles whose rows were all chosen in
// earlier blocks are skipped.  The owner of block J + 1 updates first and
// hands it to the factoring wavefront through LDS; the others update while
// the factoring wavefront works on block J + 1.  Two workgroup barriers per
// block.  The factoring wavefront runs its own loop, so the registers of its
// panel and of the others' tiles are never live together.  At the end every
// block wavefront inverts its diagonal block of P S on the matrix cores.
constexpr int MLB_PW = 17;   // LDS pitch of a 16-wide row
template <int NBT>
__host__ __device__ constexpr size_t mlu_blk_lds_bytes() {
  // Lm[2], Lp[2] (16 NBT rows each), Li[2], one tile per wavefront, the
  // pivot row; slot[2], rstep, pvt[2], live tiles[2], zero flag
  return (size_t)(4 * 16 * NBT * MLB_PW + 2 * 16 * MLB_PW + (NBT + 1) * 16 * MLB_PW + 16) * 8 +
         (size_t)(2 * 16 * NBT + 16 * NBT + 32 + 2 * NBT + 1) * 4;
}

template <int NBT>
__device__ __forceinline__ void mlu_blk_body(const KParams& k, const int bx_, const int gx_, int mbeg) {
  using Mq = Mf<double>;
  using v4 = Mq::v4;
  constexpr int NMAX = 16 * NBT, PW = MLB_PW, TS = 16 * PW, BUF = NMAX * PW;
  constexpr int RS = (NMAX + 63) / 64;   // row slots per lane in the panel layout
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* Lm = reinterpret_cast<double*>(smem_raw);   // [2][BUF] masked multipliers
  double* Lp = Lm + 2 * BUF;                           // [2][BUF] the block being factored / factored
  double* Li = Lp + 2 * BUF;                           // [2][TS] L11^{-1}
  double* Gt = Li + 2 * TS;                            // [NBT + 1][TS] one tile per wavefront
  double* rowbuf = Gt + (NBT + 1) * TS;                // [16] pivot row
  int* slot = reinterpret_cast<int*>(rowbuf + 16);     // [2][NMAX] step of a block's pivot row, else -1
  int* rstep = slot + 2 * NMAX;                        // [NMAX] step a row was chosen, -1 open, -2 padding
  int* pvt = rstep + NMAX;                             // [2][16] pivot rows of a block
  int* tlive = pvt + 32;                               // [2][NBT] tile has a row open before the block
  int* zflag = tlive + 2 * NBT;

  const MergeDesc Jm = k.merges[mbeg + bx_];
  const int n = k.ku, mi = Jm.mif;
  const int nbk = (n + 15) / 16;
  double* S = k.sfac + (int64_t)mi * n * n;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const v4 zero = {0.0, 0.0, 0.0, 0.0};
  if (tid == 0) *zflag = 0;
  for (int r = tid; r < NMAX; r += blockDim.x) rstep[r] = r < n ? -1 : -2;

  // (lane-derived indices go through opaque() so that the addresses are
  // formed where they are used, not hoisted out of the block loop and kept)
  auto mm = [&](const double* P, const v4& b, v4 d) __attribute__((always_inline)) -> v4 {
    const int ln = opaque(lane);
#pragma unroll
    for (int q = 0; q < 4; ++q) d = Mq::mma(P[(ln & 15) * PW + Mq::row(ln, q)], b[q], d);
    return d;
  };
  auto put = [&](double* P, const v4& v) __attribute__((always_inline)) {
    const int ln = opaque(lane);
#pragma unroll
    for (int q = 0; q < 4; ++q) P[Mq::row(ln, q) * PW + (ln & 15)] = v[q];
  };
  // (I + N)^{-1} = (I - N)(I + N^2)(I + N^4)(I + N^8) for a strictly
  // triangular 16 x 16 N (nilpotent: N^16 = 0), G a tile of scratch
  auto unit_inv = [&](const v4& N, double* G) __attribute__((always_inline)) -> v4 {
    const int ln = opaque(lane);
    v4 X, P = N;
#pragma unroll
    for (int q = 0; q < 4; ++q) X[q] = (Mq::row(ln, q) == (ln & 15) ? 1.0 : 0.0) - N[q];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      put(G, P);
      wave_lds_sync();
      P = mm(G, P, zero);
      wave_lds_sync();
      put(G, P);
      wave_lds_sync();
      X = mm(G, X, X);
      wave_lds_sync();
    }
    return X;
  };

  if (w == nbk) {
    // ---- the factoring wavefront
    __syncthreads();   // block 0 in Lp[0]
    for (int J = 0; J < nbk; ++J) {
      const int bb = J & 1, jb = min(16, n - 16 * J), s0 = 16 * J;
      double* Lpb = Lp + bb * BUF;
      double pr[RS][16];
      unsigned rch = 0;   // which of this lane's rows are chosen (or padding)
      {
        const int ln = opaque(lane);
#pragma unroll
        for (int s = 0; s < RS; ++s) {
          const int r = ln + 64 * s;
          const bool in = r < NMAX;
#pragma unroll
          for (int c = 0; c < 16; ++c) pr[s][c] = in ? Lpb[r * PW + c] : 0.0;
          if (!in || rstep[in ? r : 0] != -1) rch |= 1u << s;
        }
      }
      static_for<0, 16>([&](auto TI) __attribute__((always_inline)) {
        constexpr int t = decltype(TI)::value;
        if (t < jb) {
          double v[RS];
          double best = -2.0;
#pragma unroll
          for (int s = 0; s < RS; ++s) {
            double x = fabs(pr[s][t]);
            if (x != x) x = -0.5;
            if (rch & (1u << s)) x = -1.0;
            v[s] = x;
            best = fmax(best, x);
          }
          const double vmax = wave_max_f64(best);
          int p = 0;
#pragma unroll
          for (int s = RS - 1; s >= 0; --s) {
            const unsigned long long hit = __ballot(v[s] == vmax);
            if (hit) p = 64 * s + (int)__builtin_ctzll(hit);
          }
          p = __builtin_amdgcn_readfirstlane(p);
          const int sp = p >> 6, lp = p & 63;
          const int l0 = opaque(lane);
          // the pivot row through LDS (a uniform branch picks its slot)
#pragma unroll
          for (int s = 0; s < RS; ++s) {
            if (s == sp) {
              if (l0 == lp) {
#pragma unroll
                for (int c = t; c < 16; ++c) rowbuf[c] = pr[s][c];
              }
              if (l0 == lp) rch |= 1u << s;
            }
          }
          wave_lds_sync();
          const double piv = rowbuf[t];
          if (l0 == 0) {
            if (piv == 0.0) *zflag = 1;
            rstep[p] = s0 + t;
            pvt[bb * 16 + t] = p;
          }
          const double rp = piv != 0.0 ? recip(piv) : 0.0;
          double l[RS];
#pragma unroll
          for (int s = 0; s < RS; ++s) {
            const bool open = !(rch & (1u << s));
            l[s] = open ? pr[s][t] * rp : 0.0;
            pr[s][t] = open ? l[s] : pr[s][t];
            // settled here: otherwise the compiler keeps every step's
            // multipliers and old column values alive to the end of the block
            asm volatile("" : "+v"(pr[s][t]));
          }
#pragma unroll
          for (int c = t + 1; c < 16; ++c) {
            const double uc = rowbuf[c];
#pragma unroll
            for (int s = 0; s < RS; ++s) pr[s][c] = fma(-l[s], uc, pr[s][c]);
          }
          wave_lds_sync();
        }
      });
      // the block's final values, the masked multipliers and the pivot steps
      double* Lmb = Lm + bb * BUF;
      if (lane < NBT) tlive[bb * NBT + lane] = 0;
      wave_lds_sync();
      {
        const int ln = opaque(lane);
#pragma unroll
        for (int s = 0; s < RS; ++s) {
          const int r = ln + 64 * s;
          if (r < NMAX) {
            const int rs_ = rstep[r];
            const bool old = rs_ != -1 && rs_ < s0;
            const int tt = rs_ >= s0 ? rs_ - s0 : 16;
#pragma unroll
            for (int c = 0; c < 16; ++c) {
              Lpb[r * PW + c] = pr[s][c];
              Lmb[r * PW + c] = (old || c >= tt) ? 0.0 : pr[s][c];
            }
            slot[bb * NMAX + r] = rs_ >= s0 ? tt : -1;
            if (!old) tlive[bb * NBT + (r >> 4)] = 1;
          }
        }
      }
      wave_lds_sync();
      // L11^{-1}, N(t, s) the multiplier of the block's pivot row t at step s < t
      double* G = Gt + NBT * TS;   // this wavefront's own tile
      v4 N;
      {
        const int ln = opaque(lane);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int tq = Mq::row(ln, q), c3 = ln & 15;
          const int prow = tq < jb ? pvt[bb * 16 + tq] : 0;
          N[q] = (c3 < tq && tq < jb) ? Lpb[prow * PW + c3] : 0.0;
        }
      }
      const v4 X = unit_inv(N, G);
      put(Li + bb * TS, X);
      __syncthreads();   // block J published
      if (J + 1 < nbk) __syncthreads();   // block J + 1 in Lp[bb ^ 1]
    }
  } else if (w < nbk) {
    // ---- a block wavefront
    double* G = Gt + w * TS;
    v4 acc[NBT];
    {
      const int ln = opaque(lane);
#pragma unroll
      for (int R = 0; R < NBT; ++R)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = 16 * R + Mq::row(ln, q), c = 16 * w + (ln & 15);
          acc[R][q] = (r < n && c < n) ? S[r + (int64_t)c * n] : 0.0;
        }
    }
    if (w == 0) {
#pragma unroll
      for (int R = 0; R < NBT; ++R) put(Lp + R * TS, acc[R]);
    }
    __syncthreads();   // block 0 in Lp[0]
    // block J's rank-16 update of this wavefront's tiles (buffer b)
    auto update = [&](int J, int b) __attribute__((always_inline)) {
      const int jb = min(16, n - 16 * J);
      const double* Lmb = Lm + b * BUF;
      const int* sl = slot + b * NMAX;
      {
        // the block's pivot rows of this wavefront's columns into G (row = step)
        const int ln = opaque(lane), c4 = ln & 15;
#pragma unroll
        for (int R = 0; R < NBT; ++R)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int t = sl[16 * R + Mq::row(ln, q)];
            if (t >= 0) G[t * PW + c4] = acc[R][q];
          }
      }
      wave_lds_sync();
      v4 a12;
      {
        const int ln = opaque(lane), c4 = ln & 15;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int tq = Mq::row(ln, q);
          a12[q] = tq < jb ? G[tq * PW + c4] : 0.0;
        }
      }
      const v4 u12 = mm(Li + b * TS, a12, zero);
      {
        const int ln = opaque(lane);
#pragma unroll
        for (int R = 0; R < NBT; ++R) {
          if (R < nbk && tlive[b * NBT + R]) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              acc[R] = Mq::mma(-Lmb[(16 * R + (ln & 15)) * PW + Mq::row(ln, q)], u12[q], acc[R]);
          }
        }
      }
      wave_lds_sync();
    };
    for (int J = 0; J < nbk; ++J) {
      const int b = J & 1;
      __syncthreads();   // block J published
      if (w == J) {
        // the factored block back (whole vectors: the values before are dead)
        const int ln = opaque(lane);
        const double* Lpb = Lp + b * BUF;
#pragma unroll
        for (int R = 0; R < NBT; ++R) {
          const double* Lr = Lpb + (16 * R) * PW + (ln & 15);
          acc[R] = v4{Lr[Mq::row(ln, 0) * PW], Lr[Mq::row(ln, 1) * PW], Lr[Mq::row(ln, 2) * PW],
                      Lr[Mq::row(ln, 3) * PW]};
        }
      } else if (w == J + 1) {
        update(J, b);
#pragma unroll
        for (int R = 0; R < NBT; ++R) put(Lp + (b ^ 1) * BUF + R * TS, acc[R]);
      }
      if (J + 1 < nbk) __syncthreads();   // block J + 1 in Lp[b ^ 1]
      if (w > J + 1) update(J, b);        // meanwhile block J + 1 is factored
    }
    // P S = L U packed: row rstep[r] of the output is row r of S
    {
      const int ln = opaque(lane);
#pragma unroll
      for (int R = 0; R < NBT; ++R)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = 16 * R + Mq::row(ln, q), c = 16 * w + (ln & 15);
          if (r < n && c < n) S[rstep[r] + (int64_t)c * n] = acc[R][q];
        }
    }
    // the inverses of the unit lower and of the upper triangle of diagonal
    // block w of P S (the identity beyond the order), for the sweeps
    {
      const int ln = opaque(lane), c4 = ln & 15;
#pragma unroll
      for (int R = 0; R < NBT; ++R)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = 16 * R + Mq::row(ln, q);
          if (r < n) {
            const int i = rstep[r];
            if ((i >> 4) == w) G[(i & 15) * PW + c4] = acc[R][q];
          }
        }
      wave_lds_sync();
      v4 Dg;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i16 = Mq::row(ln, q);
        const bool in = 16 * w + i16 < n && 16 * w + c4 < n;
        Dg[q] = in ? G[i16 * PW + c4] : (i16 == c4 ? 1.0 : 0.0);
      }
      wave_lds_sync();
      put(G, Dg);
      wave_lds_sync();
      // lane t < 16: column t of L^{-1} by forward substitution; lane 16 + t:
      // column t of U^{-1} by back substitution (the block read from LDS)
      double* Dv = k.sdinv + ((int64_t)mi * ((n + 15) / 16) + w) * dinv_stride();
      const int t = ln & 15;
      double x[16];
      if (ln < 16) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          double a = (r == t) ? 1.0 : 0.0;
#pragma unroll
          for (int q = 0; q < r; ++q) a = fma(-G[r * PW + q], x[q], a);
          x[r] = a;
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) Dv[r * 16 + t] = x[r];
      } else if (ln < 32) {
#pragma unroll
        for (int r = 15; r >= 0; --r) {
          double a = (r == t) ? 1.0 : 0.0;
#pragma unroll
          for (int q = r + 1; q < 16; ++q) a = fma(-G[r * PW + q], x[q], a);
          x[r] = a / G[r * PW + r];
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) Dv[256 + r * 16 + t] = x[r];
      }
    }
  } else {
    // ---- wavefronts beyond the blocks (n = 0): the same barriers
    __syncthreads();
    for (int J = 0; J < nbk; ++J) {
      __syncthreads();
      if (J + 1 < nbk) __syncthreads();
    }
  }
  __syncthreads();
  // the permutation (row i of P S is row perm[i] of S)
  int* perm = k.sperm + (int64_t)mi * n;
  for (int r = tid; r < n; r += blockDim.x) perm[rstep[r]] = r;
  if (tid == 0 && *zflag) atomicMin(&k.status->iface, (unsigned long long)(mi + 1));
}
template <int NBT>
__global__ __launch_bounds__(64 * (NBT + 1)) void k_mlu_blk(KParams k, int mbeg) {
  mlu_blk_body<NBT>(k, blockIdx.x, gridDim.x, mbeg);
}
// the same for up to kMaxBatch systems: workgroup i belongs to system s
// with off[s] <= i < off[s + 1] (its parameter block at kp[s])
template <int NBT>
__global__ __launch_bounds__(64 * (NBT + 1)) void k_mlu_blk_b(BatchArgs ba) {
  const int s = batch_sys(ba, blockIdx.x);
  mlu_blk_body<NBT>(*ba.kp[s], blockIdx.x - ba.off[s], ba.off[s + 1] - ba.off[s], ba.mbeg[s]);
}

// ------------------------------------------------------- beta, delta solves
// LDS doubles of k_mtrsm<HT>.
template <int HT>
__host__ __device__ constexpr int mtrsm_lds_elems() {
  return tile_lds_elems(HT);
}

// logical workgroup (merge * 2 + job) * ncg + cg; job 0: beta = S^{-1} V_t(R),
// job 1: delta = S^{-1} Dm; columns [64 cg, 64 cg + 64).
template <int HT>
__device__ __forceinline__ void mtrsm_body(const KParams& k, const int bx_, const int gx_, int mbeg, int ncg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  const int b = xcd_grouped(bx_, gx_);
  const int cg = b % ncg, rest = b / ncg;
  const int job = rest % 2, mm = rest / 2;
  const MergeDesc J = k.merges[mbeg + mm];
  const int kl = k.kl, ku = k.ku, kw = k.kw, mi = J.mif;
  const bool nv = J.b < k.p - 1, nw = J.a > 0;
  if (job == 0 ? !nv : !nw) return;
  const int ncol = job == 0 ? ku : kl;
  const int c0 = 64 * cg;
  if (c0 >= ncol) return;
  const Tips tp{k.tips, kw, ku};
  double* C = k.coef + (int64_t)mi * kw * kw;
  double* X = job == 0 ? C + kl : C + kl + (int64_t)ku * kw;   // ld kw
  const double* src = job == 0 ? tp.Vt(J.right) : k.qw + (int64_t)mi * kw * kw;
  const int64_t lds_src = job == 0 ? kw : ku;
  const int* perm = k.sperm + (int64_t)mi * ku;
  const int cw = min(64, ncol - c0);
  batched_copy<20>(
      ku * cw, [&](int idx) { return src[perm[idx % ku] + (int64_t)(c0 + idx / ku) * lds_src]; },
      [&](int idx, double v) { X[idx % ku + (int64_t)(c0 + idx / ku) * kw] = v; });
  __syncthreads();
  const DenseAcc<double> D{k.sfac + (int64_t)mi * ku * ku, ku, ku - 1, ku - 1, ku, nullptr};
  const double* dv = k.sdinv + (int64_t)mi * ((ku + 15) / 16) * dinv_stride();
  const TSrc s = tsrc(X, 1, 1, kw, 0, ku);
  const TDst d = tdst(X, nullptr, 1, 1, kw, ku, ku, ku);
  tile_sweep<double, HT, OP_L_FWD>(D, dv, s, d, c0, ncol, lds);
  tile_sweep<double, HT, OP_U_BWD>(D, dv, s, d, c0, ncol, lds);
}
template <int HT>
__global__ __launch_bounds__(NT) void k_mtrsm(KParams k, int mbeg, int ncg) {
  mtrsm_body<HT>(k, blockIdx.x, gridDim.x, mbeg, ncg);
}
// the same for up to kMaxBatch systems: workgroup i belongs to system s
// with off[s] <= i < off[s + 1] (its parameter block at kp[s])
template <int HT>
__global__ __launch_bounds__(NT) void k_mtrsm_b(BatchArgs ba, int ncg) {
  const int s = batch_sys(ba, blockIdx.x);
  mtrsm_body<HT>(*ba.kp[s], blockIdx.x - ba.off[s], ba.off[s + 1] - ba.off[s], ba.mbeg[s], ncg);
}

// ---------------------------------------------------------------- solves
// C = alpha A B + beta C with few columns (N <= 8): one thread per entry.
__device__ inline void wg_gemm_nr(int M, int N, int K, double alpha, GM A, GM B, double beta, double* C,
                                  int64_t ldc) {
  for (int idx = threadIdx.x; idx < M * N; idx += NT) {
    const int i = idx % M, j = idx / M;
    const double* ap = A.p + (int64_t)i * A.rs;
    const double* bp = B.p + (int64_t)j * B.cs;
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int kk = 0;
    for (; kk + 7 < K; kk += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] += ap[(int64_t)(kk + u) * A.cs] * bp[(int64_t)(kk + u) * B.rs];
    }
    for (; kk < K; ++kk) a[0] += ap[(int64_t)kk * A.cs] * bp[(int64_t)kk * B.rs];
    const double sum = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    double* c = C + i + (int64_t)j * ldc;
    *c = (beta == 0.0 ? 0.0 : beta * *c) + alpha * sum;
  }
  __syncthreads();
}

// LDS doubles every reduced-solve launch provides (at least).
constexpr int kMsolveLds = 2 * 16 * 65;

// Sum of v over the wavefront, returned uniformly: row shifts within rows of
// 16 lanes, then the row broadcasts, into lane 63 (lanes without a source
// add zero); a fixed order, so the result repeats bitwise.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add_step(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
  const int slo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xf, false);
  const int shi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xf, false);
  return v + __longlong_as_double(((long long)shi << 32) | (long long)(unsigned int)slo);
}
__device__ __forceinline__ double wave_sum_f64(double v) {
  v = dpp_add_step<0x111, 0xf>(v);   // row_shr:1
  v = dpp_add_step<0x112, 0xf>(v);   // row_shr:2
  v = dpp_add_step<0x114, 0xf>(v);   // row_shr:4
  v = dpp_add_step<0x118, 0xf>(v);   // row_shr:8
  v = dpp_add_step<0x142, 0xa>(v);   // row_bcast:15
  v = dpp_add_step<0x143, 0xc>(v);   // row_bcast:31
  return lane_read(v, 63);
}

// y = alpha A x + beta y for one right-hand side, bound by the latency of
// reading A (a k x k block of the reduced system): x is staged in LDS and
// every lane keeps up to 40 loads of A in flight before using them.
// Column-major A (rs = 1): lanes run over rows, the four wavefronts over
// quarters of K, partial sums combined through LDS; row-major A (cs = 1):
// a wavefront takes 8 rows at a time with its lanes across K, then sums each
// row over the wavefront.  Needs K + 4 M <= kMsolveLds doubles of LDS (the
// caller checks); starts after and ends with a barrier.
__device__ inline void wg_gemv(int M, int K, double alpha, GM A, const double* x, double beta, double* y,
                               double* lds) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* xl = lds;
  double* part = lds + K;
  for (int kk = tid; kk < K; kk += NT) xl[kk] = gld(x + kk);
  __syncthreads();
  constexpr int LB = 40;   // loads in flight per lane
  if (A.rs == 1) {
    const int kq = (K + 3) / 4, nrc = (M + 63) / 64;
    for (int it = wave; it < 4 * nrc; it += NT / 64) {
      const int q = it % 4, i = 64 * (it / 4) + lane;
      const int k0 = q * kq, k1 = min(K, k0 + kq);
      const bool row_ok = i < M;
      double a4[4] = {0.0, 0.0, 0.0, 0.0};
      for (int kb = k0; kb < k1; kb += LB) {
        double v[LB];
#pragma unroll
        for (int u = 0; u < LB; ++u) {
          const int kk = kb + u;
          v[u] = (row_ok && kk < k1) ? gld(A.p + i + (int64_t)kk * A.cs) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < LB; ++u) {
          const int kk = kb + u;
          if (kk < k1) a4[u & 3] = fma(v[u], sld(xl + kk), a4[u & 3]);
        }
      }
      if (row_ok) part[q * M + i] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
    }
    __syncthreads();
    for (int i = tid; i < M; i += NT) {
      const double sum = (part[i] + part[M + i]) + (part[2 * M + i] + part[3 * M + i]);
      y[i] = (beta == 0.0 ? 0.0 : beta * y[i]) + alpha * sum;
    }
  } else {
    constexpr int RW = 8;                  // rows per wavefront pass
    const int nkb = (K + 63) / 64;         // loads per row and lane
    for (int i0 = RW * wave; i0 < M; i0 += RW * (NT / 64)) {
      double acc[RW];
#pragma unroll
      for (int r = 0; r < RW; ++r) acc[r] = 0.0;
      for (int kb0 = 0; kb0 < nkb; kb0 += LB / RW) {
        double v[RW][LB / RW];
#pragma unroll
        for (int r = 0; r < RW; ++r)
#pragma unroll
          for (int u = 0; u < LB / RW; ++u) {
            const int kk = 64 * (kb0 + u) + lane, i = i0 + r;
            v[r][u] = (i < M && kk < K) ? gld(A.p + (int64_t)i * A.rs + kk) : 0.0;
          }
#pragma unroll
        for (int u = 0; u < LB / RW; ++u) {
          const int kk = 64 * (kb0 + u) + lane;
          const double xv = kk < K ? sld(xl + kk) : 0.0;
#pragma unroll
          for (int r = 0; r < RW; ++r) acc[r] = fma(v[r][u], xv, acc[r]);
        }
      }
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        const double sum = wave_sum_f64(acc[r]);
        const int i = i0 + r;
        if (lane == 0 && i < M) y[i] = (beta == 0.0 ? 0.0 : beta * y[i]) + alpha * sum;
      }
    }
  }
  __syncthreads();
}

// Products of the reduced solve: one column on the latency-bound gemv (or
// per-thread dot products where its LDS does not suffice), up to 16 columns
// on one MFMA column tile, more in groups of 16.
__device__ __forceinline__ void mgemm_any(int M, int N, int K, double alpha, GM A, GM B, double beta, double* C,
                                          int64_t ldc, double* lds) {
  if (N == 1) {
    if (B.rs == 1 && (A.rs == 1 || A.cs == 1) && K + 4 * M <= kMsolveLds)
      wg_gemv(M, K, alpha, A, B.p, beta, C, lds);
    else
      wg_gemm_nr(M, N, K, alpha, A, B, beta, C, ldc);
    return;
  }
  for (int c0 = 0; c0 < N; c0 += 16) {
    wg_gemm16x<double>(M, min(16, N - c0), K, alpha, A.p, A.rs, A.cs, B.p + (int64_t)c0 * B.cs, B.rs, B.cs, beta,
                       C + (int64_t)c0 * ldc, 1, ldc);
  }
}

// Bottom-up pass of the reduced solve at merge J (see k_merge_up), with
// S^{-1} applied as U^{-1} L^{-1} P.
template <int HT>
__device__ void mup_body(const KParams& k, int d, int c0, int nrhs, double* lds) {
  if (solve_idle(k)) return;
  const MergeDesc J = k.merges[d];
  const int kl = k.kl, ku = k.ku, kw = k.kw, mi = J.mif, R = k.R;
  const int64_t co = (int64_t)c0 * kw;   // first right-hand side of this column group
  const Tips tp{k.tips, kw, ku};
  double* nvl = k.nodeval + (int64_t)J.left * kw * R + co;
  double* nvr = k.nodeval + (int64_t)J.right * kw * R + co;
  double* nvj = k.nodeval + (int64_t)(k.p + mi) * kw * R + co;
  double* s = k.st + (int64_t)mi * kw * R + co;
  double* t = s + kl;
  double* tmp = k.mtmp + (int64_t)mi * kw * R + co;
  const int* perm = k.sperm + (int64_t)mi * ku;
  wg_copy(ku, nrhs, nvr, kw, t, kw);
  wg_copy(kl, nrhs, nvl + ku, kw, s, kw);
  __syncthreads();
  mgemm_any(ku, nrhs, kl, -1.0, gm(tp.Wt(J.right), 1, kw), gm(s, 1, kw), 1.0, t, kw, lds);
  for (int idx = threadIdx.x; idx < ku * nrhs; idx += NT) {
    const int i = idx % ku, q = idx / ku;
    tmp[i + (int64_t)q * kw] = t[perm[i] + (int64_t)q * kw];
  }
  __syncthreads();
  const DenseAcc<double> D{k.sfac + (int64_t)mi * ku * ku, ku, ku - 1, ku - 1, ku, nullptr};
  const double* dv = k.sdinv + (int64_t)mi * ((ku + 15) / 16) * dinv_stride();
  leaf_sweep<double, HT, OP_L_FWD>(D, dv, tsrc(tmp, 1, 1, kw, 0, ku), tdst(tmp, nullptr, 1, 1, kw, ku, ku, ku), 0,
                                   nrhs, lds);
  leaf_sweep<double, HT, OP_U_BWD>(D, dv, tsrc(tmp, 1, 1, kw, 0, ku), tdst(t, nullptr, 1, 1, kw, ku, ku, ku), 0,
                                   nrhs, lds);
  __syncthreads();
  mgemm_any(kl, nrhs, ku, -1.0, gm(tp.Vb(J.left), 1, kw), gm(t, 1, kw), 1.0, s, kw, lds);
  if (J.a > 0) {
    wg_copy(ku, nrhs, nvl, kw, nvj, kw);
    __syncthreads();
    mgemm_any(ku, nrhs, ku, -1.0, gm(tp.Vt(J.left), 1, kw), gm(t, 1, kw), 1.0, nvj, kw, lds);
  }
  if (J.b < k.p - 1) {
    wg_copy(kl, nrhs, nvr + ku, kw, nvj + ku, kw);
    __syncthreads();
    mgemm_any(kl, nrhs, kl, -1.0, gm(tp.Wb(J.right), 1, kw), gm(s, 1, kw), 1.0, nvj + ku, kw, lds);
  }
}

// Top-down pass: interface values of J from its children's (see k_merge_down).
__device__ inline void mdown_body(const KParams& k, int d, int c0, int nrhs, double* lds) {
  if (solve_idle(k)) return;
  const MergeDesc J = k.merges[d];
  const int kl = k.kl, ku = k.ku, kw = k.kw, mi = J.mif, R = k.R;
  const int64_t co = (int64_t)c0 * kw;   // first right-hand side of this column group
  double* x = k.xint + (int64_t)mi * kw * R + co;
  const double* C = k.coef + (int64_t)mi * kw * kw;
  wg_copy(kw, nrhs, k.st + (int64_t)mi * kw * R + co, kw, x, kw);
  __syncthreads();
  if (J.b < k.p - 1)
    mgemm_any(kw, nrhs, ku, -1.0, gm(C, 1, kw), gm(k.xint + (int64_t)J.b * kw * R + kl + co, 1, kw), 1.0, x, kw, lds);
  if (J.a > 0)
    mgemm_any(kw, nrhs, kl, -1.0, gm(C + (int64_t)ku * kw, 1, kw), gm(k.xint + (int64_t)(J.a - 1) * kw * R + co, 1, kw),
              1.0, x, kw, lds);
}

// Transposed reduced solve, first pass (see k_merge_tup).
__device__ inline void mtup_body(const KParams& k, int d, int c0, int nrhs, double* lds) {
  if (solve_idle(k)) return;
  const MergeDesc J = k.merges[d];
  const int kl = k.kl, ku = k.ku, kw = k.kw, mi = J.mif, R = k.R;
  const int64_t co = (int64_t)c0 * kw;   // first right-hand side of this column group
  double* x = k.xint + (int64_t)mi * kw * R + co;
  for (int ci = k.cptr[mi]; ci < k.cptr[mi + 1]; ++ci) {
    const Contrib c = k.contrib[ci];
    const double* cr = k.crl + (int64_t)c.merge * kw * R + co;
    if (c.kind == 0) {
      for (int idx = threadIdx.x; idx < ku * nrhs; idx += NT) {
        const int r = idx % ku, q = idx / ku;
        x[kl + r + (int64_t)q * kw] -= cr[r + (int64_t)q * kw];
      }
    } else {
      for (int idx = threadIdx.x; idx < kl * nrhs; idx += NT) {
        const int r = idx % kl, q = idx / kl;
        x[r + (int64_t)q * kw] -= cr[ku + r + (int64_t)q * kw];
      }
    }
    __syncthreads();
  }
  wg_copy(kw, nrhs, x, kw, k.st + (int64_t)mi * kw * R + co, kw);
  const double* C = k.coef + (int64_t)mi * kw * kw;
  double* out = k.crl + (int64_t)d * kw * R + co;
  if (J.b < k.p - 1) mgemm_any(ku, nrhs, kw, 1.0, gm(C, kw, 1), gm(x, 1, kw), 0.0, out, kw, lds);
  if (J.a > 0) mgemm_any(kl, nrhs, kw, 1.0, gm(C + (int64_t)ku * kw, kw, 1), gm(x, 1, kw), 0.0, out + ku, kw, lds);
}

// Transposed reduced solve, second pass (see k_merge_tdown), with S^{-T}
// applied as P^T L^{-T} U^{-T}.
template <int HT>
__device__ void mtdown_body(const KParams& k, int d, int c0, int nrhs, double* lds) {
  if (solve_idle(k)) return;
  const MergeDesc J = k.merges[d];
  const int kl = k.kl, ku = k.ku, kw = k.kw, mi = J.mif, R = k.R;
  const int64_t co = (int64_t)c0 * kw;   // first right-hand side of this column group
  const Tips tp{k.tips, kw, ku};
  double* sb = k.st + (int64_t)mi * kw * R + co;
  double* tb = sb + kl;
  double* nvl = k.nodeval + (int64_t)J.left * kw * R + co;
  double* nvr = k.nodeval + (int64_t)J.right * kw * R + co;
  double* nvj = k.nodeval + (int64_t)(k.p + mi) * kw * R + co;
  double* tmp = k.mtmp + (int64_t)mi * kw * R + co;
  const int* perm = k.sperm + (int64_t)mi * ku;
  if (J.a > 0) mgemm_any(ku, nrhs, ku, -1.0, gm(tp.Vt(J.left), kw, 1), gm(nvj, 1, kw), 1.0, tb, kw, lds);
  if (J.b < k.p - 1)
    mgemm_any(kl, nrhs, kl, -1.0, gm(tp.Wb(J.right), kw, 1), gm(nvj + ku, 1, kw), 1.0, sb, kw, lds);
  mgemm_any(ku, nrhs, kl, -1.0, gm(tp.Vb(J.left), kw, 1), gm(sb, 1, kw), 1.0, tb, kw, lds);
  const DenseAcc<double> D{k.sfac + (int64_t)mi * ku * ku, ku, ku - 1, ku - 1, ku, nullptr};
  const double* dv = k.sdinv + (int64_t)mi * ((ku + 15) / 16) * dinv_stride();
  leaf_sweep<double, HT, OP_UT_FWD>(D, dv, tsrc(tb, 1, 1, kw, 0, ku), tdst(tmp, nullptr, 1, 1, kw, ku, ku, ku), 0,
                                    nrhs, lds);
  leaf_sweep<double, HT, OP_LT_BWD>(D, dv, tsrc(tmp, 1, 1, kw, 0, ku), tdst(tmp, nullptr, 1, 1, kw, ku, ku, ku), 0,
                                    nrhs, lds);
  __syncthreads();
  for (int idx = threadIdx.x; idx < ku * nrhs; idx += NT) {
    const int i = idx % ku, q = idx / ku;
    tb[perm[i] + (int64_t)q * kw] = tmp[i + (int64_t)q * kw];
  }
  __syncthreads();
  mgemm_any(kl, nrhs, ku, -1.0, gm(tp.Wt(J.right), kw, 1), gm(tb, 1, kw), 1.0, sb, kw, lds);
  wg_copy(kl, nrhs, sb, kw, nvl + ku, kw);
  wg_copy(ku, nrhs, tb, kw, nvr, kw);
  if (J.a > 0) wg_copy(ku, nrhs, nvj, kw, nvl, kw);
  if (J.b < k.p - 1) wg_copy(kl, nrhs, nvj + ku, kw, nvr + ku, kw);
}

// Single-system (merges mbeg + blockIdx.x of one level) and batched launches
// of the reduced-solve kernels.
// Every operation of the reduced solve acts on the right-hand sides column by
// column, so the single-system launches give each merge one workgroup per
// group of MCG columns (blockIdx.x = merge * groups + group).  A batched
// launch runs a merge's groups one after the other in one workgroup, with the
// same arithmetic per column.
constexpr int MCG = 16;
__device__ __forceinline__ int mcg_groups(int nrhs) { return (nrhs + MCG - 1) / MCG; }

template <int HT>
__global__ __launch_bounds__(NT) void k_mup(KParams k, int mbeg, int nrhs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ng = mcg_groups(nrhs), c0 = MCG * (blockIdx.x % ng);
  mup_body<HT>(k, mbeg + blockIdx.x / ng, c0, min(MCG, nrhs - c0), reinterpret_cast<double*>(smem_raw));
}
static __global__ __launch_bounds__(NT) void k_mdown(KParams k, int mbeg, int nrhs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ng = mcg_groups(nrhs), c0 = MCG * (blockIdx.x % ng);
  mdown_body(k, mbeg + blockIdx.x / ng, c0, min(MCG, nrhs - c0), reinterpret_cast<double*>(smem_raw));
}
static __global__ __launch_bounds__(NT) void k_mtup(KParams k, int mbeg, int nrhs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ng = mcg_groups(nrhs), c0 = MCG * (blockIdx.x % ng);
  mtup_body(k, mbeg + blockIdx.x / ng, c0, min(MCG, nrhs - c0), reinterpret_cast<double*>(smem_raw));
}
template <int HT>
__global__ __launch_bounds__(NT) void k_mtdown(KParams k, int mbeg, int nrhs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ng = mcg_groups(nrhs), c0 = MCG * (blockIdx.x % ng);
  mtdown_body<HT>(k, mbeg + blockIdx.x / ng, c0, min(MCG, nrhs - c0), reinterpret_cast<double*>(smem_raw));
}
template <int HT, int KIND>
__global__ __launch_bounds__(NT) void k_msolve_b(BatchArgs ba) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  const int s = batch_sys(ba, blockIdx.x);
  const KParams& k = *ba.kp[s];
  const int d = ba.mbeg[s] + (blockIdx.x - ba.off[s]);
  const int nrhs = ba.nrhs[s];
  for (int c0 = 0; c0 < nrhs; c0 += MCG) {
    const int nc = min(MCG, nrhs - c0);
    if (KIND == 0) mup_body<HT>(k, d, c0, nc, lds);
    else if (KIND == 1) mdown_body(k, d, c0, nc, lds);
    else if (KIND == 2) mtup_body(k, d, c0, nc, lds);
    else mtdown_body<HT>(k, d, c0, nc, lds);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- runners
template <typename K>
inline void allow_lds_m(K kernel, size_t lds) {
  (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// One level of the reduced-system factorisation for several systems of the
// same bandwidths (orders up to 160: the blocked LU); cnt[s] merges of
// system s from ba.mbeg[s] on.
template <int HT>
int run_mfactor_level_batch(BatchArgs ba, const int* cnt, int kl, int ku, hipStream_t st) {
  const int kmax = kl > ku ? kl : ku, kw = kl + ku;
  const size_t tr_lds = (size_t)mtrsm_lds_elems<HT>() * 8 + 2048;
  const int ncg = (kmax + 63) / 64;
  const int ftn = (kw + FG_T - 1) / FG_T, ftiles = ((kmax + FG_T - 1) / FG_T) * ftn;
  auto prefix = [&](int mult) {
    int tot = 0;
    for (int s = 0; s < ba.nsys; ++s) {
      ba.off[s] = tot;
      tot += cnt[s] * mult;
    }
    ba.off[ba.nsys] = tot;
    return tot;
  };
  if (prefix(1) <= 0) return 0;
  {
    ProfScope ps("k_mgemm", st);
    hipLaunchKernelGGL((k_mgemm_b<1>), dim3(prefix(fjobs(1) * ftiles)), dim3(NT), 0, st, ba, ftiles, ftn);
    SPIKE_CHECK_LAUNCH();
  }
  {
    ProfScope ps("k_mlu", st);
    const int nw = (ku + 15) / 16 + 1;
    const int nl = prefix(1);
    if (ku <= 64) {
      allow_lds_m(k_mlu_blk_b<4>, mlu_blk_lds_bytes<4>());
      hipLaunchKernelGGL((k_mlu_blk_b<4>), dim3(nl), dim3(64 * nw), mlu_blk_lds_bytes<4>(), st, ba);
    } else if (ku <= 128) {
      allow_lds_m(k_mlu_blk_b<8>, mlu_blk_lds_bytes<8>());
      hipLaunchKernelGGL((k_mlu_blk_b<8>), dim3(nl), dim3(64 * nw), mlu_blk_lds_bytes<8>(), st, ba);
    } else {
      allow_lds_m(k_mlu_blk_b<10>, mlu_blk_lds_bytes<10>());
      hipLaunchKernelGGL((k_mlu_blk_b<10>), dim3(nl), dim3(64 * nw), mlu_blk_lds_bytes<10>(), st, ba);
    }
    SPIKE_CHECK_LAUNCH();
  }
  {
    allow_lds_m(k_mtrsm_b<HT>, tr_lds);
    ProfScope ps("k_mtrsm", st);
    hipLaunchKernelGGL((k_mtrsm_b<HT>), dim3(prefix(2 * ncg)), dim3(NT), tr_lds, st, ba, ncg);
    SPIKE_CHECK_LAUNCH();
  }
  {
    ProfScope ps("k_mgemm", st);
    hipLaunchKernelGGL((k_mgemm_b<45>), dim3(prefix(fjobs(45) * ftiles)), dim3(NT), 0, st, ba, ftiles, ftn);
    SPIKE_CHECK_LAUNCH();
  }
  {
    ProfScope ps("k_mgemm", st);
    hipLaunchKernelGGL((k_mgemm_b<6>), dim3(prefix(fjobs(6) * ftiles)), dim3(NT), 0, st, ba, ftiles, ftn);
    SPIKE_CHECK_LAUNCH();
  }
  return 0;
}

template <int HT>
int run_mfactor(const KParams& k, const LaunchCfg& c, hipStream_t st) {
  const int kmax = k.kmax;
  const size_t lu_lds = (size_t)mlu_lds_elems(k.ku) * 8;
  const size_t tr_lds = (size_t)mtrsm_lds_elems<HT>() * 8 + 2048;
  allow_lds_m(k_mlu, lu_lds);
  allow_lds_m(k_mlu_blk<4>, mlu_blk_lds_bytes<4>());
  allow_lds_m(k_mlu_blk<8>, mlu_blk_lds_bytes<8>());
  allow_lds_m(k_mlu_blk<10>, mlu_blk_lds_bytes<10>());
  allow_lds_m(k_mtrsm<HT>, tr_lds);
  const int ncg = (kmax + 63) / 64;
  // fused products: rows up to kmax, kw = kl + ku columns, 64 x 64 tiles
  const int ftn = (k.kw + FG_T - 1) / FG_T, ftiles = ((kmax + FG_T - 1) / FG_T) * ftn;
  for (int l = 0; l + 1 < (int)c.level_off.size(); ++l) {
    const int beg = c.level_off[l], cnt = c.level_off[l + 1] - beg;
    if (cnt <= 0) continue;
    {
      ProfScope ps("k_mgemm", st);
      hipLaunchKernelGGL((k_mgemm<1>), dim3(cnt * fjobs(1) * ftiles), dim3(NT), 0, st, k, beg, ftiles, ftn);
      SPIKE_CHECK_LAUNCH();
    }
    {
      ProfScope ps("k_mlu", st);
      const int nw = (k.ku + 15) / 16 + 1;   // block wavefronts and the factoring one
      if (k.ku <= 64)
        hipLaunchKernelGGL((k_mlu_blk<4>), dim3(cnt), dim3(64 * nw), mlu_blk_lds_bytes<4>(), st, k, beg);
      else if (k.ku <= 128)
        hipLaunchKernelGGL((k_mlu_blk<8>), dim3(cnt), dim3(64 * nw), mlu_blk_lds_bytes<8>(), st, k, beg);
      else if (k.ku <= 160)
        hipLaunchKernelGGL((k_mlu_blk<10>), dim3(cnt), dim3(64 * nw), mlu_blk_lds_bytes<10>(), st, k, beg);
      else if (k.ku <= 192)
        hipLaunchKernelGGL((k_mlu_reg<24, 3>), dim3(cnt), dim3(NWR * 64), 0, st, k, beg);
      else
        hipLaunchKernelGGL(k_mlu, dim3(cnt), dim3(NT), lu_lds, st, k, beg);
      SPIKE_CHECK_LAUNCH();
    }
    {
      ProfScope ps("k_mtrsm", st);
      hipLaunchKernelGGL((k_mtrsm<HT>), dim3(cnt * 2 * ncg), dim3(NT), tr_lds, st, k, beg, ncg);
      SPIKE_CHECK_LAUNCH();
    }
    {
      ProfScope ps("k_mgemm", st);
      hipLaunchKernelGGL((k_mgemm<45>), dim3(cnt * fjobs(45) * ftiles), dim3(NT), 0, st, k, beg, ftiles, ftn);
      SPIKE_CHECK_LAUNCH();
    }
    {
      ProfScope ps("k_mgemm", st);
      hipLaunchKernelGGL((k_mgemm<6>), dim3(cnt * fjobs(6) * ftiles), dim3(NT), 0, st, k, beg, ftiles, ftn);
      SPIKE_CHECK_LAUNCH();
    }
  }
  return 0;
}

template <int HT>
int run_msolve(const KParams& k, const LaunchCfg& c, hipStream_t st, int nrhs, bool trans) {
  const size_t lds = (size_t)(tile_lds_elems(HT) > kMsolveLds ? tile_lds_elems(HT) : kMsolveLds) * 8 + 2048;
  allow_lds_m(k_mup<HT>, lds);
  allow_lds_m(k_mtdown<HT>, lds);
  allow_lds_m(k_mdown, lds);
  allow_lds_m(k_mtup, lds);
  const int L = (int)c.level_off.size() - 1;
  if (!trans) {
    for (int l = 0; l < L; ++l) {
      const int beg = c.level_off[l], cnt = c.level_off[l + 1] - beg;
      ProfScope ps("k_mup", st);
      hipLaunchKernelGGL((k_mup<HT>), dim3(cnt * ((nrhs + MCG - 1) / MCG)), dim3(NT), lds, st, k, beg, nrhs);
      SPIKE_CHECK_LAUNCH();
    }
    for (int l = L - 1; l >= 0; --l) {
      const int beg = c.level_off[l], cnt = c.level_off[l + 1] - beg;
      ProfScope ps("k_mdown", st);
      hipLaunchKernelGGL(k_mdown, dim3(cnt * ((nrhs + MCG - 1) / MCG)), dim3(NT), lds, st, k, beg, nrhs);
      SPIKE_CHECK_LAUNCH();
    }
  } else {
    for (int l = 0; l < L; ++l) {
      const int beg = c.level_off[l], cnt = c.level_off[l + 1] - beg;
      ProfScope ps("k_mtup", st);
      hipLaunchKernelGGL(k_mtup, dim3(cnt * ((nrhs + MCG - 1) / MCG)), dim3(NT), lds, st, k, beg, nrhs);
      SPIKE_CHECK_LAUNCH();
    }
    for (int l = L - 1; l >= 0; --l) {
      const int beg = c.level_off[l], cnt = c.level_off[l + 1] - beg;
      ProfScope ps("k_mtdown", st);
      hipLaunchKernelGGL((k_mtdown<HT>), dim3(cnt * ((nrhs + MCG - 1) / MCG)), dim3(NT), lds, st, k, beg, nrhs);
      SPIKE_CHECK_LAUNCH();
    }
  }
  return 0;
}

// One level of the reduced solve for a batch of systems (up: the first pass,
// bottom-up; else the second pass, top-down).
template <int HT>
int run_msolve_level_batch(const BatchArgs& ba, hipStream_t st, int nitems, bool trans, bool up) {
  if (nitems <= 0) return 0;
  const size_t lds = (size_t)(tile_lds_elems(HT) > kMsolveLds ? tile_lds_elems(HT) : kMsolveLds) * 8 + 2048;
  const int kind = trans ? (up ? 2 : 3) : (up ? 0 : 1);
  switch (kind) {
    case 0: {
      allow_lds_m(k_msolve_b<HT, 0>, lds);
      ProfScope ps("k_mup", st);
      hipLaunchKernelGGL((k_msolve_b<HT, 0>), dim3(nitems), dim3(NT), lds, st, ba);
      break;
    }
    case 1: {
      allow_lds_m(k_msolve_b<HT, 1>, lds);
      ProfScope ps("k_mdown", st);
      hipLaunchKernelGGL((k_msolve_b<HT, 1>), dim3(nitems), dim3(NT), lds, st, ba);
      break;
    }
    case 2: {
      allow_lds_m(k_msolve_b<HT, 2>, lds);
      ProfScope ps("k_mtup", st);
      hipLaunchKernelGGL((k_msolve_b<HT, 2>), dim3(nitems), dim3(NT), lds, st, ba);
      break;
    }
    default: {
      allow_lds_m(k_msolve_b<HT, 3>, lds);
      ProfScope ps("k_mtdown", st);
      hipLaunchKernelGGL((k_msolve_b<HT, 3>), dim3(nitems), dim3(NT), lds, st, ba);
      break;
    }
  }
  SPIKE_CHECK_LAUNCH();
  return 0;
}

}  // namespace spike
