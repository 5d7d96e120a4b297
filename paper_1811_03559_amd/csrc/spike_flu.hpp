// Block LU of a banded partition on MFMA tiles (non-pivoting; the factor
// stage of the central-concept subsection, A_i = L_i U_i, with the last
// partition factored as the LU of its reversal, pivoting-UL subsection).
//
// The partition is cut into 16 x 16 tiles; with HT = ceil(max(kl, ku) / 16)
// the active part of the right-looking elimination is a window of
// (HT + 1) x (HT + 1) tiles that slides one tile down the diagonal per step.
// A workgroup has NW = HT + 2 wavefronts; wavefront w owns the tile columns
// C = w (mod NW) and keeps the HT + 1 window tiles of its current column in
// MFMA accumulators, so a tile stays in registers from the moment it is read
// from the caller's band until it is final.  Step j (column block j is the
// panel):
//   * every other wavefront, with its column C in the window:
//       U_{j,C} = L_jj^{-1} A_{j,C}                       (row tile, stored)
//       Z       = U_jj^{-1} U_{j,C}
//       A_{i,C} -= A_{i,j} Z,  i = j+1 .. j+HT              (trailing update)
//     and one of them also forms the L tile L_{j+c,j} = A_{j+c,j} U_jj^{-1}
//     for the factor output; (A_{i,j} U_jj^{-1}) U_{j,C} = A_{i,j} Z, so the
//     trailing update needs the panel's raw tiles only;
//   * the wavefront that owns column j+1 finishes its own update first, then
//     factors the next diagonal tile in registers (16 rank-1 steps with
//     cross-lane shuffles) and forms the inverses of its unit-lower and upper
//     triangles, which it publishes in the other LDS buffer together with
//     its column's raw tiles: the panel of step j+1 overlaps the trailing
//     update of step j, and one barrier ends a step.
// The diagonal-tile inverses are also the ones the multi-RHS sweeps use, so
// they are written out as the partition's diagonal-block inverses.
//
// Boosting (threshold tau * ||A_i||_1): the first pass factors without
// boosting and accumulates the exact column sums of |A_i| as tiles are read;
// if any pivot fell below the threshold, the partition is factored again with
// boosting.  When no pivot is below the threshold the boosted factorisation
// applies no boost, so the first pass is already its result.
#pragma once
#include "spike_fast.hpp"
#include "spike_rowlu.hpp"

namespace spike {

template <typename T>
struct PivStats {
  T minpiv;
  int boosts;
  int first_zero;
};

// Wavefronts of k_flu: one per window column plus one, so that a wavefront
// that finishes its column has one idle step before the next column it owns
// enters the window, and the loads of that column are in flight meanwhile.
template <int HT>
__host__ __device__ constexpr int flu_nw() { return HT + 2; }

// The elimination of one partition; REV: the partition is the last one,
// held as the LU of its reversal (row and column order reversed).
template <typename T, int HT, bool REV>
__device__ __forceinline__ void flu_body(const KParams& k, const LeafDesc& L, T* lds) {
  using M = Mf<T>;
  using v4 = typename M::v4;
  constexpr int NW = flu_nw<HT>();
  constexpr int PADW = tile_pad();
  constexpr int TS = 16 * PADW;          // one tile in LDS
  constexpr int BUF = (HT + 2) * TS;     // L^{-1}, U^{-1}, raw panel tiles 1..HT
  __shared__ double s_norm[NW];
  __shared__ double s_minp[NW];
  __shared__ int s_boost[NW], s_zero[NW];

  const int m = L.m;
  const BandAcc<T> A = leaf_band<T>(k, L);
  T* dv = reinterpret_cast<T*>(k.dinv) + L.dinv_off;
  int* pflag = reinterpret_cast<int*>(lds + 2 * BUF);   // step whose diagonal tile is published
  const int klf = A.kl, kuf = A.kuw;
  const int64_t s = L.start;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, cl = lane & 15;
  // Wavefront w owns the tile columns C = role(w) (mod NW).  The wavefronts
  // of a workgroup are normally placed on the four SIMDs of a compute unit
  // in turn (w on SIMD w % 4; any placement gives the same results), so
  // role(w) numbers the wavefronts of SIMD 0 first, then those of SIMD 1, and
  // so on: wavefronts that share a SIMD hold neighbouring columns, and the
  // factoring wavefront of a step (window column 0) often shares its SIMD
  // with the owner of the next panel column (window column 1) or with the
  // loading wavefront (window column NW - 1), which issue few or no
  // matrix-core products while it factors, rather than with two wavefronts
  // that issue a full step of them.
  const int role = (wave % 4) * (NW / 4) + min(wave % 4, NW % 4) + wave / 4;
  constexpr int DQ = sizeof(T) == 8 ? 4 : 1;   // row step between registers
  const int nbk = (m + 15) / 16;

  // tile (R, C) of the block in the accumulator layout; entries outside the
  // order are the identity, entries outside the band zero; `cs` gathers
  // |a| of the real entries (this lane's rows of its column).  Element
  // (i, c) of the block is A(s+i, s+c), or A(s+m-1-i, s+m-1-c) reversed.
  // Issued in two halves so that a batch of tiles has all its loads in
  // flight before the first value is used: load_raw reads the band entries
  // (zero outside the band and the order), make_tile forms the tile.
  auto load_raw = [&](int R, int Cc, double (&av)[4]) __attribute__((always_inline)) {
    const int ln = opaque(lane);
    const int c = 16 * Cc + (ln & 15), i0 = 16 * R + M::row(ln, 0);
    const int64_t gc = REV ? s + m - 1 - c : s + c;
    const double* colp = k.dAB + (int64_t)k.ku + gc * k.ldab - gc + (REV ? s + m - 1 : s);   // + gi
    const double* p0 = REV ? colp - i0 : colp + i0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + DQ * q;
      const bool ok = i < m && c < m && i - c <= klf && c - i <= kuf;
      av[q] = ok ? (REV ? p0[-DQ * q] : p0[DQ * q]) : 0.0;
    }
  };
  auto make_tile = [&](int R, int Cc, const double (&av)[4], double& cs) __attribute__((always_inline)) -> v4 {
    const int ln = opaque(lane);
    const int c = 16 * Cc + (ln & 15), i0 = 16 * R + M::row(ln, 0);
    v4 v;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + DQ * q;
      v[q] = (i >= m || c >= m) ? ((i == c) ? T(1) : T(0)) : (T)av[q];
      cs += fabs(av[q]);
    }
    return v;
  };
  // all HT + 1 window tiles of column Cc from row R0 down, loads batched
  auto load_column = [&](int R0, int Cc, v4 (&acc)[HT + 1], double& cs) __attribute__((always_inline)) {
    double av[HT + 1][4];
#pragma unroll
    for (int i = 0; i <= HT; ++i) load_raw(R0 + i, Cc, av[i]);
#pragma unroll
    for (int i = 0; i <= HT; ++i) acc[i] = make_tile(R0 + i, Cc, av[i], cs);
  };
  auto store_band = [&](int R, int Cc, const v4& v) __attribute__((always_inline)) {
    const int ln = opaque(lane);
    const int c = 16 * Cc + (ln & 15), i0 = 16 * R + M::row(ln, 0);
    T* p0 = A.a + (int64_t)kuf - c + (int64_t)c * A.ldw + i0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + DQ * q;
      if (i < m && c < m && i - c <= klf && c - i <= kuf) p0[DQ * q] = v[q];
    }
  };
  auto lds_put = [&](T* P, const v4& v) __attribute__((always_inline)) {
    const int ln = opaque(lane);
#pragma unroll
    for (int q = 0; q < 4; ++q) P[M::row(ln, q) * PADW + (ln & 15)] = v[q];
  };
  // d += P * b, P a 16 x 16 tile in LDS, b in accumulator layout
  auto mm_lds_reg = [&](const T* P, const v4& b, v4 d) __attribute__((always_inline)) -> v4 {
    const int ln = opaque(lane);
#pragma unroll
    for (int q = 0; q < 4; ++q) d = M::mma(P[(ln & 15) * PADW + M::row(ln, q)], b[q], d);
    return d;
  };
  // P * Q, both tiles in LDS
  auto mm_lds_lds = [&](const T* P, const T* Q) __attribute__((always_inline)) -> v4 {
    v4 d = {T(0), T(0), T(0), T(0)};
    const int ln = opaque(lane);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = M::row(ln, q);
      d = M::mma(P[(ln & 15) * PADW + r], Q[r * PADW + (ln & 15)], d);
    }
    return d;
  };

  double anorm = 0.0;
  PivStats<T> st;
  for (int pass = 0; pass < 2; ++pass) {
    const T boost = pass == 0 ? T(0) : (T)(k.boost_tau * anorm);
    st.minpiv = T(__builtin_huge_val());
    st.boosts = 0;
    st.first_zero = -1;
    double nmax = 0.0;

    int C = role;
    v4 acc[HT + 1];
    double cs = 0.0;
    // column sums of the owner's column C, gathered over its lanes into the
    // running maximum (the 1-norm of the partition)
    auto note_colsum = [&]() __attribute__((always_inline)) {
      double cmax = cs;
      cmax += __shfl_xor(cmax, 16);
      cmax += __shfl_xor(cmax, 32);
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) cmax = fmax(cmax, __shfl_xor(cmax, off));
      nmax = fmax(nmax, cmax);
    };
    // acc holds nothing that is used before it is loaded again: an empty
    // definition tells the compiler so, which keeps the tiles out of the
    // registers the panel needs
    auto drop_tiles = [&]() __attribute__((always_inline)) {
#pragma unroll
      for (int i = 0; i <= HT; ++i) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          T x;
          asm volatile("" : "=v"(x));
          acc[i][q] = x;
        }
      }
    };
    // LU of diagonal tile jp (published in the U^{-1} slot of its buffer Pn)
    // and the inverses of its factors, by the wavefront that holds no tiles
    // in this step
    auto panel = [&](int jp, T* Pn) __attribute__((always_inline)) {
      // lane-derived indices are recomputed here rather than kept from
      // outside the step loop
      const int ln = opaque(lane), r = ln & 15;
      T ar[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) ar[c] = Pn[TS + r * PADW + c];
      wave_lds_sync();
      int nb = 0;
      lu16_rows<T>(ar, boost, m - 16 * jp, nb);
      st.boosts += nb;
      // this lane's pivot, and the statistics of the tile's pivots over its rows
      T d = ar[0];
#pragma unroll
      for (int t = 1; t < 16; ++t) d = (r == t) ? ar[t] : d;
      const T myrp = d != T(0) ? recip(d) : T(0);
      {
        const int mrem = m - 16 * jp;
        T mp = r < mrem ? (T)fabs(d) : T(__builtin_huge_val());
        int fz = (r < mrem && d == T(0)) ? r : 16;
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
          mp = fmin(mp, __shfl_xor(mp, off));
          fz = min(fz, __shfl_xor(fz, off));
        }
        st.minpiv = fmin(st.minpiv, mp);
        if (st.first_zero < 0 && fz < 16) st.first_zero = 16 * jp + fz;
      }
      T* D = dv + (int64_t)jp * dinv_stride();
      if (ln < 16) {
        const int i = 16 * jp + r;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const int cc = 16 * jp + c;
          if (i < m && cc < m && i - cc <= klf && cc - i <= kuf)
            A.a[(int64_t)kuf + i - cc + (int64_t)cc * A.ldw] = ar[c];
        }
      }
      // L^{-1} in lanes 0-15 (and 32-47); in lanes 16-31 (and 48-63)
      // (L')^{-1} for L' = J V J, J the order reversal and V = D^{-1} U unit
      // upper (row r of U times the reciprocal of its pivot): lane 16 + r'
      // takes row 15 - r' of the tile reversed, so that its row of the
      // inverse is row 15 - r' of V^{-1} reversed; U^{-1} = V^{-1} D^{-1}
      const bool hi = (ln & 16) != 0;
      const T rpm = row_mirror(myrp);
      T mv[16], xi[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const T am = row_mirror(ar[15 - c]);
        mv[c] = hi ? am * rpm : ar[c];
      }
      unit_lower_inv16_rows<T>(mv, xi);
      if (ln < 16) {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          Pn[r * PADW + c] = xi[c];
          D[r * 16 + c] = xi[c];
        }
      } else if (ln < 32) {
        const int R = 15 - r;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const T v = xi[c] * row_bcast(myrp, 15 - c);   // U^{-1}(R, 15 - c)
          Pn[TS + R * PADW + 15 - c] = v;
          D[256 + R * 16 + 15 - c] = v;
        }
      }
    };

    // The last wavefront's first column enters the window at step 1: it
    // factors diagonal tile 0 (published by the owner of column 0) and loads
    // that column in step 0; the others load theirs at once.
    const bool first_panel = role == NW - 1;
    if (!first_panel) {
      if (C < nbk) {
        load_column(0, C, acc, cs);   // rows of its first window step
      } else {
#pragma unroll
        for (int i = 0; i <= HT; ++i) acc[i] = v4{T(0), T(0), T(0), T(0)};
      }
    }
    if (role == 0) {
      note_colsum();
#pragma unroll
      for (int i = 1; i <= HT; ++i) lds_put(lds + (1 + i) * TS, acc[i]);
      lds_put(lds + TS, acc[0]);
    }
    if (tid == 0) *pflag = -1;
    __syncthreads();
    if (first_panel) {
      panel(0, lds);
      __builtin_amdgcn_sched_barrier(0);
      drop_tiles();
    }
    __syncthreads();

    // Step j: the owner of column j + 1 (window column 1) updates that
    // column first, publishes its diagonal tile and raises the flag; the
    // wavefront that finished column j (window column 0) waits for the flag,
    // factors the diagonal tile and publishes the inverses; the wavefront
    // whose column enters the window next step (window column HT + 1) loads
    // it.  One barrier ends a step; it waits for LDS operations only, so the
    // global stores of a step stay in flight across it.
    for (int j = 0; j < nbk; ++j) {
      const int c = C - j;   // window column of this wavefront's tiles
      T* Pn = lds + ((j + 1) & 1) * BUF;
      if (c == 0) {
        if (j + 1 < nbk) {
          while (__hip_atomic_load(pflag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) != j + 1)
            __builtin_amdgcn_s_sleep(1);
          __builtin_amdgcn_s_setprio(3);
          panel(j + 1, Pn);
          __builtin_amdgcn_s_setprio(0);
        }
        // column j is final; the next column of this wavefront enters the
        // window at step j + 2 and is loaded in step j + 1
        C += NW;
        cs = 0.0;
        __builtin_amdgcn_sched_barrier(0);
        drop_tiles();
      } else if (c == HT + 1) {
        if (C < nbk) load_column(C - HT, C, acc, cs);   // window from step j + 1 on
      } else if (c <= HT && C < nbk) {
        const T* P = lds + (j & 1) * BUF;
        double nav[4];
        load_raw(j + 1 + HT, C, nav);   // used at the end of the step
        const bool own = (c == 1) && (j + 1 < nbk);
        if (own) __builtin_amdgcn_s_setprio(2);
        const v4 zero = {T(0), T(0), T(0), T(0)};
        const v4 u = mm_lds_reg(P, acc[0], zero);        // U_{j,C}
        const v4 nz = -mm_lds_reg(P + TS, u, zero);      // -U_jj^{-1} U_{j,C}
        acc[1] = mm_lds_reg(P + 2 * TS, nz, acc[1]);
        if (own) {
          // the next diagonal tile is final: hand it to the factoring
          // wavefront before any other work of the step is issued
          lds_put(Pn + TS, acc[1]);
          __hip_atomic_store(pflag, j + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 2; i <= HT; ++i) acc[i] = mm_lds_reg(P + (1 + i) * TS, nz, acc[i]);
        store_band(j, C, u);
        if (j + c < nbk) store_band(j + c, j, mm_lds_lds(P + (1 + c) * TS, P + TS));   // L_{j+c,j}
#pragma unroll
        for (int i = 0; i < HT; ++i) acc[i] = acc[i + 1];
        acc[HT] = make_tile(j + 1 + HT, C, nav, cs);
        if (own) {
          note_colsum();
#pragma unroll
          for (int i = 1; i <= HT; ++i) lds_put(Pn + (1 + i) * TS, acc[i]);
          __builtin_amdgcn_s_setprio(0);
        }
      }
      lds_barrier();
    }

    if (lane == 0) {
      s_norm[wave] = nmax;
      s_minp[wave] = (double)st.minpiv;
      s_boost[wave] = st.boosts;
      s_zero[wave] = st.first_zero;
    }
    __syncthreads();
    double minp = __builtin_huge_val();
    int boosts = 0, fz = -1;
    anorm = 0.0;
    for (int w = 0; w < NW; ++w) {
      anorm = fmax(anorm, s_norm[w]);
      minp = fmin(minp, s_minp[w]);
      boosts += s_boost[w];
      if (s_zero[w] >= 0 && (fz < 0 || s_zero[w] < fz)) fz = s_zero[w];
    }
    __syncthreads();
    const bool redo = pass == 0 && k.boost_tau > 0.0 && (T)minp < (T)(k.boost_tau * anorm);
    if (!redo) {
      if (tid == 0) {
        if (fz >= 0) {
          const int64_t grow = REV ? s + m - 1 - fz : s + fz;
          atomicMin(&k.status->zero_row, (unsigned long long)(grow + 1));
        }
        if (boosts) atomicAdd(&k.status->n_boosts, boosts);
        atomicMin(&k.status->min_pivot_bits, dbits(minp));
      }
      break;
    }
  }
}

// LDS bytes of k_flu<T, HT>: two panel buffers and the hand-over flag.
template <typename T, int HT>
constexpr size_t flu_lds_bytes() {
  return (size_t)2 * (HT + 2) * 16 * tile_pad() * sizeof(T) + 16;
}

template <typename T, int HT>
__device__ __forceinline__ void flu_kernel_body(const KParams& k, const int bx_, const int gx_) {
  constexpr int NW = flu_nw<HT>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int li = bx_;
  const LeafDesc L = k.leaves[li];
  const int m = L.m;
  const BandAcc<T> A = leaf_band<T>(k, L);
  const int klf = A.kl, kuf = A.kuw;
  const int64_t s = L.start;
  const int nthr = NW * 64, tid = threadIdx.x;

  // coupling blocks: B^_i (rows s_{i+1}-ku.., cols s_{i+1}..) and C^_i
  // (rows s_i.., cols s_i-kl..), in the normal frame
  if (li < k.p - 1) {
    double* bh = k.bhat + (int64_t)li * k.ku * k.ku;
    const int64_t s1 = s + m;
    for (int idx = tid; idx < k.ku * k.ku; idx += nthr) {
      const int r = idx % k.ku, c = idx / k.ku;
      const int64_t gi = s1 - k.ku + r, gc = s1 + c;
      bh[idx] = (r >= c) ? k.dAB[(k.ku + gi - gc) + gc * k.ldab] : 0.0;
    }
  }
  if (li > 0) {
    double* ch = k.chat + (int64_t)(li - 1) * k.kl * k.kl;
    for (int idx = tid; idx < k.kl * k.kl; idx += nthr) {
      const int r = idx % k.kl, c = idx / k.kl;
      const int64_t gi = s + r, gc = s - k.kl + c;
      ch[idx] = (r <= c) ? k.dAB[(k.ku + gi - gc) + gc * k.ldab] : 0.0;
    }
  }
  // band slots that lie outside the block (top-left and bottom-right corners)
  for (int idx = tid; idx < kuf * kuf; idx += nthr) {
    const int c = idx / kuf, sr = idx % kuf;
    if (c < m && sr < kuf - c) A.a[sr + (int64_t)c * A.ldw] = T(0);
  }
  for (int idx = tid; idx < klf * (int)A.ldw; idx += nthr) {
    const int c = m - 1 - idx / (int)A.ldw, sr = idx % (int)A.ldw;
    if (c >= 0 && c + sr - kuf >= m) A.a[sr + (int64_t)c * A.ldw] = T(0);
  }
  if (L.type == LEAF_LAST) flu_body<T, HT, true>(k, L, lds);
  else flu_body<T, HT, false>(k, L, lds);
}
template <typename T, int HT>
__global__ __launch_bounds__(flu_nw<HT>() * 64) void k_flu(KParams k) {
  flu_kernel_body<T, HT>(k, blockIdx.x, gridDim.x);
}
// the same for up to kMaxBatch systems: workgroup i belongs to system s
// with off[s] <= i < off[s + 1] (its parameter block at kp[s])
template <typename T, int HT>
__global__ __launch_bounds__(flu_nw<HT>() * 64) void k_flu_b(BatchArgs ba) {
  const int s = batch_sys(ba, blockIdx.x);
  flu_kernel_body<T, HT>(*ba.kp[s], blockIdx.x - ba.off[s], ba.off[s + 1] - ba.off[s]);
}

// fills ba.off from the per-system counts
inline int batch_prefix(BatchArgs& ba, const int* cnt, int mult) {
  int tot = 0;
  for (int s = 0; s < ba.nsys; ++s) {
    ba.off[s] = tot;
    tot += cnt[s] * mult;
  }
  ba.off[ba.nsys] = tot;
  return tot;
}

template <typename T, int HT>
int run_flu_batch(BatchArgs ba, const int* cnt, hipStream_t st) {
  constexpr int NW = flu_nw<HT>();
  const size_t lds = flu_lds_bytes<T, HT>();
  const int n = batch_prefix(ba, cnt, 1);
  if (n <= 0) return 0;
  hipFuncSetAttribute((const void*)k_flu_b<T, HT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  ProfScope ps("k_flu", st);
  hipLaunchKernelGGL((k_flu_b<T, HT>), dim3(n), dim3(NW * 64), lds, st, ba);
  SPIKE_CHECK_LAUNCH();
  return 0;
}

template <typename T, int HT>
int run_flu(const KParams& k, const LaunchCfg& c, hipStream_t st) {
  constexpr int NW = flu_nw<HT>();
  const size_t lds = flu_lds_bytes<T, HT>();
  hipFuncSetAttribute((const void*)k_flu<T, HT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  ProfScope ps("k_flu", st);
  hipLaunchKernelGGL((k_flu<T, HT>), dim3(k.p), dim3(NW * 64), lds, st, k);
  SPIKE_CHECK_LAUNCH();
  return 0;
}

}  // namespace spike
