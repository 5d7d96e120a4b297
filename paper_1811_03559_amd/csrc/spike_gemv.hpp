// Banded triangular sweep of a single right-hand side (non-pivoting factors).
//
// With one column the sweep is bound by streaming the band from HBM, so it is
// organised as a sequence of matrix-vector products over 16-row blocks
// instead of MFMA tiles.  The workgroup keeps a ring of RS = 16 (HT + 1) rows
// in flight, one row per thread: the current block and the HT blocks below
// it (in sweep order) that it still updates.  Per block step:
//   1. the 16 threads whose rows form the current block publish their value
//      w to LDS (one barrier);
//   2. every wavefront forms x = D^{-1} w with the precomputed inverse of the
//      16 x 16 diagonal block (each lane multiplies four entries, two
//      cross-lane sums finish a row), so x needs no second barrier;
//   3. every other thread subtracts its row of the coupling block times x
//      (16 coefficients, prefetched PD steps ahead);
//   4. the 16 threads of the current block move to the rows entering the
//      ring, and every thread reloads its row's right-hand side into the copy
//      of this step's prefetch slot; a row's right-hand side is only combined
//      with its accumulated update when the row becomes current, so no load
//      latency lies on the chain of block steps.
// The step barrier waits for LDS operations only, so the loads issued for
// later steps stay in flight across it, and every load is issued without a
// branch (entries outside the stored data read a global zero).
// For U^T and L^T a row's 16 coefficients lie along one band column, so a
// thread reading its own row would touch a different cache line in every
// lane.  There the coefficients of a step are loaded cooperatively (16
// consecutive lanes per row, one cache line per 16 lanes), staged through
// a double-buffered LDS block one step ahead, and read back per row.
// Operations, as for the tile engine: L X (unit lower, forward), U X (upper,
// backward), U^T X (forward) and L^T X (unit, backward).
#pragma once
#include <hip/hip_runtime.h>

#include "spike_tile.hpp"

namespace spike {

// LDS elements (of T) used by gemv_sweep<HT> (at most tile_lds_elems(HT)).
__host__ __device__ constexpr int gemv_lds_elems(int HT) { return 32 + 2 * 16 * HT * 17; }

template <typename T, int HT, int OP, typename Acc>
__device__ void gemv_sweep(const Acc& A, const T* dinv, const TSrc& src, const TDst& dst, T* lds) {
  constexpr bool FWD = (OP == OP_L_FWD || OP == OP_UT_FWD);
  constexpr bool USE_U = (OP == OP_U_BWD || OP == OP_UT_FWD);
  constexpr bool TRANS = (OP == OP_UT_FWD || OP == OP_LT_BWD);
  constexpr int RS = 16 * (HT + 1);
  // prefetch depth of coefficients and block inverses, in steps; a thread's
  // row advances once every HT + 1 steps, so a prefetch PD + 1 <= HT + 1
  // steps ahead sees at most one advance
  constexpr int PD = HT < 2 ? HT : 2;
  static_assert(RS <= NT, "ring larger than the workgroup");
  const int tid = threadIdx.x, lane = tid & 63, r16 = lane & 15, g4 = lane >> 4;
  const int m = A.m, nb = (m + 15) / 16, mp = 16 * nb;
  const bool act = tid < RS;
  // band reach of the coupling entries
  const int reach = (OP == OP_L_FWD || OP == OP_LT_BWD) ? A.kl : A.kuw;

  auto row_of = [&](int pos) { return FWD ? pos : mp - 1 - pos; };
  auto blk_of = [&](int s) { return FWD ? s : nb - 1 - s; };

  int pos = tid;   // ring position of this thread's row (step 0 holds positions 0 .. RS-1)
  T upd = T(0);

  // coefficients M(i, 16 b + c), c = 0..15, of this thread's row at step sp;
  // the ring keeps every row strictly past the block (distance d >= 1), so
  // only the band reach and the order bound the entries
  auto fetch_cf = [&](int sp, T (&cf)[16]) __attribute__((always_inline)) {
    const int pp = pos >= 16 * sp ? pos : pos + RS;
    const int i = row_of(pp);
    const int b = blk_of(sp);
    const bool ok = act && sp < nb && pp >= 16 * sp + 16 && pp < mp && i < m;
    // valid c: FWD d = i - 16 b - c <= reach; BWD d = 16 b + c - i <= reach, 16 b + c < m
    const int clo = FWD ? i - 16 * b - reach : 0;
    const int chi = FWD ? 15 : min(reach + i - 16 * b, m - 1 - 16 * b);
    // every load is issued (entries outside the band read a global zero),
    // so neither a branch nor a select touches them before their use
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int cc = 16 * b + c;
      const bool in = ok && c >= clo && c <= chi;
      cf[c] = gld(in ? (TRANS ? &A.at(cc, i) : &A.at(i, cc)) : zero_entry<T>());
    }
  };
  // entries (r16, 4 g4 + c4) of the inverse of the diagonal block of step sp
  auto fetch_dv = [&](int sp, T (&dvv)[4]) __attribute__((always_inline)) {
    const int b = blk_of(sp < nb ? sp : nb - 1);
    const T* D = dinv + (int64_t)b * dinv_stride() + (USE_U ? 256 : 0);
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) {
      const int c = 4 * g4 + c4;
      dvv[c4] = gld(TRANS ? D + c * 16 + r16 : D + r16 * 16 + c);
    }
  };

  // ring of NS = PD + 1 prefetched steps; the step loop is unrolled by NS so
  // that step s always uses slot s mod NS and refills it for step s + NS
  constexpr int NS = PD + 1;
  T cf[NS][16];
  T dv[NS][4];
  // right-hand side of this thread's row, one copy per ring slot: a thread
  // moves to a new row at most once in HT + 1 >= NS steps, so the copy
  // loaded NS steps before a use holds the row it publishes
  T rv[NS];
#pragma unroll
  for (int d = 0; d < NS; ++d) {
    if constexpr (!TRANS) fetch_cf(d, cf[d]);
    fetch_dv(d, dv[d]);
    const int i = row_of(pos);
    rv[d] = (T)src.load_always(i, 0, act && pos < mp && i < m);
  }

  // transposed operators: cooperative loads of the coefficients of step sp
  // (element e = 16 q + c: row q of the ring past the block, column c),
  // staged in LDS block (sp & 1) one step before they are used
  constexpr int NQ = 16 * HT;                  // ring rows past the block
  constexpr int CPT = (NQ * 16 + NT - 1) / NT;   // staged coefficients per thread
  constexpr int CP = 17;                       // LDS pitch of a row
  T* cfl = lds + 32;
  T stg[NS][CPT];
  auto stage_load = [&](int sp, T (&r)[CPT]) __attribute__((always_inline)) {
    const int b = blk_of(sp < nb ? sp : nb - 1);
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int e = tid + NT * u, q = e >> 4, c = e & 15;
      const int pp = 16 * sp + 16 + q, i = row_of(pp), cc = 16 * b + c;
      const int d = FWD ? i - cc : cc - i;
      const bool in = q < NQ && sp < nb && pp < mp && i < m && cc < m && d >= 1 && d <= reach;
      r[u] = gld(in ? &A.at(cc, i) : zero_entry<T>());
    }
  };
  auto stage_store = [&](int sp, const T (&r)[CPT]) __attribute__((always_inline)) {
    T* blk = cfl + (sp & 1) * NQ * CP;
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int e = tid + NT * u, q = e >> 4, c = e & 15;
      if (q < NQ) sst(blk + q * CP + c, r[u]);
    }
  };
  if constexpr (TRANS) {
#pragma unroll
    for (int d = 0; d < NS; ++d) stage_load(d, stg[d]);
    stage_store(0, stg[0]);   // made visible by the first step's barrier
  }

  auto step = [&](int s, T (&cfs)[16], T (&dvs)[4], T (&stg_s)[CPT], T (&stg_n)[CPT], T& rhs) __attribute__((always_inline)) {
    const int b = blk_of(s);
    T* wb = lds + (s & 1) * 16;
    const bool cur = act && pos < 16 * s + 16;
    if (cur) sst(wb + row_of(pos) - 16 * b, rhs - upd);
    // threads exchange only LDS data within the sweep (each row's right-hand
    // side is read by the thread that later publishes it, before it is
    // stored), so the prefetches of later steps stay in flight
    lds_barrier();
    // x = D_b^{-1} w_b; lane holds x of row 16 b + r16
    T xp = T(0);
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) xp += dvs[c4] * sld(wb + 4 * g4 + c4);
    xp = pair_sum16(xp);
    xp = pair_sum32(xp);
    if (tid < 16 && 16 * b + tid < m) dst.store(16 * b + tid, 0, (double)xp);
    T xs[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) xs[c] = lane_read(xp, c);
    if (act && !cur) {
      T cv[16];
      if constexpr (TRANS) {
        const T* row = cfl + (s & 1) * NQ * CP + (pos - 16 * s - 16) * CP;
#pragma unroll
        for (int c = 0; c < 16; ++c) cv[c] = sld(row + c);
      } else {
#pragma unroll
        for (int c = 0; c < 16; ++c) cv[c] = cfs[c];
      }
      T a4[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int c = 0; c < 16; ++c) a4[c & 3] += cv[c] * xs[c];
      upd += (a4[0] + a4[1]) + (a4[2] + a4[3]);
    }
    {
      // the current block's threads move to the rows entering the ring; every
      // thread then reloads its row's right-hand side into this slot's copy,
      // so the load needs no select and is first used NS steps later
      pos = cur ? pos + RS : pos;
      upd = cur ? T(0) : upd;
      const int i = row_of(pos);
      rhs = (T)src.load_always(i, 0, act && pos < mp && i < m);
    }
    if constexpr (TRANS) {
      // step s + 1's coefficients (loaded NS - 1 steps ago) into the other
      // LDS block, read after the next barrier; then this slot's registers
      // start the loads of step s + NS
      stage_store(s + 1, stg_n);
      stage_load(s + NS, stg_s);
    } else {
      fetch_cf(s + NS, cfs);
    }
    fetch_dv(s + NS, dvs);
  };
  // whole groups of NS steps in the loop, so that every path around it
  // issues the same loads and the waits for prefetched data stay exact;
  // the last partial group after it
  int s0 = 0;
  for (; s0 + NS <= nb; s0 += NS) {
    static_for<0, NS>([&](auto D) __attribute__((always_inline)) {
      constexpr int d = decltype(D)::value;
      step(s0 + d, cf[d], dv[d], stg[d], stg[(d + 1) % NS], rv[d]);
    });
  }
  static_for<0, NS>([&](auto D) __attribute__((always_inline)) {
    constexpr int d = decltype(D)::value;
    if (s0 + d < nb) step(s0 + d, cf[d], dv[d], stg[d], stg[(d + 1) % NS], rv[d]);
  });
  __syncthreads();   // the last block's LDS reads before the caller reuses LDS
}

// Full sweep of columns [c0, ncol) of a leaf on the tile engine, or on the
// matrix-vector engine when it is a single column and the ring fits.
template <typename T, int HT, int OP, typename Acc>
__device__ __forceinline__ void leaf_sweep(const Acc& A, const T* dinv, const TSrc& src, const TDst& dst, int c0,
                                           int ncol, T* lds) {
  if constexpr (16 * (HT + 1) <= NT) {
    if (ncol - c0 == 1 && c0 == 0) {
      gemv_sweep<T, HT, OP>(A, dinv, src, dst, lds);
      return;
    }
  }
  tile_sweep<T, HT, OP>(A, dinv, src, dst, c0, ncol, lds);
}

}  // namespace spike
