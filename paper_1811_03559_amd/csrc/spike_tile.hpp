// MFMA tile engine for banded triangular sweeps with many right-hand sides.
//
// A workgroup of four wavefronts owns 64 right-hand-side columns (one 16-wide
// column tile per wavefront).  The sweep advances in 16-row blocks.  Each
// wavefront keeps, in MFMA accumulator registers, the 16 x 16 tile of the
// current block and of the HT pending blocks that the current block still
// updates (HT = ceil(bandwidth / 16)); the window shifts by one block per step
// (register moves), so no right-hand-side value is re-read from memory.
// Per step:
//   1. x_j = D_j^{-1} w_j with the 16 x 16 inverse of the diagonal block
//      (precomputed once per factorisation), an MFMA product;
//   2. x_j is written out and the pending blocks are updated,
//      W_{j+s} -= M(block j+s, block j) x_j, s = 1..HT, by MFMA products with
//      the coupling tiles of the band panel held in LDS;
//   3. the panel of the next step, loaded into registers at the start of the
//      step, is stored to the other LDS buffer; one barrier ends the step.
// The accumulator layout doubles as the B-operand layout: register i of a
// tile holds, in lane l, row r(l, i) of column l % 16, and an MFMA whose B
// operand is that register contracts over exactly those four rows when its A
// operand in lane l is A[l % 16][r(l, i)].  So x_j feeds the updates straight
// from registers.
// Operations: L X (unit lower, forward), U X (upper, backward), U^T X
// (forward) and L^T X (unit, backward), without row interchanges.
//
// MFMA operand layouts on gfx950 (16 x 16 x 4): lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16]; the result register i of lane l is
// D[(l / 16) + 4 i][l % 16] for FP64 and D[4 (l / 16) + i][l % 16] for FP32.
#pragma once
#include <hip/hip_runtime.h>

#include "spike_device.hpp"

namespace spike {

template <typename T>
struct Mf;

template <>
struct Mf<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static inline v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int l, int i) { return (l >> 4) + 4 * i; }
  // lane group (l / 16) and register of row t
  __host__ __device__ static constexpr int grp(int t) { return t & 3; }
  __host__ __device__ static constexpr int reg(int t) { return t >> 2; }
};

template <>
struct Mf<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static inline v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int l, int i) { return 4 * (l >> 4) + i; }
  __host__ __device__ static constexpr int grp(int t) { return t >> 2; }
  __host__ __device__ static constexpr int reg(int t) { return t & 3; }
};

// An opaque copy of x: values derived from it are recomputed where they are
// used instead of being hoisted out of the elimination loop and kept live.
__device__ __forceinline__ int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Orders one wavefront's LDS accesses across lanes: stores before it are
// visible to loads after it (a wavefront's LDS operations execute in order;
// the fences keep the compiler from moving accesses across the point).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// v + (the value of lane l ^ 16), resp. l ^ 32, in every lane, with the
// cross-lane swaps of gfx950 (plain VALU, no LDS crossbar).  Swapping a
// register with itself leaves the lower lanes' values in the first result
// and the upper lanes' in the second, so their sum is the pair's sum in the
// same order in both lanes of the pair.
__device__ __forceinline__ double pair_sum16(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)(b & 0xffffffffll), hi = (unsigned)((unsigned long long)b >> 32);
  const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  const double a = __longlong_as_double((long long)(((unsigned long long)h[0] << 32) | l[0]));
  const double c = __longlong_as_double((long long)(((unsigned long long)h[1] << 32) | l[1]));
  return a + c;
}
__device__ __forceinline__ double pair_sum32(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)(b & 0xffffffffll), hi = (unsigned)((unsigned long long)b >> 32);
  const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const double a = __longlong_as_double((long long)(((unsigned long long)h[0] << 32) | l[0]));
  const double c = __longlong_as_double((long long)(((unsigned long long)h[1] << 32) | l[1]));
  return a + c;
}
__device__ __forceinline__ float pair_sum16(float v) {
  const unsigned x = __float_as_uint(v);
  const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float pair_sum32(float v) {
  const unsigned x = __float_as_uint(v);
  const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// One DPP step of a max-reduction of a double: lane l combines its value with
// the value the DPP pattern `CTRL` routes to it (its own value where the
// pattern has no source lane).
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ double dpp_max_step(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
  const int slo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROW_MASK, BANK_MASK, false);
  const int shi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROW_MASK, BANK_MASK, false);
  const double o = __longlong_as_double(((long long)shi << 32) | (long long)(unsigned int)slo);
  return fmax(v, o);
}

// Maximum of v over the wavefront, returned uniformly (lane 63 gathers the
// maximum through row shifts within rows of 16 lanes and row broadcasts).
__device__ __forceinline__ double wave_max_f64(double v) {
  v = dpp_max_step<0x111, 0xf, 0xf>(v);   // row_shr:1
  v = dpp_max_step<0x112, 0xf, 0xf>(v);   // row_shr:2
  v = dpp_max_step<0x114, 0xf, 0xf>(v);   // row_shr:4
  v = dpp_max_step<0x118, 0xf, 0xf>(v);   // row_shr:8
  v = dpp_max_step<0x142, 0xa, 0xf>(v);   // row_bcast:15
  v = dpp_max_step<0x143, 0xc, 0xf>(v);   // row_bcast:31
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

// C = alpha A B + beta C for N <= 16 columns on one 16-column MFMA tile per
// 16-row block (wavefronts over the row blocks).  A(i, k) = A[i ars + k acs]
// (FP64 or FP32, used in FP64), B(k, j) = B[k brs + j bcs],
// C(i, j) = C[i crs + j ccs]; operands are read straight from global memory
// with 8 k-steps of loads in flight before their MFMAs.  Ends with a barrier.
template <typename TA>
__device__ inline void wg_gemm16x(int M, int N, int K, double alpha, const TA* A, int64_t ars, int64_t acs,
                                  const double* B, int64_t brs, int64_t bcs, double beta, double* C, int64_t crs,
                                  int64_t ccs) {
  using Mq = Mf<double>;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cl = lane & 15, kq = lane >> 4;
  const int ntile = (M + 15) / 16;
  for (int rt = wave; rt < ntile; rt += NT / 64) {
    const int i = 16 * rt + cl;
    typename Mq::v4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += 32) {
      double av[8], bv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int kk = k0 + 4 * u + kq;
        av[u] = (i < M && kk < K) ? (double)gld(A + (int64_t)i * ars + (int64_t)kk * acs) : 0.0;
        bv[u] = (cl < N && kk < K) ? gld(B + (int64_t)kk * brs + (int64_t)cl * bcs) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = Mq::mma(av[u], bv[u], acc);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 16 * rt + Mq::row(lane, q);
      if (r < M && cl < N) {
        double* c = C + (int64_t)r * crs + (int64_t)cl * ccs;
        *c = (beta == 0.0 ? 0.0 : beta * *c) + alpha * acc[q];
      }
    }
  }
  __syncthreads();
}

// The same for any N, in groups of 16 columns.
template <typename TA>
__device__ inline void wg_gemm_cols(int M, int N, int K, double alpha, const TA* A, int64_t ars, int64_t acs,
                                    const double* B, int64_t brs, int64_t bcs, double beta, double* C, int64_t crs,
                                    int64_t ccs) {
  for (int c0 = 0; c0 < N; c0 += 16)
    wg_gemm16x<TA>(M, min(16, N - c0), K, alpha, A, ars, acs, B + (int64_t)c0 * bcs, brs, bcs, beta,
                   C + (int64_t)c0 * ccs, crs, ccs);
}

// Uniform read of lane `src` (src uniform across the wavefront).
template <typename T>
__device__ __forceinline__ T lane_read(T v, int src) {
  if constexpr (sizeof(T) == 8) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
  } else {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
  }
}

enum TileOp { OP_L_FWD = 0, OP_U_BWD = 1, OP_UT_FWD = 2, OP_LT_BWD = 3 };

// Source of the right-hand side: element (r, c) at p[r * rs + c * ld] for
// rows in [lo1, hi1) or [lo2, hi2), zero elsewhere; columns below csplit are
// also zero for rows below clo.
struct TSrc {
  const void* p;
  int f64;
  int64_t rs, ld;
  int lo1, hi1, lo2, hi2;
  int csplit, clo;
  __device__ __forceinline__ double load(int r, int c) const {
    bool ok = ((r >= lo1 && r < hi1) || (r >= lo2 && r < hi2)) && (c >= csplit || r >= clo);
    if (!ok) return 0.0;
    int64_t o = (int64_t)r * rs + (int64_t)c * ld;
    return f64 ? gld(static_cast<const double*>(p) + o) : (double)gld(static_cast<const float*>(p) + o);
  }
  // load(r, c) when `want`, else 0, with the load issued either way (from a
  // global zero when the entry is not wanted or outside the source), so that
  // neither a branch nor a select touches it before its use
  __device__ __forceinline__ double load_always(int r, int c, bool want) const {
    const bool ok = want && ((r >= lo1 && r < hi1) || (r >= lo2 && r < hi2)) && (c >= csplit || r >= clo);
    const int64_t o = (int64_t)r * rs + (int64_t)c * ld;
    if (f64) return gld(ok ? static_cast<const double*>(p) + o : zero_entry<double>());
    return (double)gld(ok ? static_cast<const float*>(p) + o : zero_entry<float>());
  }
};

// Destination of the solved rows: rows [0, top) go to p1 + r*rs, rows
// [bot, m) to p2 + (r - bot)*rs, the rest are dropped.  sub != 0 subtracts
// the value from the destination instead of storing it.
struct TDst {
  void* p1;
  void* p2;
  int f64;
  int64_t rs, ld;
  int top, bot, m, sub;
  __device__ __forceinline__ void store(int r, int c, double v) const {
    if (r >= m) return;
    void* p;
    int rr;
    if (r < top) {
      p = p1;
      rr = r;
    } else if (r >= bot) {
      p = p2;
      rr = r - bot;
    } else {
      return;
    }
    int64_t o = (int64_t)rr * rs + (int64_t)c * ld;
    if (f64) {
      double* q = static_cast<double*>(p) + o;
      gst(q, sub ? gld(q) - v : v);
    } else {
      float* q = static_cast<float*>(p) + o;
      gst(q, sub ? (float)((double)gld(q) - v) : (float)v);
    }
  }
};

__host__ __device__ constexpr int tile_pad() { return 17; }   // LDS row pitch of a 16-wide tile

// LDS elements (of T) used by tile_sweep<HT>.
__host__ __device__ constexpr int tile_lds_elems(int HT) { return 2 * (HT + 1) * 16 * tile_pad(); }

// Diagonal-block inverses of a partition: block b at dinv + 512 b, the
// inverse of the unit-lower L_bb in the first 256 entries and of the upper
// U_bb in the next 256, both row-major 16 x 16 (identity beyond the order).
__host__ __device__ constexpr int dinv_stride() { return 512; }

// Value of the operator matrix M at (row i, col c) (M = L, U, U^T or L^T).
template <typename T, int OP, typename Acc>
__device__ __forceinline__ T tile_m(const Acc& A, int i, int c) {
  const int m = A.m;
  if (i < 0 || c < 0 || i >= m || c >= m) return T(0);
  if (OP == OP_L_FWD) return (i > c && A.in(i, c)) ? A.gl(i, c) : T(0);
  if (OP == OP_U_BWD) return (i <= c && A.in(i, c)) ? A.gl(i, c) : T(0);
  if (OP == OP_UT_FWD) return (c <= i && A.in(c, i)) ? A.gl(c, i) : T(0);
  return (c > i && A.in(c, i)) ? A.gl(c, i) : T(0);   // OP_LT_BWD
}

template <typename T, int HT, int OP, typename Acc>
__device__ void tile_sweep(const Acc& A, const T* dinv, const TSrc& src, const TDst& dst, int c0, int ncol,
                           T* lds) {
  using M = Mf<T>;
  using v4 = typename M::v4;
  constexpr bool FWD = (OP == OP_L_FWD || OP == OP_UT_FWD);
  constexpr bool ROWMAJOR = (OP == OP_UT_FWD || OP == OP_LT_BWD);   // panel read along band rows
  constexpr bool USE_U = (OP == OP_U_BWD || OP == OP_UT_FWD);
  constexpr bool TRANS = ROWMAJOR;
  constexpr int PADW = tile_pad();
  constexpr int PAN = (HT + 1) * 16 * PADW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = A.m, nb = (m + 15) / 16;
  const int col = c0 + 16 * wave + (lane & 15);
  const bool colok = col < ncol;
  const bool wave_active = c0 + 16 * wave < ncol;
  // this thread's element of every panel tile
  const int rr = ROWMAJOR ? (tid >> 4) : (tid & 15);
  const int cc = ROWMAJOR ? (tid & 15) : (tid >> 4);
  const int slot = rr * PADW + cc;
  const int dsrc = (USE_U ? 256 : 0) + (TRANS ? cc * 16 + rr : rr * 16 + cc);
  auto blk = [&](int step) { return FWD ? step : nb - 1 - step; };
  auto load_panel = [&](int j, T* pf) {
    pf[0] = gld(dinv + (int64_t)j * dinv_stride() + dsrc);
#pragma unroll
    for (int s = 1; s <= HT; ++s) {
      const int bi = FWD ? j + s : j - s;
      pf[s] = tile_m<T, OP>(A, 16 * bi + rr, 16 * j + cc);
    }
  };
  auto store_panel = [&](T* P, const T* pf) {
#pragma unroll
    for (int s = 0; s <= HT; ++s) sst(P + s * 16 * PADW + slot, pf[s]);
  };
  auto load_block = [&](int b) -> v4 {
    v4 v;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int r = 16 * b + M::row(lane, i);
      v[i] = (colok && b >= 0 && b < nb) ? (T)src.load(r, col) : T(0);
    }
    return v;
  };

  v4 acc[HT + 1];
#pragma unroll
  for (int s = 0; s <= HT; ++s) acc[s] = load_block(FWD ? s : nb - 1 - s);
  {
    T pf[HT + 1];
    load_panel(blk(0), pf);
    store_panel(lds, pf);
  }
  __syncthreads();

  for (int step = 0; step < nb; ++step) {
    const int j = blk(step), b = step & 1;
    const bool more = step + 1 < nb;
    T pf[HT + 1];
    if (more) load_panel(blk(step + 1), pf);
    v4 nxt = load_block(FWD ? step + HT + 1 : nb - 1 - (step + HT + 1));
    const T* P = lds + b * PAN;
    // 1. x_j = D_j^{-1} w_j
    v4 xv = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int i = 0; i < 4; ++i) xv = M::mma(sld(P + (lane & 15) * PADW + M::row(lane, i)), acc[0][i], xv);
    // 2. write x_j, update the pending blocks
    if (colok) {
#pragma unroll
      for (int i = 0; i < 4; ++i) dst.store(16 * j + M::row(lane, i), col, (double)xv[i]);
    }
    if (wave_active) {
      // the product of pending block s lands in slot s - 1 (the window
      // moves down one block per step): the last product of each chain
      // writes the register of the slot it moves to, so the window shifts
      // without register moves
      v4 t[HT + 1];
#pragma unroll
      for (int s = 1; s <= HT; ++s) t[s] = acc[s];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const T nx = -xv[i];   // (-a) b = a (-b) exactly: one negation per step, not one per product
#pragma unroll
        for (int s = 1; s <= HT; ++s)
          t[s] = M::mma(sld(P + (s * 16 + (lane & 15)) * PADW + M::row(lane, i)), nx, t[s]);
      }
#pragma unroll
      for (int s = 1; s <= HT; ++s) acc[s - 1] = t[s];
    }
    // 3. next panel into the other buffer
    if (more) store_panel(lds + (b ^ 1) * PAN, pf);
    __syncthreads();
    acc[HT] = nxt;   // (a wavefront without columns keeps zeros or stale tiles it never stores)
  }
}

// Inverses of the 16 x 16 diagonal blocks of L and U of one partition
// (non-pivoting factors), one thread per (block, column, factor): column t
// of D^{-1} by substitution.  Blocks extending beyond the order are padded
// with the identity.
template <typename T, typename Acc>
__device__ void diag_inverses(const Acc& A, T* dinv, int gtid, int gstride) {
  const int m = A.m, nb = (m + 15) / 16;
  for (int w = gtid; w < nb * 32; w += gstride) {
    const int b = w >> 5, t = w & 15;
    const bool upper = (w >> 4) & 1;
    const int o = 16 * b;
    T v[16];
    if (!upper) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        T s = (r == t) ? T(1) : T(0);
#pragma unroll
        for (int q = 0; q < r; ++q) {
          const int i = o + r, c = o + q;
          T d = (i < m && A.in(i, c)) ? A.at(i, c) : T(0);
          s -= d * v[q];
        }
        v[r] = s;
      }
    } else {
#pragma unroll
      for (int r = 15; r >= 0; --r) {
        T s = (r == t) ? T(1) : T(0);
#pragma unroll
        for (int q = r + 1; q < 16; ++q) {
          const int i = o + r, c = o + q;
          T d = (c < m && A.in(i, c)) ? A.at(i, c) : T(0);
          s -= d * v[q];
        }
        const int i = o + r;
        v[r] = i < m ? s / A.at(i, i) : s;
      }
    }
    T* D = dinv + (int64_t)b * dinv_stride() + (upper ? 256 : 0);
#pragma unroll
    for (int r = 0; r < 16; ++r) D[r * 16 + t] = v[r];
  }
}

}  // namespace spike
