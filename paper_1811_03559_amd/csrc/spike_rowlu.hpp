// Row-per-lane LU of a 16 x 16 tile and the inverses of its factors, the
// diagonal-tile work of the block LU (the factor stage of the central-concept
// subsection: each panel step needs the LU of its diagonal block and, for the
// products on the matrix cores, the inverses of its two triangles).
#pragma once
#include "spike_tile.hpp"

namespace spike {

// The diagonal tile of a panel is factored in a row-per-lane layout: lane l
// holds row l % 16 of the tile, so each 16-lane row of the wavefront holds the
// whole tile.  Step t of an elimination passes row t from lane t to the other
// lanes of its 16-lane row with a DPP row broadcast (a register-to-register
// move, no LDS traffic and no wait on other wavefronts' LDS requests).

// Value of lane t of this lane's 16-lane row (t a constant after unrolling).
template <typename T>
__device__ __forceinline__ T row_bcast(T v, int t) {
  auto b32 = [&](int x) __attribute__((always_inline)) -> int {
    switch (t) {
      case 0: return __builtin_amdgcn_update_dpp(0, x, 0x150, 0xf, 0xf, false);
      case 1: return __builtin_amdgcn_update_dpp(0, x, 0x151, 0xf, 0xf, false);
      case 2: return __builtin_amdgcn_update_dpp(0, x, 0x152, 0xf, 0xf, false);
      case 3: return __builtin_amdgcn_update_dpp(0, x, 0x153, 0xf, 0xf, false);
      case 4: return __builtin_amdgcn_update_dpp(0, x, 0x154, 0xf, 0xf, false);
      case 5: return __builtin_amdgcn_update_dpp(0, x, 0x155, 0xf, 0xf, false);
      case 6: return __builtin_amdgcn_update_dpp(0, x, 0x156, 0xf, 0xf, false);
      case 7: return __builtin_amdgcn_update_dpp(0, x, 0x157, 0xf, 0xf, false);
      case 8: return __builtin_amdgcn_update_dpp(0, x, 0x158, 0xf, 0xf, false);
      case 9: return __builtin_amdgcn_update_dpp(0, x, 0x159, 0xf, 0xf, false);
      case 10: return __builtin_amdgcn_update_dpp(0, x, 0x15a, 0xf, 0xf, false);
      case 11: return __builtin_amdgcn_update_dpp(0, x, 0x15b, 0xf, 0xf, false);
      case 12: return __builtin_amdgcn_update_dpp(0, x, 0x15c, 0xf, 0xf, false);
      case 13: return __builtin_amdgcn_update_dpp(0, x, 0x15d, 0xf, 0xf, false);
      case 14: return __builtin_amdgcn_update_dpp(0, x, 0x15e, 0xf, 0xf, false);
      default: return __builtin_amdgcn_update_dpp(0, x, 0x15f, 0xf, 0xf, false);
    }
  };
  if constexpr (sizeof(T) == 8) {
    const long long bits = __double_as_longlong(v);
    const int lo = b32((int)(bits & 0xffffffffll)), hi = b32((int)(bits >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned int)hi << 32) | (unsigned int)lo));
  } else {
    return __int_as_float(b32(__float_as_int(v)));
  }
}

// Value of lane 15 - (l % 16) of this lane's 16-lane row (row_mirror).
template <typename T>
__device__ __forceinline__ T row_mirror(T v) {
  if constexpr (sizeof(T) == 8) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(bits & 0xffffffffll), 0x140, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), 0x140, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned int)hi << 32) | (unsigned int)lo));
  } else {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xf, 0xf, false));
  }
}

// 1/x from the hardware reciprocal estimate refined by Newton's iteration
// r <- r + r (1 - x r), which about doubles the correct bits per step (two
// steps in FP64, one in FP32): a few fused operations on the pivot chain
// instead of a correctly rounded division; within a few units in the last
// place.
template <typename T>
__device__ __forceinline__ T recip(T x) {
  if constexpr (sizeof(T) == 8) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
  } else {
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
  }
}

// LU without interchanges of the tile held by rows (a[]: in A, out L\U).
// Pivots of rows at or beyond `mrem` (padding, identity) are never boosted;
// `nb` counts the boosted ones.
template <typename T>
__device__ __forceinline__ void lu16_rows(T (&a)[16], T boost, int mrem, int& nb) {
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    // the lane index is taken afresh each step, so that the compiler does not
    // keep the comparisons of all steps alive at once
    const int r = opaque(threadIdx.x & 15);
    T piv = row_bcast(a[t], t);
    T u[16];
#pragma unroll
    for (int c = t + 1; c < 16; ++c) u[c] = row_bcast(a[c], t);   // U(t, c)
    const bool bst = boost > T(0) && t < mrem && fabs(piv) < boost;
    piv = bst ? (piv >= T(0) ? piv + boost : piv - boost) : piv;
    nb = opaque(nb + (bst ? 1 : 0));   // counted here, not kept as one flag per step
    const T rp = piv != T(0) ? recip(piv) : T(0);
    // rows above t keep their values: their multiplier is zero
    const T l = (r > t) ? a[t] * rp : T(0);
    a[t] = (r > t) ? l : (r == t ? piv : a[t]);
#pragma unroll
    for (int c = t + 1; c < 16; ++c) a[c] -= l * u[c];
  }
}

// Inverse of a unit lower triangular 16 x 16 matrix held by rows (m[c] for
// c < the lane's row r; the diagonal is implicit), into x[] by rows, by
// forward substitution: at step t row t of the inverse is final and passes
// from lane t of each 16-lane row to the others, whose rows r > t subtract
// m[t] times it.  Each 16-lane row inverts its own matrix.
template <typename T>
__device__ __forceinline__ void unit_lower_inv16_rows(const T (&m)[16], T (&x)[16]) {
  const int r0 = opaque(threadIdx.x & 15);   // not hoisted out of the caller's loop
#pragma unroll
  for (int c = 0; c < 16; ++c) x[c] = (c == r0) ? T(1) : T(0);
#pragma unroll
  for (int t = 0; t < 15; ++t) {
    const int r = opaque(threadIdx.x & 15);
    T y[16];
#pragma unroll
    for (int c = 0; c < t; ++c) y[c] = row_bcast(x[c], t);
    const T f = (r > t) ? m[t] : T(0);
#pragma unroll
    for (int c = 0; c < t; ++c) x[c] -= f * y[c];
    x[t] -= f;
  }
}

}  // namespace spike
