// Workgroup-cooperative device primitives of the SPIKE solver (gfx950).
//
// Every routine here is executed by a whole workgroup of NT threads and
// synchronises with __syncthreads() between phases.  Matrices are reached
// through small accessor structs so the same code serves the banded
// partition blocks (LAPACK band storage) and the dense interface systems.
//
// Block pivoting convention.  The LU is blocked right-looking with panel
// width NB.  Inside a panel the row interchanges are applied to all NB panel
// columns; the L columns of earlier panels are not permuted.  The matching
// forward sweep therefore applies, per panel J, the panel's interchanges to
// the right-hand side, then the unit-lower diagonal block, then the
// sub-diagonal block:  L^{-1} P = prod_J (Lt_J^{-1} P_J).  The transposed
// sweep undoes it in reverse: for J from last to first, Lt_J^{-T} then P_J^T.
// Pivot rows are recorded as absolute (block-local) row numbers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "spike_types.hpp"

namespace spike {

// Loads and stores through an explicitly global (address space 1) or LDS
// (address space 3) pointer.  Device functions that receive pointers as
// generic ones would otherwise use flat instructions, which count against
// the LDS wait counter too, so that every LDS wait would also wait for the
// global loads in flight.
// f(integral_constant<int, i>) for i = B .. E-1, unrolled at compile time.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

template <typename T>
__device__ __forceinline__ T gld(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ void gst(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}
template <typename T>
__device__ __forceinline__ T sld(const T* p) {
  return *(const __attribute__((address_space(3))) T*)p;
}
template <typename T>
__device__ __forceinline__ void sst(T* p, T v) {
  *(__attribute__((address_space(3))) T*)p = v;
}

constexpr int NT = 256;      // threads per workgroup of the leaf and merge kernels
constexpr int NWAVE = NT / 64;

// Logical index of workgroup b of a G-workgroup launch such that the
// workgroups of consecutive logical indices run on one XCD: workgroups are
// handed to the XCDs round-robin (b mod NXCD), and XCD x takes the logical
// range that starts after those of XCDs 0 .. x-1.  Workgroups that read the
// same operands (the column groups of one partition, the tiles of one
// merge) then share an L2.  A bijection of [0, G) for any G.
// Zeros in global memory, never written: the address that loads of entries
// outside the stored data read instead, so that such loads need neither a
// branch nor a select on their value (both would pull the wait for a
// prefetched load to the point of issue).
__device__ double kZeroEntries[2] = {0.0, 0.0};
template <typename T>
__device__ __forceinline__ const T* zero_entry() {
  return reinterpret_cast<const T*>(kZeroEntries);
}

constexpr int NXCD = 8;

// Workgroup barrier that waits only for this wavefront's LDS (and scalar
// memory) operations.  __syncthreads() also waits for every global load in
// flight, which would pull loads issued for later steps onto each step's
// chain.  Only for loops whose threads exchange data through LDS alone; the
// memory clobber keeps the compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }
__device__ __forceinline__ int xcd_grouped(int b, int G) {
  const int x = b % NXCD, s = b / NXCD, q = G / NXCD, r = G % NXCD;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + s;
}


// Band storage: element (i, c), 0-based, at a[(kuw + i - c) + c * ldw],
// for -kuw <= i - c <= kl.  With partial pivoting kuw = kl + ku (U fill).
//
// With partial pivoting the interchanges of a panel move multipliers of
// earlier panel columns up to NB - 1 rows below the band, where band storage
// has no slot.  So a pivoting factorisation keeps each panel's L block as a
// dense (NB + kl) x NB tile (`lp`, leading dimension lpld, one tile per panel)
// and band storage holds U only.
template <typename T>
struct BandAcc {
  T* a;
  int m, kl, kuw;
  int64_t ldw;
  const int* ipiv;  // block pivots (nullptr: no pivoting)
  T* lp;            // dense L tiles of the panels (pivoting), else nullptr
  int64_t lpld;
  __device__ __forceinline__ T& at(int i, int c) const {
    return a[(int64_t)(kuw + i - c) + (int64_t)c * ldw];
  }
  __device__ __forceinline__ T gl(int i, int c) const { return gld(&a[(int64_t)(kuw + i - c) + (int64_t)c * ldw]); }
  __device__ __forceinline__ bool in(int i, int c) const {
    int d = i - c;
    return d <= kl && -d <= kuw;
  }
  __device__ __forceinline__ T* lpanel(int J, int nb) const {
    return lp ? lp + (int64_t)(J / nb) * lpld * nb : nullptr;
  }
};

// Dense column-major matrix seen as a band with full bandwidth.
template <typename T>
struct DenseAcc {
  T* a;
  int m, kl, kuw;   // kl = kuw = m - 1
  int64_t ld;
  const int* ipiv;
  int64_t lpld = 0;
  __device__ __forceinline__ T& at(int i, int c) const { return a[i + (int64_t)c * ld]; }
  __device__ __forceinline__ T gl(int i, int c) const { return gld(&a[i + (int64_t)c * ld]); }
  __device__ __forceinline__ bool in(int, int) const { return true; }
  __device__ __forceinline__ T* lpanel(int, int) const { return nullptr; }
};

// Right-hand-side block: element (r, c) at p[(r - r0) * rs + c * ld].
// rs = -1 addresses a partition in the reversed frame.
template <typename V>
struct Mat {
  V* p;
  int64_t rs, ld;
  int r0;
  __device__ __forceinline__ V& at(int r, int c) const {
    return p[(int64_t)(r - r0) * rs + (int64_t)c * ld];
  }
};

template <typename V>
__device__ __forceinline__ Mat<V> make_mat(V* p, int64_t rs, int64_t ld, int r0 = 0) {
  Mat<V> m;
  m.p = p;
  m.rs = rs;
  m.ld = ld;
  m.r0 = r0;
  return m;
}

template <typename T>
__device__ __forceinline__ void swapv(T& a, T& b) {
  T t = a;
  a = b;
  b = t;
}

// Order-preserving bits of a non-negative double (for atomicMin).
__device__ __forceinline__ unsigned long long dbits(double x) {
  return (unsigned long long)__double_as_longlong(x);
}

struct LuStats {
  int first_zero;   // local index of the first exactly-zero pivot, -1 if none
  int boosts;
  double min_piv;
};

// ---------------------------------------------------------------------------
// Blocked right-looking LU (partial pivoting when ipiv_out != nullptr),
// in place through the accessor.  `boost` > 0 enables diagonal boosting
// (non-pivoting only): |u_jj| < boost  ->  u_jj += sign(u_jj) * boost.
// LDS: (NB + kl) * NB + NB * kuw elements of T, plus 64 ints.
// Statistics are valid in thread 0.
// ---------------------------------------------------------------------------
template <int NB, typename T, typename Acc>
__device__ void wg_lu(const Acc& A, int* ipiv_out, T boost, T* lds, LuStats& st) {
  const int tid = threadIdx.x;
  const int m = A.m, kl = A.kl, kuw = A.kuw;
  const int ldP = NB + kl;
  T* P = lds;
  T* U = lds + (size_t)ldP * NB;
  int* sI = reinterpret_cast<int*>(U + (size_t)NB * (kuw > 0 ? kuw : 1));
  int* sPiv = sI + 4;
  if (tid == 0) {
    st.first_zero = -1;
    st.boosts = 0;
    st.min_piv = __builtin_huge_val();
  }
  for (int J = 0; J < m; J += NB) {
    const int jb = min(NB, m - J);
    const int prow = min(m - J, jb + kl);
    for (int idx = tid; idx < prow * jb; idx += NT) {
      int r = idx % prow, c = idx / prow;
      int i = J + r, col = J + c;
      P[r + c * ldP] = A.in(i, col) ? A.at(i, col) : T(0);
    }
    __syncthreads();
    for (int t = 0; t < jb; ++t) {
      const int rend = min(prow, t + kl + 1);
      if (ipiv_out) {
        if (tid < 64) {
          T best = T(-1);
          int bi = t;
          for (int r = t + tid; r < rend; r += 64) {
            T v = fabs(P[r + t * ldP]);
            if (v > best) { best = v; bi = r; }
          }
          for (int off = 32; off > 0; off >>= 1) {
            T ob = __shfl_xor(best, off);
            int oi = __shfl_xor(bi, off);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
          }
          if (tid == 0) { sI[0] = bi; sPiv[t] = J + bi; }
        }
        __syncthreads();
        const int r = sI[0];
        if (r != t)
          for (int c = tid; c < jb; c += NT) swapv(P[t + c * ldP], P[r + c * ldP]);
        __syncthreads();
      }
      if (tid == 0) {
        T piv = P[t + t * ldP];
        if (boost > T(0) && fabs(piv) < boost) {
          piv = piv >= T(0) ? piv + boost : piv - boost;
          P[t + t * ldP] = piv;
          st.boosts++;
        }
        double ap = (double)fabs(piv);
        if (ap < st.min_piv) st.min_piv = ap;
        if (piv == T(0) && st.first_zero < 0) st.first_zero = J + t;
      }
      __syncthreads();
      const T piv = P[t + t * ldP];
      for (int r = t + 1 + tid; r < rend; r += NT)
        P[r + t * ldP] = piv != T(0) ? P[r + t * ldP] / piv : T(0);
      __syncthreads();
      const int nr = rend - (t + 1), nc = jb - (t + 1);
      for (int idx = tid; idx < nr * nc; idx += NT) {
        int r = t + 1 + idx % nr, c = t + 1 + idx / nr;
        P[r + c * ldP] -= P[r + t * ldP] * P[t + c * ldP];
      }
      __syncthreads();
    }
    T* lpb = A.lpanel(J, NB);
    for (int idx = tid; idx < prow * jb; idx += NT) {
      int r = idx % prow, c = idx / prow;
      int i = J + r, col = J + c;
      if (lpb && r > c) lpb[r + (int64_t)c * A.lpld] = P[r + c * ldP];
      else if (A.in(i, col)) A.at(i, col) = P[r + c * ldP];
    }
    if (ipiv_out)
      for (int t = tid; t < jb; t += NT) ipiv_out[J + t] = sPiv[t];
    const int cend = min(m, J + jb + kuw);
    if (ipiv_out) {
      for (int c = J + jb + tid; c < cend; c += NT) {
        for (int t = 0; t < jb; ++t) {
          const int r1 = J + t, r2 = sPiv[t];
          if (r2 != r1 && c - r1 <= kuw) swapv(A.at(r1, c), A.at(r2, c));
        }
      }
    }
    __syncthreads();
    const int ncu = cend - (J + jb);
    if (ncu > 0) {
      for (int idx = tid; idx < jb * ncu; idx += NT) {
        int r = idx % jb, c = idx / jb;
        int i = J + r, col = J + jb + c;
        U[r + c * NB] = A.in(i, col) ? A.at(i, col) : T(0);
      }
      __syncthreads();
      for (int c = tid; c < ncu; c += NT) {
        T x[NB];
#pragma unroll
        for (int r = 0; r < NB; ++r) x[r] = r < jb ? U[r + c * NB] : T(0);
#pragma unroll
        for (int r = 1; r < NB; ++r) {
          T s = x[r];
#pragma unroll
          for (int t = 0; t < r; ++t) s -= P[r + t * ldP] * x[t];
          x[r] = s;
        }
#pragma unroll
        for (int r = 0; r < NB; ++r)
          if (r < jb) U[r + c * NB] = x[r];
      }
      __syncthreads();
      for (int idx = tid; idx < jb * ncu; idx += NT) {
        int r = idx % jb, c = idx / jb;
        int i = J + r, col = J + jb + c;
        if (A.in(i, col)) A.at(i, col) = U[r + c * NB];
      }
      const int nr2 = prow - jb;
      for (int idx = tid; idx < nr2 * ncu; idx += NT) {
        int r = jb + idx % nr2, c = idx / nr2;
        int i = J + r, col = J + jb + c;
        if (!A.in(i, col)) continue;
        T s = T(0);
        for (int t = 0; t < jb; ++t) s += P[r + t * ldP] * U[t + c * NB];
        A.at(i, col) -= s;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Forward sweep X <- L^{-1} P X (unit lower, block pivots), rows from the
// panel containing row_start to the end; rows above are neither read nor
// written (their right-hand side must be zero for the result to be exact).
// LDS: (NB + kl) * NB elements of T plus NB ints.
// ---------------------------------------------------------------------------
template <int NB, typename T, typename Acc, typename V>
__device__ void wg_lsweep(const Acc& A, const Mat<V>& X, int ncol, int row_start, T* lds) {
  const int tid = threadIdx.x;
  const int m = A.m, kl = A.kl;
  const int ldP = NB + kl;
  T* P = lds;
  int* sPiv = reinterpret_cast<int*>(P + (size_t)ldP * NB);
  for (int J = (max(row_start, 0) / NB) * NB; J < m; J += NB) {
    const int jb = min(NB, m - J);
    const int prow = min(m - J, jb + kl);
    const T* lpb = A.lpanel(J, NB);
    for (int idx = tid; idx < prow * jb; idx += NT) {
      int r = idx % prow, c = idx / prow;
      int i = J + r, col = J + c;
      P[r + c * ldP] = r <= c ? T(0)
                              : (lpb ? lpb[r + (int64_t)c * A.lpld] : (A.in(i, col) ? A.at(i, col) : T(0)));
    }
    if (A.ipiv)
      for (int t = tid; t < jb; t += NT) sPiv[t] = A.ipiv[J + t];
    __syncthreads();
    for (int q = tid; q < ncol; q += NT) {
      if (A.ipiv)
        for (int t = 0; t < jb; ++t) {
          int r2 = sPiv[t];
          if (r2 != J + t) swapv(X.at(J + t, q), X.at(r2, q));
        }
      T x[NB];
#pragma unroll
      for (int r = 0; r < NB; ++r) x[r] = r < jb ? (T)X.at(J + r, q) : T(0);
#pragma unroll
      for (int r = 1; r < NB; ++r) {
        T s = x[r];
#pragma unroll
        for (int t = 0; t < r; ++t) s -= P[r + t * ldP] * x[t];
        x[r] = s;
      }
#pragma unroll
      for (int r = 0; r < NB; ++r)
        if (r < jb) X.at(J + r, q) = (V)x[r];
    }
    __syncthreads();
    const int nr = prow - jb;
    for (int idx = tid; idx < nr * ncol; idx += NT) {
      int r = jb + idx % nr, q = idx / nr;
      T s = T(0);
      for (int t = 0; t < jb; ++t) s += P[r + t * ldP] * (T)X.at(J + t, q);
      X.at(J + r, q) = (V)((T)X.at(J + r, q) - s);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Backward sweep X <- U^{-1} X restricted to rows [row_min, m): only U
// entries with both indices >= row_min are used, so with row_min > 0 this is
// the solve with the trailing principal block of U.
// LDS: (NB + kuw) * NB elements of T.
// ---------------------------------------------------------------------------
template <int NB, typename T, typename Acc, typename V>
__device__ void wg_usweep(const Acc& A, const Mat<V>& X, int ncol, int row_min, T* lds) {
  const int tid = threadIdx.x;
  const int m = A.m, kuw = A.kuw;
  const int ldP = NB + kuw;
  T* P = lds;   // P[(i - (J - kuw)) + c * ldP] = U(i, J + c)
  if (m <= 0) return;
  for (int J = ((m - 1) / NB) * NB; J >= 0; J -= NB) {
    const int jb = min(NB, m - J);
    if (J + jb <= row_min) break;
    const int r0 = max(row_min, J - kuw);
    const int nrows = J + jb - r0;
    const int base = J - kuw;
    for (int idx = tid; idx < nrows * jb; idx += NT) {
      int rr = idx % nrows, c = idx / nrows;
      int i = r0 + rr, col = J + c;
      P[(i - base) + c * ldP] = (i <= col && A.in(i, col)) ? A.at(i, col) : T(0);
    }
    __syncthreads();
    const int lo = max(J, row_min) - J;
    for (int q = tid; q < ncol; q += NT) {
      T x[NB];
#pragma unroll
      for (int r = 0; r < NB; ++r) x[r] = (r < jb && r >= lo) ? (T)X.at(J + r, q) : T(0);
#pragma unroll
      for (int r = NB - 1; r >= 0; --r) {
        if (r < jb && r >= lo) {
          x[r] = x[r] / P[(J + r - base) + r * ldP];
#pragma unroll
          for (int t = 0; t < r; ++t) x[t] -= P[(J + t - base) + r * ldP] * x[r];
        }
      }
#pragma unroll
      for (int r = 0; r < NB; ++r)
        if (r < jb && r >= lo) X.at(J + r, q) = (V)x[r];
    }
    __syncthreads();
    const int nr = J - r0;
    for (int idx = tid; idx < nr * ncol; idx += NT) {
      int i = r0 + idx % nr, q = idx / nr;
      T s = T(0);
      for (int t = 0; t < jb; ++t) s += P[(i - base) + t * ldP] * (T)X.at(J + t, q);
      X.at(i, q) = (V)((T)X.at(i, q) - s);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Forward transposed sweep X <- U^{-T} X on rows [row_min, m), rows below
// row_min treated as zero (left-looking).  LDS: (NB + kuw) * NB elements.
// ---------------------------------------------------------------------------
template <int NB, typename T, typename Acc, typename V>
__device__ void wg_utsweep(const Acc& A, const Mat<V>& X, int ncol, int row_min, T* lds) {
  const int tid = threadIdx.x;
  const int m = A.m, kuw = A.kuw;
  const int ldP = NB + kuw;
  T* P = lds;   // P[(i - (J - kuw)) + c * ldP] = U(i, J + c)
  for (int J = (max(row_min, 0) / NB) * NB; J < m; J += NB) {
    const int jb = min(NB, m - J);
    const int r0 = max(row_min, J - kuw);
    const int base = J - kuw;
    // Rows [J, row_min) of the first panel hold zeros in P: the substitution
    // below multiplies them by the zero right-hand side, and stale LDS there
    // could be a NaN pattern.
    const int lrow = min(r0, J);
    const int nrows = J + jb - lrow;
    for (int idx = tid; idx < nrows * jb; idx += NT) {
      int rr = idx % nrows, c = idx / nrows;
      int i = lrow + rr, col = J + c;
      P[(i - base) + c * ldP] = (i >= row_min && i <= col && A.in(i, col)) ? A.at(i, col) : T(0);
    }
    __syncthreads();
    const int lo = max(J, row_min);
    const int nr = J + jb - lo, nk = J - r0;
    if (nk > 0) {
      for (int idx = tid; idx < nr * ncol; idx += NT) {
        int i = lo + idx % nr, q = idx / nr;
        T s = T(0);
        for (int c = r0; c < J; ++c) s += P[(c - base) + (i - J) * ldP] * (T)X.at(c, q);
        X.at(i, q) = (V)((T)X.at(i, q) - s);
      }
    }
    __syncthreads();
    const int lor = lo - J;
    for (int q = tid; q < ncol; q += NT) {
      T x[NB];
#pragma unroll
      for (int r = 0; r < NB; ++r) x[r] = (r < jb && r >= lor) ? (T)X.at(J + r, q) : T(0);
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        if (r < jb && r >= lor) {
          T s = x[r];
#pragma unroll
          for (int t = 0; t < r; ++t) s -= P[(J + t - base) + r * ldP] * x[t];
          x[r] = s / P[(J + r - base) + r * ldP];
        }
      }
#pragma unroll
      for (int r = 0; r < NB; ++r)
        if (r < jb && r >= lor) X.at(J + r, q) = (V)x[r];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Backward transposed sweep X <- P^T L^{-T} X (left-looking from the bottom),
// processing panels from the last one down to the panel containing row_min.
// Rows at or below the bottom of that panel's reach are exact.
// LDS: (NB + kl) * NB elements of T plus NB ints.
// ---------------------------------------------------------------------------
template <int NB, typename T, typename Acc, typename V>
__device__ void wg_ltsweep(const Acc& A, const Mat<V>& X, int ncol, int row_min, T* lds) {
  const int tid = threadIdx.x;
  const int m = A.m, kl = A.kl;
  const int ldP = NB + kl;
  T* P = lds;   // P[(i - J) + c * ldP] = L(i, J + c), i > J + c
  int* sPiv = reinterpret_cast<int*>(P + (size_t)ldP * NB);
  if (m <= 0) return;
  const int Jstop = (max(row_min, 0) / NB) * NB;
  for (int J = ((m - 1) / NB) * NB; J >= Jstop; J -= NB) {
    const int jb = min(NB, m - J);
    const int rend = min(m, J + jb + kl);
    const int nrows = rend - J;
    const T* lpb = A.lpanel(J, NB);
    for (int idx = tid; idx < nrows * jb; idx += NT) {
      int r = idx % nrows, c = idx / nrows;
      int i = J + r, col = J + c;
      P[r + c * ldP] = r <= c ? T(0)
                              : (lpb ? lpb[r + (int64_t)c * A.lpld] : (A.in(i, col) ? A.at(i, col) : T(0)));
    }
    if (A.ipiv)
      for (int t = tid; t < jb; t += NT) sPiv[t] = A.ipiv[J + t];
    __syncthreads();
    const int nk = rend - (J + jb);
    if (nk > 0) {
      for (int idx = tid; idx < jb * ncol; idx += NT) {
        int r = idx % jb, q = idx / jb;
        T s = T(0);
        for (int t = jb; t < nrows; ++t) s += P[t + r * ldP] * (T)X.at(J + t, q);
        X.at(J + r, q) = (V)((T)X.at(J + r, q) - s);
      }
    }
    __syncthreads();
    for (int q = tid; q < ncol; q += NT) {
      T x[NB];
#pragma unroll
      for (int r = 0; r < NB; ++r) x[r] = r < jb ? (T)X.at(J + r, q) : T(0);
#pragma unroll
      for (int r = NB - 1; r >= 0; --r) {
        if (r < jb) {
          T s = x[r];
#pragma unroll
          for (int t = r + 1; t < NB; ++t)
            if (t < jb) s -= P[t + r * ldP] * x[t];
          x[r] = s;
        }
      }
#pragma unroll
      for (int r = 0; r < NB; ++r)
        if (r < jb) X.at(J + r, q) = (V)x[r];
      if (A.ipiv)
        for (int t = jb - 1; t >= 0; --t) {
          int r2 = sPiv[t];
          if (r2 != J + t) swapv(X.at(J + t, q), X.at(r2, q));
        }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Workgroup GEMM on global memory: C = alpha * A * B + beta * C, with A (M x K)
// element (i, k) at A.p[i * A.rs + k * A.cs] (so transposes are stride swaps),
// B (K x N) likewise, C column-major with leading dimension ldc.  C must not
// alias A or B.  LDS: 2 * 64 * 17 doubles.
// ---------------------------------------------------------------------------
struct GM {
  const double* p;
  int64_t rs, cs;
};

__device__ __forceinline__ GM gm(const double* p, int64_t rs, int64_t cs) {
  GM g;
  g.p = p;
  g.rs = rs;
  g.cs = cs;
  return g;
}

__device__ inline void wg_gemm(int M, int N, int K, double alpha, GM A, GM B, double beta,
                               double* C, int64_t ldc, double* lds) {
  const int tid = threadIdx.x;
  double* As = lds;              // [16][64+1] : As[k * 65 + i]
  double* Bs = lds + 16 * 65;    // [16][64+1] : Bs[k * 65 + j]
  const int ti = tid % 16, tj = tid / 16;
  for (int i0 = 0; i0 < M; i0 += 64) {
    for (int j0 = 0; j0 < N; j0 += 64) {
      double acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
      for (int k0 = 0; k0 < K; k0 += 16) {
        for (int idx = tid; idx < 16 * 64; idx += NT) {
          int ii = idx % 64, kk = idx / 64;
          int gi = i0 + ii, gk = k0 + kk;
          As[kk * 65 + ii] = (gi < M && gk < K) ? A.p[(int64_t)gi * A.rs + (int64_t)gk * A.cs] : 0.0;
          int jj = idx / 16, kb = idx % 16;
          int gj = j0 + jj, gkb = k0 + kb;
          Bs[kb * 65 + jj] = (gj < N && gkb < K) ? B.p[(int64_t)gkb * B.rs + (int64_t)gj * B.cs] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
          double av[4], bv[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) av[a] = As[kk * 65 + ti + 16 * a];
#pragma unroll
          for (int b = 0; b < 4; ++b) bv[b] = Bs[kk * 65 + tj + 16 * b];
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] += av[a] * bv[b];
        }
        __syncthreads();
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          int gi = i0 + ti + 16 * a, gj = j0 + tj + 16 * b;
          if (gi < M && gj < N) {
            double* c = &C[gi + (int64_t)gj * ldc];
            *c = (beta == 0.0 ? 0.0 : beta * *c) + alpha * acc[a][b];
          }
        }
    }
  }
  __syncthreads();
}

// Copy an M x N block (column-major, leading dims lds/ldd), optional scale.
__device__ inline void wg_copy(int M, int N, const double* S, int64_t lds_, double* D, int64_t ldd,
                               double scale = 1.0) {
  for (int idx = threadIdx.x; idx < M * N; idx += NT) {
    int i = idx % M, j = idx / M;
    D[i + (int64_t)j * ldd] = scale * S[i + (int64_t)j * lds_];
  }
}

}  // namespace spike
