// Descriptors shared by the host planner and the device kernels.
#pragma once
#include <cstdint>

namespace spike {

// Leaf (partition) roles.  The last partition of a multi-partition plan is
// factored UL; we hold it as the LU factorisation of Q A_p Q (Q = reversal,
// eq. Qmat), so it is stored and swept in a reversed row/column frame and
// behaves exactly like the first partition in that frame.
enum LeafType : int32_t { LEAF_SINGLE = 0, LEAF_FIRST = 1, LEAF_MIDDLE = 2, LEAF_LAST = 3 };

struct LeafDesc {
  int64_t start;      // first global row of the partition
  int32_t m;          // partition order n_i
  int32_t type;       // LeafType
  int64_t band_off;   // element offset of the block factors in the band area
  int64_t ipiv_off;   // int offset of the block pivots
  int64_t fscr_off;   // element offset of the factor-stage spike scratch (middle)
  int64_t sscr_off;   // double offset of the per-leaf solve scratch
  int64_t lp_off;     // element offset of the dense L panel tiles (pivoting)
  int64_t dinv_off;   // element offset of the diagonal-block inverses (tile engine)
};

// A merge of two adjacent nodes L = [a..mif] and R = [mif+1..b] of the
// reduced-system tree; it owns interface mif (between leaves mif and mif+1).
struct MergeDesc {
  int32_t mif;        // interface index = index of the merge node (p + mif)
  int32_t left;       // node id of L (leaf id < p, merge node p + interface)
  int32_t right;      // node id of R
  int32_t a, b;       // leaf range of the merged node J
  int32_t level;      // 1 = merges of leaves
  int32_t pad0, pad1;
};

// Contribution of merge `merge` (its index in the merge array) to interface
// `target`: kind 0 = the right-neighbour term (t part), 1 = left-neighbour
// term (b part).  Grouped by target interface.
struct Contrib {
  int32_t merge;
  int32_t kind;
};

struct DevStatus {
  unsigned long long zero_row;  // min over blocks of (global row + 1) of an exactly-zero
                                // pivot; ULLONG_MAX = none
  unsigned long long iface;     // min (interface + 1) with a singular interface system
  int32_t n_boosts;
  int32_t refine_iters;         // correction solves in the last refined solve
  unsigned long long min_pivot_bits;  // bits of min |pivot| (non-negative double)
  double berr;                  // backward error of the last refined solve (-1: none)
  int32_t refine_active;        // refinement needed (FP32 factors or boosted pivots)
  int32_t skip;                 // refinement kernels idle (inactive or converged)
  unsigned long long anorm_inf_bits;  // ||A||_inf
  unsigned long long anorm_one_bits;  // ||A||_1
};

}  // namespace spike
