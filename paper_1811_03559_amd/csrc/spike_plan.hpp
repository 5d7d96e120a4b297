// Host planner: partition sizes, leaf roles, the reduced-system merge tree
// and the workspace layout.  Pure host code (no HIP calls), so it can be
// exercised without a GPU.
#pragma once
#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/spike.h"
#include "spike_types.hpp"

namespace spike {

struct Plan {
  int64_t n = 0;
  int kl = 0, ku = 0, p = 1;
  int pivot = 0, precision = 0, nrhs_max = 64, sizing = 0;
  double K = 1.0, boost_tau = -1.0, refine_tol = 1e-13;
  int max_refine = 10;
  int nrhs_hint = 0;

  int tsize = 8;        // bytes per element of the block factors (8 or 4)
  int nb = 16;          // panel width of the leaf kernels
  int nb_dense = 16;    // panel width of the interface LU
  int kw = 0;           // kl + ku: order of an interface system
  int ldw = 1;          // leading dimension of the stored block factors
  int kuw = 0;          // stored superdiagonals of U (ku, or kl+ku pivoting)
  int kmax = 0;         // max(kl, ku)
  int side_ld = 1;      // rows of a stored truncation side block
  int levels = 0;
  size_t leaf_lds = 0, merge_lds = 0;
  bool fast = false;    // MFMA tile engine for the full sweeps (non-pivoting)
  int ht = 0;           // its window height in 16-row tiles
  size_t fast_lds = 0;
  bool mfast = false;   // reduced system on MFMA tiles (bandwidths up to 256)
  int mht = 0;          // window height (16-row tiles) for sweeps with S's factors

  std::vector<LeafDesc> leaves;
  std::vector<MergeDesc> merges;   // grouped by level, level 1 first
  std::vector<int> level_off;      // merges of level l: [level_off[l-1], level_off[l])
  std::vector<int> contrib_ptr;    // per interface, into contrib
  std::vector<Contrib> contrib;

  // Workspace layout (byte offsets from the workspace base).
  size_t off_status = 0, off_leaves = 0, off_merges = 0, off_cptr = 0, off_contrib = 0;
  size_t off_dinv = 0;
  size_t off_band = 0, off_lpan = 0, off_ipiv = 0, off_bhat = 0, off_chat = 0, off_side = 0;
  int64_t lpld = 0;    // leading dimension of a dense L panel tile (pivoting)
  size_t off_tips = 0, off_sfac = 0, off_spiv = 0, off_coef = 0, off_qw = 0;
  size_t off_fscr = 0;
  size_t off_nodeval = 0, off_st = 0, off_xint = 0, off_ztip = 0, off_crl = 0;
  size_t off_sscr = 0, off_xacc = 0, off_res = 0, off_colred = 0;
  size_t off_sdinv = 0, off_sperm = 0, off_mtmp = 0;
  size_t off_sweeps = 0;           // instrumented sweep counters
  size_t off_kp = 0;               // device copy of the kernel parameter block
  size_t total = 0;
  size_t sscr_rows = 0;            // rows of solve scratch per leaf (max)

  int64_t reduced_size() const { return (int64_t)kw * (p - 1); }
  bool refine_enabled() const { return max_refine > 0; }
};

// Bytes reserved in the workspace for the device copy of the kernel
// parameter block (used by batched launches).
constexpr size_t kKParamsBytes = 1024;

// Fills the defaults documented in spike.h.
void default_opts(spike_opts *o);

// Builds the plan.  Returns 0, or -4 for inconsistent options / sizes
// (argument codes -1..-3 are checked by the caller).  Partial pivoting is
// limited to bandwidths whose leaf kernels fit 32-column panels (about
// max(kl, ku) <= 160 with kl = ku; see kPivotMinPanel); narrow_pivot_panels
// lifts that limit for host-side replays of the kernels only.
int make_plan(int64_t n, int kl, int ku, const spike_opts &o, Plan &plan, bool narrow_pivot_panels = false);

// Narrowest panel of the partial-pivoting leaf kernels the library runs.
// The workgroup LU with 16-column panels (pivoting, bandwidths above ~160)
// faulted the GPU once with no cause shown, so it is not launched.
constexpr int kPivotMinPanel = 32;

// R13 of the load-balancing section (first/last size over inner size).
double ratio_r13(double K, double nrhs_over_k);

}  // namespace spike
