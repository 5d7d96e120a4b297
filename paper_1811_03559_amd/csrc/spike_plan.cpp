// Host planner for the recursive SPIKE solver.
//
// Partition sizing follows the load-balancing section of the paper: equal
// sizes, or three sizes n1 (first/last), n2 (two-thread inner partitions of
// the paper layout, as two leaves of n2 / 2) and n3 (single-thread inner)
// from R12 = n1/n2 and R13 = n1/n3: eq. R13_calculation with R12 = R13/2
// (eq. R12_calculation), or given explicitly.  With the balanced tree every
// inner partition is single-threaded (x = 0, y = p - 2), so
// n1 = n R13 / (2 R13 + p - 2) and n3 = n / (2 R13 + p - 2).
//
// The reduced system is solved over a merge tree.  The balanced tree works
// for any p: at every level adjacent nodes are paired left to right and an
// odd last node is carried up unchanged.  This gives p - 1 merges (one
// 2x2-block interface system per partition interface, as the recursive-SPIKE
// section counts) over ceil(log2 p) levels, and reduces to the paper's
// halving recursion when p is a power of two.  The paper layout (the
// distribution of threads of the flexible partitioning section) takes
// p = 2^m + r leaves: the r inner two-thread partitions, allocated in order
// from the second partition, are leaf pairs (1,2), (3,4), ..., (2r-1,2r)
// that merge first, and a complete binary tree then runs over the remaining
// 2^m nodes.
// The first and last partitions stay single-threaded, so r <= 2^m - 2.
//
// With R13 sizing the two layouts give the same sizes: the paper's R12 =
// R13/2 makes each half of a two-thread partition n2/2 = n3 rows long, and
// 2 r + (2^m - 2 - r) = p - 2 inner leaves of n3 rows remain either way.
// Explicit ratios with R12 != R13/2 size the two-thread halves apart from
// the single-thread partitions, which is the (R12, R13) plane the paper's
// ratio experiments scan.
#include "spike_plan.hpp"

#include <algorithm>
#include <cmath>

namespace spike {

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

void default_opts(spike_opts *o) {
  o->p = 0;
  o->pivot = 0;
  o->precision = 0;
  o->sizing = 0;
  o->K = 0.0;
  o->nrhs_hint = 0;
  o->nrhs_max = 64;
  o->boost_tau = -1.0;
  o->max_refine = -1;
  o->refine_tol = 1e-13;
  o->tree = 0;
  o->r12 = 0.0;
  o->r13 = 0.0;
}

// Paper tree layout: is p = 2^m + r with 0 <= r <= 2^m - 2?  Sets m2 = 2^m.
static bool paper_tree_admissible(int p, int *m2) {
  if (p < 1) return false;
  int q = 1;
  while (2 * q <= p) q *= 2;
  if (m2) *m2 = q;
  return p == q || p - q <= q - 2;
}

double ratio_r13(double K, double r) {
  // 1/(1 + K r) + (3/2 + 2 r)/(1/K + r), written over a common denominator.
  return (1.0 + 1.5 * K + 2.0 * K * r) / (1.0 + K * r);
}

// LDS (elements) needed by the leaf kernels for panel width nb.
static size_t leaf_lds_elems(int nb, int klmax, int kuwmax) {
  size_t lu = (size_t)(nb + klmax) * nb + (size_t)nb * kuwmax;
  size_t up = (size_t)(nb + kuwmax) * nb;
  return std::max(lu, up);
}

static int choose_p(int64_t n, int kl, int ku) {
  int64_t kw = std::max<int64_t>(1, kl + ku);
  int64_t min_part = std::max<int64_t>(8 * kw, 512);
  int64_t p = n / min_part;
  p = std::min<int64_t>(p, 256);
  return (int)std::max<int64_t>(1, p);
}

int make_plan(int64_t n, int kl, int ku, const spike_opts &o, Plan &pl, bool narrow_pivot_panels) {
  if (o.p < 0 || (o.pivot != 0 && o.pivot != 1) || (o.precision != 0 && o.precision != 1) ||
      (o.sizing < 0 || o.sizing > 2) || (o.tree != 0 && o.tree != 1) || o.nrhs_max < 0 ||
      o.nrhs_hint < 0 || (o.sizing == 2 && !(o.r12 > 0.0 && o.r13 > 0.0)))
    return -4;
  pl = Plan();
  pl.n = n;
  pl.kl = kl;
  pl.ku = ku;
  pl.pivot = o.pivot;
  pl.precision = o.precision;
  pl.sizing = o.sizing;
  pl.nrhs_max = o.nrhs_max > 0 ? o.nrhs_max : 64;
  pl.nrhs_hint = o.nrhs_hint;
  pl.K = o.K > 0 ? o.K : 1.0;
  pl.boost_tau = o.boost_tau;
  pl.max_refine = o.max_refine >= 0 ? o.max_refine : (o.precision == 1 ? 6 : 0);
  pl.refine_tol = o.refine_tol > 0 ? o.refine_tol : 1e-13;
  pl.tsize = o.precision == 1 ? 4 : 8;
  pl.kw = kl + ku;
  pl.kmax = std::max(kl, ku);
  pl.kuw = o.pivot ? kl + ku : ku;

  int p = o.p > 0 ? o.p : choose_p(n, kl, ku);
  if (n == 0) p = 1;
  if (p > std::max<int64_t>(n, 1)) return -4;
  int m2 = 1;
  if (o.tree == 1 && !paper_tree_admissible(p, &m2)) {
    if (o.p > 0) return -4;
    p = 2 * m2 - 2;   // the largest admissible count below 2^(m+1) - 1
  }
  pl.p = p;

  // ---- partition sizes
  std::vector<int64_t> sz(p, 0);
  if (p == 1) {
    sz[0] = n;
  } else if (o.sizing != 0 && p >= 3) {
    // R12 / R13 sizing.  With the paper layout the leaves 1 .. 2x are the
    // halves of x two-thread partitions (n2 / 2 rows each), the next y
    // leaves single-thread inner partitions (n3); the balanced tree has
    // x = 0.
    double R12, R13;
    if (o.sizing == 2) {
      R12 = o.r12;
      R13 = o.r13;
    } else {
      double r = pl.nrhs_hint > 0 ? (double)pl.nrhs_hint / std::max(1, pl.kmax) : 0.0;
      R13 = ratio_r13(pl.K, r);
      R12 = 0.5 * R13;
    }
    const int x = (o.tree == 1) ? p - m2 : 0;
    const int y = p - 2 - 2 * x;
    const double denom = 2.0 * R12 * R13 + x * R13 + y * R12;
    const int64_t n1 = (int64_t)std::floor((double)n * R12 * R13 / denom);
    const int64_t n2h = (int64_t)std::floor(0.5 * (double)n * R13 / denom);
    const int64_t n3 = (int64_t)std::floor((double)n * R12 / denom);
    sz[0] = sz[p - 1] = n1;
    for (int i = 1; i <= 2 * x; ++i) sz[i] = n2h;
    for (int i = 2 * x + 1; i < p - 1; ++i) sz[i] = n3;
    int64_t rem = n;
    for (int i = 0; i < p; ++i) rem -= sz[i];
    for (int i = 1; rem > 0; i = (i % (p - 2)) + 1, --rem) sz[i] += 1;
  } else {
    int64_t base = n / p, rem = n % p;
    for (int i = 0; i < p; ++i) sz[i] = base + (i >= p - rem ? 1 : 0);
  }
  int64_t minsz = p > 1 ? std::max(1, kl + ku) : (n > 0 ? 1 : 0);
  for (int i = 0; i < p; ++i)
    if (sz[i] < minsz || sz[i] > INT32_MAX) return -4;

  // ---- panel widths (largest that keeps the leaf kernels' LDS <= 128 KiB)
  int kuw_max = o.pivot ? kl + ku : pl.kmax;
  pl.nb = 0;
  for (int nb : {32, 16, 8}) {
    if (leaf_lds_elems(nb, pl.kmax, kuw_max) * pl.tsize <= 128 * 1024) { pl.nb = nb; break; }
  }
  if (pl.nb == 0) return -4;   // bandwidth beyond the leaf kernels' LDS budget
  if (o.pivot && pl.nb < kPivotMinPanel && !narrow_pivot_panels) return -4;
  pl.leaf_lds = leaf_lds_elems(pl.nb, pl.kmax, kuw_max) * pl.tsize + 2048;
  int kd = std::max(1, ku);   // interface LU is dense of order ku
  pl.nb_dense = 0;
  for (int nb : {32, 16, 8}) {
    if (leaf_lds_elems(nb, kd, kd) * 8 <= 128 * 1024) { pl.nb_dense = nb; break; }
  }
  if (pl.nb_dense == 0) return -4;
  pl.merge_lds = std::max<size_t>(leaf_lds_elems(pl.nb_dense, kd, kd) * 8, 2 * 64 * 17 * 8) + 2048;
  // MFMA tile engine: window heights of 1, 2, 4, 8, 10 or 16 tiles of 16 rows
  pl.fast = false;
  if (!o.pivot) {
    for (int h : {1, 2, 4, 8, 10, 16})
      if (16 * h >= pl.kmax) { pl.ht = h; pl.fast = true; break; }
  }
  if (pl.fast) {
    size_t tile = (size_t)(2 * (pl.ht + 1) * 16 * 17);
    pl.fast_lds = std::max(tile, leaf_lds_elems(16, pl.kmax, kuw_max)) * pl.tsize + 2048;
    if (pl.fast_lds > 160 * 1024) pl.fast = false;
  }
  if (pl.leaf_lds > 160 * 1024 || pl.merge_lds > 160 * 1024) return -4;
  // reduced system on MFMA tiles: S (order ku) swept with a window that
  // covers all of its 16-row blocks
  pl.mfast = false;
  if (pl.kmax <= 256) {
    for (int h : {1, 2, 4, 8, 10, 16})
      if (16 * h >= std::max(1, ku)) { pl.mht = h; pl.mfast = true; break; }
  }

  // The last block is stored reversed (bandwidths swapped), so with pivoting
  // the storage must hold max(kl, ku) + kl + ku + 1 rows for either frame.
  pl.ldw = o.pivot ? kl + ku + pl.kmax + 1 : kl + ku + 1;
  pl.side_ld = std::max(1, kl + ku);

  // ---- leaves
  pl.leaves.resize(p);
  int64_t start = 0, band = 0, piv = 0, fscr = 0, sscr = 0, lpan = 0, dinv = 0;
  pl.lpld = o.pivot ? pl.nb + pl.kmax : 0;
  size_t R = (size_t)pl.nrhs_max;
  size_t extra_rows = (size_t)pl.kw + 2 * (size_t)pl.nb;
  // every leaf's solve scratch is sscr_rows x R with leading dimension sscr_rows
  pl.sscr_rows = (size_t)*std::max_element(sz.begin(), sz.end()) + extra_rows;
  for (int i = 0; i < p; ++i) {
    LeafDesc &L = pl.leaves[i];
    L.start = start;
    L.m = (int32_t)sz[i];
    L.type = p == 1 ? LEAF_SINGLE : (i == 0 ? LEAF_FIRST : (i == p - 1 ? LEAF_LAST : LEAF_MIDDLE));
    L.band_off = band;
    L.lp_off = lpan;
    L.dinv_off = dinv;
    if (pl.fast) dinv += (sz[i] + 15) / 16 * 512;
    L.ipiv_off = piv;
    L.fscr_off = fscr;
    L.sscr_off = sscr;
    start += sz[i];
    band += sz[i] * pl.ldw;
    if (o.pivot) lpan += (sz[i] + pl.nb - 1) / pl.nb * pl.lpld * pl.nb;
    piv += sz[i];
    // factor-stage scratch (m x kw, ld m): spikes of middle blocks, the
    // truncated side solves of the first and last blocks
    if (L.type != LEAF_SINGLE) fscr += sz[i] * pl.kw;
    sscr += (int64_t)(pl.sscr_rows * R);
  }

  // ---- merge tree (a merged node takes id p + its interface index)
  struct Node { int a, b, id; };
  std::vector<Node> cur;
  for (int i = 0; i < p; ++i) cur.push_back({i, i, i});
  pl.level_off.assign(1, 0);
  int level = 0;
  auto merge = [&](const Node &Lt, const Node &Rt) {
    MergeDesc md{};
    md.mif = Lt.b;
    md.left = Lt.id;
    md.right = Rt.id;
    md.a = Lt.a;
    md.b = Rt.b;
    md.level = level;
    pl.merges.push_back(md);
    return Node{Lt.a, Rt.b, p + Lt.b};
  };
  if (o.tree == 1 && p > m2) {
    // level 1: the halves of the r two-thread partitions
    const int r = p - m2;
    ++level;
    std::vector<Node> nxt{cur[0]};
    for (int j = 0; j < r; ++j) nxt.push_back(merge(cur[1 + 2 * j], cur[2 + 2 * j]));
    for (int i = 2 * r + 1; i < p; ++i) nxt.push_back(cur[i]);
    pl.level_off.push_back((int)pl.merges.size());
    cur.swap(nxt);
  }
  while (cur.size() > 1) {
    ++level;
    std::vector<Node> nxt;
    for (size_t i = 0; i < cur.size(); i += 2) {
      if (i + 1 < cur.size()) nxt.push_back(merge(cur[i], cur[i + 1]));
      else nxt.push_back(cur[i]);
    }
    pl.level_off.push_back((int)pl.merges.size());
    cur.swap(nxt);
  }
  pl.levels = level;

  // contributions of each merge to its neighbouring interfaces (transpose solve)
  int nif = std::max(0, p - 1);
  std::vector<std::vector<Contrib>> byif(nif);
  for (size_t d = 0; d < pl.merges.size(); ++d) {
    const MergeDesc &J = pl.merges[d];
    if (J.b < p - 1) byif[J.b].push_back({(int32_t)d, 0});
    if (J.a > 0) byif[J.a - 1].push_back({(int32_t)d, 1});
  }
  pl.contrib_ptr.assign(nif + 1, 0);
  for (int m = 0; m < nif; ++m) {
    pl.contrib_ptr[m + 1] = pl.contrib_ptr[m] + (int)byif[m].size();
    for (auto &c : byif[m]) pl.contrib.push_back(c);
  }

  // ---- workspace layout
  const size_t A = 256;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + std::max<size_t>(bytes, 1), A); return o; };
  size_t kw = (size_t)pl.kw, nodes = (size_t)(2 * p - 1);
  pl.off_status = take(sizeof(DevStatus));
  pl.off_leaves = take(sizeof(LeafDesc) * p);
  pl.off_merges = take(sizeof(MergeDesc) * std::max<size_t>(1, pl.merges.size()));
  pl.off_cptr = take(sizeof(int) * (nif + 1));
  pl.off_contrib = take(sizeof(Contrib) * std::max<size_t>(1, pl.contrib.size()));
  pl.off_band = take((size_t)band * pl.tsize);
  pl.off_lpan = take((size_t)lpan * pl.tsize);
  pl.off_dinv = take((size_t)dinv * pl.tsize);
  pl.off_ipiv = take(sizeof(int) * (size_t)std::max<int64_t>(1, piv));
  pl.off_bhat = take(8 * (size_t)nif * ku * ku);
  pl.off_chat = take(8 * (size_t)nif * kl * kl);
  pl.off_side = take((size_t)2 * pl.side_ld * pl.kmax * pl.tsize);
  pl.off_tips = take(8 * nodes * kw * kw);
  pl.off_sfac = take(8 * (size_t)nif * ku * ku);
  pl.off_spiv = take(sizeof(int) * (size_t)nif * std::max(1, ku));
  pl.off_coef = take(8 * (size_t)nif * kw * kw);
  pl.off_qw = take(8 * (size_t)nif * kw * kw);
  pl.off_fscr = take((size_t)fscr * pl.tsize);
  pl.off_nodeval = take(8 * nodes * kw * R);
  pl.off_st = take(8 * (size_t)nif * kw * R);
  pl.off_xint = take(8 * (size_t)nif * kw * R);
  pl.off_ztip = take(8 * (size_t)nif * kw * R);
  pl.off_crl = take(8 * (size_t)std::max<size_t>(1, pl.merges.size()) * kw * R);
  pl.off_sscr = take(8 * (size_t)sscr);
  pl.off_sdinv = take(8 * ((size_t)nif * ((ku + 15) / 16) * 512 + 512));
  pl.off_sperm = take(sizeof(int) * (size_t)nif * std::max(1, ku));
  pl.off_mtmp = take(8 * (size_t)nif * kw * R);
  pl.off_sweeps = take(8 * 3 * 4 * 2);
  pl.off_kp = take(kKParamsBytes);
  if (pl.refine_enabled()) {
    pl.off_xacc = take(8 * (size_t)n * R);
    pl.off_res = take(8 * (size_t)n * R);
    pl.off_colred = take(8 * 4 * R);
  }
  pl.total = off;
  return 0;
}

}  // namespace spike
