// CPU replay of the workgroup (non-MFMA) kernel path of the SPIKE solver:
// the partial-pivoting leaf kernels, the generic interface-merge kernels and
// the transpose G-tip kernel, compiled for the host against the stand-in HIP
// header of this directory and run under AddressSanitizer.
//
// Every workspace region of the planner's layout is its own heap allocation
// (and every dynamic LDS buffer too), so an index that leaves its region, or
// an LDS offset beyond the launch's LDS size, stops the run with a report.
//
// Usage: emu_main IN OUT.  IN holds int64 n, kl, ku, p, pivot, nrhs, trans,
// then the band (n x (kl+ku+1), column-major LAPACK storage) and F (n x
// nrhs, column-major); OUT receives int64 info, X, then the 24 sweep
// counters of the run (the layout of KParams::sweeps).
#include <cstdio>
#include <cstdlib>
#include <map>
#include <vector>

#include "spike_kernels.hpp"
#include "spike_plan.hpp"

namespace {

using namespace spike;

// One heap allocation per workspace region, of exactly the region's size
// (the sizes the planner's layout reserves, before its 256-byte rounding).
struct Regions {
  std::map<size_t, char*> r;   // offset -> allocation
  void* at(size_t off) {
    auto it = r.find(off);
    if (it == r.end()) {
      std::fprintf(stderr, "no region at offset %zu\n", off);
      std::abort();
    }
    return it->second;
  }
};

Regions carve(const Plan& pl) {
  const size_t kw = (size_t)pl.kw, p = (size_t)pl.p, nif = p > 0 ? p - 1 : 0, nodes = 2 * p - 1;
  const size_t R = (size_t)pl.nrhs_max, ts = (size_t)pl.tsize, ku = (size_t)pl.ku, kl = (size_t)pl.kl;
  size_t band = 0, lpan = 0, dinv = 0, piv = 0, fscr = 0, sscr = 0;
  for (const LeafDesc& L : pl.leaves) {
    band += (size_t)L.m * pl.ldw;
    if (pl.pivot) lpan += (size_t)((L.m + pl.nb - 1) / pl.nb) * pl.lpld * pl.nb;
    if (pl.fast) dinv += (size_t)((L.m + 15) / 16) * 512;
    piv += (size_t)L.m;
    if (L.type != LEAF_SINGLE) fscr += (size_t)L.m * kw;
    sscr += pl.sscr_rows * R;
  }
  const size_t nm = std::max<size_t>(1, pl.merges.size());
  const std::vector<std::pair<size_t, size_t>> regions = {
      {pl.off_status, sizeof(DevStatus)},
      {pl.off_leaves, sizeof(LeafDesc) * p},
      {pl.off_merges, sizeof(MergeDesc) * nm},
      {pl.off_cptr, sizeof(int) * (nif + 1)},
      {pl.off_contrib, sizeof(Contrib) * std::max<size_t>(1, pl.contrib.size())},
      {pl.off_band, band * ts},
      {pl.off_lpan, lpan * ts},
      {pl.off_dinv, dinv * ts},
      {pl.off_ipiv, sizeof(int) * std::max<size_t>(1, piv)},
      {pl.off_bhat, 8 * nif * ku * ku},
      {pl.off_chat, 8 * nif * kl * kl},
      {pl.off_side, 2 * (size_t)pl.side_ld * pl.kmax * ts},
      {pl.off_tips, 8 * nodes * kw * kw},
      {pl.off_sfac, 8 * nif * ku * ku},
      {pl.off_spiv, sizeof(int) * nif * std::max<size_t>(1, ku)},
      {pl.off_coef, 8 * nif * kw * kw},
      {pl.off_qw, 8 * nif * kw * kw},
      {pl.off_fscr, fscr * ts},
      {pl.off_nodeval, 8 * nodes * kw * R},
      {pl.off_st, 8 * nif * kw * R},
      {pl.off_xint, 8 * nif * kw * R},
      {pl.off_ztip, 8 * nif * kw * R},
      {pl.off_crl, 8 * nm * kw * R},
      {pl.off_sscr, 8 * sscr},
      {pl.off_sdinv, 8 * (nif * ((ku + 15) / 16) * 512 + 512)},
      {pl.off_sperm, sizeof(int) * nif * std::max<size_t>(1, ku)},
      {pl.off_mtmp, 8 * nif * kw * R},
  };
  Regions out;
  for (auto& x : regions) {
    char* q = static_cast<char*>(std::malloc(x.second > 0 ? x.second : 1));
    std::memset(q, 0xff, x.second);   // NaN pattern: unwritten data that is read shows up
    out.r[x.first] = q;
  }
  return out;
}

template <int NB>
int factor_and_solve(const Plan& pl, KParams& k, LaunchCfg& c, double* B, int64_t ldb, int nrhs, bool trans) {
  hipStream_t st = nullptr;
  emu::launch(dim3(1), dim3(64), 0, [=]() { k_init_status(k.status); });
  if (int e = run_leaf_factor<NB, double>(k, c, st)) return e;
  if (k.p > 1) {
    int e = 0;
    switch (c.nb_dense) {
      case 32: e = run_merge_factor<32>(k, c, st); break;
      case 16: e = run_merge_factor<16>(k, c, st); break;
      default: e = run_merge_factor<8>(k, c, st); break;
    }
    if (e) return e;
  }
  auto merge_solve = [&](bool t) {
    switch (c.nb_dense) {
      case 32: return run_merge_solve<32>(k, c, st, nrhs, t);
      case 16: return run_merge_solve<16>(k, c, st, nrhs, t);
      default: return run_merge_solve<8>(k, c, st, nrhs, t);
    }
  };
  if (!trans) {
    if (int e = run_leaf_phase<NB, double>(k, c, st, B, ldb, nrhs, 0)) return e;
    if (k.p > 1) {
      if (int e = merge_solve(false)) return e;
      if (int e = run_leaf_phase<NB, double>(k, c, st, B, ldb, nrhs, 1)) return e;
    }
  } else {
    if (int e = run_leaf_phase<NB, double>(k, c, st, B, ldb, nrhs, 2)) return e;
    if (k.p > 1) {
      const KParams kk = k;
      emu::launch(dim3(k.p - 1), dim3(NT), 0, [=]() { k_gform(kk, B, ldb, nrhs); });
      if (int e = merge_solve(true)) return e;
      if (int e = run_leaf_phase<NB, double>(k, c, st, B, ldb, nrhs, 3)) return e;
    }
  }
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t hdr[9];
  double ratios[2];
  if (std::fread(hdr, 8, 9, f) != 9 || std::fread(ratios, 8, 2, f) != 2) return 2;
  const int64_t n = hdr[0];
  const int kl = (int)hdr[1], ku = (int)hdr[2], p = (int)hdr[3], pivot = (int)hdr[4], nrhs = (int)hdr[5];
  const bool trans = hdr[6] != 0;
  const int64_t ldab = kl + ku + 1;
  std::vector<double> ab((size_t)(n * ldab)), B((size_t)(n * nrhs));
  if (std::fread(ab.data(), 8, ab.size(), f) != ab.size() || std::fread(B.data(), 8, B.size(), f) != B.size())
    return 2;
  std::fclose(f);

  spike_opts o;
  default_opts(&o);
  o.p = p;
  o.pivot = pivot;
  o.nrhs_max = std::max(1, nrhs);
  o.tree = (int)hdr[7];
  o.sizing = (int)hdr[8];
  o.r12 = ratios[0];
  o.r13 = ratios[1];
  Plan pl;
  if (make_plan(n, kl, ku, o, pl, /*narrow_pivot_panels=*/true)) return 3;
  Regions R = carve(pl);

  KParams k;
  std::memset(&k, 0, sizeof(k));
  k.n = pl.n;
  k.kl = pl.kl;
  k.ku = pl.ku;
  k.kw = pl.kw;
  k.kmax = pl.kmax;
  k.p = pl.p;
  k.pivot = pl.pivot;
  k.ldw = pl.ldw;
  k.side_ld = pl.side_ld;
  k.R = pl.nrhs_max;
  k.sscr_ld = (int64_t)pl.sscr_rows;
  k.boost_tau = pl.pivot ? 0.0 : 1.4901161194e-8;
  k.dAB = ab.data();
  k.ldab = ldab;
  k.status = static_cast<DevStatus*>(R.at(pl.off_status));
  // descriptors: copies in their own regions, as the device holds them
  std::memcpy(R.at(pl.off_leaves), pl.leaves.data(), sizeof(LeafDesc) * pl.leaves.size());
  if (!pl.merges.empty())
    std::memcpy(R.at(pl.off_merges), pl.merges.data(), sizeof(MergeDesc) * pl.merges.size());
  if (!pl.contrib_ptr.empty())
    std::memcpy(R.at(pl.off_cptr), pl.contrib_ptr.data(), sizeof(int) * pl.contrib_ptr.size());
  if (!pl.contrib.empty())
    std::memcpy(R.at(pl.off_contrib), pl.contrib.data(), sizeof(Contrib) * pl.contrib.size());
  k.leaves = static_cast<const LeafDesc*>(R.at(pl.off_leaves));
  k.merges = static_cast<const MergeDesc*>(R.at(pl.off_merges));
  k.cptr = static_cast<const int*>(R.at(pl.off_cptr));
  k.contrib = static_cast<const Contrib*>(R.at(pl.off_contrib));
  k.band = R.at(pl.off_band);
  k.lpan = R.at(pl.off_lpan);
  k.lpld = pl.lpld;
  k.ipiv = static_cast<int*>(R.at(pl.off_ipiv));
  k.bhat = static_cast<double*>(R.at(pl.off_bhat));
  k.chat = static_cast<double*>(R.at(pl.off_chat));
  k.side = R.at(pl.off_side);
  k.tips = static_cast<double*>(R.at(pl.off_tips));
  k.sfac = static_cast<double*>(R.at(pl.off_sfac));
  k.spiv = static_cast<int*>(R.at(pl.off_spiv));
  k.coef = static_cast<double*>(R.at(pl.off_coef));
  k.qw = static_cast<double*>(R.at(pl.off_qw));
  k.fscr = R.at(pl.off_fscr);
  k.nodeval = static_cast<double*>(R.at(pl.off_nodeval));
  k.st = static_cast<double*>(R.at(pl.off_st));
  k.xint = static_cast<double*>(R.at(pl.off_xint));
  k.ztip = static_cast<double*>(R.at(pl.off_ztip));
  k.crl = static_cast<double*>(R.at(pl.off_crl));
  k.sscr = static_cast<double*>(R.at(pl.off_sscr));
  k.fast_tips = 0;
  k.dinv = R.at(pl.off_dinv);
  k.sdinv = static_cast<double*>(R.at(pl.off_sdinv));
  k.sperm = static_cast<int*>(R.at(pl.off_sperm));
  k.mtmp = static_cast<double*>(R.at(pl.off_mtmp));
  std::vector<unsigned long long> sweeps(kSweepCounters, 0ull);
  k.sweeps = sweeps.data();

  LaunchCfg c;
  c.nb = pl.nb;
  c.nb_dense = pl.nb_dense;
  c.fp32 = false;
  c.leaf_lds = pl.leaf_lds;
  c.merge_lds = pl.merge_lds;
  c.level_off = pl.level_off;
  c.fast = false;
  c.flu = false;
  c.mfast = false;   // the generic interface kernels (the MFMA ones do not run here)
  int e = 0;
  switch (pl.nb) {
    case 32: e = factor_and_solve<32>(pl, k, c, B.data(), n, nrhs, trans); break;
    case 16: e = factor_and_solve<16>(pl, k, c, B.data(), n, nrhs, trans); break;
    default: e = factor_and_solve<8>(pl, k, c, B.data(), n, nrhs, trans); break;
  }
  if (e) return 4;
  const DevStatus* s = k.status;
  int64_t info = 0;
  if (s->zero_row != ULLONG_MAX) info = (int64_t)s->zero_row;
  else if (s->iface != ULLONG_MAX) info = pl.n + (int64_t)s->iface;
  FILE* g = std::fopen(argv[2], "wb");
  std::fwrite(&info, 8, 1, g);
  std::fwrite(B.data(), 8, B.size(), g);
  std::fwrite(sweeps.data(), 8, sweeps.size(), g);
  std::fclose(g);
  std::printf("replay: n=%lld kl=%d ku=%d p=%d pivot=%d nrhs=%d trans=%d nb=%d info=%lld\n", (long long)n, kl, ku,
              pl.p, pivot, nrhs, (int)trans, pl.nb, (long long)info);
  return 0;
}
