// C ABI of the SPIKE solver: argument checking, planning, workspace carving
// and stream-ordered launches.  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>
#include <new>

#include "../../include/spike.h"
#include "spike_launch.hpp"
#include "spike_plan.hpp"
#include "spike_krylov.hpp"
#include "spike_refine.hpp"

namespace {

constexpr uint32_t kMagic = 0x5e1ce5u;

// Handles made while this is set count their sweeps (spike_sweep_counting).
std::atomic<int> g_count_sweeps{0};

int check_hip(hipError_t e) { return e == hipSuccess ? 0 : SPIKE_ERR_HIP - (int)e; }

int plan_for(int64_t n, int32_t kl, int32_t ku, const spike_opts* opts, spike::Plan& pl) {
  if (n < 0) return -1;
  if (kl < 0) return -2;
  if (ku < 0) return -3;
  spike_opts o;
  if (opts) o = *opts;
  else spike::default_opts(&o);
  return spike::make_plan(n, kl, ku, o, pl);
}

}  // namespace

struct spike_handle_s {
  uint32_t magic;
  spike::Plan plan;
  char* ws;
  spike::KParams kp;
  spike::LaunchCfg cfg;
  int64_t zn = -1;   // complex order when the handle holds a complex system's real embedding
  double* zd = nullptr;   // its row rotations d_j (interleaved complex, in the workspace)
};

namespace spike {
int launch_zembed(const double* zab, int64_t ldab, int64_t n, int kl, int ku, double* R, int64_t ldr, double* Dv,
                  hipStream_t st);
int launch_zrowscale(double* B, int64_t ldb2, int64_t n, int nrhs, const double* Dv, bool conj_d,
                     const DevStatus* status, hipStream_t st);
int launch_zconj(double* B, int64_t ldb2, int64_t n, int nrhs, const DevStatus* status, hipStream_t st);
}  // namespace spike

namespace {

bool valid(spike_handle h) { return h != nullptr && h->magic == kMagic; }

template <typename P>
P* at(char* base, size_t off) { return reinterpret_cast<P*>(base + off); }

void fill_params(spike_handle h, const double* dAB, int64_t ldab) {
  const spike::Plan& pl = h->plan;
  spike::KParams& k = h->kp;
  char* w = h->ws;
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
  double tau = pl.boost_tau;
  if (tau < 0.0) tau = pl.precision == 1 ? 3.4526698300e-4 : 1.4901161194e-8;  // sqrt(unit roundoff)
  k.boost_tau = pl.pivot ? 0.0 : tau;
  k.dAB = dAB;
  k.ldab = ldab;
  k.status = at<spike::DevStatus>(w, pl.off_status);
  k.leaves = at<spike::LeafDesc>(w, pl.off_leaves);
  k.merges = at<spike::MergeDesc>(w, pl.off_merges);
  k.cptr = at<int>(w, pl.off_cptr);
  k.contrib = at<spike::Contrib>(w, pl.off_contrib);
  k.band = w + pl.off_band;
  k.lpan = w + pl.off_lpan;
  k.lpld = pl.lpld;
  k.ipiv = at<int>(w, pl.off_ipiv);
  k.bhat = at<double>(w, pl.off_bhat);
  k.chat = at<double>(w, pl.off_chat);
  k.side = w + pl.off_side;
  k.tips = at<double>(w, pl.off_tips);
  k.sfac = at<double>(w, pl.off_sfac);
  k.spiv = at<int>(w, pl.off_spiv);
  k.coef = at<double>(w, pl.off_coef);
  k.qw = at<double>(w, pl.off_qw);
  k.fscr = w + pl.off_fscr;
  k.nodeval = at<double>(w, pl.off_nodeval);
  k.st = at<double>(w, pl.off_st);
  k.xint = at<double>(w, pl.off_xint);
  k.ztip = at<double>(w, pl.off_ztip);
  k.crl = at<double>(w, pl.off_crl);
  k.sscr = at<double>(w, pl.off_sscr);
  k.fast_tips = (pl.fast && pl.p >= 3) ? 1 : 0;
  k.dinv = w + pl.off_dinv;
  k.lu_done = 0;
  k.skip = nullptr;
  k.sdinv = at<double>(w, pl.off_sdinv);
  k.sperm = at<int>(w, pl.off_sperm);
  k.mtmp = at<double>(w, pl.off_mtmp);
  k.sweeps = g_count_sweeps.load() ? at<unsigned long long>(w, pl.off_sweeps) : nullptr;

  spike::LaunchCfg& c = h->cfg;
  c.nb = pl.nb;
  c.nb_dense = pl.nb_dense;
  c.fp32 = pl.precision == 1;
  c.leaf_lds = pl.leaf_lds;
  c.merge_lds = pl.merge_lds;
  c.level_off = pl.level_off;
  c.fast = pl.fast;
  c.ht = pl.ht;
  c.fast_lds = pl.fast_lds;
  c.fast_min_nrhs = 1;
  c.flu = pl.fast && !pl.pivot && pl.ht <= 10;
  c.mfast = pl.mfast;
  c.mht = pl.mht;
  {
    int maxm = 0;
    for (auto& L : pl.leaves) maxm = L.m > maxm ? L.m : maxm;
    c.dinv_chunks = ((maxm + 15) / 16 * 32 + 255) / 256;
    if (c.dinv_chunks < 1) c.dinv_chunks = 1;
  }
}

int upload(spike_handle h, hipStream_t st) {
  const spike::Plan& pl = h->plan;
  char* w = h->ws;
  int e = 0;
  if ((e = check_hip(hipMemcpyAsync(w + pl.off_leaves, pl.leaves.data(),
                                    sizeof(spike::LeafDesc) * pl.leaves.size(),
                                    hipMemcpyHostToDevice, st))))
    return e;
  if (!pl.merges.empty() &&
      (e = check_hip(hipMemcpyAsync(w + pl.off_merges, pl.merges.data(),
                                    sizeof(spike::MergeDesc) * pl.merges.size(),
                                    hipMemcpyHostToDevice, st))))
    return e;
  if (!pl.contrib_ptr.empty() &&
      (e = check_hip(hipMemcpyAsync(w + pl.off_cptr, pl.contrib_ptr.data(),
                                    sizeof(int) * pl.contrib_ptr.size(), hipMemcpyHostToDevice, st))))
    return e;
  if (!pl.contrib.empty() &&
      (e = check_hip(hipMemcpyAsync(w + pl.off_contrib, pl.contrib.data(),
                                    sizeof(spike::Contrib) * pl.contrib.size(),
                                    hipMemcpyHostToDevice, st))))
    return e;
  static_assert(sizeof(spike::KParams) <= spike::kKParamsBytes, "parameter block slot too small");
  if ((e = check_hip(hipMemcpyAsync(w + pl.off_kp, &h->kp, sizeof(spike::KParams), hipMemcpyHostToDevice, st))))
    return e;
  return 0;
}

void to_info(const spike::Plan& pl, spike_plan_info* out) {
  out->p = pl.p;
  out->levels = pl.levels;
  out->merges = (int32_t)pl.merges.size();
  out->reduced_size = pl.reduced_size();
  out->workspace_bytes = pl.total;
}

int solve_common(spike_handle h, int32_t nrhs, double* dB, int64_t ldb, hipStream_t st, bool trans) {
  if (!valid(h)) return -1;
  if (nrhs < 0) return -2;
  if (nrhs > 0 && h->plan.n > 0 && dB == nullptr) return -3;
  if (ldb < (h->plan.n > 1 ? h->plan.n : 1)) return -4;
  if (nrhs == 0 || h->plan.n == 0) return 0;
  const int R = h->plan.nrhs_max;
  for (int c0 = 0; c0 < nrhs; c0 += R) {
    int cnt = nrhs - c0 < R ? nrhs - c0 : R;
    double* B = dB + (int64_t)c0 * ldb;
    int e = h->plan.refine_enabled()
                ? spike::refined_solve(h->kp, h->cfg, h->plan, h->ws, st, B, ldb, cnt, trans)
                : spike::launch_solve(h->kp, h->cfg, st, B, ldb, cnt, trans);
    if (e) return e;
  }
  return 0;
}

// Solves that can share batched launches: non-refined, MFMA tile engine for
// the partition sweeps, reduced system on MFMA tiles (when p > 1).
bool batchable(spike_handle h, int32_t nrhs) {
  const spike::LaunchCfg& c = h->cfg;
  return !h->plan.refine_enabled() && c.fast && nrhs >= c.fast_min_nrhs && nrhs <= h->plan.nrhs_max &&
         (h->plan.p == 1 || c.mfast) && h->plan.n > 0;
}

// One pass of the solve stage over up to kMaxBatch systems that share the
// kernel instantiation (precision, window heights) and the operation.
int batch_pass(spike_handle const* hs, const int* idx, int cnt, const int32_t* nrhs, double* const* dB,
               const int64_t* ldb, bool trans, hipStream_t st) {
  spike::BatchArgs ba;
  std::memset(&ba, 0, sizeof(ba));
  ba.nsys = cnt;
  size_t lds = 0;
  int maxL = 0;
  const spike::LaunchCfg& c0 = hs[idx[0]]->cfg;
  for (int s = 0; s < cnt; ++s) {
    spike_handle h = hs[idx[s]];
    ba.kp[s] = reinterpret_cast<const spike::KParams*>(h->ws + h->plan.off_kp);
    ba.B[s] = dB[idx[s]];
    ba.ldb[s] = ldb[idx[s]];
    ba.nrhs[s] = nrhs[idx[s]];
    if (h->cfg.fast_lds > lds) lds = h->cfg.fast_lds;
    const int L = (int)h->cfg.level_off.size() - 1;
    if (L > maxL) maxL = L;
  }
  auto leaf_items = [&](int minus) {
    int tot = 0;
    for (int s = 0; s < cnt; ++s) {
      ba.off[s] = tot;
      tot += hs[idx[s]]->plan.p - minus;
    }
    ba.off[cnt] = tot;
    return tot;
  };
  auto level_items = [&](int l) {
    int tot = 0;
    for (int s = 0; s < cnt; ++s) {
      const std::vector<int>& lo = hs[idx[s]]->cfg.level_off;
      const int L = (int)lo.size() - 1;
      ba.off[s] = tot;
      ba.mbeg[s] = l < L ? lo[l] : 0;
      tot += l < L ? lo[l + 1] - lo[l] : 0;
    }
    ba.off[cnt] = tot;
    return tot;
  };
  int e;
  const bool f32 = c0.fp32;
  const int ht = c0.ht, mht = c0.mht;
  if (!trans) {
    if ((e = spike::launch_phase_batch(ba, f32, ht, lds, st, 0, leaf_items(0)))) return e;
    for (int l = 0; l < maxL; ++l)
      if ((e = spike::launch_mlevel_batch(ba, mht, st, level_items(l), false, true))) return e;
    for (int l = maxL - 1; l >= 0; --l)
      if ((e = spike::launch_mlevel_batch(ba, mht, st, level_items(l), false, false))) return e;
    if ((e = spike::launch_phase_batch(ba, f32, ht, lds, st, 1, leaf_items(0)))) return e;
  } else {
    if ((e = spike::launch_phase_batch(ba, f32, ht, lds, st, 2, leaf_items(0)))) return e;
    if ((e = spike::run_gform_batch(ba, st, leaf_items(1)))) return e;
    for (int l = 0; l < maxL; ++l)
      if ((e = spike::launch_mlevel_batch(ba, mht, st, level_items(l), true, true))) return e;
    for (int l = maxL - 1; l >= 0; --l)
      if ((e = spike::launch_mlevel_batch(ba, mht, st, level_items(l), true, false))) return e;
    if ((e = spike::launch_phase_batch(ba, f32, ht, lds, st, 3, leaf_items(0)))) return e;
  }
  return 0;
}

int solve_batch(const spike_handle* hs, const int32_t* nrhs, double* const* dB, const int64_t* ldb,
                const int32_t* trans, int32_t count, hipStream_t st) {
  if (count < 0) return -6;
  if (count == 0) return 0;
  if (!hs) return -1;
  if (!nrhs) return -2;
  if (!dB) return -3;
  if (!ldb) return -4;
  if (!trans) return -5;
  for (int i = 0; i < count; ++i) {
    if (!valid(hs[i])) return -1;
    if (nrhs[i] < 0) return -2;
    const int64_t n = hs[i]->plan.n;
    if (nrhs[i] > 0 && n > 0 && dB[i] == nullptr) return -3;
    if (ldb[i] < (n > 1 ? n : 1)) return -4;
  }
  // group by kernel instantiation and operation; others run one by one
  std::vector<int> rest;
  std::vector<std::vector<int>> groups;
  std::vector<uint64_t> keys;
  for (int i = 0; i < count; ++i) {
    if (nrhs[i] == 0 || hs[i]->plan.n == 0) continue;
    if (!batchable(hs[i], nrhs[i])) {
      rest.push_back(i);
      continue;
    }
    const spike::LaunchCfg& c = hs[i]->cfg;
    const uint64_t key = ((uint64_t)(trans[i] != 0) << 40) | ((uint64_t)c.fp32 << 32) |
                         ((uint64_t)c.ht << 16) | (uint64_t)(c.mfast ? c.mht : 0);
    size_t g = 0;
    while (g < keys.size() && keys[g] != key) ++g;
    if (g == keys.size()) {
      keys.push_back(key);
      groups.emplace_back();
    }
    groups[g].push_back(i);
  }
  for (size_t g = 0; g < groups.size(); ++g) {
    const std::vector<int>& v = groups[g];
    const bool tr = (keys[g] >> 40) & 1;
    for (size_t b = 0; b < v.size(); b += spike::kMaxBatch) {
      const int cnt = (int)std::min<size_t>(spike::kMaxBatch, v.size() - b);
      const int e = batch_pass(hs, v.data() + b, cnt, nrhs, dB, ldb, tr, st);
      if (e) return e;
    }
  }
  for (int i : rest) {
    const int e = solve_common(hs[i], nrhs[i], dB[i], ldb[i], st, trans[i] != 0);
    if (e) return e;
  }
  return 0;
}

}  // namespace

namespace {

// Candidate plans of the autotuner: partition counts around the device's
// compute-unit count (and the planner's default), equal sizing; infeasible
// ones (partitions shorter than kl + ku) are dropped.
std::vector<spike_opts> tune_candidates(int64_t n, int32_t kl, int32_t ku, const spike_opts& base) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  std::vector<int> ps;
  spike::Plan pl0;
  spike_opts o0 = base;
  o0.p = 0;
  o0.sizing = 0;
  if (spike::make_plan(n, kl, ku, o0, pl0) == 0) ps.push_back(pl0.p);
  for (int f : {1, 2, 4}) ps.push_back(cus * f / 2);
  ps.push_back(cus);
  std::vector<spike_opts> out;
  for (int p : ps) {
    if (p < 1) continue;
    bool dup = false;
    for (auto& o : out) dup = dup || o.p == p;
    if (dup) continue;
    for (int tree : {0, 1}) {
      // the paper's layout differs from the balanced tree when p is not a
      // power of two (and is admissible for it)
      if (tree == 1 && (p & (p - 1)) == 0) continue;
      spike_opts o = base;
      o.p = p;
      o.sizing = 0;
      o.tree = tree;
      spike::Plan pl;
      if (spike::make_plan(n, kl, ku, o, pl) == 0) out.push_back(o);
    }
  }
  return out;
}

// ---- the tuning cache
using TuneKey = std::tuple<int64_t, int32_t, int32_t, int32_t, int32_t, int32_t>;
std::mutex g_tune_mu;
std::map<TuneKey, spike_tune_result> g_tune;

int32_t log2_floor(int32_t v) {
  int32_t l = 0;
  while (v > 1) {
    v >>= 1;
    ++l;
  }
  return l;
}
TuneKey tune_key(int64_t n, int32_t kl, int32_t ku, int32_t nrhs, const spike_opts& o) {
  return TuneKey{n, kl, ku, log2_floor(std::max(1, nrhs)), o.precision, o.pivot};
}

}  // namespace

struct spike_graph_s {
  uint32_t magic;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

namespace {
constexpr uint32_t kGraphMagic = 0x6a2f1bu;
}

extern "C" {

void spike_default_opts(spike_opts* opts) {
  if (opts) spike::default_opts(opts);
}

int spike_plan_query(int64_t n, int32_t kl, int32_t ku, const spike_opts* opts, spike_plan_info* out,
                     int64_t* sizes) {
  spike::Plan pl;
  int r = plan_for(n, kl, ku, opts, pl);
  if (r) return r;
  if (out) to_info(pl, out);
  if (sizes)
    for (int i = 0; i < pl.p; ++i) sizes[i] = pl.leaves[i].m;
  return 0;
}

int spike_plan_tree(int64_t n, int32_t kl, int32_t ku, const spike_opts* opts, int32_t* merges) {
  spike::Plan pl;
  int r = plan_for(n, kl, ku, opts, pl);
  if (r) return r;
  if (merges)
    for (size_t d = 0; d < pl.merges.size(); ++d) {
      const spike::MergeDesc& J = pl.merges[d];
      merges[4 * d + 0] = J.level;
      merges[4 * d + 1] = J.a;
      merges[4 * d + 2] = J.mif;
      merges[4 * d + 3] = J.b;
    }
  return 0;
}

int spike_workspace_size(int64_t n, int32_t kl, int32_t ku, const spike_opts* opts, size_t* bytes) {
  spike::Plan pl;
  int r = plan_for(n, kl, ku, opts, pl);
  if (r) return r;
  if (bytes) *bytes = pl.total;
  return 0;
}

int spike_factor(int64_t n, int32_t kl, int32_t ku, const double* dAB, int64_t ldab, const spike_opts* opts,
                 void* dWork, size_t work_bytes, hipStream_t stream, spike_handle* out) {
  if (n < 0) return -1;
  if (kl < 0) return -2;
  if (ku < 0) return -3;
  if (dAB == nullptr && n > 0) return -4;
  if (ldab < (int64_t)kl + ku + 1) return -5;
  spike::Plan pl;
  if (plan_for(n, kl, ku, opts, pl)) return -6;
  if (dWork == nullptr || (reinterpret_cast<uintptr_t>(dWork) & 255u) != 0) return -7;
  if (work_bytes < pl.total) return -8;
  if (out == nullptr) return -10;
  spike_handle h = new (std::nothrow) spike_handle_s();
  if (!h) return SPIKE_ERR_HIP - (int)hipErrorOutOfMemory;
  h->magic = kMagic;
  h->plan = std::move(pl);
  h->ws = static_cast<char*>(dWork);
  fill_params(h, dAB, ldab);
  int e = upload(h, stream);
  if (!e) e = spike::launch_init_status(h->kp.status, stream);
  if (!e && h->kp.sweeps) e = spike::run_zero_counters(h->kp.sweeps, spike::kSweepCounters, stream);
  if (!e && n > 0) e = spike::launch_factor(h->kp, h->cfg, stream);
  if (!e && n > 0 && h->plan.refine_enabled()) e = spike::prepare_refine(h->kp, h->plan, h->ws, stream);
  if (e) {
    h->magic = 0;
    delete h;
    return e;
  }
  *out = h;
  return 0;
}

int spike_factor_batch(int32_t count, const int64_t* n, const int32_t* kl, const int32_t* ku,
                       const double* const* dAB, const int64_t* ldab, const spike_opts* opts, void* const* dWork,
                       const size_t* work_bytes, hipStream_t stream, spike_handle* out) {
  if (count < 0) return -11;
  if (count == 0) return 0;
  if (!n || !kl || !ku || !dAB || !ldab || !dWork || !work_bytes || !out) return -12;
  // every system's arguments first, so that nothing starts on an error
  std::vector<spike::Plan> plans(count);
  for (int i = 0; i < count; ++i) {
    if (n[i] < 0) return -1;
    if (kl[i] < 0) return -2;
    if (ku[i] < 0) return -3;
    if (dAB[i] == nullptr && n[i] > 0) return -4;
    if (ldab[i] < (int64_t)kl[i] + ku[i] + 1) return -5;
    if (plan_for(n[i], kl[i], ku[i], opts ? &opts[i] : nullptr, plans[i])) return -6;
    if (dWork[i] == nullptr || (reinterpret_cast<uintptr_t>(dWork[i]) & 255u) != 0) return -7;
    if (work_bytes[i] < plans[i].total) return -8;
  }
  std::vector<spike_handle> hs(count, nullptr);
  auto fail = [&](int e) {
    for (auto& h : hs)
      if (h) {
        h->magic = 0;
        delete h;
        h = nullptr;
      }
    return e;
  };
  for (int i = 0; i < count; ++i) {
    spike_handle h = new (std::nothrow) spike_handle_s();
    if (!h) return fail(SPIKE_ERR_HIP - (int)hipErrorOutOfMemory);
    hs[i] = h;
    h->magic = kMagic;
    h->plan = std::move(plans[i]);
    h->ws = static_cast<char*>(dWork[i]);
    fill_params(h, dAB[i], ldab[i]);
    if (int e = upload(h, stream)) return fail(e);
  }
  // systems sharing the kernel configuration of the batched factor stage
  std::vector<std::vector<int>> groups;
  std::vector<uint64_t> keys;
  std::vector<int> rest;
  for (int i = 0; i < count; ++i) {
    const spike_handle h = hs[i];
    const spike::LaunchCfg& c = h->cfg;
    const bool ok = h->plan.n > 0 && !h->plan.pivot && c.flu && c.fast && (h->plan.p == 1 || c.mfast) &&
                    !h->kp.sweeps;
    if (!ok) {
      rest.push_back(i);
      continue;
    }
    const uint64_t key = ((uint64_t)c.fp32 << 56) | ((uint64_t)c.ht << 48) |
                         ((uint64_t)(c.mfast ? c.mht : 0) << 40) | ((uint64_t)(uint32_t)kl[i] << 20) |
                         (uint64_t)(uint32_t)ku[i];
    size_t g = 0;
    while (g < keys.size() && keys[g] != key) ++g;
    if (g == keys.size()) {
      keys.push_back(key);
      groups.emplace_back();
    }
    groups[g].push_back(i);
  }
  for (size_t g = 0; g < groups.size(); ++g) {
    const std::vector<int>& v = groups[g];
    for (size_t b0 = 0; b0 < v.size(); b0 += spike::kMaxBatch) {
      const int cnt = (int)std::min<size_t>(spike::kMaxBatch, v.size() - b0);
      spike::BatchArgs ba;
      std::memset(&ba, 0, sizeof(ba));
      ba.nsys = cnt;
      std::vector<int> p(cnt);
      std::vector<const std::vector<int>*> lo(cnt);
      for (int s = 0; s < cnt; ++s) {
        spike_handle h = hs[v[b0 + s]];
        ba.kp[s] = reinterpret_cast<const spike::KParams*>(h->ws + h->plan.off_kp);
        p[s] = h->plan.p;
        lo[s] = &h->cfg.level_off;
      }
      const spike_handle h0 = hs[v[b0]];
      if (int e = spike::launch_factor_batch(ba, p.data(), lo, h0->cfg, h0->plan.kl, h0->plan.ku, stream))
        return fail(e);
    }
  }
  for (int i : rest) {
    spike_handle h = hs[i];
    int e = spike::launch_init_status(h->kp.status, stream);
    if (!e && h->kp.sweeps) e = spike::run_zero_counters(h->kp.sweeps, spike::kSweepCounters, stream);
    if (!e && h->plan.n > 0) e = spike::launch_factor(h->kp, h->cfg, stream);
    if (e) return fail(e);
  }
  for (int i = 0; i < count; ++i) {
    spike_handle h = hs[i];
    if (h->plan.n > 0 && h->plan.refine_enabled())
      if (int e = spike::prepare_refine(h->kp, h->plan, h->ws, stream)) return fail(e);
  }
  for (int i = 0; i < count; ++i) out[i] = hs[i];
  return 0;
}

int spike_solve(spike_handle h, int32_t nrhs, double* dB, int64_t ldb, hipStream_t stream) {
  return solve_common(h, nrhs, dB, ldb, stream, false);
}

int spike_solve_transpose(spike_handle h, int32_t nrhs, double* dB, int64_t ldb, hipStream_t stream) {
  return solve_common(h, nrhs, dB, ldb, stream, true);
}

int spike_info(spike_handle h, spike_status* out) {
  if (!valid(h)) return -1;
  if (!out) return -2;
  spike::DevStatus s;
  int e = check_hip(hipMemcpy(&s, h->ws + h->plan.off_status, sizeof(s), hipMemcpyDeviceToHost));
  if (e) return e;
  std::memset(out, 0, sizeof(*out));
  const unsigned long long none = ~0ull;
  if (s.zero_row != none) out->info = (int64_t)s.zero_row;
  else if (s.iface != none) out->info = h->plan.n + (int64_t)s.iface;
  else out->info = 0;
  out->n_boosts = s.n_boosts;
  out->refine_iters = s.refine_iters;
  double mp;
  std::memcpy(&mp, &s.min_pivot_bits, sizeof(mp));
  out->min_abs_pivot = mp;
  out->berr = s.berr;
  return 0;
}

void spike_krylov_default_opts(spike_krylov_opts* o) {
  if (!o) return;
  o->restart = 30;
  o->max_iters = 300;
  o->tol = 1e-13;
}

namespace {
bool krylov_opts_ok(const spike_krylov_opts& o) {
  return o.restart >= 1 && o.restart <= 500 && o.max_iters >= 0 && o.tol > 0.0;
}
}  // namespace

int spike_krylov_workspace_size(spike_handle h, int32_t nrhs, const spike_krylov_opts* opts, size_t* bytes) {
  if (!valid(h)) return -1;
  if (nrhs < 0 || nrhs > h->plan.nrhs_max) return -2;
  spike_krylov_opts o;
  spike_krylov_default_opts(&o);
  if (opts) o = *opts;
  if (!krylov_opts_ok(o)) return -3;
  if (!bytes) return -4;
  *bytes = spike::gmres_workspace_bytes(h->plan.n, nrhs, o.restart);
  return 0;
}

int spike_solve_gmres(spike_handle h, int32_t nrhs, double* dB, int64_t ldb, int32_t trans,
                      const spike_krylov_opts* opts, void* dWork, size_t work_bytes, hipStream_t stream,
                      spike_krylov_result* out) {
  if (!valid(h)) return -1;
  if (nrhs < 0 || nrhs > h->plan.nrhs_max) return -2;
  const int64_t n = h->plan.n;
  if (nrhs > 0 && n > 0 && dB == nullptr) return -3;
  if (ldb < (n > 1 ? n : 1)) return -4;
  spike_krylov_opts o;
  spike_krylov_default_opts(&o);
  if (opts) o = *opts;
  if (!krylov_opts_ok(o)) return -6;
  if (!out) return -11;
  std::memset(out, 0, sizeof(*out));
  if (nrhs == 0 || n == 0) {
    out->converged = 1;
    return 0;
  }
  if (dWork == nullptr || (reinterpret_cast<uintptr_t>(dWork) & 255u) != 0) return -7;
  if (work_bytes < spike::gmres_workspace_bytes(n, nrhs, o.restart)) return -8;
  spike::GmresResult r{};
  const int e = spike::gmres_solve(h->kp, h->cfg, h->plan, static_cast<char*>(dWork), stream, dB, ldb, nrhs,
                                   trans != 0, o.restart, o.max_iters, o.tol, &r);
  if (e) return e;
  out->iters = r.iters;
  out->restarts = r.restarts;
  out->converged = r.converged;
  out->berr = r.berr;
  return 0;
}

namespace {
// Bytes of the embedded real band and the row rotations at the front of a
// complex workspace.
size_t zband_bytes(int64_t n, int32_t kl, int32_t ku) {
  const int64_t ldr = 2 * (int64_t)kl + 2 * (int64_t)ku + 3;
  return ((size_t)(2 * n * ldr * 8) + 255) / 256 * 256;
}
size_t zrot_bytes(int64_t n) { return ((size_t)(16 * (n > 0 ? n : 1)) + 255) / 256 * 256; }
}  // namespace

int spike_zworkspace_size(int64_t n, int32_t kl, int32_t ku, const spike_opts* opts, size_t* bytes) {
  if (n < 0) return -1;
  if (kl < 0) return -2;
  if (ku < 0) return -3;
  size_t real = 0;
  const int r = spike_workspace_size(2 * n, 2 * kl + 1, 2 * ku + 1, opts, &real);
  if (r) return r < -3 ? r : -4;
  if (bytes) *bytes = zband_bytes(n, kl, ku) + zrot_bytes(n) + real;
  return 0;
}

int spike_zfactor(int64_t n, int32_t kl, int32_t ku, const double* dAB, int64_t ldab, const spike_opts* opts,
                  void* dWork, size_t work_bytes, hipStream_t stream, spike_handle* out) {
  if (n < 0) return -1;
  if (kl < 0) return -2;
  if (ku < 0) return -3;
  if (dAB == nullptr && n > 0) return -4;
  if (ldab < (int64_t)kl + ku + 1) return -5;
  size_t need = 0;
  if (spike_zworkspace_size(n, kl, ku, opts, &need)) return -6;
  if (dWork == nullptr || (reinterpret_cast<uintptr_t>(dWork) & 255u) != 0) return -7;
  if (work_bytes < need) return -8;
  if (out == nullptr) return -10;
  const int klr = 2 * kl + 1, kur = 2 * ku + 1;
  const int64_t ldr = (int64_t)klr + kur + 1;
  double* R = static_cast<double*>(dWork);
  double* Dv = reinterpret_cast<double*>(static_cast<char*>(dWork) + zband_bytes(n, kl, ku));
  const size_t zb = zband_bytes(n, kl, ku) + zrot_bytes(n);
  int e = spike::launch_zembed(dAB, ldab, n, kl, ku, R, ldr, Dv, stream);
  if (e) return e;
  spike_handle h = nullptr;
  e = spike_factor(2 * n, klr, kur, R, ldr, opts, static_cast<char*>(dWork) + zb, work_bytes - zb, stream, &h);
  if (e) return e;
  h->zn = n;
  h->zd = Dv;
  *out = h;
  return 0;
}

int spike_zsolve(spike_handle h, int32_t nrhs, double* dB, int64_t ldb, int32_t trans, hipStream_t stream) {
  if (!valid(h) || h->zn < 0) return -1;
  if (nrhs < 0) return -2;
  if (nrhs > 0 && h->zn > 0 && dB == nullptr) return -3;
  if (ldb < (h->zn > 1 ? h->zn : 1)) return -4;
  if (trans < 0 || trans > 2) return -5;
  if (nrhs == 0 || h->zn == 0) return 0;
  // the factors are those of D A (D: the unitary row rotations)
  const int64_t ld2 = 2 * ldb, zn = h->zn;
  int e = 0;
  if (trans == 0) {   // D A z = D f
    e = spike::launch_zrowscale(dB, ld2, zn, nrhs, h->zd, false, h->kp.status, stream);
    if (!e) e = solve_common(h, nrhs, dB, ld2, stream, false);
  } else if (trans == 2) {   // (D A)^H w = f, z = conj(D) w
    e = solve_common(h, nrhs, dB, ld2, stream, true);
    if (!e) e = spike::launch_zrowscale(dB, ld2, zn, nrhs, h->zd, true, h->kp.status, stream);
  } else {   // (D A)^T w = f through (D A)^H conj(w) = conj(f); z = D w
    e = spike::launch_zconj(dB, ld2, zn, nrhs, h->kp.status, stream);
    if (!e) e = solve_common(h, nrhs, dB, ld2, stream, true);
    if (!e) e = spike::launch_zconj(dB, ld2, zn, nrhs, h->kp.status, stream);
    if (!e) e = spike::launch_zrowscale(dB, ld2, zn, nrhs, h->zd, false, h->kp.status, stream);
  }
  return e;
}

int spike_sweep_counting(int on) {
  g_count_sweeps.store(on ? 1 : 0);
  return 0;
}

int spike_sweep_counts(spike_handle h, uint64_t* out) {
  if (!valid(h)) return -1;
  if (!out) return -2;
  if (!h->kp.sweeps) return -3;
  return check_hip(hipMemcpy(out, h->kp.sweeps, sizeof(uint64_t) * spike::kSweepCounters, hipMemcpyDeviceToHost));
}

int spike_handle_plan(spike_handle h, spike_plan_info* out) {
  if (!valid(h)) return -1;
  if (!out) return -2;
  to_info(h->plan, out);
  return 0;
}

int spike_solve_batch(const spike_handle* hs, const int32_t* nrhs, double* const* dB, const int64_t* ldb,
                      const int32_t* trans, int32_t count, hipStream_t stream) {
  return solve_batch(hs, nrhs, dB, ldb, trans, count, stream);
}

int spike_graph_capture_batch(const spike_handle* hs, const int32_t* nrhs, double* const* dB,
                              const int64_t* ldb, const int32_t* trans, int32_t count, hipStream_t stream,
                              spike_graph* out) {
  if (!out) return -8;
  if (stream == nullptr) return -7;
  for (int i = 0; i < count && hs; ++i)
    if (valid(hs[i]) && hs[i]->plan.refine_enabled()) return -1;
  spike_graph g = new (std::nothrow) spike_graph_s();
  if (!g) return SPIKE_ERR_HIP - (int)hipErrorOutOfMemory;
  int e = check_hip(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
  if (e) {
    delete g;
    return e;
  }
  const int r = solve_batch(hs, nrhs, dB, ldb, trans, count, stream);
  hipGraph_t graph = nullptr;
  e = check_hip(hipStreamEndCapture(stream, &graph));
  if (r || e) {
    if (graph) (void)hipGraphDestroy(graph);
    delete g;
    return r ? r : e;
  }
  e = check_hip(hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0));
  if (e) {
    (void)hipGraphDestroy(graph);
    delete g;
    return e;
  }
  g->graph = graph;
  g->magic = kGraphMagic;
  *out = g;
  return 0;
}

int spike_graph_capture_solve(spike_handle h, int32_t nrhs, double* dB, int64_t ldb, int32_t trans,
                              hipStream_t stream, spike_graph* out) {
  return spike_graph_capture_batch(&h, &nrhs, &dB, &ldb, &trans, 1, stream, out);
}

int spike_graph_launch(spike_graph g, hipStream_t stream) {
  if (!g || g->magic != kGraphMagic) return -1;
  return check_hip(hipGraphLaunch(g->exec, stream));
}

int spike_graph_destroy(spike_graph g) {
  if (!g || g->magic != kGraphMagic) return -1;
  g->magic = 0;
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  delete g;
  return 0;
}

int spike_autotune_workspace_size(int64_t n, int32_t kl, int32_t ku, const spike_opts* base, size_t* bytes) {
  if (n < 1) return -1;
  if (kl < 0) return -2;
  if (ku < 0) return -3;
  if (!bytes) return -5;
  spike_opts b;
  if (base) b = *base;
  else spike::default_opts(&b);
  size_t best = 0;
  for (const spike_opts& o : tune_candidates(n, kl, ku, b)) {
    spike::Plan pl;
    if (spike::make_plan(n, kl, ku, o, pl) == 0) best = std::max(best, pl.total);
    spike_opts r = o;
    r.sizing = 1;
    r.K = 4.0;
    if (spike::make_plan(n, kl, ku, r, pl) == 0) best = std::max(best, pl.total);
  }
  *bytes = best;
  return best ? 0 : -4;
}

int spike_autotune(int64_t n, int32_t kl, int32_t ku, const double* dAB, int64_t ldab, int32_t nrhs,
                   const spike_opts* base, void* dWork, size_t work_bytes, double* dB, int64_t ldb,
                   hipStream_t stream, spike_tune_result* out) {
  if (n < 1) return -1;
  if (kl < 0) return -2;
  if (ku < 0) return -3;
  if (!dAB) return -4;
  if (ldab < (int64_t)kl + ku + 1) return -5;
  if (nrhs < 1) return -6;
  if (!dWork) return -8;
  if (!dB || ldb < n) return -10;
  if (!out) return -13;
  spike_opts b;
  if (base) b = *base;
  else spike::default_opts(&b);
  b.nrhs_hint = nrhs;
  if (b.nrhs_max < nrhs) b.nrhs_max = nrhs;
  const TuneKey key = tune_key(n, kl, ku, nrhs, b);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      *out = it->second;
      out->opts.nrhs_max = std::max(out->opts.nrhs_max, b.nrhs_max);
      out->cached = 1;
      return 0;
    }
  }
  hipEvent_t ev[3];
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) return SPIKE_ERR_HIP - (int)hipErrorOutOfMemory;
  auto run = [&](const spike_opts& o, double& tf, double& ts) -> int {
    size_t need = 0;
    if (spike_workspace_size(n, kl, ku, &o, &need) || need > work_bytes) return 1;
    spike_handle h = nullptr;
    (void)hipEventRecord(ev[0], stream);
    int e = spike_factor(n, kl, ku, dAB, ldab, &o, dWork, work_bytes, stream, &h);
    if (e) return e;
    (void)hipEventRecord(ev[1], stream);
    e = spike_solve(h, nrhs, dB, ldb, stream);
    (void)hipEventRecord(ev[2], stream);
    if (!e) e = check_hip(hipEventSynchronize(ev[2]));
    float a = 0.f, c = 0.f;
    (void)hipEventElapsedTime(&a, ev[0], ev[1]);
    (void)hipEventElapsedTime(&c, ev[1], ev[2]);
    tf = a;
    ts = c;
    spike_destroy(h);
    return e;
  };
  double best = 1e300, bf = 0, bs = 0;
  int ncand = 0, err = 0;
  spike_opts bo = b;
  for (const spike_opts& o : tune_candidates(n, kl, ku, b)) {
    double tf = 0, ts = 0;
    const int e = run(o, tf, ts);
    if (e > 0) continue;          // does not fit the workspace
    if (e < 0) {
      err = e;
      break;
    }
    ++ncand;
    if (tf + ts < best) {
      best = tf + ts;
      bf = tf;
      bs = ts;
      bo = o;
    }
  }
  double K = 0.0;
  if (!err && ncand > 0) {
    // machine constant of the load-balancing model: solve cost per row and
    // column over factor cost per row, per unit of bandwidth
    const double kk = std::max(1, std::max(kl, ku));
    K = bf > 0 ? (bs * kk) / (bf * nrhs) : 0.0;
    if (K > 0 && bo.p >= 3) {
      spike_opts r = bo;
      r.sizing = 1;
      r.K = K;
      double tf = 0, ts = 0;
      const int e = run(r, tf, ts);
      if (e < 0) err = e;
      if (e == 0) {
        ++ncand;
        if (tf + ts < best) {
          best = tf + ts;
          bf = tf;
          bs = ts;
          bo = r;
        }
      }
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (err) return err;
  if (ncand == 0) return -9;
  out->opts = bo;
  out->factor_ms = bf;
  out->solve_ms = bs;
  out->K = K;
  out->candidates = ncand;
  out->cached = 0;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = *out;
  }
  return 0;
}

int spike_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  return 0;
}

int spike_tune_cache_size(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return (int)g_tune.size();
}

int spike_tune_cache_save(const char* path) {
  if (!path) return -1;
  std::FILE* f = std::fopen(path, "w");
  if (!f) return -2;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& kv : g_tune) {
    const TuneKey& k = kv.first;
    const spike_tune_result& r = kv.second;
    std::fprintf(f, "%lld %d %d %d %d %d %d %d %d %.17g %d %.17g %.17g %.17g %.17g %d\n",
                 (long long)std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k),
                 std::get<5>(k), r.opts.p, r.opts.sizing, r.opts.tree, r.opts.K, r.opts.nrhs_hint, r.opts.r12,
                 r.opts.r13, r.factor_ms, r.solve_ms, r.candidates);
  }
  std::fclose(f);
  return 0;
}

int spike_tune_cache_load(const char* path) {
  if (!path) return -1;
  std::FILE* f = std::fopen(path, "r");
  if (!f) return -2;
  char line[512];
  int rc = 0;
  while (std::fgets(line, sizeof(line), f)) {
    long long n = 0;
    int kl, ku, lg, prec, piv, p, sizing, tree, nh, cand;
    double K, r12, r13, fm, sm;
    if (line[0] == '\n' || line[0] == '#') continue;
    if (std::sscanf(line, "%lld %d %d %d %d %d %d %d %d %lg %d %lg %lg %lg %lg %d", &n, &kl, &ku, &lg, &prec, &piv,
                    &p, &sizing, &tree, &K, &nh, &r12, &r13, &fm, &sm, &cand) != 16 ||
        n < 1 || kl < 0 || ku < 0 || lg < 0 || lg > 30 || (prec != 0 && prec != 1) || (piv != 0 && piv != 1) ||
        p < 1 || sizing < 0 || sizing > 2 || (tree != 0 && tree != 1)) {
      rc = -3;
      break;
    }
    spike_tune_result r;
    std::memset(&r, 0, sizeof(r));
    spike::default_opts(&r.opts);
    r.opts.p = p;
    r.opts.pivot = piv;
    r.opts.precision = prec;
    r.opts.sizing = sizing;
    r.opts.tree = tree;
    r.opts.K = K;
    r.opts.nrhs_hint = nh;
    r.opts.nrhs_max = std::max(r.opts.nrhs_max, 1 << lg);
    r.opts.r12 = r12;
    r.opts.r13 = r13;
    r.factor_ms = fm;
    r.solve_ms = sm;
    r.candidates = cand;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[TuneKey{(int64_t)n, kl, ku, lg, prec, piv}] = r;
  }
  std::fclose(f);
  return rc;
}

int spike_destroy(spike_handle h) {
  if (!valid(h)) return -1;
  h->magic = 0;
  delete h;
  return 0;
}

}  // extern "C"
