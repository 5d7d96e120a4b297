// C ABI of the SPIKE solver: argument checking, planning, workspace carving
// and stream-ordered launches.  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>

#include "../../include/spike.h"
#include "spike_launch.hpp"
#include "spike_plan.hpp"
#include "spike_refine.hpp"

namespace {

constexpr uint32_t kMagic = 0x5e1ce5u;

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
};

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
  k.sdinv = at<double>(w, pl.off_sdinv);
  k.sperm = at<int>(w, pl.off_sperm);
  k.mtmp = at<double>(w, pl.off_mtmp);

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

}  // namespace

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

int spike_handle_plan(spike_handle h, spike_plan_info* out) {
  if (!valid(h)) return -1;
  if (!out) return -2;
  to_info(h->plan, out);
  return 0;
}

int spike_destroy(spike_handle h) {
  if (!valid(h)) return -1;
  h->magic = 0;
  delete h;
  return 0;
}

}  // extern "C"
