// Stage sequencing: dispatch on the panel widths and precision chosen by the
// planner, and order the leaf and merge launches of each stage.
#include <algorithm>

#include "spike_launch.hpp"

namespace spike {

namespace {

template <typename T>
int leaf_factor(int nb, const KParams& k, const LaunchCfg& c, hipStream_t st) {
  switch (nb) {
    case 32: return run_leaf_factor<32, T>(k, c, st);
    case 16: return run_leaf_factor<16, T>(k, c, st);
    default: return run_leaf_factor<8, T>(k, c, st);
  }
}

template <typename T>
int leaf_phase(int nb, const KParams& k, const LaunchCfg& c, hipStream_t st, double* B, int64_t ldb, int nrhs,
               int phase) {
  switch (nb) {
    case 32: return run_leaf_phase<32, T>(k, c, st, B, ldb, nrhs, phase);
    case 16: return run_leaf_phase<16, T>(k, c, st, B, ldb, nrhs, phase);
    default: return run_leaf_phase<8, T>(k, c, st, B, ldb, nrhs, phase);
  }
}

template <typename T>
int fast_factor(const KParams& k, const LaunchCfg& c, hipStream_t st) {
  switch (c.ht) {
    case 1: return run_fast_factor<T, 1>(k, c, st);
    case 2: return run_fast_factor<T, 2>(k, c, st);
    case 4: return run_fast_factor<T, 4>(k, c, st);
    case 8: return run_fast_factor<T, 8>(k, c, st);
    case 10: return run_fast_factor<T, 10>(k, c, st);
    default: return run_fast_factor<T, 16>(k, c, st);
  }
}

template <typename T>
int fast_phase(const KParams& k, const LaunchCfg& c, hipStream_t st, double* B, int64_t ldb, int nrhs, int phase) {
  switch (c.ht) {
    case 1: return run_fast_phase<T, 1>(k, c, st, B, ldb, nrhs, phase);
    case 2: return run_fast_phase<T, 2>(k, c, st, B, ldb, nrhs, phase);
    case 4: return run_fast_phase<T, 4>(k, c, st, B, ldb, nrhs, phase);
    case 8: return run_fast_phase<T, 8>(k, c, st, B, ldb, nrhs, phase);
    case 10: return run_fast_phase<T, 10>(k, c, st, B, ldb, nrhs, phase);
    default: return run_fast_phase<T, 16>(k, c, st, B, ldb, nrhs, phase);
  }
}

template <typename T>
int flu(const KParams& k, const LaunchCfg& c, hipStream_t st) {
  switch (c.ht) {
    case 1: return run_flu<T, 1>(k, c, st);
    case 2: return run_flu<T, 2>(k, c, st);
    case 4: return run_flu<T, 4>(k, c, st);
    case 8: return run_flu<T, 8>(k, c, st);
    default: return run_flu<T, 10>(k, c, st);
  }
}

int mfactor(const KParams& k, const LaunchCfg& c, hipStream_t st) {
  switch (c.mht) {
    case 1: return run_mfactor<1>(k, c, st);
    case 2: return run_mfactor<2>(k, c, st);
    case 4: return run_mfactor<4>(k, c, st);
    case 8: return run_mfactor<8>(k, c, st);
    case 10: return run_mfactor<10>(k, c, st);
    default: return run_mfactor<16>(k, c, st);
  }
}

int msolve(const KParams& k, const LaunchCfg& c, hipStream_t st, int nrhs, bool trans) {
  switch (c.mht) {
    case 1: return run_msolve<1>(k, c, st, nrhs, trans);
    case 2: return run_msolve<2>(k, c, st, nrhs, trans);
    case 4: return run_msolve<4>(k, c, st, nrhs, trans);
    case 8: return run_msolve<8>(k, c, st, nrhs, trans);
    case 10: return run_msolve<10>(k, c, st, nrhs, trans);
    default: return run_msolve<16>(k, c, st, nrhs, trans);
  }
}

int merge_factor(int nbd, const KParams& k, const LaunchCfg& c, hipStream_t st) {
  switch (nbd) {
    case 32: return run_merge_factor<32>(k, c, st);
    case 16: return run_merge_factor<16>(k, c, st);
    default: return run_merge_factor<8>(k, c, st);
  }
}

int merge_solve(int nbd, const KParams& k, const LaunchCfg& c, hipStream_t st, int nrhs, bool trans) {
  switch (nbd) {
    case 32: return run_merge_solve<32>(k, c, st, nrhs, trans);
    case 16: return run_merge_solve<16>(k, c, st, nrhs, trans);
    default: return run_merge_solve<8>(k, c, st, nrhs, trans);
  }
}

}  // namespace

int launch_init_status(DevStatus* s, hipStream_t st) { return run_init_status(s, st); }

namespace {
template <typename T>
int phase_batch(const BatchArgs& ba, int ht, size_t lds, hipStream_t st, int phase, int nitems) {
  switch (ht) {
    case 1: return run_fast_phase_batch<T, 1>(ba, lds, st, phase, nitems);
    case 2: return run_fast_phase_batch<T, 2>(ba, lds, st, phase, nitems);
    case 4: return run_fast_phase_batch<T, 4>(ba, lds, st, phase, nitems);
    case 8: return run_fast_phase_batch<T, 8>(ba, lds, st, phase, nitems);
    case 10: return run_fast_phase_batch<T, 10>(ba, lds, st, phase, nitems);
    default: return run_fast_phase_batch<T, 16>(ba, lds, st, phase, nitems);
  }
}
}  // namespace

int launch_phase_batch(const BatchArgs& ba, bool fp32, int ht, size_t lds, hipStream_t st, int phase, int nitems) {
  return fp32 ? phase_batch<float>(ba, ht, lds, st, phase, nitems)
              : phase_batch<double>(ba, ht, lds, st, phase, nitems);
}

int launch_mlevel_batch(const BatchArgs& ba, int mht, hipStream_t st, int nitems, bool trans, bool up) {
  switch (mht) {
    case 1: return run_msolve_level_batch<1>(ba, st, nitems, trans, up);
    case 2: return run_msolve_level_batch<2>(ba, st, nitems, trans, up);
    case 4: return run_msolve_level_batch<4>(ba, st, nitems, trans, up);
    case 8: return run_msolve_level_batch<8>(ba, st, nitems, trans, up);
    case 10: return run_msolve_level_batch<10>(ba, st, nitems, trans, up);
    default: return run_msolve_level_batch<16>(ba, st, nitems, trans, up);
  }
}

// The factor stage of up to kMaxBatch systems with one kernel configuration
// (the MFMA block LU, the tile-engine tips and the reduced system on MFMA
// tiles, equal bandwidths, non-pivoting): every kernel launch covers all of
// them.  p[s] is system s's partition count, level_off[s] its merge levels.
int launch_factor_batch(const BatchArgs& ba0, const int* p, const std::vector<const std::vector<int>*>& level_off,
                        const LaunchCfg& c, int kl, int ku, hipStream_t st) {
  BatchArgs ba = ba0;
  const int ns = ba.nsys;
  int e;
  if ((e = run_init_status_batch(ba, st))) return e;
  std::vector<int> cnt(ns), mids(ns);
  int maxL = 0;
  for (int s = 0; s < ns; ++s) {
    cnt[s] = p[s];
    mids[s] = p[s] >= 3 ? p[s] - 2 : 0;   // middle partitions: tile-engine tips (fast_tips)
    maxL = std::max(maxL, (int)level_off[s]->size() - 1);
  }
  const bool f32 = c.fp32;
  switch (c.ht) {
#define SPIKE_FB(H)                                                                                       \
  case H:                                                                                               \
    if ((e = f32 ? run_flu_batch<float, H>(ba, cnt.data(), st) : run_flu_batch<double, H>(ba, cnt.data(), st))) \
      return e;                                                                                         \
    for (int s = 0; s < ns; ++s) cnt[s] = p[s] > 1 ? p[s] : 0;                                           \
    for (int which = 0; which < 3; ++which) {                                                           \
      const int* cc = which == 0 ? cnt.data() : mids.data();                                            \
      if ((e = f32 ? run_ftip_batch<float, H>(ba, cc, which, kl, ku, c.fast_lds, st)                     \
                   : run_ftip_batch<double, H>(ba, cc, which, kl, ku, c.fast_lds, st)))                  \
        return e;                                                                                       \
    }                                                                                                   \
    break;
    SPIKE_FB(1)
    SPIKE_FB(2)
    SPIKE_FB(4)
    SPIKE_FB(8)
    SPIKE_FB(10)
#undef SPIKE_FB
    default:
      return -1;
  }
  for (int l = 0; l < maxL; ++l) {
    for (int s = 0; s < ns; ++s) {
      const std::vector<int>& lo = *level_off[s];
      const int L = (int)lo.size() - 1;
      ba.mbeg[s] = l < L ? lo[l] : 0;
      cnt[s] = l < L ? lo[l + 1] - lo[l] : 0;
    }
    switch (c.mht) {
      case 1: e = run_mfactor_level_batch<1>(ba, cnt.data(), kl, ku, st); break;
      case 2: e = run_mfactor_level_batch<2>(ba, cnt.data(), kl, ku, st); break;
      case 4: e = run_mfactor_level_batch<4>(ba, cnt.data(), kl, ku, st); break;
      case 8: e = run_mfactor_level_batch<8>(ba, cnt.data(), kl, ku, st); break;
      case 10: e = run_mfactor_level_batch<10>(ba, cnt.data(), kl, ku, st); break;
      default: e = run_mfactor_level_batch<16>(ba, cnt.data(), kl, ku, st); break;
    }
    if (e) return e;
  }
  return 0;
}

int launch_factor(const KParams& k0, const LaunchCfg& c, hipStream_t st) {
  KParams k = k0;
  int e;
  if (c.flu) {
    if ((e = c.fp32 ? flu<float>(k, c, st) : flu<double>(k, c, st))) return e;
    k.lu_done = 1;
  }
  if (!c.flu) {   // after the MFMA block LU the tip sweeps run in fast_factor
    e = c.fp32 ? leaf_factor<float>(c.nb, k, c, st) : leaf_factor<double>(c.nb, k, c, st);
    if (e) return e;
  }
  if (c.fast) {
    e = c.fp32 ? fast_factor<float>(k, c, st) : fast_factor<double>(k, c, st);
    if (e) return e;
  }
  if (k.p > 1) return c.mfast ? mfactor(k, c, st) : merge_factor(c.nb_dense, k, c, st);
  return 0;
}

int launch_solve(const KParams& k, const LaunchCfg& c, hipStream_t st, double* B, int64_t ldb, int nrhs,
                 bool trans) {
  const bool use_fast = c.fast && nrhs >= c.fast_min_nrhs;
  auto leaf = [&](int phase) {
    if (use_fast)
      return c.fp32 ? fast_phase<float>(k, c, st, B, ldb, nrhs, phase)
                    : fast_phase<double>(k, c, st, B, ldb, nrhs, phase);
    return c.fp32 ? leaf_phase<float>(c.nb, k, c, st, B, ldb, nrhs, phase)
                  : leaf_phase<double>(c.nb, k, c, st, B, ldb, nrhs, phase);
  };
  int e;
  if (!trans) {
    if ((e = leaf(0))) return e;            // D stage
    if (k.p > 1) {
      if ((e = c.mfast ? msolve(k, c, st, nrhs, false) : merge_solve(c.nb_dense, k, c, st, nrhs, false))) return e;
      if ((e = leaf(1))) return e;          // retrieval
    }
  } else {
    if ((e = leaf(2))) return e;            // Z sweeps of the transpose S stage
    if (k.p > 1) {
      if ((e = run_gform(k, st, B, ldb, nrhs))) return e;
      if ((e = c.mfast ? msolve(k, c, st, nrhs, true) : merge_solve(c.nb_dense, k, c, st, nrhs, true))) return e;
      if ((e = leaf(3))) return e;          // transpose D stage
    }
  }
  return 0;
}

}  // namespace spike
