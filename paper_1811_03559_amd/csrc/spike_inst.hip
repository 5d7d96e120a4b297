// One translation unit per group of kernel instantiations, selected by the
// build with -DSPIKE_INST_LEAF (with SPIKE_NB, SPIKE_T), -DSPIKE_INST_MERGE
// (with SPIKE_NB) or -DSPIKE_INST_COMMON, so the kernels compile in parallel.
#include "spike_fast.hpp"
#include "spike_flu.hpp"
#include "spike_merge.hpp"
#include "spike_kernels.hpp"

namespace spike {

#if defined(SPIKE_INST_LEAF)
template int run_leaf_factor<SPIKE_NB, SPIKE_T>(const KParams&, const LaunchCfg&, hipStream_t);
template int run_leaf_phase<SPIKE_NB, SPIKE_T>(const KParams&, const LaunchCfg&, hipStream_t, double*, int64_t,
                                                int, int);
#elif defined(SPIKE_INST_MERGE)
template int run_merge_factor<SPIKE_NB>(const KParams&, const LaunchCfg&, hipStream_t);
template int run_merge_solve<SPIKE_NB>(const KParams&, const LaunchCfg&, hipStream_t, int, bool);
#elif defined(SPIKE_INST_FAST)
template int run_fast_factor<SPIKE_T, SPIKE_HT>(const KParams&, const LaunchCfg&, hipStream_t);
#if SPIKE_HT <= 10
template int run_flu<SPIKE_T, SPIKE_HT>(const KParams&, const LaunchCfg&, hipStream_t);
#endif
template int run_fast_phase<SPIKE_T, SPIKE_HT>(const KParams&, const LaunchCfg&, hipStream_t, double*, int64_t,
                                                int, int);
template int run_fast_phase_batch<SPIKE_T, SPIKE_HT>(const BatchArgs&, size_t, hipStream_t, int, int);
template int run_ftip_batch<SPIKE_T, SPIKE_HT>(BatchArgs, const int*, int, int, int, size_t, hipStream_t);
#if SPIKE_HT <= 10
template int run_flu_batch<SPIKE_T, SPIKE_HT>(BatchArgs, const int*, hipStream_t);
#endif
#elif defined(SPIKE_INST_MFAST)
template int run_mfactor<SPIKE_HT>(const KParams&, const LaunchCfg&, hipStream_t);
template int run_msolve<SPIKE_HT>(const KParams&, const LaunchCfg&, hipStream_t, int, bool);
template int run_msolve_level_batch<SPIKE_HT>(const BatchArgs&, hipStream_t, int, bool, bool);
template int run_mfactor_level_batch<SPIKE_HT>(BatchArgs, const int*, int, int, hipStream_t);
#elif defined(SPIKE_INST_COMMON)
int run_init_status(DevStatus* s, hipStream_t st) {
  hipLaunchKernelGGL(k_init_status, dim3(1), dim3(64), 0, st, s);
  SPIKE_CHECK_LAUNCH();
  return 0;
}

static __global__ void k_init_status_b(BatchArgs ba) {
  if (threadIdx.x == 0 && blockIdx.x < (unsigned)ba.nsys) init_status_fields(ba.kp[blockIdx.x]->status);
}

int run_init_status_batch(const BatchArgs& ba, hipStream_t st) {
  if (ba.nsys <= 0) return 0;
  hipLaunchKernelGGL(k_init_status_b, dim3(ba.nsys), dim3(64), 0, st, ba);
  SPIKE_CHECK_LAUNCH();
  return 0;
}

int run_zero_counters(unsigned long long* c, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, st, c, n);
  SPIKE_CHECK_LAUNCH();
  return 0;
}

int run_gform_batch(const BatchArgs& ba, hipStream_t st, int nitems) {
  if (nitems <= 0) return 0;
  ProfScope ps("k_gform", st);
  hipLaunchKernelGGL(k_gform_b, dim3(nitems), dim3(NT), 0, st, ba);
  SPIKE_CHECK_LAUNCH();
  return 0;
}

int run_gform(const KParams& k, hipStream_t st, const double* B, int64_t ldb, int nrhs) {
  ProfScope ps("k_gform", st);
  hipLaunchKernelGGL(k_gform, dim3(k.p - 1), dim3(NT), 0, st, k, B, ldb, nrhs);
  SPIKE_CHECK_LAUNCH();
  return 0;
}
#else
#error "select an instantiation group"
#endif

}  // namespace spike
