// Kernel parameter block and host launch entry points (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "spike_types.hpp"

#ifndef SPIKE_ERR_HIP
#define SPIKE_ERR_HIP (-1000)
#endif

namespace spike {

// Everything a kernel needs, passed by value.  Pointers are device pointers
// into the caller's workspace (or the caller's band for dAB).
struct KParams {
  int64_t n;
  int kl, ku, kw, kmax, p, pivot;
  int64_t ldw;
  int side_ld;
  int R;                 // columns per solve pass (workspace sizing)
  int64_t sscr_ld;       // rows of each leaf's solve scratch
  double boost_tau;      // relative boosting threshold (<= 0: off)
  const double* dAB;
  int64_t ldab;
  DevStatus* status;
  const LeafDesc* leaves;
  const MergeDesc* merges;
  const int* cptr;
  const Contrib* contrib;
  void* band;            // block factors (T)
  void* lpan;            // dense L panel tiles of pivoting factors (T)
  int64_t lpld;          // leading dimension of an L panel tile (nb + max(kl, ku))
  int* ipiv;
  double* bhat;
  double* chat;
  void* side;            // truncation side blocks (T)
  double* tips;
  double* sfac;
  int* spiv;
  double* coef;
  double* qw;
  void* fscr;            // factor-stage spike scratch (T)
  double* nodeval;
  double* st;
  double* xint;
  double* ztip;
  double* crl;
  double* sscr;
  const int32_t* skip;   // when non-null and *skip != 0 the solve kernels idle
  int fast_tips;         // middle-partition tips are formed by the MFMA tile kernels
  void* dinv;            // 16 x 16 diagonal-block inverses of L and U (T), tile engine
  int lu_done;           // the block factors are already in place (k_leaf_factor forms tips only)
  double* sdinv;         // 16 x 16 diagonal-block inverses of S's L and U, per interface
  int* sperm;            // row permutation of S's factorisation, per interface
  double* mtmp;          // reduced-solve scratch, kw x R per interface
  // Instrumented sweep counts (nullptr: off): entry (stage * 4 + leaf type) * 2
  // + full counts the triangular sweeps of one column set (a spike block or
  // the right-hand sides) over one partition's factor, full = 1 when the
  // sweep runs over all of the partition's rows; stage 0 = factorisation,
  // 1 = A X = F, 2 = A^T X = F.
  unsigned long long* sweeps;
};

constexpr int kSweepCounters = 3 * 4 * 2;

// Work items of several systems in one launch (solve-stage batching).
// System s owns the items [off[s], off[s+1]) of the launch; for a merge
// phase its items are the merges mbeg[s], mbeg[s]+1, ... of one tree level.
constexpr int kMaxBatch = 32;
struct BatchArgs {
  int nsys;
  int off[kMaxBatch + 1];
  int mbeg[kMaxBatch];
  int nrhs[kMaxBatch];
  int64_t ldb[kMaxBatch];
  double* B[kMaxBatch];
  const KParams* kp[kMaxBatch];   // device copies of the systems' parameters
};

__device__ __forceinline__ int batch_sys(const BatchArgs& ba, int item) {
  int s = 0;
  while (s + 1 < ba.nsys && item >= ba.off[s + 1]) ++s;
  return s;
}

struct LaunchCfg {
  int nb, nb_dense;
  bool fp32;
  size_t leaf_lds, merge_lds;
  std::vector<int> level_off;
  bool fast;             // MFMA tile engine usable (non-pivoting, bandwidth <= 256)
  int ht;                // its window height in 16-row tiles
  size_t fast_lds;
  int fast_min_nrhs;     // solves with at least this many columns use it
  int dinv_chunks;       // grid.y of the diagonal-inverse kernel
  bool flu;              // block LU on MFMA tiles (non-pivoting, window height <= 10 tiles)
  bool mfast;            // reduced system on MFMA tiles
  int mht;               // its sweep window height
};

template <int HT>
int run_mfactor(const KParams& k, const LaunchCfg& c, hipStream_t st);
template <int HT>
int run_msolve(const KParams& k, const LaunchCfg& c, hipStream_t st, int nrhs, bool trans);
template <typename T, int HT>
int run_fast_phase_batch(const BatchArgs& ba, size_t lds, hipStream_t st, int phase, int nitems);
template <int HT>
int run_msolve_level_batch(const BatchArgs& ba, hipStream_t st, int nitems, bool trans, bool up);
int run_gform_batch(const BatchArgs& ba, hipStream_t st, int nitems);
// Factor-stage launches for several systems of one kernel configuration;
// cnt[s] counts system s's work units (partitions, or merges of the level at
// ba.mbeg[s]); the runners fill ba.off from it.
int run_init_status_batch(const BatchArgs& ba, hipStream_t st);
template <typename T, int HT>
int run_flu_batch(BatchArgs ba, const int* cnt, hipStream_t st);
template <typename T, int HT>
int run_ftip_batch(BatchArgs ba, const int* cnt, int which, int kl, int ku, size_t lds, hipStream_t st);
template <int HT>
int run_mfactor_level_batch(BatchArgs ba, const int* cnt, int kl, int ku, hipStream_t st);
template <typename T, int HT>
int run_flu(const KParams& k, const LaunchCfg& c, hipStream_t st);
template <typename T, int HT>
int run_fast_factor(const KParams& k, const LaunchCfg& c, hipStream_t st);
template <typename T, int HT>
int run_fast_phase(const KParams& k, const LaunchCfg& c, hipStream_t st, double* B, int64_t ldb, int nrhs,
                   int phase);

// Runners, instantiated per panel width / precision in spike_inst.hip.
template <int NB, typename T>
int run_leaf_factor(const KParams& k, const LaunchCfg& c, hipStream_t st);
template <int NB, typename T>
int run_leaf_phase(const KParams& k, const LaunchCfg& c, hipStream_t st, double* B, int64_t ldb, int nrhs,
                   int phase);
template <int NBD>
int run_merge_factor(const KParams& k, const LaunchCfg& c, hipStream_t st);
template <int NBD>
int run_merge_solve(const KParams& k, const LaunchCfg& c, hipStream_t st, int nrhs, bool trans);
int run_init_status(DevStatus* s, hipStream_t st);
int run_gform(const KParams& k, hipStream_t st, const double* B, int64_t ldb, int nrhs);

int launch_init_status(DevStatus* s, hipStream_t st);
int run_zero_counters(unsigned long long* c, int n, hipStream_t st);
int launch_phase_batch(const BatchArgs& ba, bool fp32, int ht, size_t lds, hipStream_t st, int phase, int nitems);
int launch_mlevel_batch(const BatchArgs& ba, int mht, hipStream_t st, int nitems, bool trans, bool up);
int launch_factor(const KParams& k, const LaunchCfg& c, hipStream_t st);
int launch_factor_batch(const BatchArgs& ba, const int* p, const std::vector<const std::vector<int>*>& level_off,
                        const LaunchCfg& c, int kl, int ku, hipStream_t st);
int launch_solve(const KParams& k, const LaunchCfg& c, hipStream_t st, double* B, int64_t ldb, int nrhs,
                 bool trans);

}  // namespace spike
