// Host stand-in for the HIP runtime header, used only by the CPU replay of
// the workgroup kernels (tests/hostemu): every workgroup runs as blockDim.x
// host threads, __syncthreads() is a barrier over the threads of the block
// that have not returned, cross-lane shuffles exchange through a per-wave
// slot array, and every dynamic LDS buffer is its own heap allocation of the
// launch's size, so AddressSanitizer reports any access outside it.
#pragma once
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __align__(x) __attribute__((aligned(x)))
#define HIP_SYMBOL(x) (&(x))

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2 };
typedef struct ihipStream_t* hipStream_t;
typedef struct ihipEvent_t* hipEvent_t;
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };
enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2 };

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

struct EmuIdx { unsigned x, y, z; };
extern thread_local EmuIdx threadIdx, blockIdx;
extern EmuIdx blockDim, gridDim;

namespace emu {

// Barrier over the threads of a workgroup (or wavefront) that have not
// returned: arrivals spin (yielding) on a generation counter; a thread that
// returns leaves, and releases the others when it was the last one missing.
struct Barrier {
  std::mutex mu;
  std::atomic<unsigned long> gen{0};
  int active = 0, arrived = 0;
  void reset(int n) { active = n; arrived = 0; }
  void arrive() {
    unsigned long g;
    {
      std::lock_guard<std::mutex> lk(mu);
      g = gen.load();
      if (++arrived >= active) { arrived = 0; gen.fetch_add(1); return; }
    }
    while (gen.load(std::memory_order_acquire) == g) std::this_thread::yield();
  }
  void leave() {
    std::lock_guard<std::mutex> lk(mu);
    --active;
    if (arrived > 0 && arrived >= active) { arrived = 0; gen.fetch_add(1); }
  }
};

struct Block {
  Barrier block;
  Barrier wave[16];
  uint64_t slot[16][64];
  uint64_t slot2[16][64];
  uint64_t slot3[16][64][4];
  unsigned char* lds = nullptr;
};

inline Block*& cur_block() { static Block* b = nullptr; return b; }
inline std::mutex& atom_mu() { static std::mutex m; return m; }
inline int& last_error() { static int e = 0; return e; }

}  // namespace emu


inline void __syncthreads() { emu::cur_block()->block.arrive(); }
inline void __threadfence_block() {}
inline void __threadfence() {}

template <typename V>
inline V __shfl_xor(V v, int mask, int width = 64) {
  (void)width;
  emu::Block* b = emu::cur_block();
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  uint64_t bits = 0;
  std::memcpy(&bits, &v, sizeof(V));
  b->slot[w][l] = bits;
  b->wave[w].arrive();
  uint64_t o = b->slot[w][l ^ mask];
  b->wave[w].arrive();
  V r;
  std::memcpy(&r, &o, sizeof(V));
  return r;
}

namespace emu {
// Value of lane `src` of v, in every lane of the wavefront.
template <typename V>
inline V readlane(V v, int src) {
  Block* b = cur_block();
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  uint64_t bits = 0;
  std::memcpy(&bits, &v, sizeof(V));
  b->slot[w][l] = bits;
  b->wave[w].arrive();
  uint64_t o = b->slot[w][src];
  b->wave[w].arrive();
  V r;
  std::memcpy(&r, &o, sizeof(V));
  return r;
}

// D = A B + C of one 16 x 16 x 4 matrix-core step of the wavefront: lane l
// holds A(l % 16, l / 16) and B(l / 16, l % 16); its four accumulator values
// are D(row(l, v), l % 16), with row(l, v) = l / 16 + 4 v for FP64 and
// 4 (l / 16) + v for FP32 (the layouts the kernels address them with).
template <typename S, typename V>
inline V mfma16x16x4(S a, S bb, V c, bool f64) {
  Block* b = cur_block();
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  double av = (double)a, bv = (double)bb;
  std::memcpy(&b->slot[w][l], &av, 8);
  std::memcpy(&b->slot2[w][l], &bv, 8);
  b->wave[w].arrive();
  V d = c;
  const int j = l % 16;
  for (int v = 0; v < 4; ++v) {
    const int i = f64 ? l / 16 + 4 * v : 4 * (l / 16) + v;
    double s = 0.0;
    for (int k = 0; k < 4; ++k) {
      double x, y;
      std::memcpy(&x, &b->slot[w][i + 16 * k], 8);
      std::memcpy(&y, &b->slot2[w][j + 16 * k], 8);
      s += x * y;
    }
    d[v] = (S)((double)c[v] + s);
  }
  b->wave[w].arrive();
  return d;
}

// __builtin_amdgcn_update_dpp for the row controls the kernels replayed here
// use: row_newbcast:n (0x150 + n, lane n of each 16-lane row to the whole
// row) and row_mirror (0x140, lane 15 - i of each row to lane i).
inline int update_dpp(int v, int ctrl) {
  Block* b = cur_block();
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  b->slot[w][l] = (uint64_t)(uint32_t)v;
  b->wave[w].arrive();
  int src;
  if (ctrl >= 0x150 && ctrl <= 0x15f) src = (l & 48) + (ctrl - 0x150);
  else if (ctrl == 0x140) src = (l & 48) + 15 - (l & 15);
  else std::abort();
  const int r = (int)(uint32_t)b->slot[w][src];
  b->wave[w].arrive();
  return r;
}

struct Pair2 {
  unsigned v[2];
  unsigned operator[](int i) const { return v[i]; }
};
[[noreturn]] inline Pair2 unsupported_pair() { std::abort(); }
[[noreturn]] inline int unsupported_int() { std::abort(); }
}  // namespace emu

#define __builtin_amdgcn_readlane(v, s) ::emu::readlane((v), (s))
#define __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, x, y, z) ::emu::mfma16x16x4<double>((a), (b), (c), true)
#define __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, x, y, z) ::emu::mfma16x16x4<float>((a), (b), (c), false)
#define __builtin_amdgcn_permlane16_swap(...) ::emu::unsupported_pair()
#define __builtin_amdgcn_permlane32_swap(...) ::emu::unsupported_pair()
#define __builtin_amdgcn_update_dpp(old, v, ctrl, rm, bm, bc) ::emu::update_dpp((v), (ctrl))
#define __builtin_amdgcn_wave_barrier() ((void)0)
#define __builtin_amdgcn_rcp(x) (1.0 / (double)(x))
#define __builtin_amdgcn_rcpf(x) (1.0f / (float)(x))
#define __builtin_amdgcn_fence(...) ((void)0)

template <typename A, typename B> inline auto min(A a, B b) -> decltype(a < b ? a : b) { return a < b ? a : b; }
template <typename A, typename B> inline auto max(A a, B b) -> decltype(a < b ? a : b) { return a < b ? b : a; }
using std::fabs;
using std::fmax;
using std::fmin;
using std::sqrt;

template <typename V> inline V atomicMin(V* p, V v) {
  std::lock_guard<std::mutex> lk(emu::atom_mu()); V o = *p; if (v < o) *p = v; return o;
}
template <typename V> inline V atomicMax(V* p, V v) {
  std::lock_guard<std::mutex> lk(emu::atom_mu()); V o = *p; if (v > o) *p = v; return o;
}
template <typename V> inline V atomicAdd(V* p, V v) {
  std::lock_guard<std::mutex> lk(emu::atom_mu()); V o = *p; *p = o + v; return o;
}

inline long long __double_as_longlong(double x) { long long r; std::memcpy(&r, &x, 8); return r; }
inline double __longlong_as_double(long long x) { double r; std::memcpy(&r, &x, 8); return r; }
inline int __float_as_int(float x) { int r; std::memcpy(&r, &x, 4); return r; }
inline unsigned __float_as_uint(float x) { unsigned r; std::memcpy(&r, &x, 4); return r; }
inline float __int_as_float(int x) { float r; std::memcpy(&r, &x, 4); return r; }
inline float __uint_as_float(unsigned x) { float r; std::memcpy(&r, &x, 4); return r; }

inline hipError_t hipGetLastError() { int e = emu::last_error(); emu::last_error() = 0; return e; }
template <typename K> inline hipError_t hipFuncSetAttribute(K, hipFuncAttribute, int) { return hipSuccess; }

namespace emu {
// Runs `body` once per thread of every workgroup of the grid: workgroups one
// after another, the threads of a workgroup concurrently.
void launch(dim3 grid, dim3 block, size_t lds, const std::function<void()>& body);
}  // namespace emu

#define hipLaunchKernelGGL(kernel, grid, block, lds, stream, ...) \
  ::emu::launch(grid, block, lds, [=]() { kernel(__VA_ARGS__); })
