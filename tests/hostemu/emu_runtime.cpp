// The stand-in runtime's thread indices, the launch that runs a grid as
// host threads (workgroups one after another, the threads of a workgroup
// concurrently) and the profiling hooks the kernels call (off here).  Shared
// by the replay drivers of this directory.
#include <algorithm>

#include "hip/hip_runtime.h"

thread_local EmuIdx threadIdx, blockIdx;
EmuIdx blockDim, gridDim;

namespace spike {
bool prof_enabled() { return false; }
int prof_begin(const char*, hipStream_t) { return -1; }
void prof_end(int, hipStream_t) {}
}  // namespace spike

void emu::launch(dim3 grid, dim3 block, size_t lds, const std::function<void()>& body) {
  const int nt = (int)(block.x * block.y * block.z);
  gridDim = {grid.x, grid.y, grid.z};
  blockDim = {block.x, block.y, block.z};
  for (unsigned by = 0; by < grid.y; ++by)
    for (unsigned bx = 0; bx < grid.x; ++bx) {
      Block* B = new Block();
      B->lds = static_cast<unsigned char*>(std::malloc(lds > 0 ? lds : 1));
      std::memset(B->lds, 0xff, lds);   // NaN pattern, as stale LDS may hold
      B->block.reset(nt);
      for (int w = 0; w < 16; ++w) B->wave[w].reset(std::max(0, std::min(64, nt - 64 * w)));
      cur_block() = B;
      std::vector<std::thread> th;
      th.reserve(nt);
      for (int t = 0; t < nt; ++t)
        th.emplace_back([=]() {
          threadIdx = {(unsigned)t, 0, 0};
          blockIdx = {bx, by, 0};
          body();
          B->wave[t / 64].leave();
          B->block.leave();
        });
      for (auto& x : th) x.join();
      std::free(B->lds);
      delete B;
    }
}
