// CPU replay of the diagonal-tile work of the block LU: the row-per-lane LU
// without interchanges (with boosting) and the inverses of its unit-lower and
// upper factors, run by one wavefront of host threads exactly as the panel of
// k_flu runs them (lanes 0-15 invert L, lanes 16-31 the reversed, row-scaled
// upper factor, and U^{-1} is rescaled by the reciprocal pivots by column).
//
// Usage: tile_lu_main IN OUT.  IN holds int64 count, mrem, fp32, then the
// double boost and count row-major 16 x 16 tiles; OUT receives, per tile,
// L\U, L^{-1} and U^{-1} (row-major doubles), then count int64 boost counts.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "spike_rowlu.hpp"

using namespace spike;

template <typename T>
static void factor_tile(const double* in, double boost, int mrem, double* out, long long* nbout) {
  emu::launch(dim3(1), dim3(64), 0, [&] {
    const int ln = threadIdx.x & 63, r = ln & 15;
    T ar[16];
    for (int c = 0; c < 16; ++c) ar[c] = (T)in[r * 16 + c];
    int nb = 0;
    lu16_rows<T>(ar, (T)boost, mrem, nb);
    T d = ar[0];
    for (int t = 1; t < 16; ++t) d = (r == t) ? ar[t] : d;
    const T myrp = d != T(0) ? recip(d) : T(0);
    if (ln < 16)
      for (int c = 0; c < 16; ++c) out[r * 16 + c] = (double)ar[c];
    const bool hi = (ln & 16) != 0;
    const T rpm = row_mirror(myrp);
    T mv[16], xi[16];
    for (int c = 0; c < 16; ++c) {
      const T am = row_mirror(ar[15 - c]);
      mv[c] = hi ? am * rpm : ar[c];
    }
    unit_lower_inv16_rows<T>(mv, xi);
    T rpv[16];
    for (int c = 0; c < 16; ++c) rpv[c] = row_bcast(myrp, 15 - c);
    if (ln < 16) {
      for (int c = 0; c < 16; ++c) out[256 + r * 16 + c] = (double)xi[c];
    } else if (ln < 32) {
      const int R = 15 - r;
      for (int c = 0; c < 16; ++c) out[512 + R * 16 + 15 - c] = (double)(xi[c] * rpv[c]);
    }
    if (ln == 0) *nbout = nb;
  });
}

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 3;
  long long hdr[3];
  double boost;
  if (std::fread(hdr, 8, 3, f) != 3 || std::fread(&boost, 8, 1, f) != 1) return 4;
  const long long cnt = hdr[0];
  const int mrem = (int)hdr[1];
  const bool fp32 = hdr[2] != 0;
  std::vector<double> in(cnt * 256), out(cnt * 768);
  std::vector<long long> nb(cnt);
  if (std::fread(in.data(), 8, in.size(), f) != in.size()) return 5;
  std::fclose(f);
  for (long long i = 0; i < cnt; ++i) {
    if (fp32) factor_tile<float>(&in[i * 256], boost, mrem, &out[i * 768], &nb[i]);
    else factor_tile<double>(&in[i * 256], boost, mrem, &out[i * 768], &nb[i]);
  }
  f = std::fopen(argv[2], "wb");
  if (!f) return 6;
  std::fwrite(out.data(), 8, out.size(), f);
  std::fwrite(nb.data(), 8, nb.size(), f);
  std::fclose(f);
  return 0;
}
