// Host-side check of the exact integer arithmetic the tiled particle kernels use
// (pm_particles.h): the window-cell division by a high multiply, the cell
// decomposition and numbering, the fixed-point weights, the node index, the packed
// window reduction and the over-capacity window.  Prints "ok" and exits 0 on success.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "pm_particles.h"

using namespace pm;

static int fails = 0;
#define EXPECT(cond, ...)                 \
  do {                                    \
    if (!(cond)) {                        \
      if (fails < 10) printf(__VA_ARGS__); \
      ++fails;                            \
    }                                     \
  } while (0)

int main() {
  // tile_coords: a bijection from workgroup order onto the tile grid, for the grids of
  // the tiled kernels at every supported mesh size (blocked and plain orders)
  {
    const int sizes[] = {64, 128, 192, 256, 512, 1024};
    const int shapes[][4] = {{4, 8, 32, 2}, {4, 8, 32, 1}, {8, 8, 16, 1}};  // tile x, y, z, tiles per workgroup in x
    for (int n : sizes)
      for (const auto& sh : shapes) {
        const int tx = n / (sh[0] * sh[3]), ty = n / sh[1], tz = n / sh[2];
        const int64_t total = (int64_t)tx * ty * tz;
        std::vector<unsigned char> seen((size_t)total, 0);
        for (int64_t lin = 0; lin < total; ++lin) {
          int ti, tk, tl;
          tile_coords(lin, tx, ty, tz, ti, tk, tl);
          const bool in = ti >= 0 && ti < tx && tk >= 0 && tk < ty && tl >= 0 && tl < tz;
          EXPECT(in, "tile_coords out of range: n %d lin %lld -> %d %d %d\n", n, (long long)lin, ti, tk, tl);
          if (in) seen[((size_t)ti * ty + tk) * tz + tl] += 1;
        }
        for (int64_t i = 0; i < total; ++i) EXPECT(seen[(size_t)i] == 1, "tile_coords: tile %lld seen %d times\n", (long long)i, (int)seen[(size_t)i]);
      }
    // odd grids take the plain order
    for (int tx : {3, 5, 8, 12}) {
      int ti, tk, tl;
      tile_coords(7 + 5 * 4, tx, 6, 5, ti, tk, tl);
      if (tx % kTileBlock != 0) EXPECT(ti == (7 + 20) / 5 / 6 && tk == ((7 + 20) / 5) % 6 && tl == 2, "plain order\n");
    }
  }
  // WinDiv: floor(c / d) for every c, d in the window range (c < 2^14, 2 <= d < 2^14)
  for (unsigned d = 2; d < 16384; ++d) {
    const WinDiv q((int)d);
    for (unsigned c = 0; c < 16384; ++c) EXPECT(q.quot(c) == c / d, "quot %u / %u\n", c, d);
  }
  // win_cell / win_index: c = a sx + b sy + cz round trip over whole windows
  std::mt19937 rng(7);
  for (int it = 0; it < 2000; ++it) {
    const int W0 = 2 + (int)(rng() % 30), W1 = 2 + (int)(rng() % 30), W2 = 2 + (int)(rng() % 60);
    if (W0 * W1 * W2 > 6144) continue;
    const int sy = W2, sx = W1 * W2;
    const WinDiv qx(sx), qy(sy);
    for (int c = 0; c < W0 * W1 * W2; ++c) {
      int a, b, cz;
      win_cell(c, qx, qy, a, b, cz);
      EXPECT(a >= 0 && a < W0 && b >= 0 && b < W1 && cz >= 0 && cz < W2 && win_index(a, b, cz, sx, sy) == c,
             "win_cell %d in %dx%dx%d\n", c, W0, W1, W2);
    }
  }
  // to_fix_w: w 2^21 rounded to nearest-even, exactly, for every float in [0, 1]; the
  // capped form stays below 2^21, so 2048 terms cannot wrap 32 bits
  for (unsigned bits = 0; bits <= 0x3F800000u; ++bits) {
    const float w = __builtin_bit_cast(float, bits);
    const double x = (double)w * 2097152.0;  // exact
    const double want = std::nearbyint(x);   // default rounding: to nearest, ties to even
    EXPECT(to_fix_w(w) == (unsigned)want, "to_fix_w %a\n", (double)w);
    EXPECT(to_fix_w_capped(w) == (unsigned)std::min(want, 2097151.0), "to_fix_w_capped %a\n", (double)w);
  }
  EXPECT(2048.0 * 2097151.0 < 4294967296.0 && 1024.0 * 2097152.0 < 4294967296.0, "window sum bounds\n");
  // node_index: both forms against the 64-bit flat index
  for (int n : {64, 128, 192, 256, 1024}) {
    for (int it = 0; it < 100000; ++it) {
      const int i = (int)(rng() % n), j = (int)(rng() % n), l = (int)(rng() % n);
      const unsigned long long want = ((unsigned long long)i * n + j) * n + l;
      EXPECT(node_index<false>(i, j, l, n) == want, "node_index %d %d %d / %d\n", i, j, l, n);
      if ((n & (n - 1)) == 0) EXPECT(node_index<true>(i, j, l, n) == want, "node_index p2 %d %d %d / %d\n", i, j, l, n);
    }
  }
  // packed reduction of (lo, -hi): the minimum of packs is the pack of (min lo, max hi)
  for (int it = 0; it < 200000; ++it) {
    int lo = 1 << 30, hi = -(1 << 30), pk = pack_lo_nhi(1 << 30, -(1 << 30));
    const int k = (int)(rng() % 64);
    for (int s = 0; s < k; ++s) {
      const int a = (int)(rng() % 1025) - 512, b = a + (int)(rng() % 40);
      lo = a < lo ? a : lo;
      hi = b > hi ? b : hi;
      pk = min_lo_nhi(pk, pack_lo_nhi(a, b));
    }
    const int glo = (int)(short)(pk & 0xFFFF), ghi = -(int)(short)((unsigned)pk >> 16);
    if (k == 0) EXPECT(glo == 32767 && ghi == -32767, "empty pack\n");
    else EXPECT(glo == lo && ghi == hi, "pack %d %d vs %d %d\n", glo, ghi, lo, hi);
  }
  // fit_box: the window fits the capacity, keeps every side in [2, W] and stays inside the box
  for (int cap : {4096, 6144}) {
    for (int it = 0; it < 300000; ++it) {
      int W[3], o[3];
      float mean[3];
      for (int d = 0; d < 3; ++d) {
        W[d] = 2 + (int)(rng() % ((rng() & 1) ? 40 : 1100));
        o[d] = -(int)(rng() % 600);
        mean[d] = (float)o[d] + (float)(rng() % (unsigned)W[d]) + 0.37f;
      }
      const long long vol = (long long)W[0] * W[1] * W[2];
      if (vol <= cap) continue;
      int Wf[3] = {W[0], W[1], W[2]}, of[3] = {o[0], o[1], o[2]};
      fit_box(of, Wf, mean, vol, cap);
      EXPECT((long long)Wf[0] * Wf[1] * Wf[2] <= cap, "fit_box volume %d %d %d\n", Wf[0], Wf[1], Wf[2]);
      for (int d = 0; d < 3; ++d)
        EXPECT(Wf[d] >= 2 && Wf[d] <= W[d] && of[d] >= o[d] && of[d] + Wf[d] <= o[d] + W[d], "fit_box side %d\n", d);
    }
  }
  if (fails) {
    printf("%d failures\n", fails);
    return 1;
  }
  printf("ok\n");
  return 0;
}
