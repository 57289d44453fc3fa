// CIC counting-density deposit (counting density of a cloud-in-cell assignment, as
// used for every density and spectrum in the paper).
//
// Two kernels with the same cell assignment and the same float weights:
//   k_deposit        one thread per particle, 8 global float atomics each (any np);
//   k_deposit_tiled  for a full Lagrangian lattice run (np = N^3): a workgroup owns a
//                    Lagrangian tile, accumulates its particles in an LDS window in
//                    32-bit fixed point at scale 2^21, terms capped at 2^21 - 1 so that
//                    the tile's 2048 particles cannot wrap a cell (LDS integer atomics
//                    run ~20x faster than LDS float atomics on gfx950), then adds each non-empty
//                    window cell to the mesh with one global float atomic.  A window
//                    that would exceed the LDS capacity shrinks to fit_box's box of
//                    the same proportions; particles outside it use global atomics.
// The mesh is pre-filled with -1, so it holds delta = rho/nbar - 1 afterwards.
#include <math.h>

#include "pm_particles.h"
#include "pm_plan.h"

namespace pm {

namespace {

constexpr int kBlock = 256;

template <typename T>
__global__ void __launch_bounds__(kBlock) k_deposit(const T* __restrict__ pos, int64_t np, T* __restrict__ mesh, int n,
                                                    T w_scale, unsigned* __restrict__ guard,
                                                    const BoxEntry* __restrict__ tab) {
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i = blk * kBlock + threadIdx.x;
  if (i >= np) return;
  pos = box_positions(tab, np, pos);  // box of the batch
  mesh += (int64_t)blockIdx.y * n * n * n;
  T x = pos[i], y = pos[np + i], z = pos[2 * np + i];
  if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
    atomicAdd(&guard[0], 1u);
    return;
  }
  const T fn = T(n);
  if (!(x >= T(0) && x < fn && y >= T(0) && y < fn && z >= T(0) && z < fn)) {
    atomicAdd(&guard[1], 1u);
    x = wrap(x, n);
    y = wrap(y, n);
    z = wrap(z, n);
  }
  const Axis<T> ax = cic_axis(x, n), ay = cic_axis(y, n), az = cic_axis(z, n);
  const int64_t n2 = (int64_t)n * n;
  const int64_t r00 = ax.i0 * n2 + (int64_t)ay.i0 * n, r01 = ax.i0 * n2 + (int64_t)ay.i1 * n;
  const int64_t r10 = ax.i1 * n2 + (int64_t)ay.i0 * n, r11 = ax.i1 * n2 + (int64_t)ay.i1 * n;
  const T wxy00 = ax.w0 * ay.w0 * w_scale, wxy01 = ax.w0 * ay.w1 * w_scale;
  const T wxy10 = ax.w1 * ay.w0 * w_scale, wxy11 = ax.w1 * ay.w1 * w_scale;
  atomic_add(mesh + r00 + az.i0, wxy00 * az.w0);
  atomic_add(mesh + r00 + az.i1, wxy00 * az.w1);
  atomic_add(mesh + r01 + az.i0, wxy01 * az.w0);
  atomic_add(mesh + r01 + az.i1, wxy01 * az.w1);
  atomic_add(mesh + r10 + az.i0, wxy10 * az.w0);
  atomic_add(mesh + r10 + az.i1, wxy10 * az.w1);
  atomic_add(mesh + r11 + az.i0, wxy11 * az.w0);
  atomic_add(mesh + r11 + az.i1, wxy11 * az.w1);
}

// Tile of TX x TY x TZ particles (Lagrangian indices), window capacity in cells.  The
// tile is long in z so that the window's rows are long: the flush's atomics on one
// row go to the L2 in requests of up to 16 consecutive cells, so a 33-cell row costs
// 3 requests where two 17-cell rows (a 16-long tile) cost 4 or more.
constexpr int TX = 8, TY = 8, TZ = 32;
constexpr int TPP = TX * TY * TZ / kBlock;  // particles per thread
constexpr int WCAP = 8192;                  // LDS window cells (32-bit fixed point, to_fix_w_capped)

// np = N^3, particle (i N + k) N + l started in cell (i, k, l).  The window is the
// bounding box of the tile's CIC cells when it fits in WCAP cells, else fit_box's
// smaller box of the same proportions; particles whose cells fall outside the window
// go to global atomics.  All window arithmetic is integer on the base nodes floor(x).
template <bool P2>
__global__ void __launch_bounds__(kBlock) k_deposit_tiled(const float* __restrict__ pos, float* __restrict__ mesh,
                                                          int n, double w_scale, unsigned* __restrict__ guard,
                                                          const BoxEntry* __restrict__ tab) {
  static_assert((double)TX * TY * TZ * (kFixW - 1.0f) < 4294967296.0, "a window cell could wrap");
  __shared__ unsigned win[WCAP];
  __shared__ int wlo[kBlock / 64][3], whi[kBlock / 64][3];
  __shared__ float wsum[kBlock / 64][3];
  const int64_t np = (int64_t)n * n * n;
  pos = box_positions(tab, np, pos);  // box of the batch
  mesh += (int64_t)blockIdx.y * np;
  const int tpx = n / TX, tpy = n / TY, tpz = n / TZ;
  int ti, tk, tl;
  tile_coords(xcd_block(blockIdx.x, gridDim.x), tpx, tpy, tpz, ti, tk, tl);
  const int org[3] = {ti * TX, tk * TY, tl * TZ};
  const int t = threadIdx.x;
  const float fn = float(n);
  float x[TPP], y[TPP], z[TPP];
  int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
  float sum[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int p = 0; p < TPP; ++p) {
    const int loc = t + kBlock * p;
    const int li = loc / (TY * TZ), lk = (loc / TZ) % TY, ll = loc % TZ;
    const unsigned j = node_index<P2>(org[0] + li, org[1] + lk, org[2] + ll, n);
    x[p] = ldg32(pos, j);
    y[p] = ldg32(pos + np, j);
    z[p] = ldg32(pos + 2 * np, j);
  }
#pragma unroll
  for (int p = 0; p < TPP; ++p) {
    if (!(isfinite(x[p]) && isfinite(y[p]) && isfinite(z[p]))) {
      atomicAdd(&guard[0], 1u);
      x[p] = -1.f;  // marks a skipped particle
      continue;
    }
    if (!(x[p] >= 0.f && x[p] < fn && y[p] >= 0.f && y[p] < fn && z[p] >= 0.f && z[p] < fn)) {
      atomicAdd(&guard[1], 1u);
      x[p] = wrap_n<P2>(x[p], n);
      y[p] = wrap_n<P2>(y[p], n);
      z[p] = wrap_n<P2>(z[p], n);
    }
    const int r[3] = {idiff_n<P2>((int)floorf(x[p]), org[0], n), idiff_n<P2>((int)floorf(y[p]), org[1], n),
                      idiff_n<P2>((int)floorf(z[p]), org[2], n)};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = min(lo[d], r[d]);
      hi[d] = max(hi[d], r[d]);
      sum[d] += float(r[d]);
    }
  }
  int o[3], W[3];
  block_window(lo, hi, sum, TX * TY * TZ, WCAP, wlo, whi, wsum, o, W);
  const int wtot = W[0] * W[1] * W[2];
  for (int c = t; c < wtot; c += kBlock) win[c] = 0u;
  __syncthreads();
  const int sy = W[2], sx = W[1] * W[2];
  const int64_t n2 = (int64_t)n * n;
#pragma unroll
  for (int p = 0; p < TPP; ++p) {
    if (x[p] < 0.f) continue;
    const Axis<float> ax = cic_axis_n<P2>(x[p], n), ay = cic_axis_n<P2>(y[p], n), az = cic_axis_n<P2>(z[p], n);
    const int rx = idiff_n<P2>(ax.i0, org[0], n) - o[0], ry = idiff_n<P2>(ay.i0, org[1], n) - o[1],
              rz = idiff_n<P2>(az.i0, org[2], n) - o[2];
    const float wxy00 = ax.w0 * ay.w0, wxy01 = ax.w0 * ay.w1;
    const float wxy10 = ax.w1 * ay.w0, wxy11 = ax.w1 * ay.w1;
    if (rx >= 0 && rx <= W[0] - 2 && ry >= 0 && ry <= W[1] - 2 && rz >= 0 && rz <= W[2] - 2) {
      unsigned* w = win + win_index(rx, ry, rz, sx, sy);
      atomicAdd(w, to_fix_w_capped(wxy00 * az.w0));
      atomicAdd(w + 1, to_fix_w_capped(wxy00 * az.w1));
      atomicAdd(w + sy, to_fix_w_capped(wxy01 * az.w0));
      atomicAdd(w + sy + 1, to_fix_w_capped(wxy01 * az.w1));
      atomicAdd(w + sx, to_fix_w_capped(wxy10 * az.w0));
      atomicAdd(w + sx + 1, to_fix_w_capped(wxy10 * az.w1));
      atomicAdd(w + sx + sy, to_fix_w_capped(wxy11 * az.w0));
      atomicAdd(w + sx + sy + 1, to_fix_w_capped(wxy11 * az.w1));
    } else {
      const float ws = float(w_scale);
      const int64_t r00 = ax.i0 * n2 + (int64_t)ay.i0 * n, r01 = ax.i0 * n2 + (int64_t)ay.i1 * n;
      const int64_t r10 = ax.i1 * n2 + (int64_t)ay.i0 * n, r11 = ax.i1 * n2 + (int64_t)ay.i1 * n;
      atomic_add(mesh + r00 + az.i0, wxy00 * az.w0 * ws);
      atomic_add(mesh + r00 + az.i1, wxy00 * az.w1 * ws);
      atomic_add(mesh + r01 + az.i0, wxy01 * az.w0 * ws);
      atomic_add(mesh + r01 + az.i1, wxy01 * az.w1 * ws);
      atomic_add(mesh + r10 + az.i0, wxy10 * az.w0 * ws);
      atomic_add(mesh + r10 + az.i1, wxy10 * az.w1 * ws);
      atomic_add(mesh + r11 + az.i0, wxy11 * az.w0 * ws);
      atomic_add(mesh + r11 + az.i1, wxy11 * az.w1 * ws);
    }
  }
  __syncthreads();
  const double scale = w_scale / (double)kFixW;  // in FP64: a float 1/S would bias the total mass
  const WinDiv qsx(sx), qsy(sy);
  for (int c = t; c < wtot; c += kBlock) {
    const unsigned v = win[c];
    if (v == 0u) continue;
    int a, b, cz;
    win_cell(c, qsx, qsy, a, b, cz);
    const unsigned idx = node_index<P2>(fold_n<P2>(org[0] + o[0] + a, n), fold_n<P2>(org[1] + o[1] + b, n),
                                        fold_n<P2>(org[2] + o[2] + cz, n), n);
    atomic_add(mesh + idx, (float)((double)v * scale));
  }
}

inline unsigned nblocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

int launch_deposit(const pm_plan* p, const void* pos, int64_t np, void* mesh, hipStream_t s) {
  ProfScope ps(p, PK_DEPOSIT, s);
  if (np <= 0) return PM_OK;
  const int n = p->n;
  const double n3 = (double)n * n * n;
  const double w = n3 / (double)np;  // 1 / nbar
  if (p->dtype == PM_F32 && (int64_t)n * n * n == np && n >= 64 && n <= 1024 && n % TZ == 0 && n % TX == 0) {
    const unsigned tiles = (unsigned)((n / TX) * (n / TY) * (n / TZ));
    // a power-of-two N wraps without a division (same results)
    auto kern = (n & (n - 1)) == 0 ? k_deposit_tiled<true> : k_deposit_tiled<false>;
    hipLaunchKernelGGL(kern, dim3(tiles, (unsigned)p->nb), dim3(kBlock), 0, s, static_cast<const float*>(pos),
                       static_cast<float*>(mesh), n, w, p->guard, p->box_tab);
  } else if (p->dtype == PM_F32) {
    hipLaunchKernelGGL(k_deposit<float>, dim3(nblocks(np), (unsigned)p->nb), dim3(kBlock), 0, s, static_cast<const float*>(pos), np,
                       static_cast<float*>(mesh), n, (float)w, p->guard, p->box_tab);
  } else {
    hipLaunchKernelGGL(k_deposit<double>, dim3(nblocks(np), (unsigned)p->nb), dim3(kBlock), 0, s, static_cast<const double*>(pos), np,
                       static_cast<double*>(mesh), n, w, p->guard, p->box_tab);
  }
  return hip_check(hipGetLastError(), "deposit");
}

}  // namespace pm
