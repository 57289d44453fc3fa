// Particle kernels: fill, CIC gather (plain and fused with kick and drift), the
// GR-minus-Newton displacement combination and the lattice step of the initial
// conditions.  One thread per particle; particles are in Lagrangian order, so
// neighbouring threads touch neighbouring cells, and blocks are mapped
// XCD-contiguous so each XCD's L2 sees a contiguous slab of the mesh.
#include <math.h>

#include "pm_particles.h"
#include "pm_plan.h"

namespace pm {

namespace {

constexpr int kBlock = 256;

inline unsigned nblocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// 16-byte stores over the 16-byte aligned body of p[0, count), element stores for the
// head and the tail.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill(T* __restrict__ p, int64_t count, T v) {
  constexpr int V = 16 / (int)sizeof(T);
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t to_align = (int64_t)((16u - (unsigned)(reinterpret_cast<uintptr_t>(p) & 15u)) & 15u) / (int64_t)sizeof(T);
  const int64_t head = to_align < count ? to_align : count;
  const int64_t nvec = (count - head) / V;
  for (int64_t i = tid; i < head; i += stride) p[i] = v;
  if constexpr (V == 4) {
    float4* q = reinterpret_cast<float4*>(p + head);
    const float4 w = make_float4(v, v, v, v);
    for (int64_t i = tid; i < nvec; i += stride) q[i] = w;
  } else {
    double2* q = reinterpret_cast<double2*>(p + head);
    const double2 w = make_double2(v, v);
    for (int64_t i = tid; i < nvec; i += stride) q[i] = w;
  }
  for (int64_t i = head + nvec * V + tid; i < count; i += stride) p[i] = v;
}

// sum over the 8 CIC corners of the three force components
// f: three meshes n3 = fstride elements apart
template <typename T>
__device__ __forceinline__ void cic_interp3(const T* __restrict__ f, int n, int64_t n3, T x, T y, T z, T& fx, T& fy,
                                            T& fz) {
  const Axis<T> ax = cic_axis(x, n), ay = cic_axis(y, n), az = cic_axis(z, n);
  const int64_t n2 = (int64_t)n * n;
  const int64_t r[4] = {ax.i0 * n2 + (int64_t)ay.i0 * n, ax.i0 * n2 + (int64_t)ay.i1 * n,
                        ax.i1 * n2 + (int64_t)ay.i0 * n, ax.i1 * n2 + (int64_t)ay.i1 * n};
  const T w[4] = {ax.w0 * ay.w0, ax.w0 * ay.w1, ax.w1 * ay.w0, ax.w1 * ay.w1};
  T sx = 0, sy = 0, sz = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int64_t a0 = r[c] + az.i0, a1 = r[c] + az.i1;
    const T w0 = w[c] * az.w0, w1 = w[c] * az.w1;
    sx += w0 * f[a0] + w1 * f[a1];
    sy += w0 * f[n3 + a0] + w1 * f[n3 + a1];
    sz += w0 * f[2 * n3 + a0] + w1 * f[2 * n3 + a1];
  }
  fx = sx;
  fy = sy;
  fz = sz;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_gather(const T* __restrict__ force, const T* __restrict__ pos, int64_t np,
                                                   int n, T* __restrict__ acc) {
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i = blk * kBlock + threadIdx.x;
  if (i >= np) return;
  T fx, fy, fz;
  cic_interp3(force, n, (int64_t)n * n * n, wrap(pos[i], n), wrap(pos[np + i], n), wrap(pos[2 * np + i], n), fx, fy,
              fz);
  acc[i] = fx;
  acc[np + i] = fy;
  acc[2 * np + i] = fz;
}

// Box blockIdx.y of a batch: particles [3][np] at pos/mom + 3 np box, force components
// fstride elements apart, box offset N^3.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_gather_kdk(const T* __restrict__ force, T* __restrict__ pos,
                                                       T* __restrict__ mom, int64_t np, int n, int64_t fstride, T kick,
                                                       T drift, const BoxEntry* __restrict__ tab) {
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i = blk * kBlock + threadIdx.x;
  if (i >= np) return;
  box_arrays(tab, np, pos, mom, kick, drift);
  force += (int64_t)blockIdx.y * n * n * n;
  T x = wrap(pos[i], n), y = wrap(pos[np + i], n), z = wrap(pos[2 * np + i], n);
  T fx, fy, fz;
  cic_interp3(force, n, fstride, x, y, z, fx, fy, fz);
  T px = mom[i] + kick * fx, py = mom[np + i] + kick * fy, pz = mom[2 * np + i] + kick * fz;
  mom[i] = px;
  mom[np + i] = py;
  mom[2 * np + i] = pz;
  pos[i] = wrap(x + drift * px, n);
  pos[np + i] = wrap(y + drift * py, n);
  pos[2 * np + i] = wrap(z + drift * pz, n);
}

// Gather + kick + drift for a full Lagrangian lattice run (np = N^3).  A workgroup
// owns a Lagrangian tile of GTX x GTY x GTZ particles, loads the three force meshes
// over the bounding box of the tile's CIC cells into LDS with row-contiguous loads
// (neighbouring tiles on the same XCD re-read overlapping rows from L2), and
// interpolates from LDS.  If the box exceeds the LDS capacity, fit_box's smaller box
// of the same proportions is staged and particles outside it read the meshes directly.
// Once the particles have moved apart (late, clustered cycles) most of the bounding
// box is cells no particle of the tile touches: a box of more than GSPARSE cells is
// staged sparsely -- the particles first mark their eight CIC cells in a byte map of
// the box, and only marked cells are loaded (the others are never read).
// Weights and arithmetic are those of k_gather_kdk.
constexpr int GTX = 4, GTY = 8, GTZ = 32;
constexpr int GPP = GTX * GTY * GTZ / kBlock;  // particles per thread
constexpr int GCAP = 4096;                     // staged cells (x3 components, float)
// the dense box of an undisplaced tile is (GTX + 1)(GTY + 1)(GTZ + 1) = 1485 cells
constexpr int GSPARSE = 2048;
static_assert(GCAP == 16 * kBlock, "the byte map is cleared with one 16-byte store per thread");

// DEPOSIT: after the drift, the tile's new positions are also deposited into `dens`
// (pre-filled with -1, box offset N^3) like the standalone tiled deposit -- an LDS
// window over the bounding box of their CIC cells, one global atomic per non-empty
// cell, global atomics for particles outside the window -- so the next cycle need not
// read the positions again.  The window reuses the force window's LDS as DCAP cells of
// 32-bit fixed point (to_fix_w_capped): half the LDS traffic of 64-bit cells and twice
// the cells; the window holds at most 2048 particles of capped terms, so a cell cannot
// wrap.
constexpr int DCAP = 3 * GCAP * (int)sizeof(float) / (int)sizeof(unsigned);
// Gather + kick + drift of one GTX x GTY x GTZ Lagrangian tile at `org` (block-wide):
// stages the three force meshes over the tile's CIC bounding box in `win`, updates
// (pos, mom) and leaves the drifted, wrapped positions in (x, y, z).  GUARD counts
// non-finite drifted positions in guard[0].
template <bool GUARD, bool P2>
__device__ __forceinline__ void gather_tile(const float* __restrict__ force, float* __restrict__ pos,
                                            float* __restrict__ mom, int n, int64_t fstride, float kick, float drift,
                                            const int (&org)[3], float* win, unsigned char* mark, int (*wlo)[3],
                                            int (*whi)[3], float (*wsum)[3], float (&x)[GPP], float (&y)[GPP],
                                            float (&z)[GPP], unsigned* __restrict__ guard) {
  const int64_t np = (int64_t)n * n * n, n2 = (int64_t)n * n;
  const int t = threadIdx.x;
  unsigned jj[GPP];
  float *const pos1 = pos + np, *const pos2 = pos + 2 * np, *const mom1 = mom + np, *const mom2 = mom + 2 * np;
  const float *const force1 = force + fstride, *const force2 = force + 2 * fstride;
  int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
  float sum[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int p = 0; p < GPP; ++p) {
    const int loc = t + kBlock * p;
    const int li = loc / (GTY * GTZ), lk = (loc / GTZ) % GTY, ll = loc % GTZ;
    jj[p] = node_index<P2>(org[0] + li, org[1] + lk, org[2] + ll, n);
    x[p] = ldg32(pos, jj[p]);
    y[p] = ldg32(pos1, jj[p]);
    z[p] = ldg32(pos2, jj[p]);
  }
  wrap_all<P2>(x, y, z, n);
#pragma unroll
  for (int p = 0; p < GPP; ++p) {
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
  reinterpret_cast<uint4*>(mark)[t] = make_uint4(0u, 0u, 0u, 0u);  // GCAP bytes, 16 per thread
  block_window(lo, hi, sum, GTX * GTY * GTZ, GCAP, wlo, whi, wsum, o, W);
  const int wtot = W[0] * W[1] * W[2];
  const int sy = W[2], sx = W[1] * W[2];
  // sparse box: mark the CIC cells of the particles inside it (plain byte stores into
  // the map cleared before block_window's barriers)
  const bool sparse = wtot > GSPARSE;  // the same in every thread
  if (sparse) {
#pragma unroll
    for (int p = 0; p < GPP; ++p) {
      const int rx = idiff_n<P2>((int)floorf(x[p]), org[0], n) - o[0];
      const int ry = idiff_n<P2>((int)floorf(y[p]), org[1], n) - o[1];
      const int rz = idiff_n<P2>((int)floorf(z[p]), org[2], n) - o[2];
      if (rx >= 0 && rx <= W[0] - 2 && ry >= 0 && ry <= W[1] - 2 && rz >= 0 && rz <= W[2] - 2) {
        unsigned char* m = mark + win_index(rx, ry, rz, sx, sy);
        m[0] = 1;
        m[1] = 1;
        m[sy] = 1;
        m[sy + 1] = 1;
        m[sx] = 1;
        m[sx + 1] = 1;
        m[sx + sy] = 1;
        m[sx + sy + 1] = 1;
      }
    }
    __syncthreads();
  }
  // the momenta are needed only after the window: start their loads now
  float mx[GPP], my[GPP], mz[GPP];
#pragma unroll
  for (int p = 0; p < GPP; ++p) {
    mx[p] = ldg32(mom, jj[p]);
    my[p] = ldg32(mom1, jj[p]);
    mz[p] = ldg32(mom2, jj[p]);
  }
  // stage the force window (row-contiguous along z): all of a thread's loads are
  // issued before its first LDS store, so they are in flight together
  // (cells a sparse box skips are stored as zeros; no particle reads them)
  float fa[GCAP / kBlock] = {}, fb[GCAP / kBlock] = {}, fc[GCAP / kBlock] = {};
  const WinDiv qsx(sx), qsy(sy);
#pragma unroll
  for (int k = 0; k < GCAP / kBlock; ++k) {
    const int c = t + kBlock * k;
    if (c < wtot && (!sparse || mark[c])) {
      int a, b, cz;
      win_cell(c, qsx, qsy, a, b, cz);
      const unsigned idx = node_index<P2>(fold_n<P2>(org[0] + o[0] + a, n), fold_n<P2>(org[1] + o[1] + b, n),
                                          fold_n<P2>(org[2] + o[2] + cz, n), n);
      fa[k] = ldg32(force, idx);
      fb[k] = ldg32(force1, idx);
      fc[k] = ldg32(force2, idx);
    }
  }
#pragma unroll
  for (int k = 0; k < GCAP / kBlock; ++k) {
    const int c = t + kBlock * k;
    if (c < wtot) {
      win[c] = fa[k];
      win[GCAP + c] = fb[k];
      win[2 * GCAP + c] = fc[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < GPP; ++p) {
    const Axis<float> ax = cic_axis_n<P2>(x[p], n), ay = cic_axis_n<P2>(y[p], n), az = cic_axis_n<P2>(z[p], n);
    const int rx = idiff_n<P2>(ax.i0, org[0], n) - o[0], ry = idiff_n<P2>(ay.i0, org[1], n) - o[1],
              rz = idiff_n<P2>(az.i0, org[2], n) - o[2];
    const float w[4] = {ax.w0 * ay.w0, ax.w0 * ay.w1, ax.w1 * ay.w0, ax.w1 * ay.w1};
    float fx = 0.f, fy = 0.f, fz = 0.f;
    if (rx >= 0 && rx <= W[0] - 2 && ry >= 0 && ry <= W[1] - 2 && rz >= 0 && rz <= W[2] - 2) {
      const int base = win_index(rx, ry, rz, sx, sy);
      const int r[4] = {base, base + sy, base + sx, base + sx + sy};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float w0 = w[c] * az.w0, w1 = w[c] * az.w1;
        fx += w0 * win[r[c]] + w1 * win[r[c] + 1];
        fy += w0 * win[GCAP + r[c]] + w1 * win[GCAP + r[c] + 1];
        fz += w0 * win[2 * GCAP + r[c]] + w1 * win[2 * GCAP + r[c] + 1];
      }
    } else {
      const int64_t r[4] = {ax.i0 * n2 + (int64_t)ay.i0 * n, ax.i0 * n2 + (int64_t)ay.i1 * n,
                            ax.i1 * n2 + (int64_t)ay.i0 * n, ax.i1 * n2 + (int64_t)ay.i1 * n};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int64_t a0 = r[c] + az.i0, a1 = r[c] + az.i1;
        const float w0 = w[c] * az.w0, w1 = w[c] * az.w1;
        fx += w0 * force[a0] + w1 * force[a1];
        fy += w0 * force[fstride + a0] + w1 * force[fstride + a1];
        fz += w0 * force[2 * fstride + a0] + w1 * force[2 * fstride + a1];
      }
    }
    const unsigned j = jj[p];
    const float px = mx[p] + kick * fx, py = my[p] + kick * fy, pz = mz[p] + kick * fz;
    stg32(mom, j, px);
    stg32(mom1, j, py);
    stg32(mom2, j, pz);
    const float ux = x[p] + drift * px, uy = y[p] + drift * py, uz = z[p] + drift * pz;
    if (GUARD && !(isfinite(ux) && isfinite(uy) && isfinite(uz))) atomicAdd(&guard[0], 1u);
    // the new positions replace the old ones in registers (used by the deposit below)
    x[p] = ux;
    y[p] = uy;
    z[p] = uz;
    wrap_one<P2>(x[p], y[p], z[p], n);
    stg32(pos, j, x[p]);
    stg32(pos1, j, y[p]);
    stg32(pos2, j, z[p]);
  }
}

// One workgroup per NT tiles adjacent along x (NT = 2 with DEPOSIT: their deposit
// windows are merged, so the halo they share is flushed once).
template <bool DEPOSIT, bool P2>
__global__ void __launch_bounds__(kBlock, 3) k_gather_kdk_tiled(const float* __restrict__ force, float* __restrict__ pos,
                                                             float* __restrict__ mom, int n, int64_t fstride,
                                                             float kick, float drift, float* __restrict__ dens,
                                                             float w_scale, unsigned* __restrict__ guard,
                                                             const BoxEntry* __restrict__ tab) {
  constexpr int NT = DEPOSIT ? 2 : 1;
  __shared__ __attribute__((aligned(16))) float win[3 * GCAP];
  __shared__ __attribute__((aligned(16))) unsigned char mark[GCAP];  // sparse staging map
  __shared__ int wlo[kBlock / 64][3], whi[kBlock / 64][3];
  __shared__ float wsum[kBlock / 64][3];
  const int64_t np = (int64_t)n * n * n, n2 = (int64_t)n * n;
  box_arrays(tab, np, pos, mom, kick, drift);  // box of the batch
  force += (int64_t)blockIdx.y * np;
  if (DEPOSIT) dens += (int64_t)blockIdx.y * np;
  const int tpy = n / GTY, tpz = n / GTZ;
  int ti, tk, tl;  // ti counts groups of NT tiles along x
  tile_coords(xcd_block(blockIdx.x, gridDim.x), n / (GTX * NT), tpy, tpz, ti, tk, tl);
  const int t = threadIdx.x;
  float x[NT * GPP], y[NT * GPP], z[NT * GPP];
#pragma unroll
  for (int sub = 0; sub < NT; ++sub) {
    const int orgs[3] = {(ti * NT + sub) * GTX, tk * GTY, tl * GTZ};
    float xs[GPP], ys[GPP], zs[GPP];
    if (sub > 0) __syncthreads();  // the previous tile is done with the window
    gather_tile<DEPOSIT, P2>(force, pos, mom, n, fstride, kick, drift, orgs, win, mark, wlo, whi, wsum, xs, ys, zs,
                             guard);
#pragma unroll
    for (int p = 0; p < GPP; ++p) {
      x[sub * GPP + p] = xs[p];
      y[sub * GPP + p] = ys[p];
      z[sub * GPP + p] = zs[p];
    }
  }
  if (!DEPOSIT) return;
  __syncthreads();  // every thread is done with the force window
  static_assert((double)NT * GTX * GTY * GTZ * (kFixW - 1.0f) < 4294967296.0, "a window cell could wrap");
  unsigned* dwin = reinterpret_cast<unsigned*>(win);
  const int org[3] = {ti * NT * GTX, tk * GTY, tl * GTZ};
  const TileWindow dw = tile_window<NT * GPP, P2>(x, y, z, n, org, DCAP, NT * GTX * GTY * GTZ, wlo, whi, wsum);
  const int D0 = dw.W[0], D1 = dw.W[1], D2 = dw.W[2];
  const int dtot = D0 * D1 * D2;
  for (int c = t; c < dtot; c += kBlock) dwin[c] = 0u;
  __syncthreads();
  const int dsy = D2, dsx = D1 * D2;
#pragma unroll
  for (int p = 0; p < NT * GPP; ++p) {
    const Axis<float> ax = cic_axis_n<P2>(x[p], n), ay = cic_axis_n<P2>(y[p], n), az = cic_axis_n<P2>(z[p], n);
    const int rx = idiff_n<P2>(ax.i0, org[0], n) - dw.o[0], ry = idiff_n<P2>(ay.i0, org[1], n) - dw.o[1],
              rz = idiff_n<P2>(az.i0, org[2], n) - dw.o[2];
    const float wxy00 = ax.w0 * ay.w0, wxy01 = ax.w0 * ay.w1;
    const float wxy10 = ax.w1 * ay.w0, wxy11 = ax.w1 * ay.w1;
    if (rx >= 0 && rx <= D0 - 2 && ry >= 0 && ry <= D1 - 2 && rz >= 0 && rz <= D2 - 2) {
      unsigned* w = dwin + win_index(rx, ry, rz, dsx, dsy);
      atomicAdd(w, to_fix_w_capped(wxy00 * az.w0));
      atomicAdd(w + 1, to_fix_w_capped(wxy00 * az.w1));
      atomicAdd(w + dsy, to_fix_w_capped(wxy01 * az.w0));
      atomicAdd(w + dsy + 1, to_fix_w_capped(wxy01 * az.w1));
      atomicAdd(w + dsx, to_fix_w_capped(wxy10 * az.w0));
      atomicAdd(w + dsx + 1, to_fix_w_capped(wxy10 * az.w1));
      atomicAdd(w + dsx + dsy, to_fix_w_capped(wxy11 * az.w0));
      atomicAdd(w + dsx + dsy + 1, to_fix_w_capped(wxy11 * az.w1));
    } else {
      const int64_t r00 = ax.i0 * n2 + (int64_t)ay.i0 * n, r01 = ax.i0 * n2 + (int64_t)ay.i1 * n;
      const int64_t r10 = ax.i1 * n2 + (int64_t)ay.i0 * n, r11 = ax.i1 * n2 + (int64_t)ay.i1 * n;
      atomic_add(dens + r00 + az.i0, wxy00 * az.w0 * w_scale);
      atomic_add(dens + r00 + az.i1, wxy00 * az.w1 * w_scale);
      atomic_add(dens + r01 + az.i0, wxy01 * az.w0 * w_scale);
      atomic_add(dens + r01 + az.i1, wxy01 * az.w1 * w_scale);
      atomic_add(dens + r10 + az.i0, wxy10 * az.w0 * w_scale);
      atomic_add(dens + r10 + az.i1, wxy10 * az.w1 * w_scale);
      atomic_add(dens + r11 + az.i0, wxy11 * az.w0 * w_scale);
      atomic_add(dens + r11 + az.i1, wxy11 * az.w1 * w_scale);
    }
  }
  __syncthreads();
  const double scale = (double)w_scale / (double)kFixW;  // in FP64: a float 1/S would bias the total mass
  const WinDiv qsx(dsx), qsy(dsy);
  for (int c = t; c < dtot; c += kBlock) {
    const unsigned v = dwin[c];
    if (v == 0u) continue;
    int a, b, cz;
    win_cell(c, qsx, qsy, a, b, cz);
    const unsigned idx = node_index<P2>(fold_n<P2>(org[0] + dw.o[0] + a, n), fold_n<P2>(org[1] + dw.o[1] + b, n),
                                        fold_n<P2>(org[2] + dw.o[2] + cz, n), n);
    atomic_add(dens + idx, (float)((double)v * scale));
  }
}

// eq. xiGR (minimum image, coarse cells) interpolated in Lagrangian coordinates to
// the fine lattice and added to the fine positions (eq. combined).
template <typename T>
__device__ __forceinline__ T min_image(T d, int n) {
  const T fn = T(n);
  const T s = d + T(0.5) * fn;
  return s - fn * floor(s / fn) - T(0.5) * fn;
}

// Coarse-lattice coordinate of fine particle j along one axis:
// u = ((2j+1) nc - nf) / (2 nf), base node i0 = floor(u) (in [-1, nc)), weight t = u - i0,
// from an integer floor division and its exact remainder.
template <typename T>
__device__ __forceinline__ int lagr_base(int j, int nc, int nf, T& t) {
  const int num = (2 * j + 1) * nc - nf;
  const int den = 2 * nf;
  const int q = num >= 0 ? num / den : -((-num + den - 1) / den);
  t = T(num - q * den) / T(den);
  return q;
}

// Block (x, y, z) of 256 threads handles the fine particles (z, G y + g, 256 x + t),
// g < G: runs along the fine z axis on G adjacent fine y-rows, whose CIC corners lie on
// two coarse x-rows times at most G + 1 coarse y-rows.  The block first stages xi =
// min-image (x_gr - x_newton) on those rows (the coarse cells its particles touch, zc
// cells per row) in LDS, then interpolates; the weights and the summation order are
// those of a direct per-particle evaluation.  G > 1 shares the staged rows between the
// fine rows and keeps 3 G fine loads per thread in flight during the staging.
constexpr int kCombineZ = kBlock + 4;  // staged coarse cells per row (nc <= nf)
// XI: xg already holds xi (coarse cells) and xn is unused.
template <typename T, bool XI, int G>
__global__ void __launch_bounds__(kBlock) k_combine(const T* __restrict__ xg, const T* __restrict__ xn, int nc,
                                                    const T* __restrict__ xf, int nf, T* __restrict__ out) {
  __shared__ T xs[3][2 * (G + 1)][kCombineZ];
  const int jx = blockIdx.z, jy0 = blockIdx.y * G, jz0 = blockIdx.x * kBlock;
  const int jz = jz0 + threadIdx.x;
  const int gy = nf - jy0 < G ? nf - jy0 : G;  // fine y-rows of this block (fewer in a ragged last group)
  auto wrap_c = [nc](int i) { return i < 0 ? i + nc : (i >= nc ? i - nc : i); };
  T tx, tdummy;
  const int qx = lagr_base(jx, nc, nf, tx);
  const int ix[2] = {wrap_c(qx), wrap_c(qx + 1)};
  const int qy0 = lagr_base(jy0, nc, nf, tdummy);
  const int ny = lagr_base(jy0 + gy - 1, nc, nf, tdummy) - qy0 + 2;  // staged coarse y-rows, <= G + 1
  const int zlo = lagr_base(jz0, nc, nf, tdummy);
  const int jlast = min(jz0 + kBlock, nf) - 1;
  const int zc = lagr_base(jlast, nc, nf, tdummy) - zlo + 2;  // <= 256 nc/nf + 2
  // the fine positions do not depend on the staging: load them first
  const int64_t npf = (int64_t)nf * nf * nf, npc = (int64_t)nc * nc * nc;
  const int jzc = jz < nf ? jz : nf - 1;
  T xfj[G][3];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int64_t j = ((int64_t)jx * nf + (g < gy ? jy0 + g : jy0)) * nf + jzc;
#pragma unroll
    for (int d = 0; d < 3; ++d) xfj[g][d] = xf[d * npf + j];
  }
  for (int e = threadIdx.x; e < 2 * ny * zc; e += kBlock) {
    const int r = e / zc, k = e - r * zc;  // staged row r = cx ny + (coarse y-row - qy0)
    const int cx = r / ny;
    const int64_t id = ((int64_t)ix[cx] * nc + wrap_c(qy0 + r - cx * ny)) * nc + wrap_c(zlo + k);
#pragma unroll
    for (int d = 0; d < 3; ++d)
      xs[d][r][k] = XI ? xg[d * npc + id] : min_image(xg[d * npc + id] - xn[d * npc + id], nc);
  }
  __syncthreads();
  if (jz >= nf) return;
  T tz;
  const int kz = lagr_base(jz, nc, nf, tz) - zlo;
  const T ratio = T(nf) / T(nc);
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if (g >= gy) break;
    const int jy = jy0 + g;
    T ty;
    const int ry = lagr_base(jy, nc, nf, ty) - qy0;
    const T t[3] = {tx, ty, tz};
    T xi[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int cx_ = (c >> 2) & 1, cy_ = (c >> 1) & 1, cz_ = c & 1;
      const T w = (cx_ ? t[0] : T(1) - t[0]) * (cy_ ? t[1] : T(1) - t[1]) * (cz_ ? t[2] : T(1) - t[2]);
#pragma unroll
      for (int d = 0; d < 3; ++d) xi[d] += w * xs[d][cx_ * ny + ry + cy_][kz + cz_];
    }
    const int64_t j = ((int64_t)jx * nf + jy) * nf + jz;
#pragma unroll
    for (int d = 0; d < 3; ++d) out[d * npf + j] = wrap(xfj[g][d] + ratio * xi[d], nf);
  }
}

// Lattice step of the initial conditions: pos = wrap(q + disp), mom = c * disp,
// q = (i, j, l) + 1/2 for particle (i N + j) N + l.
// Box blockIdx.y of a batch of gridDim.y: disp is [3][nbox][N^3], pos/mom [nbox][3][N^3].
template <typename T>
__global__ void __launch_bounds__(kBlock) k_ic_lattice(const T* __restrict__ disp, T* __restrict__ pos,
                                                       T* __restrict__ mom, int n, T mom_factor,
                                                       const BoxEntry* __restrict__ tab) {
  const int64_t np = (int64_t)n * n * n;
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= np) return;
  const int64_t dstride = (int64_t)gridDim.y * np;
  disp += (int64_t)blockIdx.y * np;
  T unused_kick = T(0), unused_drift = T(0);
  box_arrays(tab, np, pos, mom, unused_kick, unused_drift);
  const int q[3] = {(int)(j / ((int64_t)n * n)), (int)((j / n) % n), (int)(j % n)};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const T s = disp[d * dstride + j];
    pos[d * np + j] = wrap(T(q[d]) + T(0.5) + s, n);
    mom[d * np + j] = mom_factor * s;
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_lpt2_source(const T* __restrict__ h, T* __restrict__ s, int64_t n3,
                                                        int pass) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= n3) return;
  const double a = (double)h[j], b = (double)h[n3 + j], c = (double)h[2 * n3 + j];
  // FP64 products: S is a small difference of such products where the field is nearly planar
  if (pass == 0)
    s[j] = T(a * b + a * c + b * c);
  else
    s[j] = T((double)s[j] - (a * a + b * b + c * c));
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_ic_lattice2(const T* __restrict__ psi1, const T* psi2, T* __restrict__ pos,
                                                        T* mom, int n, T f1, T f2) {
  const int64_t np = (int64_t)n * n * n;
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= np) return;
  const int q[3] = {(int)(j / ((int64_t)n * n)), (int)((j / n) % n), (int)(j % n)};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const T s1 = psi1[d * np + j], s2 = psi2[d * np + j];   // psi2 may alias mom: read before the write
    pos[d * np + j] = wrap(T(q[d]) + T(0.5) + (s1 + s2), n);
    mom[d * np + j] = f1 * s1 + f2 * s2;
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_ic_gauge_lattice(const T* __restrict__ xi, const T* __restrict__ pn,
                                                             const T* __restrict__ mn, T* __restrict__ pg,
                                                             T* __restrict__ mg, int n, T mom_factor) {
  const int64_t np = (int64_t)n * n * n;
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= np) return;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const T s = xi[d * np + j];
    pg[d * np + j] = wrap(pn[d * np + j] + s, n);
    mg[d * np + j] = mn[d * np + j] + mom_factor * s;
  }
}

}  // namespace

int launch_fill(const pm_plan* p, void* mesh, int64_t count, double value, hipStream_t s) {
  ProfScope ps(p, PK_FILL, s);
  if (count <= 0) return PM_OK;
  // one 16-byte store per thread and pass (4 floats or 2 doubles)
  const int64_t vec = p->dtype == PM_F32 ? 4 : 2;
  const unsigned g = (unsigned)std::min<int64_t>((count + vec * kBlock - 1) / (vec * kBlock), 65536);
  if (p->dtype == PM_F32)
    hipLaunchKernelGGL(k_fill<float>, dim3(g), dim3(kBlock), 0, s, static_cast<float*>(mesh), count, (float)value);
  else
    hipLaunchKernelGGL(k_fill<double>, dim3(g), dim3(kBlock), 0, s, static_cast<double*>(mesh), count, value);
  return hip_check(hipGetLastError(), "fill");
}

int launch_gather(const pm_plan* p, const void* force, const void* pos, int64_t np, void* acc, hipStream_t s) {
  ProfScope ps(p, PK_GATHER, s);
  if (np <= 0) return PM_OK;
  if (p->dtype == PM_F32)
    hipLaunchKernelGGL(k_gather<float>, dim3(nblocks(np)), dim3(kBlock), 0, s, static_cast<const float*>(force),
                       static_cast<const float*>(pos), np, p->n, static_cast<float*>(acc));
  else
    hipLaunchKernelGGL(k_gather<double>, dim3(nblocks(np)), dim3(kBlock), 0, s, static_cast<const double*>(force),
                       static_cast<const double*>(pos), np, p->n, static_cast<double*>(acc));
  return hip_check(hipGetLastError(), "gather");
}

bool gather_kdk_can_deposit(const pm_plan* p, int64_t np) {
  const int n = p->n;
  return p->dtype == PM_F32 && (int64_t)n * n * n == np && n >= 64 && n <= 1024 && n % GTZ == 0;
}

int launch_gather_kdk(const pm_plan* p, const void* force, void* pos, void* mom, int64_t np, double kick,
                      double drift, void* dens, hipStream_t s) {
  ProfScope ps(p, dens ? PK_GATHER_KDK_DEPOSIT : PK_GATHER_KDK, s);
  if (np <= 0) return PM_OK;
  const int n = p->n;
  const int64_t fstride = (int64_t)p->nb * n * n * n;  // force meshes are [3][nb][N^3]
  if (dens && !gather_kdk_can_deposit(p, np)) return set_error(PM_ERR_ARG, "fused deposit needs a full FP32 lattice");
  if (gather_kdk_can_deposit(p, np)) {  // a full FP32 lattice, 64 <= N <= 1024
    const unsigned tiles = (unsigned)((n / GTX) * (n / GTY) * (n / GTZ));
    const float w = (float)((double)n * n * n / (double)np);  // 1 / nbar
    // a power-of-two N wraps without a division (same results)
    const bool p2 = (n & (n - 1)) == 0;
    const dim3 grid(dens ? tiles / 2 : tiles, (unsigned)p->nb);
    auto kern = dens ? (p2 ? k_gather_kdk_tiled<true, true> : k_gather_kdk_tiled<true, false>)
                     : (p2 ? k_gather_kdk_tiled<false, true> : k_gather_kdk_tiled<false, false>);
    hipLaunchKernelGGL(kern, grid, dim3(kBlock), 0, s, static_cast<const float*>(force), static_cast<float*>(pos),
                       static_cast<float*>(mom), n, fstride, (float)kick, (float)drift,
                       dens ? static_cast<float*>(dens) : nullptr, dens ? w : 0.f, dens ? p->guard : nullptr,
                       p->box_tab);
  } else if (p->dtype == PM_F32)
    hipLaunchKernelGGL(k_gather_kdk<float>, dim3(nblocks(np), (unsigned)p->nb), dim3(kBlock), 0, s,
                       static_cast<const float*>(force), static_cast<float*>(pos), static_cast<float*>(mom), np, p->n,
                       fstride, (float)kick, (float)drift, p->box_tab);
  else
    hipLaunchKernelGGL(k_gather_kdk<double>, dim3(nblocks(np), (unsigned)p->nb), dim3(kBlock), 0, s,
                       static_cast<const double*>(force), static_cast<double*>(pos), static_cast<double*>(mom), np, p->n,
                       fstride, kick, drift, p->box_tab);
  return hip_check(hipGetLastError(), "gather-kick-drift");
}

int launch_combine(const void* x_gr, const void* x_n, int nc, const void* x_f, int nf, int dtype, void* x_out,
                   hipStream_t s) {
  // x_n == nullptr: x_gr holds xi itself
  // FP32: four fine y-rows per block (31 KB of LDS); FP64: one (25 KB)
  constexpr int G4 = 4;
  const unsigned gz = (unsigned)((nf + kBlock - 1) / kBlock);
  if (dtype == PM_F32) {
    const dim3 grid(gz, (unsigned)((nf + G4 - 1) / G4), (unsigned)nf);
    auto kern = x_n ? k_combine<float, false, G4> : k_combine<float, true, G4>;
    hipLaunchKernelGGL(kern, grid, dim3(kBlock), 0, s, static_cast<const float*>(x_gr), static_cast<const float*>(x_n),
                       nc, static_cast<const float*>(x_f), nf, static_cast<float*>(x_out));
  } else {
    const dim3 grid(gz, (unsigned)nf, (unsigned)nf);
    auto kern = x_n ? k_combine<double, false, 1> : k_combine<double, true, 1>;
    hipLaunchKernelGGL(kern, grid, dim3(kBlock), 0, s, static_cast<const double*>(x_gr),
                       static_cast<const double*>(x_n), nc, static_cast<const double*>(x_f), nf,
                       static_cast<double*>(x_out));
  }
  return hip_check(hipGetLastError(), "displacement combine");
}

int launch_ic_lattice(const pm_plan* p, const void* disp, void* pos, void* mom, double mom_factor, hipStream_t s) {
  ProfScope ps(p, PK_IC, s);
  const int64_t np = (int64_t)p->n * p->n * p->n;
  const dim3 grid(nblocks(np), (unsigned)p->nb);
  if (p->dtype == PM_F32)
    hipLaunchKernelGGL(k_ic_lattice<float>, grid, dim3(kBlock), 0, s, static_cast<const float*>(disp),
                       static_cast<float*>(pos), static_cast<float*>(mom), p->n, (float)mom_factor, p->box_tab);
  else
    hipLaunchKernelGGL(k_ic_lattice<double>, grid, dim3(kBlock), 0, s, static_cast<const double*>(disp),
                       static_cast<double*>(pos), static_cast<double*>(mom), p->n, mom_factor, p->box_tab);
  return hip_check(hipGetLastError(), "ic lattice");
}

int launch_lpt2_source(const pm_plan* p, const void* h, void* s_out, int pass, hipStream_t s) {
  ProfScope ps(p, PK_IC, s);
  const int64_t n3 = (int64_t)p->n * p->n * p->n;
  if (p->dtype == PM_F32)
    hipLaunchKernelGGL(k_lpt2_source<float>, dim3(nblocks(n3)), dim3(kBlock), 0, s, static_cast<const float*>(h),
                       static_cast<float*>(s_out), n3, pass);
  else
    hipLaunchKernelGGL(k_lpt2_source<double>, dim3(nblocks(n3)), dim3(kBlock), 0, s, static_cast<const double*>(h),
                       static_cast<double*>(s_out), n3, pass);
  return hip_check(hipGetLastError(), "lpt2 source");
}

int launch_ic_lattice2(const pm_plan* p, const void* psi1, const void* psi2, void* pos, void* mom, double f1,
                       double f2, hipStream_t s) {
  ProfScope ps(p, PK_IC, s);
  const int64_t np = (int64_t)p->n * p->n * p->n;
  if (p->dtype == PM_F32)
    hipLaunchKernelGGL(k_ic_lattice2<float>, dim3(nblocks(np)), dim3(kBlock), 0, s, static_cast<const float*>(psi1),
                       static_cast<const float*>(psi2), static_cast<float*>(pos), static_cast<float*>(mom), p->n,
                       (float)f1, (float)f2);
  else
    hipLaunchKernelGGL(k_ic_lattice2<double>, dim3(nblocks(np)), dim3(kBlock), 0, s,
                       static_cast<const double*>(psi1), static_cast<const double*>(psi2), static_cast<double*>(pos),
                       static_cast<double*>(mom), p->n, f1, f2);
  return hip_check(hipGetLastError(), "ic lattice 2lpt");
}

int launch_ic_gauge_lattice(const pm_plan* p, const void* xi, const void* pos_n, const void* mom_n, void* pos_gr,
                            void* mom_gr, double mom_factor, hipStream_t s) {
  ProfScope ps(p, PK_IC, s);
  const int64_t np = (int64_t)p->n * p->n * p->n;
  if (p->dtype == PM_F32)
    hipLaunchKernelGGL(k_ic_gauge_lattice<float>, dim3(nblocks(np)), dim3(kBlock), 0, s, static_cast<const float*>(xi),
                       static_cast<const float*>(pos_n), static_cast<const float*>(mom_n),
                       static_cast<float*>(pos_gr), static_cast<float*>(mom_gr), p->n, (float)mom_factor);
  else
    hipLaunchKernelGGL(k_ic_gauge_lattice<double>, dim3(nblocks(np)), dim3(kBlock), 0, s,
                       static_cast<const double*>(xi), static_cast<const double*>(pos_n),
                       static_cast<const double*>(mom_n), static_cast<double*>(pos_gr), static_cast<double*>(mom_gr),
                       p->n, mom_factor);
  return hip_check(hipGetLastError(), "ic gauge lattice");
}

}  // namespace pm
