// Kernels of the reverse-mode (adjoint) PM step and of the initial-condition and
// power-spectrum adjoints.  The forward map of one cycle is
//   F(x) = gather_x( A deposit(x) ),  p' = p + K F(x),  x' = wrap(x + Dr p'),
// with A the linear mesh operator density -> force meshes (Green's function and
// gradient in Fourier space).  Given cotangents (lx', lp') of (x', p'):
//   lp = lp' + Dr lx',   v = K lp,
//   lx = lx' + sum_d v_d grad(F_d)(x)                       (force-field term)
//           + (1/nbar) grad_x( W * h )(x),  h = A^T deposit_v (density term)
// where deposit_v spreads each particle's v with the CIC weights (the adjoint of
// the gather) and grad_x(W * h) differentiates the CIC weights (the adjoint of the
// deposit).  CIC weight derivatives are the right derivatives at cell edges,
// consistent with the floor() in the assignment.  One thread per particle.
#include <math.h>

#include "fft_kernels.h"
#include "pm_particles.h"
#include "pm_plan.h"

namespace pm {

namespace {

constexpr int kBlock = 256;

inline unsigned nblocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Adjoint of gather + kick + drift: updates (lam_pos, lam_mom) by the force-field
// term and deposits v = kick (lam_mom + drift lam_pos) into g ([3][N^3], pre-zeroed).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_adj_gather_kdk(const T* __restrict__ force, const T* __restrict__ pos,
                                                           int64_t np, int n, T kick, T drift, T* __restrict__ lam_pos,
                                                           T* __restrict__ lam_mom, T* __restrict__ g) {
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i = blk * kBlock + threadIdx.x;
  if (i >= np) return;
  const int64_t n2 = (int64_t)n * n, n3 = n2 * n;
  const Axis<T> ax = cic_axis(wrap(pos[i], n), n), ay = cic_axis(wrap(pos[np + i], n), n),
                az = cic_axis(wrap(pos[2 * np + i], n), n);
  T lx[3], lp[3], v[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lx[d] = lam_pos[d * np + i];
    lp[d] = lam_mom[d * np + i] + drift * lx[d];
    v[d] = kick * lp[d];
  }
  T gx = 0, gy = 0, gz = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int bx = (c >> 2) & 1, by = (c >> 1) & 1, bz = c & 1;
    const int64_t idx = (bx ? ax.i1 : ax.i0) * n2 + (int64_t)(by ? ay.i1 : ay.i0) * n + (bz ? az.i1 : az.i0);
    const T wx = bx ? ax.w1 : ax.w0, wy = by ? ay.w1 : ay.w0, wz = bz ? az.w1 : az.w0;
    const T s = v[0] * force[idx] + v[1] * force[n3 + idx] + v[2] * force[2 * n3 + idx];
    // d/dx of the weight: -1 at the base node, +1 at the next one
    gx += (bx ? s : -s) * wy * wz;
    gy += (by ? s : -s) * wx * wz;
    gz += (bz ? s : -s) * wx * wy;
    const T w = wx * wy * wz;
    atomic_add(g + idx, w * v[0]);
    atomic_add(g + n3 + idx, w * v[1]);
    atomic_add(g + 2 * n3 + idx, w * v[2]);
  }
  lam_mom[i] = lp[0];
  lam_mom[np + i] = lp[1];
  lam_mom[2 * np + i] = lp[2];
  lam_pos[i] = lx[0] + gx;
  lam_pos[np + i] = lx[1] + gy;
  lam_pos[2 * np + i] = lx[2] + gz;
}

// Full-lattice (np = N^3, FP32) variant, one workgroup per Lagrangian tile of
// AX x AY x AZ particles.  The force-field term is computed with the three force
// meshes staged in LDS over the tile's CIC bounding box (as in the forward gather);
// then, with the positions still in registers, v = kick * lam_mom (the updated lam_mom)
// is deposited like the counting density: the same box becomes an LDS window of the
// three components in 32-bit fixed point with a per-tile, per-component scale
// 2^(20 - e_d) (e_d the exponent of the tile's largest |v_d|): every term is rounded to
// the nearest multiple of 2^(e_d - 20) (a relative 1e-6 of the tile's largest |v_d|)
// and no window cell can overflow, since the tile's 1024 particles add at most 2^30 in
// magnitude.  Then one global atomic per non-empty cell and component; particles
// outside the window (a box past ACAP cells, shrunk by fit_box) read the force meshes
// and deposit with global atomics directly.  g must not overlap force.
constexpr int AX = 4, AY = 8, AZ = 32;
constexpr int APP = AX * AY * AZ / kBlock;
constexpr int ACAP = 4096;
// a box of more than ASPARSE cells (the undisplaced tile's is 1485) stages only the
// cells its particles touch, marked in a byte map, as the forward gather does
constexpr int ASPARSE = 2048;
static_assert(ACAP == 16 * kBlock, "the byte map is cleared with one 16-byte store per thread");

template <bool P2>
__global__ void __launch_bounds__(kBlock) k_adj_gather_tiled(const float* __restrict__ force, const float* __restrict__ pos,
                                                             int n, float kick, float drift, float* __restrict__ lam_pos,
                                                             float* __restrict__ lam_mom, float* __restrict__ g) {
  static_assert(AX * AY * AZ <= 1024, "the fixed-point headroom assumes at most 2^10 particles per tile");
  __shared__ float win[3 * ACAP];
  __shared__ __attribute__((aligned(16))) unsigned char mark[ACAP];
  __shared__ int wlo[4][3], whi[4][3];
  __shared__ float wsum[4][3];
  __shared__ float wmax[4][3];
  const int64_t np = (int64_t)n * n * n, n2 = (int64_t)n * n;
  const int tpy = n / AY, tpz = n / AZ;
  int ti, tk, tl;
  tile_coords(xcd_block(blockIdx.x, gridDim.x), n / AX, tpy, tpz, ti, tk, tl);
  const int org[3] = {ti * AX, tk * AY, tl * AZ};
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  float x[APP], y[APP], z[APP];
  unsigned jj[APP];
#pragma unroll
  for (int p = 0; p < APP; ++p) {
    const int loc = t + kBlock * p;
    const int li = loc / (AY * AZ), lk = (loc / AZ) % AY, ll = loc % AZ;
    jj[p] = node_index<P2>(org[0] + li, org[1] + lk, org[2] + ll, n);
    x[p] = ldg32(pos, jj[p]);
    y[p] = ldg32(pos + np, jj[p]);
    z[p] = ldg32(pos + 2 * np, jj[p]);
  }
  wrap_all<P2>(x, y, z, n);
  reinterpret_cast<uint4*>(mark)[t] = make_uint4(0u, 0u, 0u, 0u);  // before tile_window's barriers
  const TileWindow tw = tile_window<APP, P2>(x, y, z, n, org, ACAP, AX * AY * AZ, wlo, whi, wsum);
  const int W0 = tw.W[0], W1 = tw.W[1], W2 = tw.W[2];
  const int sy = W2, sx = W1 * W2;
  const int wtot = W0 * W1 * W2;
  const bool sparse = wtot > ASPARSE;  // the same in every thread
  if (sparse) {
#pragma unroll
    for (int p = 0; p < APP; ++p) {
      const int rx = idiff_n<P2>((int)floorf(x[p]), org[0], n) - tw.o[0];
      const int ry = idiff_n<P2>((int)floorf(y[p]), org[1], n) - tw.o[1];
      const int rz = idiff_n<P2>((int)floorf(z[p]), org[2], n) - tw.o[2];
      if (rx >= 0 && rx <= W0 - 2 && ry >= 0 && ry <= W1 - 2 && rz >= 0 && rz <= W2 - 2) {
        unsigned char* m = mark + rx * sx + ry * sy + rz;
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
  // stage the window: all of a thread's loads in flight before its first LDS store
  // (cells a sparse box skips are stored as zeros; no particle reads them)
  float fa[ACAP / kBlock] = {}, fb[ACAP / kBlock] = {}, fc[ACAP / kBlock] = {};
  const WinDiv qsx(sx), qsy(sy);
#pragma unroll
  for (int k = 0; k < ACAP / kBlock; ++k) {
    const int c = t + kBlock * k;
    if (c < wtot && (!sparse || mark[c])) {
      int a, b, cz;
      win_cell(c, qsx, qsy, a, b, cz);
      const unsigned idx = node_index<P2>(fold_n<P2>(org[0] + tw.o[0] + a, n), fold_n<P2>(org[1] + tw.o[1] + b, n),
                                          fold_n<P2>(org[2] + tw.o[2] + cz, n), n);
      fa[k] = ldg32(force, idx);
      fb[k] = ldg32(force + np, idx);
      fc[k] = ldg32(force + 2 * np, idx);
    }
  }
#pragma unroll
  for (int k = 0; k < ACAP / kBlock; ++k) {
    const int c = t + kBlock * k;
    if (c < wtot) {
      win[c] = fa[k];
      win[ACAP + c] = fb[k];
      win[2 * ACAP + c] = fc[k];
    }
  }
  __syncthreads();
  float v[3][APP];
  float vmax[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int p = 0; p < APP; ++p) {
    const unsigned j = jj[p];
    float lx[3], lp[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lx[d] = ldg32(lam_pos + d * np, j);
      lp[d] = ldg32(lam_mom + d * np, j) + drift * lx[d];
      v[d][p] = kick * lp[d];
      vmax[d] = fmaxf(vmax[d], fabsf(v[d][p]));
    }
    const Axis<float> ax = cic_axis_n<P2>(x[p], n), ay = cic_axis_n<P2>(y[p], n), az = cic_axis_n<P2>(z[p], n);
    const int rx = idiff_n<P2>(ax.i0, org[0], n) - tw.o[0], ry = idiff_n<P2>(ay.i0, org[1], n) - tw.o[1],
              rz = idiff_n<P2>(az.i0, org[2], n) - tw.o[2];
    const bool inside = rx >= 0 && rx <= W0 - 2 && ry >= 0 && ry <= W1 - 2 && rz >= 0 && rz <= W2 - 2;
    float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int bx = (c >> 2) & 1, by = (c >> 1) & 1, bz = c & 1;
      float s;
      if (inside) {
        const int w = (rx + bx) * sx + (ry + by) * sy + rz + bz;
        s = v[0][p] * win[w] + v[1][p] * win[ACAP + w] + v[2][p] * win[2 * ACAP + w];
      } else {
        const int64_t idx = (bx ? ax.i1 : ax.i0) * n2 + (int64_t)(by ? ay.i1 : ay.i0) * n + (bz ? az.i1 : az.i0);
        s = v[0][p] * force[idx] + v[1][p] * force[np + idx] + v[2][p] * force[2 * np + idx];
      }
      const float wx = bx ? ax.w1 : ax.w0, wy = by ? ay.w1 : ay.w0, wz = bz ? az.w1 : az.w0;
      gx += (bx ? s : -s) * wy * wz;
      gy += (by ? s : -s) * wx * wz;
      gz += (bz ? s : -s) * wx * wy;
    }
    stg32(lam_mom, j, lp[0]);
    stg32(lam_mom + np, j, lp[1]);
    stg32(lam_mom + 2 * np, j, lp[2]);
    stg32(lam_pos, j, lx[0] + gx);
    stg32(lam_pos + np, j, lx[1] + gy);
    stg32(lam_pos + 2 * np, j, lx[2] + gz);
  }
  // deposit of v over the same box: the force window's LDS becomes the fixed-point window
#pragma unroll
  for (int d = 0; d < 3; ++d)
    for (int off = 32; off > 0; off >>= 1) vmax[d] = fmaxf(vmax[d], __shfl_xor(vmax[d], off, 64));
  if (lane == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) wmax[wave][d] = vmax[d];
  }
  __syncthreads();  // every thread is done with the force window
  unsigned* dwin = reinterpret_cast<unsigned*>(win);
#pragma unroll
  for (int d = 0; d < 3; ++d)
    for (int c = t; c < wtot; c += kBlock) dwin[d * ACAP + c] = 0u;
  __syncthreads();
  float scale[3], inv[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float m = fmaxf(fmaxf(wmax[0][d], wmax[1][d]), fmaxf(wmax[2][d], wmax[3][d]));
    int e = 0;
    (void)frexpf(m, &e);  // m < 2^e
    scale[d] = m > 0.f ? ldexpf(1.f, 20 - e) : 0.f;
    inv[d] = m > 0.f ? ldexpf(1.f, e - 20) : 0.f;
  }
#pragma unroll
  for (int p = 0; p < APP; ++p) {
    const Axis<float> ax = cic_axis_n<P2>(x[p], n), ay = cic_axis_n<P2>(y[p], n), az = cic_axis_n<P2>(z[p], n);
    const int rx = idiff_n<P2>(ax.i0, org[0], n) - tw.o[0], ry = idiff_n<P2>(ay.i0, org[1], n) - tw.o[1],
              rz = idiff_n<P2>(az.i0, org[2], n) - tw.o[2];
    const bool inside = rx >= 0 && rx <= W0 - 2 && ry >= 0 && ry <= W1 - 2 && rz >= 0 && rz <= W2 - 2;
    const float wxy[4] = {ax.w0 * ay.w0, ax.w0 * ay.w1, ax.w1 * ay.w0, ax.w1 * ay.w1};
    if (inside) {
      const int base = rx * sx + ry * sy + rz;
      const int off[4] = {0, sy, sx, sx + sy};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const float vs = v[d][p] * scale[d];  // |vs| < 2^20, exact power-of-two scaling
        unsigned* wd = dwin + d * ACAP + base;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          atomicAdd(wd + off[q], (unsigned)(int)rintf(wxy[q] * az.w0 * vs));
          atomicAdd(wd + off[q] + 1, (unsigned)(int)rintf(wxy[q] * az.w1 * vs));
        }
      }
    } else {
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int bx = (c >> 2) & 1, by = (c >> 1) & 1, bz = c & 1;
        const int64_t idx = (bx ? ax.i1 : ax.i0) * n2 + (int64_t)(by ? ay.i1 : ay.i0) * n + (bz ? az.i1 : az.i0);
        const float w = wxy[2 * bx + by] * (bz ? az.w1 : az.w0);
#pragma unroll
        for (int d = 0; d < 3; ++d) atomic_add(g + d * np + idx, w * v[d][p]);
      }
    }
  }
  __syncthreads();
  for (int c = t; c < wtot; c += kBlock) {
    const int q0 = (int)dwin[c], q1 = (int)dwin[ACAP + c], q2 = (int)dwin[2 * ACAP + c];
    if ((q0 | q1 | q2) == 0) continue;
    int a, b, cz;
    win_cell(c, qsx, qsy, a, b, cz);
    const unsigned idx = node_index<P2>(fold_n<P2>(org[0] + tw.o[0] + a, n), fold_n<P2>(org[1] + tw.o[1] + b, n),
                                        fold_n<P2>(org[2] + tw.o[2] + cz, n), n);
    if (q0) atomic_add(g + idx, (float)q0 * inv[0]);
    if (q1) atomic_add(g + np + idx, (float)q1 * inv[1]);
    if (q2) atomic_add(g + 2 * np + idx, (float)q2 * inv[2]);
  }
}

// lam_pos (+)= scale * grad_x sum_c W(x - c) h(c): the adjoint of the CIC deposit
// applied to a cotangent mesh h.
template <typename T, bool P2>
__global__ void __launch_bounds__(kBlock) k_grad_gather(const T* __restrict__ h, const T* __restrict__ pos, int64_t np,
                                                        int n, T scale, T* __restrict__ lam_pos, int accumulate) {
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i = blk * kBlock + threadIdx.x;
  if (i >= np) return;
  const int64_t n2 = (int64_t)n * n;
  const Axis<T> ax = cic_axis_n<P2>(wrap_n<P2>(pos[i], n), n), ay = cic_axis_n<P2>(wrap_n<P2>(pos[np + i], n), n),
                az = cic_axis_n<P2>(wrap_n<P2>(pos[2 * np + i], n), n);
  T gx = 0, gy = 0, gz = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int bx = (c >> 2) & 1, by = (c >> 1) & 1, bz = c & 1;
    const int64_t idx = (bx ? ax.i1 : ax.i0) * n2 + (int64_t)(by ? ay.i1 : ay.i0) * n + (bz ? az.i1 : az.i0);
    const T wx = bx ? ax.w1 : ax.w0, wy = by ? ay.w1 : ay.w0, wz = bz ? az.w1 : az.w0;
    const T s = h[idx];
    gx += (bx ? s : -s) * wy * wz;
    gy += (by ? s : -s) * wx * wz;
    gz += (bz ? s : -s) * wx * wy;
  }
  const T gs[3] = {scale * gx, scale * gy, scale * gz};
#pragma unroll
  for (int d = 0; d < 3; ++d) lam_pos[d * np + i] = accumulate ? lam_pos[d * np + i] + gs[d] : gs[d];
}

// Transposed Newtonian force operator on three spectra (natural [N][N][hp] layout):
// c0 <- coef / k^2 * sum_d conj(D_d(n)) c_d, zero at k = 0.  The forward operator
// multiplies by D_d coef / k^2 (coef = (3/2) Omega_m / N^3, which also carries the
// 1/N^3 of the inverse transform); its transpose multiplies by the conjugate.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_div_newton(cx<T>* __restrict__ c0, const cx<T>* __restrict__ c1,
                                                       const cx<T>* __restrict__ c2, int n, int hp, int grad, T coef) {
  const int64_t total = (int64_t)n * n * hp;
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= total) return;
  const int iz = (int)(idx % hp);
  if (iz > n / 2) return;
  const int iy = (int)((idx / hp) % n);
  const int ix = (int)(idx / ((int64_t)hp * n));
  const int nx = ix < n / 2 ? ix : ix - n, ny = iy < n / 2 ? iy : iy - n, nz = iz;
  const T kx = T(2.0 * kPi / n) * T(nx), ky = T(2.0 * kPi / n) * T(ny), kz = T(2.0 * kPi / n) * T(nz);
  const T k2s = kx * kx + ky * ky + kz * kz;
  cx<T> out = mk(T(0), T(0));
  if (nx != 0 || ny != 0 || nz != 0) {
    const cx<T> dx = conjg(grad_symbol<T>(nx, n, grad)), dy = conjg(grad_symbol<T>(ny, n, grad)),
                dz = conjg(grad_symbol<T>(nz, n, grad));
    const cx<T> s = dx * ldc(c0 + idx) + dy * ldc(c1 + idx) + dz * ldc(c2 + idx);
    out = scale(s, coef / k2s);
  }
  stc(c0 + idx, out);
}

// Cotangent of the Zel'dovich displacement from those of (pos, mom):
// lam_psi = lam_pos + mom_factor lam_mom.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_ic_lattice_adj(const T* __restrict__ lam_pos, const T* __restrict__ lam_mom,
                                                           T* __restrict__ lam_psi, int64_t count, T mom_factor) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= count) return;
  lam_psi[j] = lam_pos[j] + mom_factor * lam_mom[j];
}

// Adjoint of the second-order source S = sum_{i<j} (h_ii h_jj - h_ij^2) for a
// cotangent g of S: dS/dh_aa = sum_{b != a} h_bb, dS/dh_ab = -2 h_ab (a < b).  h holds
// [xx, yy, zz, xy, xz, yz] and is overwritten with the six cotangents g dS/dh.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_lpt2_source_adj(T* __restrict__ h, const T* __restrict__ g,
                                                            int64_t n3) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= n3) return;
  const double gj = (double)g[j];
  const double xx = (double)h[j], yy = (double)h[n3 + j], zz = (double)h[2 * n3 + j];
  h[j] = T(gj * (yy + zz));
  h[n3 + j] = T(gj * (xx + zz));
  h[2 * n3 + j] = T(gj * (xx + yy));
#pragma unroll
  for (int d = 3; d < 6; ++d) h[d * n3 + j] = T(-2.0 * gj * (double)h[d * n3 + j]);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_accumulate(T* __restrict__ y, const T* __restrict__ x, int64_t count) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j < count) y[j] += x[j];
}

}  // namespace

int launch_lpt2_source_adj(const pm_plan* p, void* h, const void* g, hipStream_t s) {
  ProfScope ps(p, PK_ADJ_SYMBOL, s);
  const int64_t n3 = (int64_t)p->n * p->n * p->n;
  if (p->dtype == PM_F32)
    hipLaunchKernelGGL(k_lpt2_source_adj<float>, dim3(nblocks(n3)), dim3(kBlock), 0, s, static_cast<float*>(h),
                       static_cast<const float*>(g), n3);
  else
    hipLaunchKernelGGL(k_lpt2_source_adj<double>, dim3(nblocks(n3)), dim3(kBlock), 0, s, static_cast<double*>(h),
                       static_cast<const double*>(g), n3);
  return hip_check(hipGetLastError(), "lpt2 source adjoint");
}

int launch_accumulate(const pm_plan* p, void* y, const void* x, int64_t count, hipStream_t s) {
  if (p->dtype == PM_F32)
    hipLaunchKernelGGL(k_accumulate<float>, dim3(nblocks(count)), dim3(kBlock), 0, s, static_cast<float*>(y),
                       static_cast<const float*>(x), count);
  else
    hipLaunchKernelGGL(k_accumulate<double>, dim3(nblocks(count)), dim3(kBlock), 0, s, static_cast<double*>(y),
                       static_cast<const double*>(x), count);
  return hip_check(hipGetLastError(), "accumulate");
}

int launch_adj_gather_kdk(const pm_plan* p, const void* force, const void* pos, int64_t np, double kick, double drift,
                          void* lam_pos, void* lam_mom, void* g, hipStream_t s) {
  if (np <= 0) return PM_OK;
  const int n = p->n;
  if (p->dtype == PM_F32 && (int64_t)n * n * n == np && n >= 64 && n <= 1024 && n % AZ == 0) {
    ProfScope ps(p, PK_ADJ_GATHER, s);
    const unsigned tiles = (unsigned)((n / AX) * (n / AY) * (n / AZ));
    // a power-of-two N wraps without a division (same results)
    auto kern = (n & (n - 1)) == 0 ? k_adj_gather_tiled<true> : k_adj_gather_tiled<false>;
    hipLaunchKernelGGL(kern, dim3(tiles), dim3(kBlock), 0, s, static_cast<const float*>(force),
                       static_cast<const float*>(pos), n, (float)kick, (float)drift, static_cast<float*>(lam_pos),
                       static_cast<float*>(lam_mom), static_cast<float*>(g));
    return hip_check(hipGetLastError(), "adjoint gather-kick-drift");
  }
  ProfScope ps(p, PK_ADJ_GATHER, s);
  if (p->dtype == PM_F32)
    hipLaunchKernelGGL(k_adj_gather_kdk<float>, dim3(nblocks(np)), dim3(kBlock), 0, s,
                       static_cast<const float*>(force), static_cast<const float*>(pos), np, p->n, (float)kick,
                       (float)drift, static_cast<float*>(lam_pos), static_cast<float*>(lam_mom),
                       static_cast<float*>(g));
  else
    hipLaunchKernelGGL(k_adj_gather_kdk<double>, dim3(nblocks(np)), dim3(kBlock), 0, s,
                       static_cast<const double*>(force), static_cast<const double*>(pos), np, p->n, kick, drift,
                       static_cast<double*>(lam_pos), static_cast<double*>(lam_mom), static_cast<double*>(g));
  return hip_check(hipGetLastError(), "adjoint gather-kick-drift");
}

int launch_grad_gather(const pm_plan* p, const void* h, const void* pos, int64_t np, double scale, void* lam_pos,
                       bool accumulate, hipStream_t s) {
  ProfScope ps(p, PK_GRAD_GATHER, s);
  if (np <= 0) return PM_OK;
  const bool p2 = (p->n & (p->n - 1)) == 0;  // a power-of-two N wraps without a division
  if (p->dtype == PM_F32) {
    auto kern = p2 ? k_grad_gather<float, true> : k_grad_gather<float, false>;
    hipLaunchKernelGGL(kern, dim3(nblocks(np)), dim3(kBlock), 0, s, static_cast<const float*>(h),
                       static_cast<const float*>(pos), np, p->n, (float)scale, static_cast<float*>(lam_pos),
                       accumulate ? 1 : 0);
  } else {
    auto kern = p2 ? k_grad_gather<double, true> : k_grad_gather<double, false>;
    hipLaunchKernelGGL(kern, dim3(nblocks(np)), dim3(kBlock), 0, s, static_cast<const double*>(h),
                       static_cast<const double*>(pos), np, p->n, scale, static_cast<double*>(lam_pos),
                       accumulate ? 1 : 0);
  }
  return hip_check(hipGetLastError(), "gradient gather");
}

int launch_div_newton(const pm_plan* p, int grad, double coef, hipStream_t s) {
  ProfScope ps(p, PK_ADJ_SYMBOL, s);
  const int n = p->n;
  const int64_t total = (int64_t)n * n * p->hp;
  const unsigned g = (unsigned)((total + kBlock - 1) / kBlock);
  if (p->dtype == PM_F32)
    hipLaunchKernelGGL(k_div_newton<float>, dim3(g), dim3(kBlock), 0, s, static_cast<cx<float>*>(cbuf(p, 0)),
                       static_cast<const cx<float>*>(cbuf(p, 1)), static_cast<const cx<float>*>(cbuf(p, 2)), n, p->hp,
                       grad, (float)coef);
  else
    hipLaunchKernelGGL(k_div_newton<double>, dim3(g), dim3(kBlock), 0, s, static_cast<cx<double>*>(cbuf(p, 0)),
                       static_cast<const cx<double>*>(cbuf(p, 1)), static_cast<const cx<double>*>(cbuf(p, 2)), n,
                       p->hp, grad, coef);
  return hip_check(hipGetLastError(), "adjoint force symbol");
}

int launch_ic_lattice_adj(const pm_plan* p, const void* lam_pos, const void* lam_mom, void* lam_psi,
                          double mom_factor, hipStream_t s) {
  ProfScope ps(p, PK_IC, s);
  const int64_t count = 3 * (int64_t)p->n * p->n * p->n;
  if (p->dtype == PM_F32)
    hipLaunchKernelGGL(k_ic_lattice_adj<float>, dim3(nblocks(count)), dim3(kBlock), 0, s,
                       static_cast<const float*>(lam_pos), static_cast<const float*>(lam_mom),
                       static_cast<float*>(lam_psi), count, (float)mom_factor);
  else
    hipLaunchKernelGGL(k_ic_lattice_adj<double>, dim3(nblocks(count)), dim3(kBlock), 0, s,
                       static_cast<const double*>(lam_pos), static_cast<const double*>(lam_mom),
                       static_cast<double*>(lam_psi), count, mom_factor);
  return hip_check(hipGetLastError(), "ic lattice adjoint");
}

}  // namespace pm
