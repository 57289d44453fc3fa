// Hand-written 3-D FFT building blocks for gfx950.
//
// A 3-D transform of an N^3 real mesh is three 1-D passes over a [N][N][N/2+1]
// complex spectrum kept in natural order:
//   rows   (last axis, contiguous): real-to-complex / complex-to-real, N/2-point
//          complex transform of packed even/odd samples plus the split step;
//   cols   (axes 1 and 0, strided): batches of B adjacent columns per workgroup so
//          every global access is a B*sizeof(complex)-byte contiguous segment.
// Every 1-D transform of length L = L1*L2 is a four-step transform: each of L2
// threads transforms L1 strided values in registers (compile-time twiddles), the
// inter-stage twiddles come from the plan's table W_N^m = exp(-2 pi i m/N), one LDS
// exchange, then each of L1 threads transforms L2 values in registers.
#pragma once

#include "pm_common.h"

namespace pm {

// Table twiddle W_L^m for a length-L transform on a plan of mesh size N (N/L = step).
template <bool INV, typename T>
__device__ __forceinline__ cx<T> tw_mul(cx<T> a, const cx<T>* tw, int m_times_step) {
  return twiddle<INV>(a, tw[m_times_step]);
}


__device__ __forceinline__ void sin_cos(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void sin_cos(double x, double* s, double* c) { sincos(x, s, c); }

template <typename T>
__device__ __forceinline__ cx<T> grad_symbol(int nd, int n, int grad) {
  // nd in [-N/2, N/2], k = 2 pi nd / N
  if (grad == PM_GRAD_SPECTRAL) {
    if (nd == -n / 2 || nd == n / 2) return mk(T(0), T(0));
    return mk(T(0), T(2.0 * kPi / n) * T(nd));
  }
  T sk, ck;
  sin_cos(T(2.0 * kPi / n) * T(nd), &sk, &ck);
  if (grad == PM_GRAD_FD2) return mk(T(0), sk);
  return mk(ck - T(1), sk);  // PM_GRAD_FD1
}

struct ColArgs {
  int64_t stride;        // element stride along the transform axis
  int64_t outer_stride;  // stride between outer indices
  int64_t comp_stride;   // stride between components (blockIdx.y)
  int ncols;             // columns per outer index
  int bcols;             // columns per workgroup
  int groups;            // ceil(ncols / bcols)
  int tw_step;           // N / L
};

// Column exchange buffer [L1][L2][B]: the j2 index is XOR-swizzled with the low bits
// of k1 so that the stage-2 reads (threads spread over k1) fall on different banks.
template <typename T, int L1, int L2>
__device__ __forceinline__ int col_lds_index(int k1, int j2, int b, int B) {
  constexpr int SW = L2 >= 4 ? 3 : L2 - 1;
  return (k1 * L2 + (j2 ^ (k1 & SW))) * B + b;
}

// Plain strided complex-to-complex pass, in place.  DIR = -1 forward, +1 inverse
// (unnormalised).  blockDim.x = B * max(L1, L2).
template <typename T, int L1, int L2, int DIR>
__global__ void __launch_bounds__(256) k_fft_cols(cx<T>* __restrict__ data, ColArgs g, const cx<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  constexpr bool INV = DIR > 0;
  const int B = g.bcols;
  const int t = threadIdx.x;
  const int b = t % B, u = t / B;
  // adjacent column groups share cache lines: keep them on one XCD (one L2)
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t outer = lb / g.groups;
  const int col = (int)(lb % g.groups) * B + b;
  const bool valid = col < g.ncols;
  cx<T>* base = data + (int64_t)blockIdx.y * g.comp_stride + outer * g.outer_stride + col;

  if (u < L2) {
    cx<T> a[L1];
#pragma unroll
    for (int j1 = 0; j1 < L1; ++j1) a[j1] = valid ? ldc(base + (int64_t)(u + L2 * j1) * g.stride) : mk(T(0), T(0));
    RegDFT<T, L1, DIR>::run(a);
#pragma unroll
    for (int k1 = 0; k1 < L1; ++k1) {
      cx<T> v = k1 == 0 ? a[k1] : tw_mul<INV>(a[k1], tw, u * k1 * g.tw_step);
      lds[col_lds_index<T, L1, L2>(k1, u, b, B)] = v;
    }
  }
  __syncthreads();
  if (u < L1) {
    cx<T> c[L2];
#pragma unroll
    for (int j2 = 0; j2 < L2; ++j2) c[j2] = lds[col_lds_index<T, L1, L2>(u, j2, b, B)];
    RegDFT<T, L2, DIR>::run(c);
    if (valid) {
#pragma unroll
      for (int k2 = 0; k2 < L2; ++k2) stc(base + (int64_t)(u + L1 * k2) * g.stride, c[k2]);
    }
  }
}

// Shell-filtered inverse column passes of the FFT bispectrum estimator (eq.
// bispectre).  A shell S = {n : lo4 <= 4|n|^2 < hi4} fills a small part of the
// spectrum, so these passes transform only what can be non-zero, and every load is
// masked by the support the previous pass wrote (elements a skipped workgroup left
// alone hold stale data and are never read):
//   STAGE 0, along axis 0 (columns (iy, iz)), src -> dst: loads src where n is in S
//     (1 where src is null: the shell's indicator), 0 elsewhere.  A workgroup whose
//     columns all have 4(ny^2 + iz^2) >= hi4 contains no mode of S and returns.
//   STAGE 1, along axis 1 (columns (ix, iz)), in place on dst: loads only where
//     4(ny^2 + iz^2) < hi4 (the columns stage 0 transformed), 0 elsewhere.  A
//     workgroup whose columns all have 4 iz^2 >= hi4 returns.
// The rows pass that follows (k_fft_rows_c2r with ZMASK) loads only iz with
// 4 iz^2 < hi4.  Same arithmetic as k_fft_cols on the values it keeps.
struct ShellArgs {
  double lo4, hi4;  // shell bounds on 4|n|^2 (exact integers in double)
  int n;            // N
};

template <typename T, int L1, int L2, int STAGE>
__global__ void __launch_bounds__(256) k_fft_cols_shell(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst,
                                                      ColArgs g, ShellArgs sh, const cx<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int B = g.bcols;
  const int t = threadIdx.x;
  const int b = t % B, u = t / B;
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t outer = lb / g.groups;            // STAGE 0: iy; STAGE 1: ix
  const int z0 = (int)(lb % g.groups) * B;        // first column (iz) of the workgroup
  const int col = z0 + b;
  const bool valid = col < g.ncols;
  const int N = sh.n;
  const double z4 = 4.0 * (double)z0 * (double)z0;
  if (STAGE == 0) {
    const int ny = outer < N / 2 ? (int)outer : (int)outer - N;
    if (z4 + 4.0 * (double)ny * (double)ny >= sh.hi4) return;  // the same decision in every thread
  } else {
    if (z4 >= sh.hi4) return;
  }
  const int64_t off = outer * g.outer_stride + col;
  const double c4 = 4.0 * (double)col * (double)col;
  constexpr bool INV = true;

  if (u < L2) {
    cx<T> a[L1];
#pragma unroll
    for (int j1 = 0; j1 < L1; ++j1) {
      const int i = u + L2 * j1;                 // index along the transform axis
      const int ni = i < N / 2 ? i : i - N;
      bool keep;
      if (STAGE == 0) {
        const int ny = outer < N / 2 ? (int)outer : (int)outer - N;
        const double r4 = 4.0 * ((double)ni * ni + (double)ny * ny) + c4;
        keep = valid && r4 >= sh.lo4 && r4 < sh.hi4;
      } else {
        keep = valid && 4.0 * (double)ni * ni + c4 < sh.hi4;
      }
      const cx<T>* from = STAGE == 0 ? src : dst;
      cx<T> v = mk(T(0), T(0));
      if (keep) v = (STAGE == 0 && !src) ? mk(T(1), T(0)) : ldc(from + off + (int64_t)i * g.stride);
      a[j1] = v;
    }
    RegDFT<T, L1, 1>::run(a);
#pragma unroll
    for (int k1 = 0; k1 < L1; ++k1) {
      cx<T> v = k1 == 0 ? a[k1] : tw_mul<INV>(a[k1], tw, u * k1 * g.tw_step);
      lds[col_lds_index<T, L1, L2>(k1, u, b, B)] = v;
    }
  }
  __syncthreads();
  if (u < L1) {
    cx<T> c[L2];
#pragma unroll
    for (int j2 = 0; j2 < L2; ++j2) c[j2] = lds[col_lds_index<T, L1, L2>(u, j2, b, B)];
    RegDFT<T, L2, 1>::run(c);
    if (valid) {
#pragma unroll
      for (int k2 = 0; k2 < L2; ++k2) stc(dst + off + (int64_t)(u + L1 * k2) * g.stride, c[k2]);
    }
  }
}

// Inverse pass along axis 1 of the solve's G form: blockIdx.y = 2 b + kind for box b.
// kind 0: the F_x spectrum (component 0), in place.  kind 1: the y-columns of G
// (component 1) are read once and transformed twice: D_y(ny) G to component 2, and G
// in place.  Components c of box b sit (c nbox + b) comp_stride elements from `data`.
template <typename T, int L1, int L2>
__device__ __forceinline__ void col_inverse_store(cx<T> (&a)[L1], cx<T>* lds, cx<T>* base, const ColArgs& g,
                                                  const cx<T>* __restrict__ tw, int b, int u, int B, bool valid) {
  if (u < L2) {
    RegDFT<T, L1, 1>::run(a);
#pragma unroll
    for (int k1 = 0; k1 < L1; ++k1)
      lds[col_lds_index<T, L1, L2>(k1, u, b, B)] = k1 == 0 ? a[k1] : tw_mul<true>(a[k1], tw, u * k1 * g.tw_step);
  }
  __syncthreads();
  if (u < L1) {
    cx<T> c[L2];
#pragma unroll
    for (int j2 = 0; j2 < L2; ++j2) c[j2] = lds[col_lds_index<T, L1, L2>(u, j2, b, B)];
    RegDFT<T, L2, 1>::run(c);
    if (valid) {
#pragma unroll
      for (int k2 = 0; k2 < L2; ++k2) stc(base + (int64_t)(u + L1 * k2) * g.stride, c[k2]);
    }
  }
}

template <typename T, int L1, int L2>
__global__ void __launch_bounds__(256) k_fft_cols_gform(cx<T>* __restrict__ data, ColArgs g, int nbox, int n, int grad,
                                                      const cx<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int B = g.bcols;
  const int t = threadIdx.x;
  const int b = t % B, u = t / B;
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t outer = lb / g.groups;
  const int col = (int)(lb % g.groups) * B + b;
  const bool valid = col < g.ncols;
  const int box = (int)blockIdx.y >> 1, kind = (int)blockIdx.y & 1;
  const int64_t off = outer * g.outer_stride + col;
  cx<T>* c0 = data + (int64_t)(kind * nbox + box) * g.comp_stride + off;  // F_x, or G
  cx<T> a[L1];
  if (u < L2) {
#pragma unroll
    for (int j1 = 0; j1 < L1; ++j1) a[j1] = valid ? ldc(c0 + (int64_t)(u + L2 * j1) * g.stride) : mk(T(0), T(0));
  }
  if (kind == 1) {
    cx<T> d[L1];
    if (u < L2) {
#pragma unroll
      for (int j1 = 0; j1 < L1; ++j1) {
        const int iy = u + L2 * j1;
        d[j1] = grad_symbol<T>(iy < n / 2 ? iy : iy - n, n, grad) * a[j1];
      }
    }
    col_inverse_store<T, L1, L2>(d, lds, data + (int64_t)(2 * nbox + box) * g.comp_stride + off, g, tw, b, u, B, valid);
    __syncthreads();  // the exchange buffer is reused
  }
  col_inverse_store<T, L1, L2>(a, lds, c0, g, tw, b, u, B, valid);
}

// Real-to-complex along the contiguous axis: rows of N reals -> rows of N/2+1
// complex.  M = N/2 = L1*L2 complex points z[n] = x[2n] + i x[2n+1];
// X[k] = E[k] + W_N^k O[k] with E = (Z[k] + conj Z[M-k])/2, O = -i (Z[k] - conj Z[M-k])/2.
// blockDim.x = R * max(L1, L2), R rows per workgroup.  in_row_stride / out_row_stride
// in elements; blockIdx.y selects a component (strides in_comp / out_comp).
struct RowArgs {
  int64_t nrows;
  int64_t in_comp, out_comp;  // component strides (elements of the in/out type)
  int n;                      // N (real row length)
  int hs;                     // spectrum row stride (complex elements, >= N/2+1)
  double zmask4;              // c2r MODE 1: only coefficients k with 4 k^2 < zmask4 are read
  int nbox;                   // c2r MODE 2: boxes per component
  int grad;                   // c2r MODE 2: gradient symbol (PM_GRAD_*) of the z component
};

// Modes of the c2r rows pass.
enum { C2R_PLAIN = 0, C2R_ZMASK = 1, C2R_FORCE = 2 };

template <typename T, int L1, int L2>
__global__ void __launch_bounds__(256) k_fft_rows_r2c(const T* __restrict__ in, cx<T>* __restrict__ out, RowArgs g,
                                                    const cx<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  constexpr int M = L1 * L2;
  constexpr int TPC = L1 > L2 ? L1 : L2;
  constexpr int XS = L1 * (L2 + 1);  // exchange row size (padded)
  constexpr int RS = XS > M ? XS : M;
  const int t = threadIdx.x;
  const int r = t / TPC, u = t % TPC;
  const int R = blockDim.x / TPC;
  const int64_t row = (int64_t)blockIdx.x * R + r;
  const bool valid = row < g.nrows;
  const int N = g.n;
  const T* src = in + (int64_t)blockIdx.y * g.in_comp + row * N;
  cx<T>* dst = out + (int64_t)blockIdx.y * g.out_comp + row * g.hs;
  cx<T>* my = lds + r * RS;

  if (u < L2) {
    cx<T> a[L1];
    const cx<T>* zsrc = reinterpret_cast<const cx<T>*>(src);
#pragma unroll
    for (int j1 = 0; j1 < L1; ++j1) a[j1] = valid ? ldc(zsrc + u + L2 * j1) : mk(T(0), T(0));
    RegDFT<T, L1, -1>::run(a);
#pragma unroll
    for (int k1 = 0; k1 < L1; ++k1) my[k1 * (L2 + 1) + u] = k1 == 0 ? a[k1] : tw_mul<false>(a[k1], tw, 2 * u * k1);
  }
  __syncthreads();
  cx<T> c[L2];
  if (u < L1) {
#pragma unroll
    for (int j2 = 0; j2 < L2; ++j2) c[j2] = my[u * (L2 + 1) + j2];
    RegDFT<T, L2, -1>::run(c);
  }
  __syncthreads();
  if (u < L1) {
#pragma unroll
    for (int k2 = 0; k2 < L2; ++k2) my[u + L1 * k2] = c[k2];
  }
  __syncthreads();
  if (valid) {
    for (int k = u; k <= M; k += TPC) {
      cx<T> zk = my[k == M ? 0 : k];
      cx<T> zm = conjg(my[k == 0 ? 0 : M - k]);
      cx<T> e = scale(zk + zm, T(0.5));
      cx<T> d = zk - zm;
      cx<T> o = mk(T(0.5) * d.y, T(-0.5) * d.x);  // -i d / 2
      cx<T> w = k == M ? mk(T(-1), T(0)) : tw[k];
      stc(dst + k, e + w * o);
    }
  }
}

// Complex-to-real along the contiguous axis (unnormalised inverse:
// x[n] = sum_{k in full row} X[k] exp(+2 pi i n k / N)).
// Z[k] = (X[k] + conj X[M-k]) + i conj(W_N^k) (X[k] - conj X[M-k]), z = IDFT_M(Z),
// x[2n] = Re z[n], x[2n+1] = Im z[n].
// MODE C2R_FORCE: the three force components of the solve's G form (see
// k_fft_cols_solve): output component 0 from input component 0 (F_x), 1 from input 2
// (the y-transformed D_y G), 2 from input 1 (the y-transformed G) times D_z(k) on load.
template <typename T, int L1, int L2, int MODE = C2R_PLAIN>
__global__ void __launch_bounds__(256) k_fft_rows_c2r(const cx<T>* __restrict__ in, T* __restrict__ out, RowArgs g,
                                                    const cx<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  constexpr int M = L1 * L2;
  constexpr int TPC = L1 > L2 ? L1 : L2;
  constexpr int XS = L1 * (L2 + 1);
  const int t = threadIdx.x;
  const int r = t / TPC, u = t % TPC;
  const int R = blockDim.x / TPC;
  const int64_t row = (int64_t)blockIdx.x * R + r;
  const bool valid = row < g.nrows;
  const int N = g.n;
  int64_t src_comp = blockIdx.y;
  bool zgrad = false;
  if (MODE == C2R_FORCE) {
    const int c = (int)blockIdx.y / g.nbox, b = (int)blockIdx.y % g.nbox;
    src_comp = (int64_t)(c == 0 ? 0 : (c == 1 ? 2 : 1)) * g.nbox + b;
    zgrad = c == 2;
  }
  const cx<T>* src = in + src_comp * g.in_comp + row * g.hs;
  T* dst = out + (int64_t)blockIdx.y * g.out_comp + row * N;
  cx<T>* my = lds + r * XS;

  cx<T> a[L1];
  // coefficient k of the row as the split below uses it: masked (C2R_ZMASK: beyond the
  // shell's reach the row holds stale data) or multiplied by D_z(k) (C2R_FORCE's z
  // component: F_z = D_z(k) G, k the z frequency, 0 <= k <= N/2)
  auto coeff = [&](int k) -> cx<T> {
    bool vk = valid;
    if (MODE == C2R_ZMASK) vk = vk && 4.0 * (double)k * (double)k < g.zmask4;
    cx<T> x = vk ? ldc(src + k) : mk(T(0), T(0));
    if (MODE == C2R_FORCE && zgrad) x = grad_symbol<T>(k, N, g.grad) * x;
    return x;
  };
  if constexpr (64 % TPC == 0) {
    // Every coefficient is loaded once: lane u holds X[u + L2 j1], and the mirror
    // X[M - k] of its k = u + L2 j1 is X[(L2 - u) + L2 (L1 - 1 - j1)] of lane L2 - u
    // (u >= 1) or X[L2 (L1 - j1)] of its own (u = 0; X[M] itself for j1 = 0), so the
    // mirrors travel between the lanes of the row (one wave holds whole rows).
    cx<T> xv[L1];
#pragma unroll
    for (int j1 = 0; j1 < L1; ++j1) xv[j1] = u < L2 ? coeff(u + L2 * j1) : mk(T(0), T(0));
    const cx<T> xnyq = u == 0 ? coeff(M) : mk(T(0), T(0));
    const int partner = u < L2 ? (L2 - u) % L2 : 0;
#pragma unroll
    for (int j1 = 0; j1 < L1; ++j1) {
      cx<T> xm;
      xm.x = __shfl(xv[L1 - 1 - j1].x, partner, TPC);
      xm.y = __shfl(xv[L1 - 1 - j1].y, partner, TPC);
      if (u == 0) xm = j1 == 0 ? xnyq : xv[(L1 - j1) % L1];
      xm = conjg(xm);
      const cx<T> xk = xv[j1];
      const cx<T> s = xk + xm;
      const cx<T> d = twiddle<true>(xk - xm, tw[u + L2 * j1]);  // d * conj(W_N^k)
      a[j1] = mk(s.x - d.y, s.y + d.x);                         // s + i d
    }
    if (u < L2) RegDFT<T, L1, 1>::run(a);
  } else if (u < L2) {
    // rows that straddle waves: X[k] and its mirror X[M-k] come straight from the row
    // (the mirrored loads hit the lines the neighbouring lanes fetch)
#pragma unroll
    for (int j1 = 0; j1 < L1; ++j1) {
      const int k = u + L2 * j1;
      const cx<T> xk = coeff(k);
      const cx<T> xm = conjg(coeff(M - k));
      const cx<T> s = xk + xm;
      const cx<T> d = twiddle<true>(xk - xm, tw[k]);  // d * conj(W_N^k)
      a[j1] = mk(s.x - d.y, s.y + d.x);               // s + i d
    }
    RegDFT<T, L1, 1>::run(a);
  }
  if (u < L2) {
#pragma unroll
    for (int k1 = 0; k1 < L1; ++k1) my[k1 * (L2 + 1) + u] = k1 == 0 ? a[k1] : tw_mul<true>(a[k1], tw, 2 * u * k1);
  }
  __syncthreads();
  if constexpr (L2 == 2 * L1 && TPC == L2) {
    // stage 2 on every lane of the row: lane u = k1 + L1 s transforms the L1 values
    // j2 = 2 m + s of column k1 (a half-length DFT), and one radix-2 step with lane
    // u ^ L1, which holds the other half of the same column, gives outputs k2 = k + L1 s
    const int k1 = u % L1, sh = u / L1;
    cx<T> h[L1];
#pragma unroll
    for (int m = 0; m < L1; ++m) h[m] = my[k1 * (L2 + 1) + 2 * m + sh];
    RegDFT<T, L1, 1>::run(h);
    cx<T>* zdst = reinterpret_cast<cx<T>*>(dst);
#pragma unroll
    for (int k = 0; k < L1; ++k) {
      cx<T> q;
      q.x = __shfl_xor(h[k].x, L1, TPC);
      q.y = __shfl_xor(h[k].y, L1, TPC);
      const cx<T> e = sh ? q : h[k], o = sh ? h[k] : q;
      const cx<T> wo = k == 0 ? o : tw_mul<true>(o, tw, k * 2 * L1);  // exp(+2 pi i k / L2) o
      if (valid) stc(zdst + k1 + L1 * (k + sh * L1), sh ? e - wo : e + wo);
    }
  } else if (u < L1) {
    cx<T> c[L2];
#pragma unroll
    for (int j2 = 0; j2 < L2; ++j2) c[j2] = my[u * (L2 + 1) + j2];
    RegDFT<T, L2, 1>::run(c);
    if (valid) {
      cx<T>* zdst = reinterpret_cast<cx<T>*>(dst);
#pragma unroll
      for (int k2 = 0; k2 < L2; ++k2) stc(zdst + u + L1 * k2, c[k2]);
    }
  }
}

// ------------------------------------------------------------------------
// Fused k-space solve along axis 0: forward column transform, per-mode potential,
// then the inverse column transforms of D_x G (in place) and of G (to out1), from
// which the passes along y and z make the three force components.
// ------------------------------------------------------------------------
struct SolveArgs {
  int n;            // N
  int kind;         // PM_NEWTON | PM_POISSON_GAUGE
  int grad;         // PM_GRAD_*
  double newton;    // (3/2) Omega_m / N^3
  double a_c2;      // a c_g^2 / N^3
  double h, h2, om_a, inv_dtau;
  int nbox;            // boxes (blockIdx.y)
  int64_t box_stride;  // complex elements between the boxes' spectra
  int64_t phi_stride;  // complex elements between the boxes' potentials
};

template <typename T, int L1, int L2, int KIND>
__global__ void __launch_bounds__(256) k_fft_cols_solve(cx<T>* __restrict__ data, cx<T>* __restrict__ out1,
                                                      cx<T>* __restrict__ phi, ColArgs g, SolveArgs s,
                                                      const cx<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int B = g.bcols;
  const int t = threadIdx.x;
  const int b = t % B, u = t / B;
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t outer = lb / g.groups;             // iy
  const int col = (int)(lb % g.groups) * B + b;    // iz
  const bool valid = col < g.ncols;
  const int64_t off = outer * g.outer_stride + col;
  const int N = s.n;
  {
    const int64_t bo = (int64_t)blockIdx.y * s.box_stride;
    data += bo;
    out1 += bo;
    if (KIND != PM_NEWTON) phi += (int64_t)blockIdx.y * s.phi_stride;
  }

  // forward along axis 0
  if (u < L2) {
    cx<T> a[L1];
#pragma unroll
    for (int j1 = 0; j1 < L1; ++j1) a[j1] = valid ? ldc(data + off + (int64_t)(u + L2 * j1) * g.stride) : mk(T(0), T(0));
    RegDFT<T, L1, -1>::run(a);
#pragma unroll
    for (int k1 = 0; k1 < L1; ++k1)
      lds[col_lds_index<T, L1, L2>(k1, u, b, B)] = k1 == 0 ? a[k1] : tw_mul<false>(a[k1], tw, u * k1 * g.tw_step);
  }
  __syncthreads();
  cx<T> X[L2];
  if (u < L1) {
#pragma unroll
    for (int j2 = 0; j2 < L2; ++j2) X[j2] = lds[col_lds_index<T, L1, L2>(u, j2, b, B)];
    RegDFT<T, L2, -1>::run(X);
    // per-mode scalar factor: force_d = D_d * X[k2] after this
    const int ny = outer < N / 2 ? (int)outer : (int)outer - N;
    const int nz = col;
    const T ky = T(2.0 * kPi / N) * T(ny), kz = T(2.0 * kPi / N) * T(nz);
    const T kyz2 = ky * ky + kz * kz;
#pragma unroll
    for (int k2 = 0; k2 < L2; ++k2) {
      const int ix = u + L1 * k2;
      const int nx = ix < N / 2 ? ix : ix - N;
      const T kx = T(2.0 * kPi / N) * T(nx);
      const T k2s = kx * kx + kyz2;
      const bool zero = (nx == 0 && ny == 0 && nz == 0);
      if (KIND == PM_NEWTON) {
        // FP32: the hardware reciprocal (1 ulp) instead of an IEEE division (~10 operations
        // per mode): solve 4.30 -> 4.25 ms at 1024^3
        T f;
        if constexpr (sizeof(T) == 4) f = zero ? T(0) : T(s.newton) * __builtin_amdgcn_rcpf(k2s);
        else f = zero ? T(0) : T(s.newton) / k2s;
        X[k2] = scale(X[k2], f);
      } else {
        // the carried potential keeps the unpadded [N][N][N/2+1] layout of the C ABI
        const int64_t pidx = ((int64_t)ix * N + outer) * (N / 2 + 1) + col;
        const cx<T> pstored = valid ? ldc(phi + pidx) : mk(T(0), T(0));
        const T h = T(s.h), h2 = T(s.h2);
        const T den = -k2s - T(3) * h2 - T(3) * h * T(s.inv_dtau) - T(4.5) * h2 * T(s.om_a);
        const cx<T> num = scale(X[k2], T(1.5) * h2 * T(s.om_a)) - scale(pstored, T(3) * h * T(s.inv_dtau));
        const cx<T> pnew = zero ? mk(T(0), T(0)) : scale(num, T(1) / den);  // phi_old -> phi_new
        if (valid) stc(phi + pidx, pnew);
        X[k2] = scale(pnew, -T(s.a_c2));
      }
    }
  }
  // Inverse transforms.  Along axis 0 the y and z gradient symbols are constants, so
  //   F_x = IDFT(D_x G),  F_y = D_y IDFT(G),  F_z = D_z IDFT(G)
  // (G here the potential times its prefactor).  F_x is written in place and IDFT(G)
  // to out1 (the "G form"): D_y is applied by the inverse pass along y and D_z by the
  // c2r rows pass, so F_y and F_z never exist as spectra of their own.
  {
    __syncthreads();  // every thread has read its forward data from LDS
    if (u < L1) {
      cx<T> Y[L2];
#pragma unroll
      for (int k2 = 0; k2 < L2; ++k2) {
        const int ix = u + L1 * k2;
        Y[k2] = grad_symbol<T>(ix < N / 2 ? ix : ix - N, N, s.grad) * X[k2];
      }
      RegDFT<T, L2, 1>::run(Y);
#pragma unroll
      for (int ja = 0; ja < L2; ++ja)
        lds[col_lds_index<T, L1, L2>(u, ja, b, B)] = ja == 0 ? Y[ja] : tw_mul<true>(Y[ja], tw, u * ja * g.tw_step);
    }
    __syncthreads();
    if (u < L2) {
      cx<T> c[L1];
#pragma unroll
      for (int k1 = 0; k1 < L1; ++k1) c[k1] = lds[col_lds_index<T, L1, L2>(k1, u, b, B)];
      RegDFT<T, L1, 1>::run(c);
      if (valid) {
#pragma unroll
        for (int jb = 0; jb < L1; ++jb) stc(data + off + (int64_t)(u + L2 * jb) * g.stride, c[jb]);
      }
    }
  }
  __syncthreads();  // every thread has read the F_x exchange from LDS
  if (u < L1) {
    RegDFT<T, L2, 1>::run(X);
#pragma unroll
    for (int ja = 0; ja < L2; ++ja)
      lds[col_lds_index<T, L1, L2>(u, ja, b, B)] = ja == 0 ? X[ja] : tw_mul<true>(X[ja], tw, u * ja * g.tw_step);
  }
  __syncthreads();
  if (u < L2) {
    cx<T> c[L1];
#pragma unroll
    for (int k1 = 0; k1 < L1; ++k1) c[k1] = lds[col_lds_index<T, L1, L2>(k1, u, b, B)];
    RegDFT<T, L1, 1>::run(c);
    if (valid) {
#pragma unroll
      for (int jb = 0; jb < L1; ++jb) stc(out1 + off + (int64_t)(u + L2 * jb) * g.stride, c[jb]);
    }
  }
}

}  // namespace pm
