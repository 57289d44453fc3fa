// Device helpers shared by the particle kernels (deposit, gather, combine, ICs).
#pragma once

#include "pm_common.h"

namespace pm {

// Periodic wrap into [0, N): x - N floor(x/N); a rounded quotient that overshoots
// (possible when N is not a power of two) is corrected by +N, and a result that
// rounds to N becomes 0.  Non-finite input maps to 0, so every derived cell index
// stays inside the mesh.
template <typename T>
__device__ __forceinline__ T wrap(T x, int n) {
  const T fn = T(n);
  T y = x - fn * floor(x / fn);
  if (y < T(0)) y += fn;
  return (y >= fn || !(y >= T(0))) ? T(0) : y;
}

// wrap for a power-of-two N: x / N is exact as x 2^-log2(N), so the same result
// without a division
template <typename T>
__device__ __forceinline__ T wrap_pow2(T x, int n) {
  const T fn = T(n);
  T y = x - fn * floor(ldexp(x, -(int)__builtin_ctz((unsigned)n)));
  if (y < T(0)) y += fn;
  return (y >= fn || !(y >= T(0))) ? T(0) : y;
}
template <bool P2, typename T>
__device__ __forceinline__ T wrap_n(T x, int n) {
  if constexpr (P2) return wrap_pow2(x, n);
  else return wrap(x, n);
}

// wrap_n of one particle's coordinates (wrap_one) or of all of a thread's (wrap_all).
// Both wraps return x unchanged for x in [0, N), so when every coordinate of the wave
// is already there (positions this library wrote, and almost every drift) the wave
// skips them: a wave-uniform branch on a few compares instead of ~10 operations per
// coordinate.  Non-finite values fail the compares and take the wrap.
template <bool P2>
__device__ __forceinline__ void wrap_one(float& x, float& y, float& z, int n) {
  const float fn = float(n);
  if (__all(x >= 0.f && x < fn && y >= 0.f && y < fn && z >= 0.f && z < fn)) return;
  x = wrap_n<P2>(x, n);
  y = wrap_n<P2>(y, n);
  z = wrap_n<P2>(z, n);
}
template <bool P2, int PP>
__device__ __forceinline__ void wrap_all(float (&x)[PP], float (&y)[PP], float (&z)[PP], int n) {
  const float fn = float(n);
  bool in = true;
#pragma unroll
  for (int p = 0; p < PP; ++p)
    in = in && x[p] >= 0.f && x[p] < fn && y[p] >= 0.f && y[p] < fn && z[p] >= 0.f && z[p] < fn;
  if (__all(in)) return;
#pragma unroll
  for (int p = 0; p < PP; ++p) {
    x[p] = wrap_n<P2>(x[p], n);
    y[p] = wrap_n<P2>(y[p], n);
    z[p] = wrap_n<P2>(z[p], n);
  }
}

// Load and store of element i < 2^30 of a float array in device memory at a
// wave-uniform base.  The access goes through a global-address-space pointer: a
// pointer the compiler cannot trace to a kernel argument (e.g. one read from a box
// table) would otherwise be accessed with flat instructions, which also count
// against the LDS counter, so every wait for an LDS result would wait for them too.
// The byte offset fits 32 bits, so the address is the scalar base plus a 32-bit lane
// offset, without per-lane 64-bit address arithmetic.
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) char gchar;
__device__ __forceinline__ float ldg32(const float* base, unsigned i) {
  return *reinterpret_cast<const gfloat*>((const gchar*)base + (i << 2));
}
__device__ __forceinline__ void stg32(float* base, unsigned i, float v) {
  *reinterpret_cast<gfloat*>((gchar*)base + (i << 2)) = v;
}

// CIC base node and weights of one coordinate (x in [0, N)): node floor(x) gets
// 1 - t and node floor(x) + 1 (mod N) gets t = x - floor(x).
template <typename T>
struct Axis {
  int i0, i1;
  T w0, w1;
};
template <typename T>
__device__ __forceinline__ Axis<T> cic_axis(T x, int n) {
  Axis<T> a;
  const T f = floor(x);
  a.i0 = (int)f;
  a.i1 = a.i0 + 1 == n ? 0 : a.i0 + 1;
  a.w1 = x - f;
  a.w0 = T(1) - a.w1;
  return a;
}
template <bool P2, typename T>
__device__ __forceinline__ Axis<T> cic_axis_n(T x, int n) {
  if constexpr (P2) {
    Axis<T> a;
    const T f = floor(x);
    a.i0 = (int)f;
    a.i1 = (a.i0 + 1) & (n - 1);
    a.w1 = x - f;
    a.w0 = T(1) - a.w1;
    return a;
  } else {
    return cic_axis(x, n);
  }
}

template <typename T>
__device__ __forceinline__ void atomic_add(T* p, T v) {
  unsafeAtomicAdd(p, v);
}

// LDS deposit windows accumulate CIC weights (<= 1) as 32-bit fixed point with scale
// S = 2^21 (integer LDS atomics are much faster than float ones on gfx950): w S is
// exact in float and to_fix_w rounds it to nearest-even, so the terms carry no bias;
// each is at most 2^21, so a window of up to 2048 particles reaches 2^32 in a cell only
// if all of them sit exactly on the same node (to_fix_w_capped, for such windows,
// keeps every term below 2^21).  The quantum 2^-21 ~ 4.8e-7 of a particle is far
// below the FP32 rounding of the density it is flushed into.
// The rounding: for 0 <= w <= 1, w S + 2^23 in one fused multiply-add is rounded to
// nearest-even once and lands in [2^23, 2^24), where the floats are the integers, so
// its bits minus those of 2^23 are rint(w S) (one operation instead of a multiply, a
// rounding and a conversion).
constexpr float kFixW = 2097152.0f;
__host__ __device__ __forceinline__ unsigned to_fix_w(float w) {
  return __builtin_bit_cast(unsigned, __builtin_fmaf(w, kFixW, 8388608.0f)) - 0x4B000000u;
}
__host__ __device__ __forceinline__ unsigned to_fix_w_capped(float w) {
  const unsigned v = to_fix_w(w);
  return v < 2097151u ? v : 2097151u;
}

// Product of two factors below 2^24 (the masks let the compiler use the full-rate
// 24-bit multiplier, where a 32-bit multiply is quarter rate)
__host__ __device__ __forceinline__ unsigned mul24(unsigned a, unsigned b) { return (a & 0xFFFFFFu) * (b & 0xFFFFFFu); }

// Flat index (i N + j) N + l of a mesh node (i, j, l in [0, N)) as a 32-bit value
// (N <= 1024, so below 2^30): shifts for a power-of-two N, else 24-bit multiplies.
template <bool P2>
__host__ __device__ __forceinline__ unsigned node_index(int i, int j, int l, int n) {
  if constexpr (P2) {
    const int k = __builtin_ctz((unsigned)n);
    return ((((unsigned)i << k) | (unsigned)j) << k) | (unsigned)l;
  } else {
    return mul24(mul24((unsigned)i, (unsigned)n) + (unsigned)j, (unsigned)n) + (unsigned)l;
  }
}

// Window cell number a sx + b sy + c of in-window offsets (all products below 2^24)
__host__ __device__ __forceinline__ int win_index(int a, int b, int c, int sx, int sy) {
  return (int)(mul24((unsigned)a, (unsigned)sx) + mul24((unsigned)b, (unsigned)sy)) + c;
}

// Window cells are numbered c = (a W1 + b) W2 + cz.  Their decomposition divides by
// runtime extents, which a high multiply does exactly in the range windows use
// (2 <= d < 2^14, 0 <= c < 2^14; the largest window has 12288 cells): with
// m = floor((2^32 - 1) / d) + 1 the product c m / 2^32 exceeds c / d by less than
// c / 2^32 < 2^-18, while c / d stays at least 1/d > 2^-14 below the next integer,
// so floor(c m / 2^32) = floor(c / d).
struct WinDiv {
  unsigned d, m;
  __host__ __device__ __forceinline__ explicit WinDiv(int dd) : d((unsigned)dd), m(0xFFFFFFFFu / (unsigned)dd + 1u) {}
  __host__ __device__ __forceinline__ unsigned quot(unsigned c) const {
    return (unsigned)(((unsigned long long)c * m) >> 32);
  }
};
// c -> (a, b, cz) for the strides sx = W1 W2 (in qx) and sy = W2 (in qy)
__host__ __device__ __forceinline__ void win_cell(int c, const WinDiv& qx, const WinDiv& qy, int& a, int& b,
                                                  int& cz) {
  const unsigned ua = qx.quot((unsigned)c);
  const unsigned r = (unsigned)c - mul24(ua, qx.d);
  const unsigned ub = qy.quot(r);
  a = (int)ua;
  b = (int)ub;
  cz = (int)(r - mul24(ub, qy.d));
}

// v in (-N, 2N) -> [0, N)
__device__ __forceinline__ int fold(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
// minimum-image difference of two cell indices in [0, N): result in [-N/2, N/2]
__device__ __forceinline__ int idiff(int a, int b, int n) {
  int d = a - b;
  if (d > n / 2) d -= n;
  else if (d < -n / 2) d += n;
  return d;
}
// The same for a power-of-two N (P2) with masks instead of compares and selects.
// idiff_n<true> returns [-N/2, N/2) (a difference of exactly N/2 comes out as -N/2):
// a kernel uses one of the two forms throughout, so tile-relative coordinates stay
// consistent.
template <bool P2>
__device__ __forceinline__ int fold_n(int v, int n) {
  if constexpr (P2) return (v + n) & (n - 1);
  else return fold(v, n);
}
template <bool P2>
__device__ __forceinline__ int idiff_n(int a, int b, int n) {
  if constexpr (P2) return ((a - b + n / 2) & (n - 1)) - n / 2;
  else return idiff(a, b, n);
}

// Window of a tile whose bounding box (origin o, extents W, volume vol) exceeds the
// LDS capacity `cap` (>= 8): the same proportions scaled by (cap/vol)^(1/3), each side
// at least 2; while the volume still exceeds cap the longest side is cut to
// cap / (product of the other two) (at least 2), which fits after at most three cuts;
// centred on the tile's mean base cell and kept inside the bounding box.  Particles
// outside it take the direct global path; for late-time (clustered) tiles this leaves
// about a tenth of the particles a fixed cube would.  Every thread computes the same
// box.
__host__ __device__ __forceinline__ void fit_box(int (&o)[3], int (&W)[3], const float (&mean)[3], int64_t vol,
                                                 int cap) {
  const float f = cbrtf((float)cap / (float)vol);
  int Wf[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int w = (int)((float)W[d] * f);
    Wf[d] = w < 2 ? 2 : (w > W[d] ? W[d] : w);
  }
#pragma unroll
  for (int it = 0; it < 3; ++it) {
    const int m = Wf[0] >= Wf[1] ? (Wf[0] >= Wf[2] ? 0 : 2) : (Wf[1] >= Wf[2] ? 1 : 2);
    const int rest = Wf[m == 0 ? 1 : 0] * Wf[m == 2 ? 1 : 2];
    if (Wf[m] * rest > cap) Wf[m] = cap / rest < 2 ? 2 : cap / rest;
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int c = (int)rintf(mean[d]) - Wf[d] / 2, hi = o[d] + W[d] - Wf[d];
    o[d] = c < o[d] ? o[d] : (c > hi ? hi : c);
    W[d] = Wf[d];
  }
}

// Block-wide (256 threads) window from per-thread ranges [lo_d, hi_d] of tile-relative
// base cells and per-thread sums of them over `count` particles: o = the block's
// minimum, W = max - min + 2 (a 2-cell box at 0 when no thread saw a particle); if the
// volume exceeds `cap`, the sums are reduced too and fit_box shrinks the window.
// Within a wave lo and -hi travel together as two 16-bit halves (|values| < 2^15):
// one shuffle and one packed minimum per step.  wlo/whi/wsum: __shared__ [4][3]
// scratch, free again on return; every thread must call.
__host__ __device__ __forceinline__ int pack_lo_nhi(int lo, int hi) {
  const int a = lo < -32767 ? -32767 : (lo > 32767 ? 32767 : lo);
  const int b = -hi < -32767 ? -32767 : (-hi > 32767 ? 32767 : -hi);
  return (int)((unsigned)(unsigned short)a | ((unsigned)(unsigned short)b << 16));
}
__host__ __device__ __forceinline__ int min_lo_nhi(int u, int v) {
  typedef short s16x2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(int, __builtin_elementwise_min(__builtin_bit_cast(s16x2, u), __builtin_bit_cast(s16x2, v)));
}
__device__ __forceinline__ void block_window(const int (&lo)[3], const int (&hi)[3], const float (&sum)[3], int count,
                                             int cap, int (*wlo)[3], int (*whi)[3], float (*wsum)[3], int (&o)[3],
                                             int (&W)[3]) {
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  int pk[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    pk[d] = pack_lo_nhi(lo[d], hi[d]);
    for (int off = 32; off > 0; off >>= 1) pk[d] = min_lo_nhi(pk[d], __shfl_xor(pk[d], off, 64));
  }
  if (lane == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      wlo[wave][d] = (int)(short)(pk[d] & 0xFFFF);
      whi[wave][d] = -(int)(short)((unsigned)pk[d] >> 16);
    }
  }
  __syncthreads();
  int64_t vol = 1;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int a = wlo[0][d], b = whi[0][d];
    for (int k = 1; k < 4; ++k) {
      a = min(a, wlo[k][d]);
      b = max(b, whi[k][d]);
    }
    if (b < a) a = b = 0;  // no particle: an empty 2-cell box at the origin
    o[d] = a;
    W[d] = b - a + 2;
    vol *= W[d];
  }
  if (vol > cap) {  // the same decision in every thread
    float sm[3] = {sum[0], sum[1], sum[2]};
#pragma unroll
    for (int d = 0; d < 3; ++d)
      for (int off = 32; off > 0; off >>= 1) sm[d] += __shfl_xor(sm[d], off, 64);
    if (lane == 0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) wsum[wave][d] = sm[d];
    }
    __syncthreads();
    float mean[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) mean[d] = (wsum[0][d] + wsum[1][d] + wsum[2][d] + wsum[3][d]) / float(count);
    fit_box(o, W, mean, vol, cap);
  }
  __syncthreads();  // the scratch may be reused after return
}

// Window of a Lagrangian tile (one 256-thread block, PP particles per thread): the
// bounding box of the particles' CIC base cells floor(x), relative to the tile
// origin `org` (minimum image), widened by one cell so the +1 CIC neighbours fit:
// cells [o_d, o_d + W_d).  If its volume exceeds `cap` cells, fit_box's smaller box
// is used instead.  Particles with x < 0 are skipped.  Block-wide
// (every thread must call); wlo/whi/wsum are __shared__ [4][3] scratch.
struct TileWindow {
  int o[3], W[3];
};
template <int PP, bool P2>
__device__ __forceinline__ TileWindow tile_window(const float (&x)[PP], const float (&y)[PP], const float (&z)[PP],
                                                  int n, const int (&org)[3], int cap, int count,
                                                  int (*wlo)[3], int (*whi)[3], float (*wsum)[3]) {
  int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
  float sum[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int p = 0; p < PP; ++p) {
    if (x[p] < 0.f) continue;
    const int r[3] = {idiff_n<P2>((int)floorf(x[p]), org[0], n), idiff_n<P2>((int)floorf(y[p]), org[1], n),
                      idiff_n<P2>((int)floorf(z[p]), org[2], n)};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = min(lo[d], r[d]);
      hi[d] = max(hi[d], r[d]);
      sum[d] += float(r[d]);
    }
  }
  TileWindow w;
  block_window(lo, hi, sum, count, cap, wlo, whi, wsum, w.o, w.W);
  return w;
}

// Particle arrays (and, with a table, kick and drift) of box blockIdx.y: the table's
// entry when a table is given, else the arrays at a stride of 3 np from the pointers.
template <typename T>
__device__ __forceinline__ void box_arrays(const BoxEntry* tab, int64_t np, T* __restrict__& pos, T* __restrict__& mom,
                                           T& kick, T& drift) {
  if (tab) {
    const BoxEntry& e = tab[blockIdx.y];
    pos = static_cast<T*>(e.pos);
    mom = static_cast<T*>(e.mom);
    kick = T(e.kick);
    drift = T(e.drift);
  } else {
    pos += (int64_t)blockIdx.y * 3 * np;
    mom += (int64_t)blockIdx.y * 3 * np;
  }
}
template <typename T>
__device__ __forceinline__ const T* box_positions(const BoxEntry* tab, int64_t np, const T* pos) {
  return tab ? static_cast<const T*>(tab[blockIdx.y].pos) : pos + (int64_t)blockIdx.y * 3 * np;
}

// Order of a tiled kernel's workgroups over its grid of tx x ty x tz Lagrangian tile
// columns (z fastest).  Consecutive workgroups (of one XCD, after xcd_block) take the
// z-run of one column, then the next column of a block of kTileBlock x kTileBlock
// columns in (x, y), block after block: the columns whose windows share halo rows with
// a column in x or y were processed at most about kTileBlock^2 z-runs earlier, so those
// rows are still in the L2 or the last-level cache instead of being fetched from HBM
// again (in plain z-y-x order the x neighbour comes ty z-runs later).  Grids whose tx
// or ty is not a multiple of the block size keep the plain order.
constexpr int kTileBlock = 8;
__host__ __device__ __forceinline__ void tile_coords(int64_t lin, int tx, int ty, int tz, int& ti, int& tk, int& tl) {
  tl = (int)(lin % tz);
  int64_t r = lin / tz;
  if (tx % kTileBlock == 0 && ty % kTileBlock == 0) {
    const int xl = (int)(r % kTileBlock);
    r /= kTileBlock;
    const int yl = (int)(r % kTileBlock);
    r /= kTileBlock;
    const int nbx = tx / kTileBlock;
    ti = (int)(r % nbx) * kTileBlock + xl;
    tk = (int)(r / nbx) * kTileBlock + yl;
  } else {
    tk = (int)(r % ty);
    ti = (int)(r / ty);
  }
}

}  // namespace pm
