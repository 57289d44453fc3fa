// Internal device/host helpers shared by the pmhip kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pmhip.h"

namespace pm {

// Particle arrays and kick/drift factors of one box of an uneven ensemble's size group
// (pm_batch): the particle kernels of a group plan read box blockIdx.y's entry from a
// device table instead of taking the plan's arrays at a stride of 3 N^3.
struct BoxEntry {
  void* pos;
  void* mom;
  double kick;
  double drift;
};

// ------------------------------------------------------------------ complex --

template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T a, T b) {
  cx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return mk(a.x * s, a.y * s); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> conjg(cx<T> a) { return mk(a.x, -a.y); }
// multiply by +i (dir = +1) or -i (dir = -1)
template <int DIR, typename T>
__host__ __device__ __forceinline__ cx<T> mul_i(cx<T> a) {
  return DIR > 0 ? mk(-a.y, a.x) : mk(a.y, -a.x);
}
// a * conj(w) when INV, a * w otherwise
template <bool INV, typename T>
__host__ __device__ __forceinline__ cx<T> twiddle(cx<T> a, cx<T> w) {
  return INV ? mk(a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y) : a * w;
}

// Vector memory types for 8/16-byte complex loads.
template <typename T>
struct vec2;
template <>
struct vec2<float> {
  typedef float2 type;
};
template <>
struct vec2<double> {
  typedef double2 type;
};

template <typename T>
__device__ __forceinline__ cx<T> ldc(const cx<T>* p) {
  typedef typename vec2<T>::type V;
  V v = *reinterpret_cast<const V*>(p);
  return mk(v.x, v.y);
}
template <typename T>
__device__ __forceinline__ void stc(cx<T>* p, cx<T> a) {
  typedef typename vec2<T>::type V;
  V v;
  v.x = a.x;
  v.y = a.y;
  *reinterpret_cast<V*>(p) = v;
}

// ------------------------------------------------- compile-time twiddles --
// cos / sin of 2 pi m / n evaluated at compile time: the angle is reduced exactly
// (integer octant arithmetic) to |x| <= pi/4 and the Taylor series of sin and cos
// is summed to well below double rounding.
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int i = 1; i < 14; ++i) {
    term *= -x * x / double((2 * i) * (2 * i + 1));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int i = 1; i < 14; ++i) {
    term *= -x * x / double((2 * i - 1) * (2 * i));
    sum += term;
  }
  return sum;
}
// angle 2 pi m / n = (pi/2) q + x, q = nearest quarter turn
constexpr double ct_cos(long m, long n) {
  long mm = ((m % n) + n) % n;
  long q = (4 * mm + n / 2) / n;  // round(4 mm / n)
  double x = 2.0 * kPi * (double(4 * mm - q * n) / double(4 * n));
  double c = taylor_cos(x), s = taylor_sin(x);
  switch (q & 3) {
    case 0: return c;
    case 1: return -s;
    case 2: return -c;
    default: return s;
  }
}
constexpr double ct_sin(long m, long n) {
  long mm = ((m % n) + n) % n;
  long q = (4 * mm + n / 2) / n;
  double x = 2.0 * kPi * (double(4 * mm - q * n) / double(4 * n));
  double c = taylor_cos(x), s = taylor_sin(x);
  switch (q & 3) {
    case 0: return s;
    case 1: return c;
    case 2: return -s;
    default: return -c;
  }
}

// ----------------------------------------------------- register DFTs --
// In-place DFT of N values held in registers, natural order in and out:
//   X[k] = sum_n a[n] exp(DIR * 2 pi i n k / N), DIR = -1 forward, +1 inverse.
// Decimation in time with radix 4, 3 or 2 at every level; every twiddle is a
// compile-time constant.

template <typename T, int N, int DIR>
struct RegDFT;

template <typename T, int DIR>
struct RegDFT<T, 1, DIR> {
  __device__ __forceinline__ static void run(cx<T>*) {}
};

template <typename T, int DIR>
struct RegDFT<T, 2, DIR> {
  __device__ __forceinline__ static void run(cx<T>* a) {
    cx<T> t = a[0];
    a[0] = t + a[1];
    a[1] = t - a[1];
  }
};

template <typename T, int DIR>
struct RegDFT<T, 3, DIR> {
  __device__ __forceinline__ static void run(cx<T>* a) {
    const T s3 = T(0.86602540378443864676372317075293618);
    cx<T> s = a[1] + a[2];
    cx<T> d = a[1] - a[2];
    cx<T> m = a[0] - scale(s, T(0.5));
    cx<T> r = scale(mul_i<DIR>(d), s3);  // DIR i (sqrt3/2)(a1 - a2)
    a[0] = a[0] + s;
    a[1] = m + r;
    a[2] = m - r;
  }
};

template <typename T, int DIR>
struct RegDFT<T, 4, DIR> {
  __device__ __forceinline__ static void run(cx<T>* a) {
    cx<T> s0 = a[0] + a[2], d0 = a[0] - a[2];
    cx<T> s1 = a[1] + a[3], d1 = mul_i<DIR>(a[1] - a[3]);
    a[0] = s0 + s1;
    a[2] = s0 - s1;
    a[1] = d0 + d1;
    a[3] = d0 - d1;
  }
};

template <int N>
struct Radix {
  static constexpr int value = (N % 4 == 0) ? 4 : (N % 3 == 0 ? 3 : 2);
};

template <typename T, int N, int DIR>
struct RegDFT {
  static constexpr int R = Radix<N>::value;
  static constexpr int M = N / R;
  __device__ __forceinline__ static void run(cx<T>* a) {
    cx<T> sub[R][M];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int m = 0; m < M; ++m) sub[r][m] = a[r + R * m];
#pragma unroll
    for (int r = 0; r < R; ++r) RegDFT<T, M, DIR>::run(sub[r]);
#pragma unroll
    for (int k = 0; k < M; ++k) {
      cx<T> t[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (r == 0 || k == 0) {
          t[r] = sub[r][k];
        } else if (4L * r * k == N) {
          t[r] = mul_i<DIR>(sub[r][k]);  // W_N^(N/4) = DIR i exactly: no multiply
        } else {
          const T wc = T(ct_cos(long(r) * k, N));
          const T ws = T(DIR * ct_sin(long(r) * k, N));
          t[r] = sub[r][k] * mk(wc, ws);
        }
      }
      RegDFT<T, R, DIR>::run(t);
#pragma unroll
      for (int q = 0; q < R; ++q) a[k + M * q] = t[q];
    }
  }
};

// --------------------------------------------------------- FFT shapes --
// A length-L transform is done as L = L1 * L2: L2 threads each transform L1
// strided values in registers, exchange through LDS, then L1 threads transform L2
// values.  Threads per transform = max(L1, L2).
struct Shape {
  int L, L1, L2;
};
__host__ __device__ constexpr Shape shape_for(int L) {
  return L == 4      ? Shape{4, 2, 2}
         : L == 8    ? Shape{8, 4, 2}
         : L == 16   ? Shape{16, 4, 4}
         : L == 32   ? Shape{32, 8, 4}
         : L == 64   ? Shape{64, 8, 8}
         : L == 96   ? Shape{96, 8, 12}
         : L == 128  ? Shape{128, 16, 8}
         : L == 192  ? Shape{192, 16, 12}
         : L == 256  ? Shape{256, 16, 16}
         : L == 512  ? Shape{512, 16, 32}
         : L == 1024 ? Shape{1024, 32, 32}
                     : Shape{0, 0, 0};
}

// Row stride (complex elements) of the library's internal [N][N][N/2+1] spectra: N/2+1
// rounded up to a 128-byte multiple, so every row starts on a cache-line boundary and
// a batch of adjacent columns maps onto whole lines.
__host__ __device__ inline int padded_half(int n, int esize) {
  const int per_line = 128 / (2 * esize);
  const int h = n / 2 + 1;
  return (h + per_line - 1) / per_line * per_line;
}

__host__ __device__ inline bool mesh_supported(int n) {
  return n == 8 || n == 16 || n == 32 || n == 64 || n == 128 || n == 192 || n == 256 || n == 512 || n == 1024;
}

// XCD-aware block index: consecutive logical blocks land on the same XCD (the
// hardware deals workgroups round-robin over the 8 XCDs), so each XCD's L2 sees a
// contiguous slice of the work.
__device__ __forceinline__ int64_t xcd_block(int64_t bid, int64_t nblocks) {
  const int64_t nx = 8;
  int64_t per = nblocks / nx;
  if (per == 0) return bid;
  int64_t full = per * nx;
  if (bid >= full) return bid;
  return (bid % nx) * per + bid / nx;
}

}  // namespace pm
