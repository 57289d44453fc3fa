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

template <typename T>
__device__ __forceinline__ void atomic_add(T* p, T v) {
  unsafeAtomicAdd(p, v);
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

}  // namespace pm
