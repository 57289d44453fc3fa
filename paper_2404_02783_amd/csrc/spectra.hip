// Fourier-space kernels that are not FFT passes: the initial-condition symbol,
// the power-spectrum shell reduction and the bispectrum shell filter / triple sums.
#include <math.h>

#include <algorithm>

#include "pm_common.h"
#include "pm_plan.h"

namespace pm {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int signed_freq(int i, int n) { return i < n / 2 ? i : i - n; }

// Eisenstein & Hu (1998) no-wiggle transfer function (their sound-horizon fit, the
// alpha_Gamma suppression, the effective shape Gamma and T0(q)); k in h/Mpc.
__device__ double eh98_transfer(double k, double om, double ob, double h, double tcmb) {
  const double omh2 = om * h * h, obh2 = ob * h * h, fb = ob / om, th = tcmb / 2.7;
  const double s = 44.5 * log(9.83 / omh2) / sqrt(1.0 + 10.0 * pow(obh2, 0.75));
  const double al = 1.0 - 0.328 * log(431.0 * omh2) * fb + 0.38 * log(22.3 * omh2) * fb * fb;
  const double ks = 0.43 * k * h * s;
  const double gam = om * h * (al + (1.0 - al) / (1.0 + ks * ks * ks * ks));
  const double q = k * th * th / gam;
  const double l0 = log(2.0 * 2.718281828459045235360287 + 1.8 * q);
  const double c0 = 14.2 + 731.0 / (1.0 + 62.5 * q);
  return l0 / (l0 + c0 * q * q);
}

// Zel'dovich / gauge-shift symbol on the natural [N][N][N/2+1] layout.  Input
// cbuf(0) = DFT(noise).  delta_L = w_hat sqrt(P(k)/dx^3) growth (zero at k = 0 and on
// Nyquist planes); output component d = coef * i k_d delta_L / k^(2 kpow) *
// exp(i (k_x + k_y + k_z)/2) into cbuf(d), i.e. S_d(n) w_hat(n).
// ADJ: the transposed map, cbuf(0) <- sum_d conj(S_d(n)) cbuf(d) (inputs are the
// spectra of the displacement cotangents).
template <typename T, bool ADJ>
__global__ void __launch_bounds__(kBlock) k_ic_symbol(cx<T>* __restrict__ c0, cx<T>* __restrict__ c1,
                                                      cx<T>* __restrict__ c2, int n, int hp, int64_t cs, IcSymbol sy) {
  const int h = hp;  // padded row stride; columns iz > N/2 are padding
  const int64_t total = (int64_t)n * n * h;
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= total) return;
  c0 += (int64_t)blockIdx.y * cs;  // box of the batch (spectra cs elements apart)
  c1 += (int64_t)blockIdx.y * cs;
  c2 += (int64_t)blockIdx.y * cs;
  const int iz = (int)(idx % h);
  if (iz > n / 2) return;
  const int iy = (int)((idx / h) % n);
  const int ix = (int)(idx / ((int64_t)h * n));
  const int nx = signed_freq(ix, n), ny = signed_freq(iy, n), nz = iz;
  const bool nyq = (nx == -n / 2) || (ny == -n / 2) || (nz == n / 2);
  const int64_t n2 = (int64_t)nx * nx + (int64_t)ny * ny + (int64_t)nz * nz;
  cx<T> out[3] = {mk(T(0), T(0)), mk(T(0), T(0)), mk(T(0), T(0))};
  if (sy.mode == 3 && !nyq && n2 > 0) {
    // gradient of a field sampled on the lattice: i k_d coef w_hat / k^2; adjoint:
    // sum_d conj(i k_d) coef c_d / k^2
    const double s = 2.0 * kPi / n;
    const double kd[3] = {s * nx, s * ny, s * nz};
    const double f = sy.coef / (kd[0] * kd[0] + kd[1] * kd[1] + kd[2] * kd[2]);
    if (ADJ) {
      double qr = 0.0, qi = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const cx<T> cdd = ldc((d == 0 ? c0 : d == 1 ? c1 : c2) + idx);
        qr += kd[d] * (double)cdd.x;
        qi += kd[d] * (double)cdd.y;
      }
      out[0] = mk(T(f * qi), T(-f * qr));  // -i q
    } else {
      const cx<T> w = ldc(c0 + idx);
#pragma unroll
      for (int d = 0; d < 3; ++d) out[d] = mk(T(-kd[d] * f * (double)w.y), T(kd[d] * f * (double)w.x));
    }
  } else if (sy.mode != 3 && !nyq && n2 > 0) {
    const double kmag = sy.kf * sqrt((double)n2);
    double pk = sy.amp * pow(kmag, sy.index);
    if (sy.pk_kind == PM_PK_EH98) {
      const double tk = eh98_transfer(kmag, sy.om, sy.ob, sy.h, sy.tcmb);
      pk *= tk * tk;
    }
    const double amp = sqrt(pk * sy.inv_dx3) * sy.growth;
    const double s = 2.0 * kPi / n;
    const double kx = s * nx, ky = s * ny, kz = s * nz;
    const double k2 = kx * kx + ky * ky + kz * kz;
    const double inv = sy.kpow == 1 ? 1.0 / k2 : 1.0 / (k2 * k2);
    double sn, cs;
    sincos(0.5 * (kx + ky + kz), &sn, &cs);
    const double f = amp * inv * sy.coef;
    const double kd[3] = {kx, ky, kz};
    if (ADJ && sy.mode != 0) {
      // sum_d conj(h_d f e^{i phase}) c_d = f e^{-i phase} sum_d h_d c_d (h_d real:
      // -k_d^2, or -k_a k_b for the pairs xy, xz, yz)
      const cx<T> cd[3] = {ldc(c0 + idx), ldc(c1 + idx), ldc(c2 + idx)};
      const int ia[3] = {0, 0, 1}, ib[3] = {1, 2, 2};
      double qr = 0.0, qi = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double h = sy.mode == 1 ? -kd[d] * kd[d] : -kd[ia[d]] * kd[ib[d]];
        qr += h * (double)cd[d].x;
        qi += h * (double)cd[d].y;
      }
      out[0] = mk(T(f * (qr * cs + qi * sn)), T(f * (qi * cs - qr * sn)));
    } else if (ADJ) {
      // sum_d conj(i k_d f e^{i phase}) c_d = f e^{-i phase} (-i) sum_d k_d c_d
      const cx<T> cd[3] = {ldc(c0 + idx), ldc(c1 + idx), ldc(c2 + idx)};
      double qr = 0.0, qi = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        qr += kd[d] * (double)cd[d].x;
        qi += kd[d] * (double)cd[d].y;
      }
      const double rr = qi, ri = -qr;  // -i q
      out[0] = mk(T(f * (rr * cs + ri * sn)), T(f * (ri * cs - rr * sn)));
    } else {
      const cx<T> w = ldc(c0 + idx);
      // base = w * amp * inv * coef * e^{i phase}; component d = i k_d base, or a
      // Hessian component -k_a k_b base
      const double br = f * ((double)w.x * cs - (double)w.y * sn);
      const double bi = f * ((double)w.x * sn + (double)w.y * cs);
      if (sy.mode == 0) {
#pragma unroll
        for (int d = 0; d < 3; ++d) out[d] = mk(T(-kd[d] * bi), T(kd[d] * br));
      } else {
        const int ia[3] = {0, 0, 1}, ib[3] = {1, 2, 2};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double h = sy.mode == 1 ? -kd[d] * kd[d] : -kd[ia[d]] * kd[ib[d]];
          out[d] = mk(T(h * br), T(h * bi));
        }
      }
    }
  }
  stc(c0 + idx, out[0]);
  if (!ADJ) {
    stc(c1 + idx, out[1]);
    stc(c2 + idx, out[2]);
  }
}

// Power-spectrum shell reduction.  Bin b of mode n: N^2 (2b+1)^2 <= 16 nb^2 |n|^2 <
// N^2 (2b+3)^2, found from a floating estimate and settled with integer tests.
// Per block: LDS accumulators (sum w |dhat|^2, sum w |n|, count); then one global
// atomic per touched bin.  sums layout: [0, nb) power, [nb, 2nb) |n| sums,
// [2nb, 3nb) counts (as unsigned 64-bit integers reinterpreted).
__device__ __forceinline__ int pk_bin(int64_t n2, int n, int nb) {
  const int64_t s = 16LL * nb * nb * n2;
  const int64_t nn = (int64_t)n * n;
  // (2b+1) <= 4 nb |n| / N  -> b ~ floor((4 nb |n|/N - 1)/2), a first guess that the
  // exact integer tests below correct
  int b = (int)floor((sqrt((double)n2) * (4.0 * nb / n) - 1.0) * 0.5);
  if (b < 0) b = 0;
  for (int it = 0; it < 3; ++it) {
    const int64_t lo = nn * (2LL * b + 1) * (2LL * b + 1);
    const int64_t hi = nn * (2LL * b + 3) * (2LL * b + 3);
    if (s < lo) {
      if (b == 0) return -1;
      --b;
    } else if (s >= hi) {
      ++b;
    } else {
      return b < nb ? b : -1;
    }
  }
  return -1;
}

// CROSS: the power of the pair (dhat, bhat), Re(dhat conj(bhat)), in place of |dhat|^2.
template <typename T, bool CROSS>
__global__ void __launch_bounds__(kBlock) k_pk_reduce(const cx<T>* __restrict__ dhat, const cx<T>* __restrict__ bhat,
                                                      int n, int hp, int64_t cs, int nb, double* __restrict__ sums) {
  extern __shared__ double sh[];
  dhat += (int64_t)blockIdx.y * cs;  // box of the batch
  if (CROSS) bhat += (int64_t)blockIdx.y * cs;
  sums += (int64_t)blockIdx.y * 3 * nb;
  double* sp = sh;
  double* sk = sh + nb;
  unsigned long long* sc = reinterpret_cast<unsigned long long*>(sh + 2 * nb);
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    sp[b] = 0.0;
    sk[b] = 0.0;
    sc[b] = 0ull;
  }
  __syncthreads();
  const int h = hp;  // padded row stride; columns iz > N/2 are padding
  // One wave per spectrum row (ix, iy), its lanes along iz (coalesced): the row's
  // coordinates are computed once, not recovered per mode by divisions.  Each thread's
  // runs of the same bin are merged in registers.
  const int lane = threadIdx.x & 63, waves = blockDim.x >> 6;
  const int nrows = n * n;
  int cur = -1;
  double ap = 0.0, ak = 0.0;
  unsigned long long ac = 0;
  for (int row = blockIdx.x * waves + (threadIdx.x >> 6); row < nrows; row += gridDim.x * waves) {
    const int ix = row / n, iy = row - ix * n;
    const int nx = signed_freq(ix, n), ny = signed_freq(iy, n);
    const int64_t nxy2 = (int64_t)nx * nx + (int64_t)ny * ny;
    const cx<T>* drow = dhat + (int64_t)row * h;
    const cx<T>* brow = CROSS ? bhat + (int64_t)row * h : nullptr;
    for (int iz = lane; iz <= n / 2; iz += 64) {
      const int64_t n2 = nxy2 + (int64_t)iz * iz;
      const int b = n2 > 0 ? pk_bin(n2, n, nb) : -1;
      if (b < 0) continue;
      const int wgt = (iz == 0 || iz == n / 2) ? 1 : 2;
      const cx<T> v = ldc(drow + iz);
      double p2;
      if (CROSS) {
        const cx<T> u = ldc(brow + iz);
        p2 = (double)v.x * u.x + (double)v.y * u.y;
      } else {
        p2 = (double)v.x * v.x + (double)v.y * v.y;
      }
      if (b != cur) {
        if (cur >= 0) {
          atomicAdd(&sp[cur], ap);
          atomicAdd(&sk[cur], ak);
          atomicAdd(&sc[cur], ac);
        }
        cur = b;
        ap = ak = 0.0;
        ac = 0;
      }
      ap += wgt * p2;
      ak += wgt * sqrt((double)n2);
      ac += (unsigned long long)wgt;
    }
  }
  if (cur >= 0) {
    atomicAdd(&sp[cur], ap);
    atomicAdd(&sk[cur], ak);
    atomicAdd(&sc[cur], ac);
  }
  __syncthreads();
  unsigned long long* gc = reinterpret_cast<unsigned long long*>(sums + 2 * nb);
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    if (sc[b] == 0ull) continue;
    atomicAdd(&sums[b], sp[b]);
    atomicAdd(&sums[nb + b], sk[b]);
    atomicAdd(&gc[b], sc[b]);
  }
}

__global__ void k_pk_finalize(const double* __restrict__ sums, int nb, int n, double box, double* __restrict__ k_mean,
                              double* __restrict__ pk, int64_t* __restrict__ n_modes) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  sums += (int64_t)blockIdx.y * 3 * nb;  // box of the batch
  k_mean += (int64_t)blockIdx.y * nb;
  pk += (int64_t)blockIdx.y * nb;
  n_modes += (int64_t)blockIdx.y * nb;
  const unsigned long long c = reinterpret_cast<const unsigned long long*>(sums + 2 * nb)[b];
  const double kf = 2.0 * kPi / box;
  const double vol = box * box * box;
  const double n6 = (double)n * n * n * (double)n * n * n;
  k_mean[b] = c ? kf * sums[nb + b] / (double)c : 0.0;
  pk[b] = c ? vol / n6 * sums[b] / (double)c : 0.0;
  n_modes[b] = (int64_t)c;
}

// Cotangent of the binned power spectrum pulled back to the spectrum:
// dhat(n) <- beta_b dhat(n), beta_b = 2 V dP_b / (N^6 count_b) for the bin b of n and
// 0 outside every bin (P_b is a quadratic form in dhat; the factor 2 and the full-cube
// count come from summing |dhat|^2 over n and -n).  Counts are those left in `sums` by
// the reduction of the same spectrum.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_pk_adjoint_weight(cx<T>* __restrict__ dhat, int n, int hp, int nb,
                                                              const double* __restrict__ sums,
                                                              const double* __restrict__ dpk, double coef) {
  const int64_t total = (int64_t)n * n * hp;
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= total) return;
  const int iz = (int)(idx % hp);
  if (iz > n / 2) return;
  const int iy = (int)((idx / hp) % n);
  const int ix = (int)(idx / ((int64_t)hp * n));
  const int nx = signed_freq(ix, n), ny = signed_freq(iy, n);
  const int64_t n2 = (int64_t)nx * nx + (int64_t)ny * ny + (int64_t)iz * iz;
  const int b = n2 > 0 ? pk_bin(n2, n, nb) : -1;
  double beta = 0.0;
  if (b >= 0) {
    const unsigned long long c = reinterpret_cast<const unsigned long long*>(sums + 2 * nb)[b];
    beta = c ? coef * dpk[b] / (double)c : 0.0;
  }
  const cx<T> v = ldc(dhat + idx);
  stc(dhat + idx, mk(T(beta * (double)v.x), T(beta * (double)v.y)));
}

// Coarse spectrum from a fine one on the natural layouts: coarse mode n (signed, all
// |n_i| < Nc/2) takes fine mode n times `scale`; the coarse Nyquist planes are zero.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_truncate_spectrum(const cx<T>* __restrict__ fine, int nf, int hpf,
                                                              cx<T>* __restrict__ coarse, int nc, int hpc, T scale) {
  const int64_t total = (int64_t)nc * nc * hpc;
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= total) return;
  const int iz = (int)(idx % hpc);
  if (iz > nc / 2) return;
  const int iy = (int)((idx / hpc) % nc);
  const int ix = (int)(idx / ((int64_t)hpc * nc));
  const int nx = signed_freq(ix, nc), ny = signed_freq(iy, nc);
  cx<T> v = mk(T(0), T(0));
  if (nx != -nc / 2 && ny != -nc / 2 && iz != nc / 2) {
    const int fx = nx < 0 ? nx + nf : nx, fy = ny < 0 ? ny + nf : ny;
    const cx<T> w = ldc(fine + ((int64_t)fx * nf + fy) * hpf + iz);
    v = mk(w.x * scale, w.y * scale);
  }
  stc(coarse + idx, v);
}

// Paired-and-fixed noise: every stored mode keeps its phase and takes the modulus
// `target` (N^(3/2) times the inverse transform's 1/N^3); exact zeros stay zero.
// Box b of the batch is negated when `negate_mask` has its bit (b & 1) set
// (bit 0: even boxes, bit 1: odd boxes).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fix_spectrum(cx<T>* __restrict__ c, int n, int hp, int64_t cs,
                                                         double target, int negate_mask) {
  const int64_t total = (int64_t)n * n * hp;
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= total) return;
  if ((int)(idx % hp) > n / 2) return;
  c += (int64_t)blockIdx.y * cs;
  const cx<T> v = ldc(c + idx);
  const double re = (double)v.x, im = (double)v.y;
  const double m = sqrt(re * re + im * im);
  double f = m > 0.0 ? target / m : 0.0;
  if ((negate_mask >> (blockIdx.y & 1)) & 1) f = -f;
  stc(c + idx, mk(T(re * f), T(im * f)));
}

// One pass over up to four shell fields accumulating up to four triangle sums
// sum_x f_a f_b f_c (FP64 products and sums of the fields' values); each thread reads
// 16-byte vectors of every field.  count is a multiple of the vector width.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_triple_multi(TriPass tp, int64_t count) {
  constexpr int VW = 16 / (int)sizeof(T);
  typedef T vec_t __attribute__((ext_vector_type(VW)));
  __shared__ double red[kMaxTriPerPass][kBlock / 64];
  double acc[kMaxTriPerPass] = {0.0, 0.0, 0.0, 0.0};
  const int64_t nvec = count / VW;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += stride) {
    vec_t v[kMaxFieldsPerPass];
#pragma unroll
    for (int f = 0; f < kMaxFieldsPerPass; ++f)
      v[f] = f < tp.nf ? reinterpret_cast<const vec_t*>(tp.field[f])[i] : vec_t(T(0));
#pragma unroll
    for (int t = 0; t < kMaxTriPerPass; ++t) {
      if (t >= tp.nt) break;
      const int ia = tp.idx[t][0], ib = tp.idx[t][1], ic = tp.idx[t][2];
      // the indices are uniform: selects, not dynamic register indexing
      const vec_t a = ia == 0 ? v[0] : (ia == 1 ? v[1] : (ia == 2 ? v[2] : v[3]));
      const vec_t b = ib == 0 ? v[0] : (ib == 1 ? v[1] : (ib == 2 ? v[2] : v[3]));
      const vec_t c = ic == 0 ? v[0] : (ic == 1 ? v[1] : (ic == 2 ? v[2] : v[3]));
#pragma unroll
      for (int e = 0; e < VW; ++e) acc[t] += (double)a[e] * (double)b[e] * (double)c[e];
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < kMaxTriPerPass; ++t) {
    double v = acc[t];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[t][wave] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < tp.nt) {
    const int t = threadIdx.x;
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) v += red[t][w];
    atomicAdd(tp.slot[t], v);
  }
}

__global__ void k_bk_finalize(const double* __restrict__ sums, int n_tri, int n, double box, double* __restrict__ bk,
                              double* __restrict__ ntri_out, const double* __restrict__ ntri_known) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tri) return;
  // sums[t]: sum_x d_a d_b d_c with fields scaled to the unnormalised inverse (x N^3 each);
  // sums[n_tri + t]: same for the indicator fields, unless ntri_known is given.
  const double n3 = (double)n * n * n;
  const double n9 = n3 * n3 * n3;
  const double ntri = ntri_known ? ntri_known[t] : sums[n_tri + t] / n3;  // N^6 sum_x I I I (I = IDFT(1_S))
  const double num = sums[t] / (n3 * n3 * n3);                             // sum_x d d d (d = IDFT(...))
  const double den = ntri / (n3 * n3);
  const double vol = box * box * box;
  bk[t] = den != 0.0 ? vol * vol / n9 * num / den : 0.0;
  ntri_out[t] = ntri;
}

__global__ void k_zero_d(double* __restrict__ d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = 0.0;
}

}  // namespace

int launch_ic_symbol(const pm_plan* p, const IcSymbol& sym, bool adjoint, hipStream_t s) {
  ProfScope ps(p, PK_IC, s);
  const int n = p->n;
  const int64_t total = (int64_t)n * n * p->hp;
  const dim3 g((unsigned)((total + kBlock - 1) / kBlock), (unsigned)p->nb);
  const int64_t cs = cstride(p);
  cx<float>* f[3] = {static_cast<cx<float>*>(cbuf(p, 0)), static_cast<cx<float>*>(cbuf(p, 1)),
                     static_cast<cx<float>*>(cbuf(p, 2))};
  cx<double>* d[3] = {static_cast<cx<double>*>(cbuf(p, 0)), static_cast<cx<double>*>(cbuf(p, 1)),
                      static_cast<cx<double>*>(cbuf(p, 2))};
  if (p->dtype == PM_F32 && adjoint)
    hipLaunchKernelGGL((k_ic_symbol<float, true>), g, dim3(kBlock), 0, s, f[0], f[1], f[2], n, p->hp, cs, sym);
  else if (p->dtype == PM_F32)
    hipLaunchKernelGGL((k_ic_symbol<float, false>), g, dim3(kBlock), 0, s, f[0], f[1], f[2], n, p->hp, cs, sym);
  else if (adjoint)
    hipLaunchKernelGGL((k_ic_symbol<double, true>), g, dim3(kBlock), 0, s, d[0], d[1], d[2], n, p->hp, cs, sym);
  else
    hipLaunchKernelGGL((k_ic_symbol<double, false>), g, dim3(kBlock), 0, s, d[0], d[1], d[2], n, p->hp, cs, sym);
  return hip_check(hipGetLastError(), "ic symbol");
}

int launch_fix_spectrum(const pm_plan* p, double target, int negate_mask, hipStream_t s) {
  ProfScope ps(p, PK_IC, s);
  const int n = p->n;
  const int64_t total = (int64_t)n * n * p->hp;
  const dim3 g((unsigned)((total + kBlock - 1) / kBlock), (unsigned)p->nb);
  if (p->dtype == PM_F32)
    hipLaunchKernelGGL(k_fix_spectrum<float>, g, dim3(kBlock), 0, s, static_cast<cx<float>*>(cbuf(p, 0)), n, p->hp,
                       cstride(p), target, negate_mask);
  else
    hipLaunchKernelGGL(k_fix_spectrum<double>, g, dim3(kBlock), 0, s, static_cast<cx<double>*>(cbuf(p, 0)), n,
                       p->hp, cstride(p), target, negate_mask);
  return hip_check(hipGetLastError(), "fix spectrum");
}

int launch_zero_doubles(double* d, int64_t n, hipStream_t s) {
  if (n <= 0) return PM_OK;
  hipLaunchKernelGGL(k_zero_d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, n);
  return hip_check(hipGetLastError(), "zero");
}

int launch_pk_reduce(const pm_plan* p, const void* dhat, int n_bins, hipStream_t s, const void* bhat) {
  ProfScope ps(p, PK_PK, s);
  const int n = p->n;
  const int64_t total = (int64_t)n * n * p->hp;
  int64_t g = (total + kBlock * 16 - 1) / (kBlock * 16);  // ~16 modes per thread
  if (g < 1) g = 1;
  if (g > 65535) g = 65535;
  const size_t shm = (size_t)n_bins * 3 * sizeof(double);
  const dim3 grid((unsigned)g, (unsigned)p->nb);
  if (p->dtype == PM_F32) {
    auto kern = bhat ? k_pk_reduce<float, true> : k_pk_reduce<float, false>;
    hipLaunchKernelGGL(kern, grid, dim3(kBlock), shm, s, static_cast<const cx<float>*>(dhat),
                       static_cast<const cx<float>*>(bhat), n, p->hp, cstride(p), n_bins, p->sums);
  } else {
    auto kern = bhat ? k_pk_reduce<double, true> : k_pk_reduce<double, false>;
    hipLaunchKernelGGL(kern, grid, dim3(kBlock), shm, s, static_cast<const cx<double>*>(dhat),
                       static_cast<const cx<double>*>(bhat), n, p->hp, cstride(p), n_bins, p->sums);
  }
  return hip_check(hipGetLastError(), "pk reduce");
}

int launch_pk_finalize(const pm_plan* p, int n_bins, double* k_mean, double* pk, int64_t* n_modes, hipStream_t s) {
  ProfScope ps(p, PK_PK, s);
  hipLaunchKernelGGL(k_pk_finalize, dim3((unsigned)((n_bins + 63) / 64), (unsigned)p->nb), dim3(64), 0, s, p->sums,
                     n_bins, p->n, p->box,
                     k_mean, pk, n_modes);
  return hip_check(hipGetLastError(), "pk finalize");
}

int launch_pk_adjoint_weight(const pm_plan* p, void* dhat, int n_bins, const double* dpk, hipStream_t s) {
  ProfScope ps(p, PK_PK, s);
  const int n = p->n;
  const int64_t total = (int64_t)n * n * p->hp;
  const unsigned g = (unsigned)((total + kBlock - 1) / kBlock);
  const double n3 = (double)n * n * n;
  const double coef = 2.0 * p->box * p->box * p->box / (n3 * n3);
  if (p->dtype == PM_F32)
    hipLaunchKernelGGL(k_pk_adjoint_weight<float>, dim3(g), dim3(kBlock), 0, s, static_cast<cx<float>*>(dhat), n,
                       p->hp, n_bins, p->sums, dpk, coef);
  else
    hipLaunchKernelGGL(k_pk_adjoint_weight<double>, dim3(g), dim3(kBlock), 0, s, static_cast<cx<double>*>(dhat), n,
                       p->hp, n_bins, p->sums, dpk, coef);
  return hip_check(hipGetLastError(), "pk adjoint weight");
}

int launch_truncate_spectrum(const pm_plan* fine, const pm_plan* coarse, hipStream_t s) {
  ProfScope ps(coarse, PK_IC, s);
  const int nc = coarse->n, nf = fine->n;
  const int64_t total = (int64_t)nc * nc * coarse->hp;
  const unsigned g = (unsigned)((total + kBlock - 1) / kBlock);
  // (Nc/Nf)^(3/2) keeps the physical field on the shared modes; 1/Nc^3 is the inverse transform's
  const double scale = std::pow((double)nc / nf, 1.5) / ((double)nc * nc * nc);
  if (fine->dtype == PM_F32)
    hipLaunchKernelGGL(k_truncate_spectrum<float>, dim3(g), dim3(kBlock), 0, s,
                       static_cast<const cx<float>*>(cbuf(fine, 0)), nf, fine->hp,
                       static_cast<cx<float>*>(cbuf(coarse, 0)), nc, coarse->hp, (float)scale);
  else
    hipLaunchKernelGGL(k_truncate_spectrum<double>, dim3(g), dim3(kBlock), 0, s,
                       static_cast<const cx<double>*>(cbuf(fine, 0)), nf, fine->hp,
                       static_cast<cx<double>*>(cbuf(coarse, 0)), nc, coarse->hp, scale);
  return hip_check(hipGetLastError(), "truncate spectrum");
}

int launch_triple_multi(const pm_plan* p, const TriPass& tp, hipStream_t s) {
  ProfScope ps(p, PK_BK, s);
  const int64_t count = (int64_t)p->n * p->n * p->n;
  const int vw = p->dtype == PM_F32 ? 4 : 2;
  int64_t g = (count / vw + kBlock * 16 - 1) / (kBlock * 16);
  g = std::max<int64_t>(1, std::min<int64_t>(g, 8192));
  if (p->dtype == PM_F32)
    hipLaunchKernelGGL(k_triple_multi<float>, dim3((unsigned)g), dim3(kBlock), 0, s, tp, count);
  else
    hipLaunchKernelGGL(k_triple_multi<double>, dim3((unsigned)g), dim3(kBlock), 0, s, tp, count);
  return hip_check(hipGetLastError(), "triple sums");
}

int launch_bk_finalize(const pm_plan* p, int n_tri, const double* sums, double* bk, double* ntri_out,
                       const double* ntri_known, hipStream_t s) {
  ProfScope ps(p, PK_BK, s);
  hipLaunchKernelGGL(k_bk_finalize, dim3((unsigned)((n_tri + 63) / 64)), dim3(64), 0, s, sums, n_tri, p->n, p->box, bk,
                     ntri_out, ntri_known);
  return hip_check(hipGetLastError(), "bk finalize");
}

}  // namespace pm
