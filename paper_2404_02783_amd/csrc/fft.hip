// Launchers of the hand-written FFT passes (see fft_kernels.h).
#include <algorithm>

#include "fft_kernels.h"
#include "pm_plan.h"

namespace pm {

namespace {

template <typename T>
int cols_per_block(int n) {
  const Shape sh = shape_for(n);
  const int tpc = std::max(sh.L1, sh.L2);
  int b = 256 / tpc;
  const int by_lds = 65536 / (n * (int)sizeof(cx<T>));
  b = std::min(b, std::max(by_lds, 1));
  const int h = n / 2 + 1;
  int cap = 1;
  while (cap < h) cap <<= 1;
  b = std::min(b, cap);
  int p2 = 1;
  while (p2 * 2 <= b) p2 <<= 1;
  return p2;
}

template <typename T, int L1, int L2>
void launch_cols_t(cx<T>* data, const ColArgs& g, int dir, int ncomp, int outer, const cx<T>* tw, hipStream_t s) {
  const int tpc = std::max(L1, L2);
  dim3 grid((unsigned)(outer * g.groups), (unsigned)ncomp);
  dim3 block((unsigned)(g.bcols * tpc));
  size_t shm = (size_t)L1 * L2 * g.bcols * sizeof(cx<T>);
  if (dir < 0)
    hipLaunchKernelGGL((k_fft_cols<T, L1, L2, -1>), grid, block, shm, s, data, g, tw);
  else
    hipLaunchKernelGGL((k_fft_cols<T, L1, L2, 1>), grid, block, shm, s, data, g, tw);
}

template <typename T, int L1, int L2>
void launch_r2c_t(const T* in, cx<T>* out, const RowArgs& g, int ncomp, const cx<T>* tw, int rows, hipStream_t s) {
  constexpr int M = L1 * L2;
  constexpr int TPC = L1 > L2 ? L1 : L2;
  constexpr int XS = L1 * (L2 + 1);
  constexpr int RS = XS > M ? XS : M;
  const int R = rows > 0 ? rows : 256 / TPC;
  dim3 grid((unsigned)((g.nrows + R - 1) / R), (unsigned)ncomp);
  dim3 block((unsigned)(R * TPC));
  hipLaunchKernelGGL((k_fft_rows_r2c<T, L1, L2>), grid, block, (size_t)R * RS * sizeof(cx<T>), s, in, out, g, tw);
}

template <typename T, int L1, int L2, int MODE = C2R_PLAIN>
void launch_c2r_t(const cx<T>* in, T* out, const RowArgs& g, int ncomp, const cx<T>* tw, int rows, hipStream_t s) {
  constexpr int M = L1 * L2;
  constexpr int TPC = L1 > L2 ? L1 : L2;
  constexpr int XS = L1 * (L2 + 1);
  (void)M;
  const int R = rows > 0 ? rows : 256 / TPC;
  dim3 grid((unsigned)((g.nrows + R - 1) / R), (unsigned)ncomp);
  dim3 block((unsigned)(R * TPC));
  hipLaunchKernelGGL((k_fft_rows_c2r<T, L1, L2, MODE>), grid, block, (size_t)R * XS * sizeof(cx<T>), s, in, out, g,
                     tw);
}

template <typename T, int L1, int L2>
void launch_c2r_force_t(const cx<T>* in, T* out, const RowArgs& g, int ncomp, const cx<T>* tw, int rows,
                        hipStream_t s) {
  launch_c2r_t<T, L1, L2, C2R_FORCE>(in, out, g, ncomp, tw, rows, s);
}

template <typename T, int L1, int L2>
void launch_cols_gform_t(cx<T>* data, const ColArgs& g, int nbox, int n, int grad, int outer, const cx<T>* tw,
                         hipStream_t s) {
  const int tpc = std::max(L1, L2);
  size_t shm = (size_t)L1 * L2 * g.bcols * sizeof(cx<T>);
  hipLaunchKernelGGL((k_fft_cols_gform<T, L1, L2>), dim3((unsigned)(outer * g.groups), (unsigned)(2 * nbox)),
                     dim3((unsigned)(g.bcols * tpc)), shm, s, data, g, nbox, n, grad, tw);
}

template <typename T, int L1, int L2>
void launch_c2r_zmask_t(const cx<T>* in, T* out, const RowArgs& g, int ncomp, const cx<T>* tw, int rows,
                        hipStream_t s) {
  launch_c2r_t<T, L1, L2, C2R_ZMASK>(in, out, g, ncomp, tw, rows, s);
}

template <typename T, int L1, int L2>
void launch_cols_shell0_t(const cx<T>* src, cx<T>* dst, const ColArgs& g, const ShellArgs& sh, int outer,
                          const cx<T>* tw, hipStream_t s) {
  const int tpc = std::max(L1, L2);
  size_t shm = (size_t)L1 * L2 * g.bcols * sizeof(cx<T>);
  hipLaunchKernelGGL((k_fft_cols_shell<T, L1, L2, 0>), dim3((unsigned)(outer * g.groups)),
                     dim3((unsigned)(g.bcols * tpc)), shm, s, src, dst, g, sh, tw);
}

template <typename T, int L1, int L2>
void launch_cols_shell1_t(cx<T>* data, const ColArgs& g, const ShellArgs& sh, int outer, const cx<T>* tw,
                          hipStream_t s) {
  const int tpc = std::max(L1, L2);
  size_t shm = (size_t)L1 * L2 * g.bcols * sizeof(cx<T>);
  hipLaunchKernelGGL((k_fft_cols_shell<T, L1, L2, 1>), dim3((unsigned)(outer * g.groups)),
                     dim3((unsigned)(g.bcols * tpc)), shm, s, static_cast<const cx<T>*>(nullptr), data, g, sh, tw);
}

template <typename T, int L1, int L2>
void launch_solve_t(cx<T>* data, cx<T>* o1, cx<T>* phi, const ColArgs& g, const SolveArgs& a, int outer,
                    const cx<T>* tw, hipStream_t s) {
  const int tpc = std::max(L1, L2);
  dim3 grid((unsigned)(outer * g.groups), (unsigned)a.nbox);
  dim3 block((unsigned)(g.bcols * tpc));
  size_t shm = (size_t)L1 * L2 * g.bcols * sizeof(cx<T>);
  // one launch: forward transform, symbol, both inverse transforms
  if (a.kind == PM_NEWTON)
    hipLaunchKernelGGL((k_fft_cols_solve<T, L1, L2, PM_NEWTON>), grid, block, shm, s, data, o1, phi, g, a, tw);
  else
    hipLaunchKernelGGL((k_fft_cols_solve<T, L1, L2, PM_POISSON_GAUGE>), grid, block, shm, s, data, o1, phi, g, a, tw);
}

#define PM_TRY_HIP(expr, what)                  \
  do {                                          \
    const int rc_ = hip_check((expr), (what));  \
    if (rc_ != PM_OK) return rc_;               \
  } while (0)

// Dispatch on a transform length L to the compile-time (L1, L2) instantiation.
#define PM_DISPATCH_LEN(L, FN, ...)                  \
  switch (L) {                                       \
    case 4: FN<T, 2, 2>(__VA_ARGS__); break;         \
    case 8: FN<T, 4, 2>(__VA_ARGS__); break;         \
    case 16: FN<T, 4, 4>(__VA_ARGS__); break;        \
    case 32: FN<T, 8, 4>(__VA_ARGS__); break;        \
    case 64: FN<T, 8, 8>(__VA_ARGS__); break;        \
    case 96: FN<T, 8, 12>(__VA_ARGS__); break;       \
    case 128: FN<T, 16, 8>(__VA_ARGS__); break;      \
    case 192: FN<T, 16, 12>(__VA_ARGS__); break;     \
    case 256: FN<T, 16, 16>(__VA_ARGS__); break;     \
    case 512: FN<T, 16, 32>(__VA_ARGS__); break;     \
    case 1024: FN<T, 32, 32>(__VA_ARGS__); break;    \
    default: return set_error(PM_ERR_SIZE, "unsupported transform length %d", (int)(L)); \
  }

// Strides of the internal spectrum [N][N][hp] (hp = padded N/2+1) for a pass along
// axis 1 (columns (ix, iz)) or axis 0 (columns (iy, iz)); N/2+1 columns are valid.
ColArgs col_args(int n, int hp, int axis, int bcols) {
  const int64_t h = n / 2 + 1;
  ColArgs g;
  g.stride = axis == 1 ? hp : (int64_t)n * hp;
  g.outer_stride = axis == 1 ? (int64_t)n * hp : hp;
  g.comp_stride = 0;
  g.ncols = (int)h;
  g.bcols = bcols;
  g.groups = (int)((h + bcols - 1) / bcols);
  g.tw_step = 1;
  return g;
}

template <typename T>
int cols_t(const pm_plan* p, void* data, int axis, int dir, int ncomp, int64_t comp_stride, hipStream_t s) {
  const int n = p->n;
  ColArgs g = col_args(n, p->hp, axis, p->tune[0] > 0 ? p->tune[0] : cols_per_block<T>(n));
  g.comp_stride = comp_stride;
  cx<T>* d = static_cast<cx<T>*>(data);
  const cx<T>* tw = static_cast<const cx<T>*>(p->tw);
  PM_DISPATCH_LEN(n, launch_cols_t, d, g, dir, ncomp, n, tw, s)
  return hip_check(hipGetLastError(), "fft column pass");
}

template <typename T>
int r2c_t(const pm_plan* p, int count, const void* in, void* out, hipStream_t s) {
  const int n = p->n;
  RowArgs g;
  g.nrows = (int64_t)n * n;
  g.in_comp = (int64_t)n * n * n;
  g.out_comp = cstride(p);
  g.n = n;
  g.hs = p->hp;
  const cx<T>* tw = static_cast<const cx<T>*>(p->tw);
  PM_DISPATCH_LEN(n / 2, launch_r2c_t, static_cast<const T*>(in), static_cast<cx<T>*>(out), g, count, tw, p->tune[2],
                  s)
  return hip_check(hipGetLastError(), "fft r2c rows");
}

template <typename T>
int c2r_t(const pm_plan* p, int ncomp, const void* in, int64_t in_comp, void* out, hipStream_t s) {
  const int n = p->n;
  RowArgs g;
  g.nrows = (int64_t)n * n;
  g.in_comp = in_comp;
  g.out_comp = (int64_t)n * n * n;
  g.n = n;
  g.hs = p->hp;
  const cx<T>* tw = static_cast<const cx<T>*>(p->tw);
  PM_DISPATCH_LEN(n / 2, launch_c2r_t, static_cast<const cx<T>*>(in), static_cast<T*>(out), g, ncomp, tw, p->tune[3],
                  s)
  return hip_check(hipGetLastError(), "fft c2r rows");
}

// Inverse transform of one shell of the spectrum `src` (or of its indicator when src
// is null) into the real mesh `out`, through the complex buffer `work`.
template <typename T>
int shell_c2r_t(const pm_plan* p, const void* src, void* work, void* out, double lo4, double hi4, hipStream_t s) {
  const int n = p->n;
  const int bc = p->tune[0] > 0 ? p->tune[0] : cols_per_block<T>(n);
  const cx<T>* tw = static_cast<const cx<T>*>(p->tw);
  ShellArgs sh;
  sh.lo4 = lo4;
  sh.hi4 = hi4;
  sh.n = n;
  cx<T>* w = static_cast<cx<T>*>(work);
  const ColArgs g0 = col_args(n, p->hp, 0, bc);
  PM_DISPATCH_LEN(n, launch_cols_shell0_t, static_cast<const cx<T>*>(src), w, g0, sh, n, tw, s)
  PM_TRY_HIP(hipGetLastError(), "shell column pass (axis 0)");
  const ColArgs g1 = col_args(n, p->hp, 1, bc);
  PM_DISPATCH_LEN(n, launch_cols_shell1_t, w, g1, sh, n, tw, s)
  PM_TRY_HIP(hipGetLastError(), "shell column pass (axis 1)");
  RowArgs g;
  g.nrows = (int64_t)n * n;
  g.in_comp = 0;
  g.out_comp = (int64_t)n * n * n;
  g.n = n;
  g.hs = p->hp;
  g.zmask4 = hi4;
  PM_DISPATCH_LEN(n / 2, launch_c2r_zmask_t, static_cast<const cx<T>*>(w), static_cast<T*>(out), g, 1, tw,
                  p->tune[3], s)
  return hip_check(hipGetLastError(), "shell c2r rows");
}

template <typename T>
int solve_t(const pm_plan* p, const pm_solve_params* sp, void* phi, hipStream_t s) {
  const int n = p->n;
  ColArgs g = col_args(n, p->hp, 0, p->tune[1] > 0 ? p->tune[1] : cols_per_block<T>(n));
  SolveArgs a;
  const double n3 = (double)n * n * n;
  a.n = n;
  a.kind = sp->kind;
  a.grad = sp->grad;
  a.newton = 1.5 * sp->omega_m / n3;
  a.a_c2 = sp->a * sp->c_g * sp->c_g / n3;
  a.h = sp->calh;
  a.h2 = sp->calh * sp->calh;
  a.om_a = sp->om_a;
  a.inv_dtau = sp->inv_dtau;
  a.nbox = p->nb;
  a.box_stride = cstride(p);
  a.phi_stride = (int64_t)n * n * (n / 2 + 1);
  cx<T>* c0 = static_cast<cx<T>*>(cbuf(p, 0));
  cx<T>* c1 = static_cast<cx<T>*>(cbuf(p, 1));
  const cx<T>* tw = static_cast<const cx<T>*>(p->tw);
  PM_DISPATCH_LEN(n, launch_solve_t, c0, c1, static_cast<cx<T>*>(phi), g, a, n, tw, s)
  return hip_check(hipGetLastError(), "fft solve pass");
}

// Launch shapes of tuning slot `kind` that stay within the kernels' limits: at most
// 256 threads per workgroup (their launch bounds) and 64 KiB of LDS, columns per
// workgroup no more than the next power of two above the N/2+1 columns.
template <typename T>
int tune_candidates_t(const pm_plan* p, int kind, int* out, int cap) {
  const int n = p->n;
  const size_t cxs = sizeof(cx<T>);
  int cnt = 0;
  auto push = [&](int v) {
    if (cnt < cap) out[cnt] = v;
    ++cnt;
  };
  if (kind == 0 || kind == 1) {
    const Shape sh = shape_for(n);
    const int tpc = std::max(sh.L1, sh.L2);
    const int h = n / 2 + 1;
    int colcap = 1;
    while (colcap < h) colcap <<= 1;
    for (int b = 1; b * tpc <= 256 && b <= colcap; b <<= 1)
      if ((size_t)sh.L1 * sh.L2 * b * cxs <= 65536) push(b);
  } else {
    const Shape sh = shape_for(n / 2);
    const int tpc = std::max(sh.L1, sh.L2);
    const int xs = sh.L1 * (sh.L2 + 1);
    const int rs = kind == 2 ? std::max(xs, sh.L) : xs;
    const int def = 256 / tpc;  // the built-in choice (not always a power of two)
    bool def_done = false;
    for (int r = 1; r * tpc <= 256; r <<= 1) {
      if (!def_done && def < r) {
        push(def);
        def_done = true;
      }
      if (r == def) def_done = true;
      if ((size_t)r * rs * cxs <= 65536 || r == def) push(r);
    }
    if (!def_done) push(def);
  }
  return cnt;
}

}  // namespace

int fft_tune_default(const pm_plan* p, int kind) {
  if (kind == 0 || kind == 1) return p->dtype == PM_F32 ? cols_per_block<float>(p->n) : cols_per_block<double>(p->n);
  const Shape sh = shape_for(p->n / 2);
  return 256 / std::max(sh.L1, sh.L2);
}

int fft_tune_candidates(const pm_plan* p, int kind, int* out, int cap) {
  if (kind < 0 || kind > 3) return 0;
  return p->dtype == PM_F32 ? tune_candidates_t<float>(p, kind, out, cap) : tune_candidates_t<double>(p, kind, out, cap);
}

int fft_pass_cols(const pm_plan* p, void* data, int axis, int dir, int ncomp, int64_t comp_stride, hipStream_t s) {
  const int kind = axis == 1 ? (dir < 0 ? PK_COLS_FWD_AXIS1 : PK_COLS_INV_AXIS1)
                             : (dir < 0 ? PK_COLS_FWD_AXIS0 : PK_COLS_INV_AXIS0);
  ProfScope ps(p, kind, s);
  return p->dtype == PM_F32 ? cols_t<float>(p, data, axis, dir, ncomp, comp_stride, s)
                            : cols_t<double>(p, data, axis, dir, ncomp, comp_stride, s);
}

int fft_pass_rows_r2c(const pm_plan* p, int count, const void* in, void* out, hipStream_t s) {
  ProfScope ps(p, PK_R2C_ROWS, s);
  return p->dtype == PM_F32 ? r2c_t<float>(p, count, in, out, s) : r2c_t<double>(p, count, in, out, s);
}

int fft_pass_rows_c2r(const pm_plan* p, int ncomp, const void* in, int64_t in_comp, void* out, hipStream_t s) {
  ProfScope ps(p, PK_C2R_ROWS, s);
  return p->dtype == PM_F32 ? c2r_t<float>(p, ncomp, in, in_comp, out, s) : c2r_t<double>(p, ncomp, in, in_comp, out, s);
}

// Inverse passes of the solve's G form: along axis 1 (F_x in place; G read once, D_y G
// to the third region and G in place), then the rows to the three real force meshes
// [3][nb][N^3] with D_z applied to the transformed G on load.
template <typename T>
int force_inverse_t(const pm_plan* p, int grad, void* force, hipStream_t s) {
  const int n = p->n;
  const cx<T>* tw = static_cast<const cx<T>*>(p->tw);
  ColArgs g = col_args(n, p->hp, 1, p->tune[0] > 0 ? p->tune[0] : cols_per_block<T>(n));
  g.comp_stride = cstride(p);
  {
    ProfScope ps(p, PK_COLS_INV_AXIS1, s);
    PM_DISPATCH_LEN(n, launch_cols_gform_t, static_cast<cx<T>*>(cbuf(p, 0)), g, p->nb, n, grad, n, tw, s)
    PM_TRY_HIP(hipGetLastError(), "fft column pass (G form)");
  }
  ProfScope ps(p, PK_C2R_ROWS, s);
  RowArgs r;
  r.nrows = (int64_t)n * n;
  r.in_comp = cstride(p);
  r.out_comp = (int64_t)n * n * n;
  r.n = n;
  r.hs = p->hp;
  r.zmask4 = 0.0;
  r.nbox = p->nb;
  r.grad = grad;
  PM_DISPATCH_LEN(n / 2, launch_c2r_force_t, static_cast<const cx<T>*>(cbuf(p, 0)), static_cast<T*>(force), r,
                  3 * p->nb, tw, p->tune[3], s)
  return hip_check(hipGetLastError(), "fft c2r rows (force)");
}

int fft3_c2r_shell(const pm_plan* p, const void* src, void* work, void* out, double lo4, double hi4, hipStream_t s) {
  ProfScope ps(p, PK_BK, s);
  return p->dtype == PM_F32 ? shell_c2r_t<float>(p, src, work, out, lo4, hi4, s)
                            : shell_c2r_t<double>(p, src, work, out, lo4, hi4, s);
}

int fft_force_inverse(const pm_plan* p, int grad, void* force, hipStream_t s) {
  return p->dtype == PM_F32 ? force_inverse_t<float>(p, grad, force, s) : force_inverse_t<double>(p, grad, force, s);
}

int fft_pass_solve(const pm_plan* p, const pm_solve_params* sp, void* phi, hipStream_t s) {
  ProfScope ps(p, PK_SOLVE_AXIS0, s);
  return p->dtype == PM_F32 ? solve_t<float>(p, sp, phi, s) : solve_t<double>(p, sp, phi, s);
}

int fft3_r2c_n(const pm_plan* p, int count, const void* real_in, void* cplx_out, hipStream_t s) {
  int rc = fft_pass_rows_r2c(p, count, real_in, cplx_out, s);
  if (rc) return rc;
  rc = fft_pass_cols(p, cplx_out, 1, -1, count, cstride(p), s);
  if (rc) return rc;
  return fft_pass_cols(p, cplx_out, 0, -1, count, cstride(p), s);
}

int fft3_r2c(const pm_plan* p, const void* real_in, void* cplx_out, hipStream_t s) {
  return fft3_r2c_n(p, p->nb, real_in, cplx_out, s);
}

int fft3_c2r(const pm_plan* p, int ncomp, void* cplx_in, int64_t comp_stride, void* real_out, hipStream_t s) {
  int rc = fft_pass_cols(p, cplx_in, 0, 1, ncomp, comp_stride, s);
  if (rc) return rc;
  rc = fft_pass_cols(p, cplx_in, 1, 1, ncomp, comp_stride, s);
  if (rc) return rc;
  return fft_pass_rows_c2r(p, ncomp, cplx_in, comp_stride, real_out, s);
}

}  // namespace pm
