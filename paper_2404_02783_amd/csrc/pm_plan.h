// Plan object and internal launch entry points of the pmhip library.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/pmhip.h"

namespace pm {
// Largest batch of equal-size boxes in one plan (grid.y of the batched launches).
constexpr int kMaxBatch = 4096;
// Kernel kinds timed by the optional per-plan profiler.
enum ProfKind {
  PK_FILL = 0,
  PK_DEPOSIT,
  PK_R2C_ROWS,
  PK_COLS_FWD_AXIS1,
  PK_COLS_FWD_AXIS0,
  PK_SOLVE_AXIS0,
  PK_COLS_INV_AXIS0,
  PK_COLS_INV_AXIS1,
  PK_C2R_ROWS,
  PK_GATHER,
  PK_GATHER_KDK,
  PK_GATHER_KDK_DEPOSIT,
  PK_COMBINE,
  PK_IC,
  PK_PK,
  PK_BK,
  PK_ADJ_GATHER,
  PK_ADJ_DEPOSIT,
  PK_GRAD_GATHER,
  PK_ADJ_SYMBOL,
  PK_COUNT
};
struct ProfState;
struct BoxEntry;
}  // namespace pm

struct pm_plan {
  pm::ProfState* prof;  // null unless profiling is enabled
  int n;             // mesh cells per axis
  int nb;            // boxes of the batch (all of side n), >= 1
  int dtype;         // PM_F32 | PM_F64
  double box;        // Mpc/h
  size_t esize;      // sizeof(real)
  void* ws;          // workspace: three regions of nb [N][N][hp] complex spectra, then
                     // the density meshes [nb][N^3] (real)
  size_t ws_bytes;
  size_t cbytes;     // bytes of one complex buffer (256-byte aligned)
  int hp;            // row stride of the internal spectra (padded N/2+1)
  bool own_ws;
  void* tw;          // device twiddle table W_N^m, m < N, complex of the plan's type
  unsigned* guard;   // device counters: [0] non-finite positions, [1] wrapped positions
  double* sums;      // device reduction scratch (estimators)
  size_t sums_cap;   // doubles in `sums`
  int device;
  // density of which positions the second workspace region holds (left by a
  // pm_step with PM_STEP_DEPOSIT_NEXT); any other use of the workspace clears it
  const void* dens_pos;
  int64_t dens_np;
  bool dens_valid;
  // launch shapes of the FFT passes picked by pm_plan_autotune (0: built-in choice):
  // [0] columns per workgroup of the plain column passes, [1] of the fused solve pass,
  // [2] rows per workgroup of the r2c rows pass, [3] of the c2r rows pass
  int tune[4];
  // device table of the boxes' particle arrays (a pm_batch size group), or null: the
  // particle kernels then take box b's arrays at b * 3 N^3 from the pointers passed
  const pm::BoxEntry* box_tab;
  // the density meshes [nb][N^3] (in the workspace after the spectra) that pm_step
  // hands from one cycle to the next
  void* dens;
};

namespace pm {

// Error helpers (api.cpp)
int set_error(int code, const char* fmt, ...);
int hip_check(hipError_t e, const char* what);

// Region i (0..2) of the workspace: nb spectra of cbytes each, box b at + b * cbytes.
inline void* cbuf(const pm_plan* p, int i) {
  return static_cast<char*>(p->ws) + (size_t)i * (size_t)p->nb * p->cbytes;
}
// Complex elements between consecutive spectra of the workspace.
inline int64_t cstride(const pm_plan* p) { return (int64_t)(p->cbytes / (2 * p->esize)); }

// Records a start/stop HIP event pair around the launches in its scope when the
// plan's profiler is on (api.cpp).
void prof_begin(const pm_plan* p, int kind, hipStream_t s);
void prof_end(const pm_plan* p, hipStream_t s);
struct ProfScope {
  const pm_plan* p;
  hipStream_t s;
  ProfScope(const pm_plan* plan, int kind, hipStream_t stream) : p(plan), s(stream) {
    if (p && p->prof) prof_begin(p, kind, s);
  }
  ~ProfScope() {
    if (p && p->prof) prof_end(p, s);
  }
};

// ---------------------------------------------------------------- api.cpp --
// The launches of one force-kick-drift cycle of pm_step on all of the plan's boxes
// (arguments checked, density bookkeeping left to the caller).
int step_cycle(pm_plan* p, void* pos, void* mom, int64_t np, const pm_step_params* st, void* force_scratch,
               void* phi_state, hipStream_t s);

// ---------------------------------------------------------------- fft.hip --
// Forward 3-D r2c of the plan's nb boxes: real [nb][N][N][N] -> complex [nb][N][N][hp]
// spaced cstride apart (unnormalised).
int fft3_r2c(const pm_plan* p, const void* real_in, void* cplx_out, hipStream_t s);
// Same for `count` boxes (1 <= count <= nb).
int fft3_r2c_n(const pm_plan* p, int count, const void* real_in, void* cplx_out, hipStream_t s);
// Inverse 3-D c2r of `ncomp` spectra spaced comp_stride complex elements apart
// (destroyed) -> ncomp real meshes spaced N^3 apart (unnormalised: N^3 times the
// inverse DFT).
int fft3_c2r(const pm_plan* p, int ncomp, void* cplx_in, int64_t comp_stride, void* real_out, hipStream_t s);
// Inverse 3-D transform of the shell lo4 <= 4|n|^2 < hi4 of the spectrum `src`
// ([N][N][hp], unchanged; null: the shell's indicator) into the real mesh `out`
// (unnormalised), through the complex buffer `work` (overwritten); only the columns
// and coefficients the shell can reach are transformed.
int fft3_c2r_shell(const pm_plan* p, const void* src, void* work, void* out, double lo4, double hi4, hipStream_t s);
// Forward column pass along axis 0 only (used after r2c rows + axis-1 pass).
int fft_pass_cols(const pm_plan* p, void* data, int axis, int dir, int ncomp, int64_t comp_stride, hipStream_t s);
int fft_pass_rows_r2c(const pm_plan* p, int count, const void* in, void* out, hipStream_t s);
int fft_pass_rows_c2r(const pm_plan* p, int ncomp, const void* in, int64_t in_comp, void* out, hipStream_t s);
// Fused solve pass along axis 0 on cbuf(0) (all nb boxes): writes the F_x spectrum
// in place and that of G (the potential times its prefactor) to cbuf 1, both
// transformed back along axis 0; phi_state holds nb unpadded [N][N][N/2+1] potentials.
int fft_pass_solve(const pm_plan* p, const pm_solve_params* sp, void* phi_state, hipStream_t s);
// After fft_pass_solve: the inverse passes along axis 1 and the rows that turn its
// output (F_x and G spectra in the first two regions; the third is scratch) into the
// three real force meshes [3][nb][N^3], with the gradient symbols D_y, D_z applied.
int fft_force_inverse(const pm_plan* p, int grad, void* force, hipStream_t s);

// ---------------------------------------------------------- particles.hip --
int launch_fill(const pm_plan* p, void* mesh, int64_t count, double value, hipStream_t s);
int launch_deposit(const pm_plan* p, const void* pos, int64_t np, void* mesh, hipStream_t s);
int launch_gather(const pm_plan* p, const void* force, const void* pos, int64_t np, void* acc, hipStream_t s);
// Gather + kick + drift; with dens non-NULL (pre-filled with -1; requires
// gather_kdk_can_deposit) the new positions are also deposited into it.
int launch_gather_kdk(const pm_plan* p, const void* force, void* pos, void* mom, int64_t np, double kick,
                      double drift, void* dens, hipStream_t s);
bool gather_kdk_can_deposit(const pm_plan* p, int64_t np);
int launch_combine(const void* x_gr, const void* x_n, int nc, const void* x_f, int nf, int dtype, void* x_out,
                   hipStream_t s);
int launch_ic_lattice(const pm_plan* p, const void* disp, void* pos, void* mom, double mom_factor, hipStream_t s);
int launch_ic_gauge_lattice(const pm_plan* p, const void* xi, const void* pos_n, const void* mom_n, void* pos_gr,
                            void* mom_gr, double mom_factor, hipStream_t s);
// Second-order source from three Hessian components h ([3][N^3]):
// pass 0: s = h0 h1 + h0 h2 + h1 h2; pass 1: s -= h0^2 + h1^2 + h2^2.
int launch_lpt2_source(const pm_plan* p, const void* h, void* s_out, int pass, hipStream_t s);
// pos = wrap(q + 1/2 + psi1 + psi2), mom = f1 psi1 + f2 psi2 (psi2 may alias mom).
int launch_ic_lattice2(const pm_plan* p, const void* psi1, const void* psi2, void* pos, void* mom, double f1,
                       double f2, hipStream_t s);

// Launch shapes the FFT passes accept for tuning slot `kind` (see pm_plan::tune),
// ascending; returns their number (at most `cap` written).  The built-in choice is
// always among them.
int fft_tune_candidates(const pm_plan* p, int kind, int* out, int cap);
int fft_tune_default(const pm_plan* p, int kind);

// ------------------------------------------------------------ spectra.hip --
struct IcSymbol {
  int pk_kind;
  double amp, index;         // P(k) = amp k^index T(k)^2
  double om, ob, h, tcmb;    // cosmology for T(k)
  double kf;                 // 2 pi / L (h/Mpc)
  double inv_dx3;            // 1 / dx^3
  double growth;             // D(a_init)/D(a_norm)
  double coef;               // multiplies the displacement symbol (includes 1/N^3)
  int kpow;                  // 1: i k / k^2 (Zel'dovich), 2: i k / k^4 (gauge shift)
  // 0: the displacement i k_d A w_hat / k^(2 kpow) on the lattice (A: sqrt(P/dx^3) D);
  // 1: Hessian diagonal -k_d^2 A w_hat / k^2 on the lattice (d = x, y, z);
  // 2: Hessian off-diagonal -k_a k_b A w_hat / k^2 on the lattice ((a, b) = xy, xz, yz);
  // 3: i k_d w_hat / k^2 of a field already sampled on the lattice (no A, no phase).
  int mode;
};
// Forward: cbuf(0) holds DFT(noise); writes the three displacement spectra S_d w_hat
// to cbuf 0, 1, 2.  Adjoint: cbuf(0) <- sum_d conj(S_d) cbuf(d).
int launch_ic_symbol(const pm_plan* p, const IcSymbol& sym, bool adjoint, hipStream_t s);
// bhat non-NULL: cross power Re(dhat conj(bhat)) of the pair.
int launch_pk_reduce(const pm_plan* p, const void* dhat, int n_bins, hipStream_t s, const void* bhat = nullptr);
int launch_pk_finalize(const pm_plan* p, int n_bins, double* k_mean, double* pk, int64_t* n_modes, hipStream_t s);
// Up to four triangle sums sum_x f_a f_b f_c over up to four distinct shell fields in
// one pass: field[0..nf) are [N^3] reals of the plan's type; triangle t multiplies
// fields idx[t][0..2] and adds its FP64 sum to *slot[t].
constexpr int kMaxFieldsPerPass = 4, kMaxTriPerPass = 4;
struct TriPass {
  const void* field[kMaxFieldsPerPass];
  double* slot[kMaxTriPerPass];
  int idx[kMaxTriPerPass][3];
  int nf, nt;
};
int launch_triple_multi(const pm_plan* p, const TriPass& tp, hipStream_t s);
int launch_bk_finalize(const pm_plan* p, int n_tri, const double* sums, double* bk, double* ntri_out,
                       const double* ntri_known, hipStream_t s);
int launch_zero_doubles(double* d, int64_t n, hipStream_t s);
// cbuf(0) of every box: modulus set to target, phase kept; box b negated when bit
// (b & 1) of negate_mask is set.
int launch_fix_spectrum(const pm_plan* p, double target, int negate_mask, hipStream_t s);
// cbuf(coarse, 0) <- the shared modes of cbuf(fine, 0) scaled by (Nc/Nf)^(3/2) / Nc^3.
int launch_truncate_spectrum(const pm_plan* fine, const pm_plan* coarse, hipStream_t s);
// dhat <- beta_b dhat with beta from dP (device [n_bins]) and the counts of the last reduction.
int launch_pk_adjoint_weight(const pm_plan* p, void* dhat, int n_bins, const double* dpk, hipStream_t s);

// ------------------------------------------------------------ adjoint.hip --
// Adjoint of gather + kick + drift (see adjoint.hip); g: [3][N^3] pre-zeroed.
int launch_adj_gather_kdk(const pm_plan* p, const void* force, const void* pos, int64_t np, double kick, double drift,
                          void* lam_pos, void* lam_mom, void* g, hipStream_t s);
// lam_pos (+)= scale * grad_x (W * h)(x_p)
int launch_grad_gather(const pm_plan* p, const void* h, const void* pos, int64_t np, double scale, void* lam_pos,
                       bool accumulate, hipStream_t s);
// cbuf(0) <- coef/k^2 sum_d conj(D_d) cbuf(d)
int launch_div_newton(const pm_plan* p, int grad, double coef, hipStream_t s);
int launch_ic_lattice_adj(const pm_plan* p, const void* lam_pos, const void* lam_mom, void* lam_psi,
                          double mom_factor, hipStream_t s);
// h [6][N^3] (xx, yy, zz, xy, xz, yz) <- g dS/dh for the second-order source S.
int launch_lpt2_source_adj(const pm_plan* p, void* h, const void* g, hipStream_t s);
// y[0, count) += x[0, count) (the plan's dtype).
int launch_accumulate(const pm_plan* p, void* y, const void* x, int64_t count, hipStream_t s);

}  // namespace pm
