/*
 * pmhip -- particle-mesh hot path of the relativistic-plus-Newtonian combination
 * method (Montandon, Hahn & Stahl, arXiv:2404.02783) as hand-written HIP kernels for
 * AMD MI355X (gfx950).
 *
 * C ABI.  Conventions shared by every entry point:
 *   - Status: every call returns 0 (PM_OK) or a negative PM_ERR_* code.  Argument
 *     errors are detected before anything is enqueued.  pm_last_error() returns a
 *     thread-local message describing the last failure.
 *   - Memory: every array argument is a DEVICE pointer allocated and owned by the
 *     caller unless the comment says "host".  The library never frees a caller
 *     pointer and keeps none past the call.
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     All device work is enqueued asynchronously on it; results are valid once the
 *     stream has been synchronised.  Calls on one plan must not run concurrently.
 *   - Precision: a plan computes in float (PM_F32) or double (PM_F64); every real
 *     array of a call on that plan uses the plan's type ("real" below), complex
 *     arrays are interleaved (re, im) pairs of it.
 *   - Units (grid units): positions lie in [0, N) cells; momenta are
 *     p = a^2 (dx/dt) / H0 in cells; a kick adds kick * F, a drift adds drift * p.
 *   - Layouts: particle arrays are structure-of-arrays [3][np] (x block, y block,
 *     z block); particle j of an N^3 lattice run has Lagrangian index
 *     j = (i N + k) N + l.  Real meshes are [N][N][N] row-major (last index
 *     fastest); spectra are [N][N][N/2+1] complex with the forward transform
 *     unnormalised (dhat(n) = sum_x d(x) exp(-2 pi i n.x/N)).
 *   - Supported mesh sizes N: 8, 16, 32, 64, 128, 192, 256, 512, 1024.
 */
#ifndef PMHIP_H
#define PMHIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PM_OK = 0,
  PM_ERR_ARG = -1,    /* bad argument (null pointer, negative size, mismatch) */
  PM_ERR_SIZE = -2,   /* unsupported mesh size */
  PM_ERR_NOMEM = -3,  /* workspace too small or device allocation failed */
  PM_ERR_HIP = -4,    /* a HIP runtime call failed */
  PM_ERR_STATE = -5   /* a device-side guard tripped (non-finite or out-of-box particle) */
};

enum { PM_F32 = 0, PM_F64 = 1 };

/* Potential solve kinds. */
enum { PM_NEWTON = 0, PM_POISSON_GAUGE = 1 };

/* Gradient symbols D_d(n) used for F = -grad(phi) in Fourier space. */
enum {
  PM_GRAD_SPECTRAL = 0, /* i k_d, zero on the Nyquist plane of axis d */
  PM_GRAD_FD2 = 1,      /* i sin(k_d): second-order central difference */
  PM_GRAD_FD1 = 2       /* exp(i k_d) - 1: first-order one-sided difference */
};

typedef struct pm_plan pm_plan;

/* Scalars of one force evaluation.
 * PM_NEWTON (Sec. 2: the N-body-gauge equations are the Newtonian ones):
 *   laplacian(phi) = (3/2) omega_m delta; uses omega_m only.
 * PM_POISSON_GAUGE (weak-field scalar sector; the paper gives the linear relation
 *   delta_count = delta_phys - 3 phi, eq. physical_density, and its consequences,
 *   eqs. b1 and bgr; the field equation is the linear 00 Einstein equation with
 *   psi = phi and a backward difference for phi'):
 *   phi_new = [(3/2) calh^2 om_a dhat_c - 3 calh inv_dtau phi_old]
 *           / [-k^2 - 3 calh^2 - 3 calh inv_dtau - (9/2) calh^2 om_a],
 *   force = -grad(a c_g^2 phi_new).  calh: conformal Hubble rate in 1/cells;
 *   c_g: speed of light in cells per (1/H0); inv_dtau: 1/(conformal time since the
 *   previous evaluation, cells), 0 for a quasi-static first solve. */
typedef struct {
  int kind;        /* PM_NEWTON | PM_POISSON_GAUGE */
  int grad;        /* PM_GRAD_* */
  double omega_m;  /* Omega_m today (Newtonian prefactor) */
  double a;        /* scale factor of the evaluation */
  double om_a;     /* Omega_m(a) */
  double calh;     /* conformal Hubble rate, 1/cells */
  double c_g;      /* speed of light, cells per (1/H0) */
  double inv_dtau; /* 1 / conformal-time step, 1/cells; 0 = quasi-static */
} pm_solve_params;

/* One force-kick-drift cycle: F = force(x); p += kick * F(x); x = wrap(x + drift * p).
 * A kick-drift-kick leapfrog is a chain of cycles with kick = K2(previous step) +
 * K1(this step) and a closing cycle with drift = 0 (see pm_kdk_factors).
 * flags (0 = plain cycle):
 *   PM_STEP_DEPOSIT_NEXT  after the drift, also deposit the new positions into the
 *                         plan's density buffer (fused into the gather where the
 *                         layout allows), for the next cycle;
 *   PM_STEP_DENSITY_READY the plan's density buffer already holds the density of
 *                         `pos`, left by the previous pm_step on this plan with the
 *                         same pos pointer and PM_STEP_DEPOSIT_NEXT; the caller
 *                         asserts the positions were not modified since.  If the
 *                         plan holds no such density the call fails with
 *                         PM_ERR_STATE.  Every other call on the plan discards it. */
#define PM_STEP_DEPOSIT_NEXT 1
#define PM_STEP_DENSITY_READY 2
typedef struct {
  double kick;
  double drift;
  pm_solve_params solve;
  int flags;
} pm_step_params;

/* Flat LCDM background without radiation (Sec. 3 of the paper). */
typedef struct {
  double omega_m;
  double omega_b;
  double h;
  double t_cmb;
} pm_cosmology;

/* Linear power spectrum at a = a_norm: P(k) = amp * k^index * T(k)^2 with k in h/Mpc,
 * T = 1 (kind 0, power law) or the Eisenstein & Hu (1998) no-wiggle transfer (kind 1). */
enum { PM_PK_POWERLAW = 0, PM_PK_EH98 = 1 };

typedef struct {
  int pk_kind;
  double amp;
  double index;
  double a_init;        /* scale factor of the initial conditions */
  double a_norm;        /* scale factor at which the spectrum above is linear */
  pm_cosmology cosmo;
} pm_ic_params;

/* ---------------------------------------------------------------- plans ------ */

/* Bytes of device workspace a plan of mesh size n and dtype needs: three complex
 * spectrum buffers (density and force components), each [N][N][hp] with the row
 * length N/2+1 padded to a 128-byte multiple hp, and one real density mesh (the
 * density pm_step hands from one cycle to the next); the layout is internal. */
size_t pm_plan_workspace_bytes(int n_mesh, int dtype);

/* Create a plan for an N^3 mesh of a periodic box of side box_mpch (Mpc/h).
 * workspace: caller device buffer of ws_bytes >= pm_plan_workspace_bytes(), aligned
 * to 256 bytes (as hipMalloc returns), or NULL to let the plan allocate (and free) its
 * own.  The plan also allocates a few KB of twiddle tables and counters.  Errors:
 * PM_ERR_SIZE for an unsupported N, PM_ERR_NOMEM if ws_bytes is too small,
 * PM_ERR_ARG for a misaligned workspace, PM_ERR_HIP if an allocation fails. */
int pm_plan_create(pm_plan** out, int n_mesh, double box_mpch, int dtype, void* workspace, size_t ws_bytes);
int pm_plan_destroy(pm_plan* plan);

/* Batched plans: n_batch independent periodic boxes of the same mesh and side (an
 * ensemble of realisations, as used for the paper's ensemble error bars; batching is
 * not in the paper).  Every box is advanced by the same launches (the box index is a
 * grid dimension), so a group of small boxes fills the GPU like one large box.
 * Entry points that accept a batched plan and their layouts:
 *   pm_deposit       pos [n_batch][3][np], delta [n_batch][N][N][N]
 *   pm_solve         delta [n_batch][N^3] -> force [3][n_batch][N^3];
 *                    phi_state [n_batch][N][N][N/2+1]
 *   pm_step          pos, mom [n_batch][3][N^3] (np must be N^3 when n_batch > 1),
 *                    force_scratch [3][n_batch][N^3]
 *   pk_estimate      delta [n_batch][N^3] -> k_mean, pk, n_modes [n_batch][n_bins]
 *   pm_ic_zeldovich  noise [n_batch][N^3] -> disp_scratch [3][n_batch][N^3],
 *                    pos, mom [n_batch][3][N^3]
 * Every other entry point requires n_batch == 1 (PM_ERR_ARG otherwise).  All boxes of
 * a call share its scalar parameters (kick, drift, solve, IC parameters).
 * n_batch in [1, 4096]; workspace bytes from pm_plan_workspace_bytes_batch (0 for an
 * unsupported N, dtype or n_batch).  pm_plan_create is the n_batch = 1 case. */
size_t pm_plan_workspace_bytes_batch(int n_mesh, int dtype, int n_batch);
int pm_plan_create_batch(pm_plan** out, int n_mesh, double box_mpch, int dtype, int n_batch, void* workspace,
                         size_t ws_bytes);

/* ------------------------------------------------------- uneven ensembles --- */
/* An ensemble of independent periodic boxes of uneven mesh sizes advanced together
 * (the ensembles of realisations behind the paper's error bars on the scale-dependent
 * bias, Sec. 5.2; batching is not in the paper).  Boxes of equal mesh size and side
 * form a size group with one internal batched plan: every call issues each kernel of
 * the operation once per group for all of the group's boxes (box index in the grid),
 * and the particle kernels read each box's particle arrays and its kick and drift
 * from the group's device table, which a small kernel refreshes at every call (the
 * calls can be captured in a HIP graph; the pointer arrays are read at call time).
 * Groups are ordered by decreasing mesh size, then by side.
 * n_mesh, box_mpch: host arrays of n_box (sizes as pm_plan_create); box i holds
 * n_mesh[i]^3 particles on its lattice.  flags: PM_BATCH_CONCURRENT runs each group on
 * a stream of its own (default priority), forked from and joined back into the call's
 * stream, so that small groups' launches overlap large groups' kernels.  The batch
 * owns its plans, force meshes and staging buffers (allocated here, freed by
 * pm_batch_destroy).  Calls on one batch must not run concurrently.
 * Errors: PM_ERR_SIZE for an unsupported mesh size, PM_ERR_ARG for bad arguments,
 * PM_ERR_NOMEM / PM_ERR_HIP when an allocation fails. */
typedef struct pm_batch pm_batch;
#define PM_BATCH_CONCURRENT 1
int pm_batch_create(pm_batch** out, int n_box, const int* n_mesh, const double* box_mpch, int dtype, int flags);
int pm_batch_destroy(pm_batch* batch);
/* Number of size groups, and group g's mesh size, side, number of boxes and internal
 * plan (host outputs, each may be NULL).  The plan may be given to the FFT launch-shape
 * tuning calls (pm_plan_autotune, pm_plan_{get,set}_tuning) and to the profiler only. */
int pm_batch_num_groups(const pm_batch* batch);
int pm_batch_group(const pm_batch* batch, int group, int* n_mesh, double* box_mpch, int* n_boxes, pm_plan** plan);
/* One force-kick-drift cycle (Sec. 2's PM cycle, as pm_step) of every box, in place.
 * pos, mom: host arrays of n_box device pointers to box i's [3][n_mesh[i]^3] arrays of
 * the batch's dtype.  per_box: host array of n_box step parameters; kick and drift
 * may differ between boxes; the solve parameters (PM_NEWTON only) and the flags must
 * be equal within a size group (PM_ERR_ARG otherwise).  flags as pm_step:
 * PM_STEP_DEPOSIT_NEXT leaves each group's density of the drifted positions for the
 * next call; PM_STEP_DENSITY_READY requires the previous pm_batch_step to have left
 * it for the same pointers (PM_ERR_STATE otherwise); any other call discards it. */
int pm_batch_step(pm_batch* batch, void* const* pos, void* const* mom, const pm_step_params* per_box, void* stream);
/* Zel'dovich initial conditions of every box (as pm_ic_zeldovich, same parameters for
 * all boxes): noise[i] box i's [n^3] unit white noise (read only), pos[i], mom[i] its
 * [3][n^3] outputs. */
int pm_batch_ic_zeldovich(pm_batch* batch, const void* const* noise, const pm_ic_params* ic, void* const* pos,
                          void* const* mom, void* stream);
/* P(k) of every box (eq. powerspectrum, as pm_deposit then pk_estimate) from its
 * particles pos[i]: n_bins[i] bins (host; equal within a size group, at most 4 N);
 * box i's k_mean, pk (double) and n_modes (int64) are written at offset
 * sum_{j<i} n_bins[j] of the device arrays. */
int pm_batch_pk_estimate(pm_batch* batch, const void* const* pos, const int* n_bins, double* k_mean, double* pk,
                         int64_t* n_modes, void* stream);

/* Reads and clears the device guard counters (synchronises `stream`).
 * Returns PM_ERR_STATE if, since the last check, the deposit met a non-finite
 * position (skipped) or a position outside [0, N) (wrapped back in). */
int pm_check(pm_plan* plan, void* stream);

/* Thread-local description of the last error ("" if none). */
const char* pm_last_error(void);
/* Not in the paper: the build record, "pmhip <offload arch> sources <sha256>" with
 * the digest of the library's sources taken when it was compiled (a static string;
 * callers compare it with the sources they hold to tell a stale build). */
const char* pm_build_info(void);

/* Per-kernel timing.  While enabled, every kernel launch of the plan is bracketed by
 * a pair of HIP events recorded on the call's stream (so it also times work inside a
 * graph-free stream sequence).  Off by default; enabling costs two event records per
 * launch. */
int pm_profile_enable(pm_plan* plan, int on);
/* Sums the recorded launch durations per kernel kind and clears them (waits for the
 * recorded events).  names: host char[n_max][32]; ms: host double[n_max] (total
 * milliseconds); count: host int64[n_max] (launches).  Returns the number of kinds
 * written, or a negative error code (PM_ERR_ARG if profiling is off). */
int pm_profile_read(pm_plan* plan, int n_max, char* names, double* ms, int64_t* count);

/* ------------------------------------------------------------ measurement --- */
/* Not in the paper: a reference rate for the deposits' global atomics.  Adds 1.0f to
 * each of buf[0, n) (device floats, caller-owned) `passes` times with unreturned
 * float atomics, consecutive threads on consecutive cells -- the pattern in which the
 * deposits flush their LDS windows -- asynchronously on `stream`; atomics per second
 * = n * passes / the launch's duration.  Errors: PM_ERR_ARG for null buf, n <= 0 or
 * passes <= 0. */
int pm_microbench_atomics(void* buf, int64_t n, int passes, void* stream);

/* ------------------------------------------------- FFT launch-shape tuning --- */
/* Not in the paper (the transforms are this library's).  Four tuning slots pick the
 * launch shape of the FFT passes of a plan: 0 columns per workgroup of the plain
 * column passes, 1 of the fused solve pass, 2 rows per workgroup of the r2c rows pass,
 * 3 of the c2r rows pass.  Every shape computes the same numbers (each column or row
 * is transformed by the same arithmetic), only the speed differs. */

/* Writes up to `cap` allowed shapes of slot `kind` (powers of two within 256 threads
 * and 64 KiB of LDS per workgroup, the built-in choice always included), ascending, to
 * host `out`; returns how many there are (may exceed cap), or a negative error. */
int pm_plan_tuning_candidates(const pm_plan* plan, int kind, int* out, int cap);
/* Host int[4]: the shapes the plan uses now (the built-in choice where none is set). */
int pm_plan_get_tuning(const pm_plan* plan, int* shapes);
/* Host int[4]: sets the shapes (0 = built-in choice); PM_ERR_ARG, and nothing changed,
 * if any is not an allowed shape of its slot. */
int pm_plan_set_tuning(pm_plan* plan, const int* shapes);
/* Measures every allowed shape of every slot on this device (reps timed launches of
 * the pass after one warm launch, HIP events on `stream`; waits for them) and keeps the
 * fastest.  mesh_scratch: [boxes][N^3] real of the plan's dtype (overwritten); the
 * plan's workspace is overwritten.  The choice is cached per (device, N, dtype, boxes)
 * for the process; with use_cache non-zero a cached choice is applied without
 * measuring.  best_ms: optional host double[4], the fastest time per launch of each
 * slot (-1 when taken from the cache).  A setup call: it synchronises the stream. */
int pm_plan_autotune(pm_plan* plan, void* mesh_scratch, int reps, int use_cache, double* best_ms, void* stream);

/* ----------------------------------------------------------- hot path ------- */

/* CIC counting density (Sec. 4: counting density of a cloud-in-cell assignment):
 * delta(c) = sum_p W(x_p - c) / nbar - 1, nbar = np / N^3, with trilinear weights
 * (1 - t, t) per axis around the base node floor(x).  pos: [3][np] real in [0, N);
 * delta: [N][N][N] real, overwritten.  np may be 0 (delta = -1).  Summation order
 * is that of device atomics (not bitwise reproducible; the assignment is). */
int pm_deposit(pm_plan* plan, const void* pos, int64_t np, void* delta, void* stream);

/* Potential solve and PM force meshes for a density contrast mesh.
 * delta: [N][N][N] real (read only); force: [3][N][N][N] real, written with
 * F_d = IDFT(-D_d(n) phi_hat(n)).  phi_state: [N][N][N/2+1] complex potential
 * phi_hat carried between calls for PM_POISSON_GAUGE (read, then overwritten with
 * phi_new); ignored (may be NULL) for PM_NEWTON. */
int pm_solve(pm_plan* plan, const void* delta, const pm_solve_params* sp, void* phi_state, void* force,
             void* stream);

/* Force interpolation of the particle-mesh method (Sec. 2: the relativistic and the
 * Newtonian run of the combination are made with a particle-mesh code, whose forces
 * come from the mesh; Sec. 4.1 traces their small-scale deficit to it): CIC
 * interpolation of the three force meshes to the
 * particles with the deposit's weights, acc[d][p] = sum_c W(x_p - c) force[d](c).
 * force: [3][N][N][N] real (read only); pos: [3][np] in [0, N); acc: [3][np]
 * (written).  Single-box plans only (PM_ERR_ARG otherwise). */
int pm_gather(pm_plan* plan, const void* force, const void* pos, int64_t np, void* acc, void* stream);

/* One cycle of the particle-mesh method (Sec. 2: the relativistic and Newtonian runs
 * are particle-mesh simulations; the time integrator is not stated and is read as
 * a kick-drift-kick leapfrog, see pm_step_params) in place on (pos, mom) [3][np]:
 * deposit -> solve (Newtonian, or the Poisson-gauge field of pm_solve) -> gather ->
 * kick -> drift, with the periodic wrap x <- x - N floor(x/N) and a result equal to N
 * set to 0.  force_scratch: [3][N][N][N] real (holds the force meshes on return);
 * phi_state as in pm_solve.  Errors: PM_ERR_ARG for bad arguments or flags,
 * PM_ERR_STATE for PM_STEP_DENSITY_READY without a handed-over density. */
int pm_step(pm_plan* plan, void* pos, void* mom, int64_t np, const pm_step_params* st, void* force_scratch,
            void* phi_state, void* stream);

/* Reverse-mode (adjoint) of one Newtonian pm_step; not in the paper: the exact
 * vector-Jacobian product of the discrete cycle x -> (x', p') defined by pm_step
 * (Sec. 2's particle-mesh force; deposit, Green's function and gradient, gather,
 * kick, drift).  With F(x) the gathered force and (lam_pos, lam_mom) the cotangents
 * of the cycle's outputs on entry:
 *   lam_mom <- lam_mom + Dr lam_pos,   v = K lam_mom,
 *   lam_pos <- lam_pos + (dF/dx)^T v
 * where (dF/dx)^T v has a force-field part (gradient of the CIC interpolation
 * weights against the force meshes) and a density part (v deposited with the CIC
 * weights, the transposed Green's/gradient operator applied in Fourier space, and
 * the result differentiated through the CIC weights of the deposit, scaled by
 * 1/nbar).  CIC weight derivatives are right derivatives at cell edges.
 * pos: [3][np] the positions the forward cycle started from (read only).
 * st: the forward cycle's parameters; st->solve.kind must be PM_NEWTON (PM_ERR_ARG
 * otherwise).  force: [3][N][N][N] the force meshes the forward cycle used (as left
 * in pm_step's force_scratch), or NULL to recompute them from pos.  mesh_scratch:
 * device real scratch of 3 N^3 elements, or 6 N^3 when force is NULL.
 * lam_pos, lam_mom: [3][np] cotangents, updated in place.  Summation order of the
 * deposit of v is that of device atomics. */
int pm_step_adjoint(pm_plan* plan, const void* pos, int64_t np, const pm_step_params* st, const void* force,
                    void* mesh_scratch, void* lam_pos, void* lam_mom, void* stream);

/* Allocation-free variant of pm_step_adjoint, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments and results as pm_step_adjoint without mesh_scratch:
 * the 3 N^3 reals of scratch (6 N^3 when force is NULL) come from a static device
 * array of PM_STATIC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends (its address is taken at plan creation).  The call makes no
 * allocation (with the plan's profiler off, the default; pm_profile_enable creates
 * HIP events).  Limit: PM_ERR_NOMEM when pm_step_adjoint_noalloc_bytes exceeds
 * PM_STATIC_SCRATCH_BYTES (64 MiB: N <= 128 in FP32, and in FP64 with the force
 * meshes given).  All calls on one GPU share the array, which keeps the last call's
 * contents (each call clears what it needs): calls that overlap in time on one GPU,
 * from any plan or stream, race and must be serialised by the caller. */
#define PM_STATIC_SCRATCH_BYTES (64u << 20)
size_t pm_step_adjoint_noalloc_bytes(int n_mesh, int dtype, int with_force);
int pm_step_adjoint_noalloc(pm_plan* plan, const void* pos, int64_t np, const pm_step_params* st, const void* force,
                            void* lam_pos, void* lam_mom, void* stream);

/* eq. xiGR and eq. combined: xi = minimum-image (x_gr - x_newton) on the coarse
 * lattice (n_coarse^3 particles, coarse cells), interpolated with CIC weights in
 * Lagrangian coordinates to the fine lattice (n_fine^3 particles; fine particle j
 * per axis sits at coarse coordinate ((2j+1) n_c - n_f)/(2 n_f)), scaled to fine
 * cells and added: x_out = wrap(x_fine + (n_f/n_c) xi_f).  Requires n_fine to be a
 * multiple of n_coarse.  x_out may alias x_fine.  All arrays [3][n^3] of `dtype`. */
int displacement_combine(const void* x_gr, const void* x_newton, int n_coarse, const void* x_fine, int n_fine,
                         int dtype, void* x_out, void* stream);

/* eq. combined with a given displacement field: x_out = wrap(x_fine + (n_f/n_c) xi_f),
 * xi ([3][n_coarse^3], coarse cells, on the coarse lattice) interpolated to the fine
 * lattice exactly as in displacement_combine (e.g. xi = pm_xi_linear's output).  x_out
 * may alias x_fine. */
int displacement_add(const void* xi, int n_coarse, const void* x_fine, int n_fine, int dtype, void* x_out,
                     void* stream);

/* Power spectrum (eq. powerspectrum), raw estimator without shot-noise subtraction or
 * deconvolution.  Bin width w = (N/2)/n_bins (units of k_f = 2 pi/L); bin b holds
 * modes with N^2 (2b+1)^2 <= 16 n_bins^2 |n|^2 < N^2 (2b+3)^2 (integer decision).
 * Outputs (device, n_bins each): k_mean [h/Mpc] (double), pk [(Mpc/h)^3] (double),
 * n_modes (int64, modes of the full cube).  delta: [N][N][N] real. */
int pk_estimate(pm_plan* plan, const void* delta, int n_bins, double* k_mean, double* pk, int64_t* n_modes,
                void* stream);

/* Cross power spectrum of two meshes of the same box(es): P_ab = (V/N^6)
 * <Re(a_hat conj(b_hat))> over the bins of pk_estimate (the halo-matter cross power of
 * the bias fits, Sec. 5, here of any two fields, e.g. combined and Newtonian).
 * delta_a, delta_b: [boxes][N][N][N] real (read only); outputs as pk_estimate.  Uses
 * two spectra of the plan's workspace. */
int pk_cross_estimate(pm_plan* plan, const void* delta_a, const void* delta_b, int n_bins, double* k_mean,
                      double* pk, int64_t* n_modes, void* stream);

/* Scale-dependent linear bias (eq. b1 and the scale dependence of Sec. 5): fits
 * ratio(k) = b1 + b1_GR calh^2/k^2 (+ c2 k^2 when with_k2) by least squares weighted
 * with the mode counts, over the bins with n_modes > 0 and 0 < k < k_cut after
 * dropping the first `skip` of them (the paper drops two).  Host arrays of n_bins: k
 * [h/Mpc], ratio (e.g. P_cross / P_auto), n_modes; calh = aH/c in h/Mpc.  Writes coef[3]
 * = (b1, b1_GR, c2) (c2 = 0 without the k^2 term).  PM_ERR_ARG when fewer bins than
 * parameters remain or the system is singular.  Host computation only. */
int bias_fit(const double* k, const double* ratio, const int64_t* n_modes, int n_bins, double k_cut, double calh,
             int skip, int with_k2, double* coef);

/* Adjoint of positions -> CIC counting density -> pk_estimate (eq. powerspectrum);
 * not in the paper.  dpk: device double [n_bins], the cotangent dL/dP_b.  Writes
 * lam_pos[d][p] = dL/dx_{p,d} (overwritten): the spectrum of the particles' density
 * is weighted per bin by 2 V dP_b / (N^6 count_b), transformed back, and
 * differentiated through the CIC weights (right derivatives at cell edges) with the
 * factor 1/nbar.  pos: [3][np]; n_bins and binning as pk_estimate. */
int pk_adjoint(pm_plan* plan, const void* pos, int64_t np, int n_bins, const double* dpk, void* lam_pos,
               void* stream);

/* FFT bispectrum estimator (eq. bispectre).  Shell s holds modes with
 * (2c_s - w)^2 <= 4|n|^2 < (2c_s + w)^2 (float64 decision, c_s and w in units of k_f).
 * For triangle t = (a, b, c): B_t = (V^2/N^9) sum_x d_a d_b d_c / sum_x I_a I_b I_c
 * with d_s = IDFT(dhat 1_s), I_s = IDFT(1_s); ntri_t = N^6 sum_x I_a I_b I_c.
 * shell_center_kf: host [n_shells]; tri: host [n_tri][3] shell ids; bk, ntri_out:
 * device double [n_tri].  shell_ws: device scratch for cached shell fields of
 * shell_ws_bytes >= 3 N^3 sizeof(real) (more bytes = fewer recomputed shells).
 * If ntri_known is non-NULL (device double [n_tri] from an earlier call with the same
 * N, shells and triangles) the indicator pass is skipped and it is copied to ntri_out. */
int bk_estimate(pm_plan* plan, const void* delta, int n_shells, const double* shell_center_kf,
                double shell_width_kf, const int32_t* tri, int n_tri, double* bk, double* ntri_out,
                const double* ntri_known, void* shell_ws, size_t shell_ws_bytes, void* stream);

/* ------------------------------------------------- initial conditions ------- */

/* Zel'dovich initial conditions on the half-cell-offset lattice (same random phases
 * for every run, Secs. 2 and 3; first-order displacement).  noise: [N][N][N] real
 * unit white noise (read only).  delta_L_hat = DFT(noise) sqrt(P(k)/dx^3)
 * D(a_init)/D(a_norm), zero at k = 0 and on every Nyquist plane; Psi_hat =
 * i k delta_L_hat / k^2 evaluated at q = (i,j,l) + 1/2; pos = wrap(q + Psi),
 * mom = a^2 E f Psi.  disp_scratch: [3][N][N][N] real, overwritten with Psi. */
int pm_ic_zeldovich(pm_plan* plan, const void* noise, const pm_ic_params* ic, void* disp_scratch, void* pos,
                    void* mom, void* stream);

/* Second-order Lagrangian (2LPT) Newtonian set (Sec. 3 starts the runs from
 * second-order ICs; continuous-2LPT reading of that start).  With chi_hat =
 * delta_L_hat / k^2 (delta_L as in pm_ic_zeldovich, so Psi1 = grad chi is the
 * Zel'dovich displacement): S = sum_{i<j} (chi_ii chi_jj - chi_ij^2) sampled on the
 * lattice, Psi2_hat = c2 i k DFT(S) / k^2 (k = 0 and Nyquist planes dropped, no
 * de-aliasing), c2 = (3/7) Omega_m(a_init)^(-1/143); pos = wrap(q + Psi1 + Psi2),
 * mom = a^2 E (f Psi1 + f2 Psi2), f2 = 2f + (3/143)(1 - Omega_m).  noise [N][N][N]
 * (read only); disp_scratch [3][N][N][N] (overwritten with Psi1); pos and mom
 * [3][N^3] (written; mom also holds intermediate Hessian fields).  The four buffers
 * must be distinct (PM_ERR_ARG).  Single-box plans only.  Four forward and twelve
 * inverse transforms of N^3. */
int pm_ic_2lpt(pm_plan* plan, const void* noise, const pm_ic_params* ic, void* disp_scratch, void* pos, void* mom,
               void* stream);

/* Paired-and-fixed white noise (the pairing method cited in Sec. 4 for the
 * bispectrum).  Every Fourier mode of every box keeps its phase and takes the
 * expected modulus of unit white noise, |DFT(noise)| = N^(3/2) (exact zeros stay
 * zero).  pair_mode 0: fixed only; 1: fixed and negated (the partner realisation);
 * 2: fixed, and every odd box of the batch negated, so that boxes (2j, 2j+1) given the
 * same noise become a pair (needs an even number of boxes).  noise: [boxes][N^3]
 * (read only); noise_out: same shape (written; may alias noise).  Uses the plan's
 * spectrum workspace. */
int pm_noise_fix(pm_plan* plan, const void* noise, int pair_mode, void* noise_out, void* stream);

/* Adjoint of pm_ic_2lpt with respect to the noise; not in the paper (the
 * differentiable model with the second-order start).  The set is quadratic in the
 * noise, so the noise itself is an input: with Psi1 = A w, chi_ab = H_ab w and
 * Psi2 = c2 G S(chi), lam_noise = A^T(lam_pos + m1 lam_mom) + sum_ab H_ab^T(g_ab),
 * g_ab = (c2 G^T(lam_pos + m2 lam_mom)) dS/dchi_ab (m1, m2 = a^2 E f, a^2 E f2;
 * transposes are the conjugate symbols).  noise [N^3], lam_pos, lam_mom [3][N^3]
 * (read only); scratch [9][N^3] of the plan's dtype (overwritten); lam_noise [N^3]
 * (written; must not alias noise or scratch).  Single-box plans only. */
int pm_ic_2lpt_adjoint(pm_plan* plan, const void* noise, const pm_ic_params* ic, const void* lam_pos,
                       const void* lam_mom, void* scratch, void* lam_noise, void* stream);

/* Adjoint of pm_ic_zeldovich with respect to the noise; not in the paper.  The
 * forward map noise -> (pos, mom) is affine: pos = wrap(q + Psi), mom = m Psi with
 * Psi_d = IDFT(S_d DFT(noise)).  Given the cotangents lam_pos, lam_mom [3][N^3]
 * (read only), writes lam_noise [N][N][N] = sum_d IDFT(conj(S_d) DFT(lam_pos_d +
 * m lam_mom_d)) scaled as the transpose of the forward map.  disp_scratch:
 * [3][N][N][N] real, overwritten. */
int pm_ic_zeldovich_adjoint(pm_plan* plan, const pm_ic_params* ic, const void* lam_pos, const void* lam_mom,
                            void* disp_scratch, void* lam_noise, void* stream);

/* White noise of a coarser run sharing the fine run's random phases (Secs. 2 and 3:
 * every simulation starts from the same phases; reading for runs of different
 * resolution).  DFT(noise_coarse)(n) = DFT(noise_fine)(n) (Nc/Nf)^(3/2) for every mode
 * with all |n_i| < Nc/2, zero on the coarse Nyquist planes, so that the physical
 * linear field (V/N^3) delta_hat is the same on the shared modes.  noise_fine:
 * [Nf][Nf][Nf] (read only); noise_coarse: [Nc][Nc][Nc] (written).  Both plans
 * single-box, same dtype, Nc dividing Nf (PM_ERR_ARG otherwise); uses both plans'
 * workspaces. */
int pm_noise_truncate(pm_plan* fine, const void* noise_fine, pm_plan* coarse, void* noise_coarse, void* stream);

/* Poisson-gauge partner set of pm_ic_zeldovich's (or pm_ic_2lpt's) output (linear reading of eqs.
 * physical_density, b1, bgr): xi_hat = i k g(a_init) delta_L_hat / k^4 on the same
 * lattice with g = (3f + (9/2) Omega_m(a)) calh^2; pos_gr = wrap(pos_n + xi),
 * mom_gr = mom_n + a^2 E (dg/dlna / g) xi.  disp_scratch as above. */
int pm_ic_gauge(pm_plan* plan, const void* noise, const pm_ic_params* ic, void* disp_scratch,
                const void* pos_n, const void* mom_n, void* pos_gr, void* mom_gr, void* stream);

/* The linear Poisson-gauge displacement at scale factor a (the same reading of eqs.
 * physical_density, b1 and bgr as pm_ic_gauge): xi_lin(a) = g(a) IDFT(i k delta_L_hat /
 * k^4) on the half-cell lattice, g(a) = (3f + (9/2) Omega_m(a)) calh(a)^2 D(a)/D(a_init),
 * with delta_L at a_init from `noise` and `ic` as in pm_ic_zeldovich.  Added to a
 * Newtonian run with displacement_add it gives the combination with linear theory in
 * place of the GR-minus-Newton displacement of eq. xiGR.  xi: [3][N^3] of the plan's
 * dtype, in cells (written; also serves as the transform's output scratch).
 * Single-box plans only. */
int pm_xi_linear(pm_plan* plan, const void* noise, const pm_ic_params* ic, double a, void* xi, void* stream);

/* --------------------------------------------------- host cosmology --------- */
/* Host-side double-precision scalars that parameterise the kernels.  Growth D(a) is
 * the Heath integral (5 Om/2) E(a) int_0^a da'/(a' E)^3; f = dlnD/dlna.  Kick and
 * drift factors: K = int da/(a^2 E), Dr = int da/(a^3 E). */
double pm_cosmo_hubble_e(const pm_cosmology* c, double a);
double pm_cosmo_omega_m_a(const pm_cosmology* c, double a);
double pm_cosmo_growth(const pm_cosmology* c, double a);
double pm_cosmo_growth_rate(const pm_cosmology* c, double a);
double pm_cosmo_kick(const pm_cosmology* c, double a0, double a1);
double pm_cosmo_drift(const pm_cosmology* c, double a0, double a1);
/* Leapfrog factors of one step a0 -> a1 with half step sqrt(a0 a1): out[0] = K(a0, ah),
 * out[1] = Dr(a0, a1), out[2] = K(ah, a1). */
void pm_kdk_factors(const pm_cosmology* c, double a0, double a1, double out[3]);
/* Scale factors of a run of n_steps steps equally spaced in ln a (the step-spacing
 * reading of the PM runs of Sec. 2 and 4): a[j] = exp(ln a_start + (ln a_end -
 * ln a_start) j / n_steps), j = 0..n_steps, into host array a[n_steps + 1].  Returns
 * PM_OK, or PM_ERR_ARG for null a, n_steps < 1 or a_start, a_end not positive. */
int pm_log_steps(double a_start, double a_end, int n_steps, double* a);
/* The kick-drift-kick leapfrog over a[0..n_steps] (host, increasing) as the chain of
 * pm_step cycles: cycle j < n_steps kicks by kick[j] = K(a_{j-1/2}, a_j) + K(a_j,
 * a_{j+1/2}) (the first term 0 for j = 0) and drifts by drift[j] = Dr(a_j, a_{j+1});
 * the closing cycle j = n_steps kicks by K(a_{n-1/2}, a_n) and has drift[n_steps] = 0
 * (a_{j+1/2} = sqrt(a_j a_{j+1}), factors of pm_kdk_factors).  kick and drift: host
 * arrays of n_steps + 1.  Returns PM_OK, or PM_ERR_ARG for null arrays, n_steps < 1
 * or a not positive and increasing. */
int pm_leapfrog_factors(const pm_cosmology* c, const double* a, int n_steps, double* kick, double* drift);
/* Solve parameters of a Poisson-gauge evaluation at a (box side box_mpch, mesh n);
 * a_prev <= 0 marks the first (quasi-static) evaluation. */
void pm_gauge_params(const pm_cosmology* c, double box_mpch, int n_mesh, double a, double a_prev,
                     pm_solve_params* out);
/* Amplitude of the EH98 no-wiggle spectrum with sigma(8 Mpc/h) = sigma8 at a = 1. */
double pm_power_eh98_amplitude(const pm_cosmology* c, double n_s, double sigma8);
/* Amplitude of P = A k^index giving an expected 3-D rms Zel'dovich displacement of
 * rms_cells over the discrete non-Nyquist modes of an N^3 box of side box_mpch. */
double pm_power_law_amplitude(int n_mesh, double box_mpch, double rms_cells, double index);

#ifdef __cplusplus
}
#endif
#endif /* PMHIP_H */
