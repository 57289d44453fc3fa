// C ABI of the pmhip library: argument checking, plans and the orchestration of the
// kernels of fft.hip, particles.hip and spectra.hip on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "pm_common.h"
#include "pm_plan.h"

namespace pm {

static thread_local char g_err[512] = "";

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return PM_OK;
  return set_error(PM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

static size_t complex_bytes(int n, int dtype) {
  const size_t es = dtype == PM_F32 ? 4 : 8;
  return align256((size_t)n * n * padded_half(n, (int)es) * 2 * es);
}

static int check_plan(const pm_plan* p) {
  if (!p) return set_error(PM_ERR_ARG, "null plan");
  return PM_OK;
}

// Scratch of pm_step_adjoint_noalloc: one file-scope device array, which every GPU the
// library runs on holds (its own copy at its own address) until the process ends.
// In host code `scratch` names a host-side stand-in, never the device memory: the
// device address of each GPU's copy is taken once per device with hipGetSymbolAddress
// (static_scratch_init, called at plan creation with that device current) and only
// that address is handed to kernels.
constexpr size_t kStaticScratchBytes = size_t(PM_STATIC_SCRATCH_BYTES);
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
static void* g_scratch_dev[kMaxDevices];
static std::mutex g_scratch_mu;

static int static_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return set_error(PM_ERR_ARG, "device %d out of range", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[device]) return PM_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_check(e, "static scratch address");
  if (!ptr) return set_error(PM_ERR_HIP, "static scratch address: null");
  g_scratch_dev[device] = ptr;
  return PM_OK;
}

static void* static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_dev[device];
}

// Every entry point other than pm_step may reuse the workspace: the density left for
// the next cycle is discarded.
static void drop_density(pm_plan* p) {
  if (p) p->dens_valid = false;
}

// Entry points that work on one box only.
static int check_single(const pm_plan* p, const char* who) {
  if (!p) return set_error(PM_ERR_ARG, "%s: null plan", who);
  if (p->nb != 1) return set_error(PM_ERR_ARG, "%s: needs a single-box plan (this plan holds %d boxes)", who, p->nb);
  return PM_OK;
}

// ------------------------------------------------------------ profiling ----
static const char* kProfNames[PK_COUNT] = {
    "fill",          "deposit",        "fft_r2c_rows",   "fft_cols_fwd_axis1", "fft_cols_fwd_axis0",
    "fft_solve_axis0", "fft_cols_inv_axis0", "fft_cols_inv_axis1", "fft_c2r_rows", "gather",
    "gather_kick_drift", "gather_kick_drift_deposit", "combine", "ic", "pk", "bk",
    "adjoint_gather_kick_drift", "adjoint_deposit", "grad_gather", "adjoint_symbol"};

struct ProfRec {
  int kind;
  hipEvent_t start, stop;
};

struct ProfState {
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  int open_kind = -1;
  hipEvent_t open_start = nullptr;
  double ms[PK_COUNT] = {0};
  int64_t count[PK_COUNT] = {0};
  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
};

void prof_begin(const pm_plan* p, int kind, hipStream_t s) {
  ProfState* ps = p->prof;
  if (ps->open_kind >= 0) return;  // nested scope: the outer one times it
  ps->open_kind = kind;
  ps->open_start = ps->take();
  (void)hipEventRecord(ps->open_start, s);
}

void prof_end(const pm_plan* p, hipStream_t s) {
  ProfState* ps = p->prof;
  if (ps->open_kind < 0) return;
  hipEvent_t stop = ps->take();
  (void)hipEventRecord(stop, s);
  ps->recs.push_back(ProfRec{ps->open_kind, ps->open_start, stop});
  ps->open_kind = -1;
  // Fold completed records so the list stays short in long runs.
  if (ps->recs.size() > 4096) {
    for (auto& r : ps->recs) {
      (void)hipEventSynchronize(r.stop);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, r.start, r.stop);
      ps->ms[r.kind] += ms;
      ps->count[r.kind] += 1;
      ps->pool.push_back(r.start);
      ps->pool.push_back(r.stop);
    }
    ps->recs.clear();
  }
}

}  // namespace pm

using namespace pm;

#define PM_TRY(expr)             \
  do {                           \
    int _rc = (expr);            \
    if (_rc != PM_OK) return _rc; \
  } while (0)

extern "C" {

#ifndef PM_SOURCE_DIGEST
#define PM_SOURCE_DIGEST "unknown"
#endif
#ifndef PM_OFFLOAD_ARCH
#define PM_OFFLOAD_ARCH "unknown"
#endif
const char* pm_build_info(void) { return "pmhip " PM_OFFLOAD_ARCH " sources " PM_SOURCE_DIGEST; }

const char* pm_last_error(void) { return g_err; }

static size_t density_bytes(int n_mesh, int dtype, int n_batch) {
  return align256((size_t)n_batch * n_mesh * n_mesh * n_mesh * (dtype == PM_F32 ? 4 : 8));
}

size_t pm_plan_workspace_bytes_batch(int n_mesh, int dtype, int n_batch) {
  if (!mesh_supported(n_mesh) || (dtype != PM_F32 && dtype != PM_F64) || n_batch < 1 || n_batch > kMaxBatch) return 0;
  return 3 * (size_t)n_batch * complex_bytes(n_mesh, dtype) + density_bytes(n_mesh, dtype, n_batch);
}

size_t pm_plan_workspace_bytes(int n_mesh, int dtype) { return pm_plan_workspace_bytes_batch(n_mesh, dtype, 1); }

int pm_plan_create(pm_plan** out, int n_mesh, double box_mpch, int dtype, void* workspace, size_t ws_bytes) {
  return pm_plan_create_batch(out, n_mesh, box_mpch, dtype, 1, workspace, ws_bytes);
}

int pm_plan_create_batch(pm_plan** out, int n_mesh, double box_mpch, int dtype, int n_batch, void* workspace,
                         size_t ws_bytes) {
  g_err[0] = 0;
  if (!out) return set_error(PM_ERR_ARG, "pm_plan_create: null output pointer");
  *out = nullptr;
  if (!mesh_supported(n_mesh)) return set_error(PM_ERR_SIZE, "pm_plan_create: unsupported mesh size %d", n_mesh);
  if (dtype != PM_F32 && dtype != PM_F64) return set_error(PM_ERR_ARG, "pm_plan_create: bad dtype %d", dtype);
  if (!(box_mpch > 0.0)) return set_error(PM_ERR_ARG, "pm_plan_create: box must be positive");
  if (n_batch < 1 || n_batch > kMaxBatch)
    return set_error(PM_ERR_ARG, "pm_plan_create: batch of %d boxes outside [1, %d]", n_batch, kMaxBatch);
  const size_t need = pm_plan_workspace_bytes_batch(n_mesh, dtype, n_batch);
  if (workspace && ws_bytes < need)
    return set_error(PM_ERR_NOMEM, "pm_plan_create: workspace of %zu bytes < %zu needed", ws_bytes, need);
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return set_error(PM_ERR_ARG, "pm_plan_create: workspace not aligned to 256 bytes");
  pm_plan* p = new (std::nothrow) pm_plan();
  if (!p) return set_error(PM_ERR_NOMEM, "pm_plan_create: host allocation failed");
  p->n = n_mesh;
  p->nb = n_batch;
  p->dtype = dtype;
  p->box = box_mpch;
  p->esize = dtype == PM_F32 ? 4 : 8;
  p->cbytes = complex_bytes(n_mesh, dtype);
  p->hp = padded_half(n_mesh, (int)p->esize);
  (void)hipGetDevice(&p->device);
  int rc = PM_OK;
  if (workspace) {
    p->ws = workspace;
    p->ws_bytes = ws_bytes;
    p->own_ws = false;
  } else {
    if (hipMalloc(&p->ws, need) != hipSuccess) rc = set_error(PM_ERR_NOMEM, "pm_plan_create: workspace allocation");
    p->ws_bytes = need;
    p->own_ws = true;
  }
  // twiddle table W_N^m = exp(-2 pi i m / N)
  if (rc == PM_OK) {
    std::vector<double> twd(2 * (size_t)n_mesh);
    for (int m = 0; m < n_mesh; ++m) {
      // exact quarter-turn values, double-precision trig elsewhere
      const double ang = 2.0 * kPi * (double)m / (double)n_mesh;
      double c = std::cos(ang), s = -std::sin(ang);
      if ((4 * m) % n_mesh == 0) {
        const int q = (4 * m) / n_mesh;
        c = q == 0 ? 1.0 : (q == 2 ? -1.0 : 0.0);
        s = q == 1 ? -1.0 : (q == 3 ? 1.0 : 0.0);
      }
      twd[2 * m] = c;
      twd[2 * m + 1] = s;
    }
    const size_t tb = 2 * (size_t)n_mesh * p->esize;
    if (hipMalloc(&p->tw, tb) != hipSuccess) {
      rc = set_error(PM_ERR_NOMEM, "pm_plan_create: twiddle allocation");
    } else if (dtype == PM_F32) {
      std::vector<float> twf(twd.begin(), twd.end());
      rc = hip_check(hipMemcpy(p->tw, twf.data(), tb, hipMemcpyHostToDevice), "pm_plan_create: twiddle upload");
    } else {
      rc = hip_check(hipMemcpy(p->tw, twd.data(), tb, hipMemcpyHostToDevice), "pm_plan_create: twiddle upload");
    }
  }
  if (rc == PM_OK) {
    if (hipMalloc(&p->guard, 4 * sizeof(unsigned)) != hipSuccess)
      rc = set_error(PM_ERR_NOMEM, "pm_plan_create: guard allocation");
    else
      rc = hip_check(hipMemset(p->guard, 0, 4 * sizeof(unsigned)), "pm_plan_create: guard init");
  }
  if (rc == PM_OK) p->dens = static_cast<char*>(p->ws) + 3 * (size_t)n_batch * p->cbytes;
  if (rc == PM_OK) rc = static_scratch_init(p->device);
  if (rc == PM_OK) {
    p->sums_cap = (size_t)n_batch * 3 * (size_t)std::max(n_mesh, 512) + 2 * 4096;
    if (hipMalloc(&p->sums, p->sums_cap * sizeof(double)) != hipSuccess)
      rc = set_error(PM_ERR_NOMEM, "pm_plan_create: reduction scratch allocation");
  }
  if (rc != PM_OK) {
    pm_plan_destroy(p);
    return rc;
  }
  *out = p;
  return PM_OK;
}

// ------------------------------------------------------------------ tuning --

namespace {
std::mutex g_tune_mu;
// (device, N, dtype, boxes) -> launch shapes picked by a measurement in this process
std::map<std::tuple<int, int, int, int>, std::vector<int>> g_tune_cache;

bool tune_value_ok(const pm_plan* p, int kind, int v) {
  if (v == 0) return true;
  int c[16];
  const int nc = std::min(fft_tune_candidates(p, kind, c, 16), 16);
  for (int i = 0; i < nc; ++i)
    if (c[i] == v) return true;
  return false;
}

// One timed instance of the pass of tuning slot `kind` on the plan's workspace.
int tune_run(pm_plan* p, int kind, void* mesh, hipStream_t s) {
  switch (kind) {
    case 0:
      PM_TRY(fft_pass_cols(p, cbuf(p, 0), 1, -1, p->nb, cstride(p), s));
      return fft_pass_cols(p, cbuf(p, 0), 0, 1, p->nb, cstride(p), s);
    case 1: {
      pm_solve_params sp{};
      sp.kind = PM_NEWTON;
      sp.grad = PM_GRAD_SPECTRAL;
      sp.omega_m = 0.3;
      return fft_pass_solve(p, &sp, nullptr, s);
    }
    case 2:
      return fft_pass_rows_r2c(p, p->nb, mesh, cbuf(p, 0), s);
    default:
      return fft_pass_rows_c2r(p, p->nb, cbuf(p, 0), cstride(p), mesh, s);
  }
}
}  // namespace

int pm_plan_tuning_candidates(const pm_plan* p, int kind, int* out, int cap) {
  PM_TRY(check_plan(p));
  if (kind < 0 || kind > 3 || cap < 0 || (cap > 0 && !out)) return set_error(PM_ERR_ARG, "bad tuning slot or buffer");
  return fft_tune_candidates(p, kind, out, cap);
}

int pm_plan_get_tuning(const pm_plan* p, int* shapes) {
  PM_TRY(check_plan(p));
  if (!shapes) return set_error(PM_ERR_ARG, "pm_plan_get_tuning: null pointer");
  for (int k = 0; k < 4; ++k) shapes[k] = p->tune[k] > 0 ? p->tune[k] : fft_tune_default(p, k);
  return PM_OK;
}

int pm_plan_set_tuning(pm_plan* p, const int* shapes) {
  PM_TRY(check_plan(p));
  if (!shapes) return set_error(PM_ERR_ARG, "pm_plan_set_tuning: null pointer");
  for (int k = 0; k < 4; ++k)
    if (!tune_value_ok(p, k, shapes[k]))
      return set_error(PM_ERR_ARG, "pm_plan_set_tuning: %d is not a launch shape of slot %d", shapes[k], k);
  for (int k = 0; k < 4; ++k) p->tune[k] = shapes[k];
  return PM_OK;
}

int pm_plan_autotune(pm_plan* p, void* mesh_scratch, int reps, int use_cache, double* best_ms, void* stream) {
  PM_TRY(check_plan(p));
  if (!mesh_scratch) return set_error(PM_ERR_ARG, "pm_plan_autotune: null scratch mesh");
  if (reps < 1 || reps > 1000) return set_error(PM_ERR_ARG, "pm_plan_autotune: reps %d out of range", reps);
  drop_density(p);
  const auto key = std::make_tuple(p->device, p->n, p->dtype, p->nb);
  if (use_cache) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      for (int k = 0; k < 4; ++k) p->tune[k] = it->second[k];
      if (best_ms)
        for (int k = 0; k < 4; ++k) best_ms[k] = -1.0;
      return PM_OK;
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  // defined contents: a zero mesh and its (zero) spectrum
  PM_TRY(launch_fill(p, mesh_scratch, (int64_t)p->nb * p->n * p->n * p->n, 0.0, s));
  PM_TRY(fft_pass_rows_r2c(p, p->nb, mesh_scratch, cbuf(p, 0), s));
  hipEvent_t e0, e1;
  PM_TRY(hip_check(hipEventCreate(&e0), "autotune event"));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return set_error(PM_ERR_HIP, "autotune event");
  }
  int rc = PM_OK;
  for (int k = 0; k < 4 && rc == PM_OK; ++k) {
    int c[16];
    const int nc = std::min(fft_tune_candidates(p, k, c, 16), 16);
    int best = 0;
    float best_t = 0.0f;
    for (int i = 0; i < nc && rc == PM_OK; ++i) {
      p->tune[k] = c[i];
      rc = tune_run(p, k, mesh_scratch, s);  // warm
      if (rc) break;
      rc = hip_check(hipEventRecord(e0, s), "autotune record");
      for (int r = 0; r < reps && rc == PM_OK; ++r) rc = tune_run(p, k, mesh_scratch, s);
      if (rc) break;
      rc = hip_check(hipEventRecord(e1, s), "autotune record");
      if (rc) break;
      rc = hip_check(hipEventSynchronize(e1), "autotune sync");
      if (rc) break;
      float ms = 0.0f;
      rc = hip_check(hipEventElapsedTime(&ms, e0, e1), "autotune elapsed");
      if (rc) break;
      if (best == 0 || ms < best_t) {
        best = c[i];
        best_t = ms;
      }
    }
    p->tune[k] = best;
    if (best_ms) best_ms[k] = best_t / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) {
    for (int k = 0; k < 4; ++k) p->tune[k] = 0;
    return rc;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = std::vector<int>(p->tune, p->tune + 4);
  return PM_OK;
}

int pm_profile_enable(pm_plan* p, int on) {
  PM_TRY(check_plan(p));
  if (on && !p->prof) {
    p->prof = new (std::nothrow) ProfState();
    if (!p->prof) return set_error(PM_ERR_NOMEM, "pm_profile_enable: host allocation");
  } else if (!on && p->prof) {
    for (auto& r : p->prof->recs) {
      (void)hipEventSynchronize(r.stop);
      (void)hipEventDestroy(r.start);
      (void)hipEventDestroy(r.stop);
    }
    for (auto e : p->prof->pool) (void)hipEventDestroy(e);
    delete p->prof;
    p->prof = nullptr;
  }
  return PM_OK;
}

int pm_profile_read(pm_plan* p, int n_max, char* names, double* ms, int64_t* count) {
  PM_TRY(check_plan(p));
  if (!p->prof) return set_error(PM_ERR_ARG, "pm_profile_read: profiling is off");
  if (n_max < 0 || (n_max > 0 && (!names || !ms || !count))) return set_error(PM_ERR_ARG, "pm_profile_read: bad output");
  ProfState* ps = p->prof;
  for (auto& r : ps->recs) {
    PM_TRY(hip_check(hipEventSynchronize(r.stop), "pm_profile_read: event"));
    float t = 0.f;
    PM_TRY(hip_check(hipEventElapsedTime(&t, r.start, r.stop), "pm_profile_read: elapsed"));
    ps->ms[r.kind] += t;
    ps->count[r.kind] += 1;
    ps->pool.push_back(r.start);
    ps->pool.push_back(r.stop);
  }
  ps->recs.clear();
  int w = 0;
  for (int k = 0; k < PK_COUNT && w < n_max; ++k) {
    if (ps->count[k] == 0) continue;
    std::snprintf(names + 32 * (size_t)w, 32, "%s", kProfNames[k]);
    ms[w] = ps->ms[k];
    count[w] = ps->count[k];
    ++w;
  }
  for (int k = 0; k < PK_COUNT; ++k) {
    ps->ms[k] = 0.0;
    ps->count[k] = 0;
  }
  return w;
}

int pm_plan_destroy(pm_plan* p) {
  if (!p) return PM_OK;
  if (p->prof) pm_profile_enable(p, 0);
  if (p->own_ws && p->ws) (void)hipFree(p->ws);
  if (p->tw) (void)hipFree(p->tw);
  if (p->guard) (void)hipFree(p->guard);
  if (p->sums) (void)hipFree(p->sums);
  delete p;
  return PM_OK;
}

int pm_check(pm_plan* p, void* stream) {
  PM_TRY(check_plan(p));
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned h[4] = {0, 0, 0, 0};
  static const unsigned zeros[4] = {0, 0, 0, 0};
  PM_TRY(hip_check(hipMemcpyAsync(h, p->guard, sizeof(h), hipMemcpyDeviceToHost, s), "pm_check: read guards"));
  PM_TRY(hip_check(hipMemcpyAsync(p->guard, zeros, sizeof(zeros), hipMemcpyHostToDevice, s), "pm_check: reset"));
  PM_TRY(hip_check(hipStreamSynchronize(s), "pm_check: synchronise"));
  if (h[0] || h[1])
    return set_error(PM_ERR_STATE, "pm_check: %u non-finite positions skipped, %u positions outside [0,N) wrapped",
                     h[0], h[1]);
  return PM_OK;
}

// ------------------------------------------------------------- hot path ----

int pm_deposit(pm_plan* p, const void* pos, int64_t np, void* delta, void* stream) {
  PM_TRY(check_plan(p));
  drop_density(p);
  if (np < 0) return set_error(PM_ERR_ARG, "pm_deposit: negative particle count");
  if (!delta || (np > 0 && !pos)) return set_error(PM_ERR_ARG, "pm_deposit: null pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n3 = (int64_t)p->n * p->n * p->n;
  PM_TRY(launch_fill(p, delta, n3 * p->nb, -1.0, s));
  return launch_deposit(p, pos, np, delta, s);
}

// cbuf(0) holds the nb spectra after the row pass; writes force [3][nb][N^3].
static int solve_from_c0(pm_plan* p, const pm_solve_params* sp, void* phi, void* force, hipStream_t s) {
  const int64_t cs = cstride(p);
  PM_TRY(fft_pass_cols(p, cbuf(p, 0), 1, -1, p->nb, cs, s));
  PM_TRY(fft_pass_solve(p, sp, phi, s));
  return fft_force_inverse(p, sp->grad, force, s);
}

static int check_solve_params(const pm_solve_params* sp, const void* phi, const char* who) {
  if (!sp) return set_error(PM_ERR_ARG, "%s: null solve parameters", who);
  if (sp->kind != PM_NEWTON && sp->kind != PM_POISSON_GAUGE) return set_error(PM_ERR_ARG, "%s: bad kind", who);
  if (sp->grad < PM_GRAD_SPECTRAL || sp->grad > PM_GRAD_FD1) return set_error(PM_ERR_ARG, "%s: bad gradient", who);
  if (sp->kind == PM_POISSON_GAUGE) {
    if (!phi) return set_error(PM_ERR_ARG, "%s: Poisson-gauge solve needs phi_state", who);
    if (!(sp->c_g > 0.0)) return set_error(PM_ERR_ARG, "%s: c_g must be positive", who);
  }
  return PM_OK;
}

int pm_solve(pm_plan* p, const void* delta, const pm_solve_params* sp, void* phi_state, void* force, void* stream) {
  PM_TRY(check_plan(p));
  drop_density(p);
  if (!delta || !force) return set_error(PM_ERR_ARG, "pm_solve: null pointer");
  PM_TRY(check_solve_params(sp, phi_state, "pm_solve"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  PM_TRY(fft_pass_rows_r2c(p, p->nb, delta, cbuf(p, 0), s));
  return solve_from_c0(p, sp, phi_state, force, s);
}

int pm_gather(pm_plan* p, const void* force, const void* pos, int64_t np, void* acc, void* stream) {
  PM_TRY(check_single(p, "pm_gather"));
  drop_density(p);
  if (np < 0) return set_error(PM_ERR_ARG, "pm_gather: negative particle count");
  if (np > 0 && (!force || !pos || !acc)) return set_error(PM_ERR_ARG, "pm_gather: null pointer");
  return launch_gather(p, force, pos, np, acc, static_cast<hipStream_t>(stream));
}

int pm_step(pm_plan* p, void* pos, void* mom, int64_t np, const pm_step_params* st, void* force_scratch,
            void* phi_state, void* stream) {
  PM_TRY(check_plan(p));
  if (np < 0) return set_error(PM_ERR_ARG, "pm_step: negative particle count");
  if (!st || !force_scratch || (np > 0 && (!pos || !mom))) return set_error(PM_ERR_ARG, "pm_step: null pointer");
  PM_TRY(check_solve_params(&st->solve, phi_state, "pm_step"));
  if (st->flags & ~(PM_STEP_DEPOSIT_NEXT | PM_STEP_DENSITY_READY)) return set_error(PM_ERR_ARG, "pm_step: bad flags");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n3 = (int64_t)p->n * p->n * p->n;
  if (p->nb > 1 && np != n3) return set_error(PM_ERR_ARG, "pm_step: a batch needs N^3 particles per box");
  const bool ready = p->dens_valid && p->dens_pos == pos && p->dens_np == np;
  if ((st->flags & PM_STEP_DENSITY_READY) && !ready) {
    p->dens_valid = false;
    return set_error(PM_ERR_STATE, "pm_step: the plan holds no density of these positions from a previous step");
  }
  p->dens_valid = false;
  PM_TRY(step_cycle(p, pos, mom, np, st, force_scratch, phi_state, s));
  if (st->flags & PM_STEP_DEPOSIT_NEXT) {
    p->dens_valid = true;
    p->dens_pos = pos;
    p->dens_np = np;
  }
  return PM_OK;
}

}  // extern "C"

namespace pm {

// The launches of one force-kick-drift cycle on all of the plan's boxes (arguments
// already checked; the density bookkeeping is the caller's): with
// PM_STEP_DENSITY_READY the plan's density meshes must hold the density of `pos`;
// with PM_STEP_DEPOSIT_NEXT they hold that of the drifted positions on return.  When
// the fused gather kernel deposits the next density, the meshes are refilled with -1
// as soon as the r2c pass has read them.
int step_cycle(pm_plan* p, void* pos, void* mom, int64_t np, const pm_step_params* st, void* force_scratch,
               void* phi_state, hipStream_t s) {
  const int64_t n3 = (int64_t)p->n * p->n * p->n;
  void* delta = p->dens;
  if (!(st->flags & PM_STEP_DENSITY_READY)) {
    PM_TRY(launch_fill(p, delta, n3 * p->nb, -1.0, s));
    PM_TRY(launch_deposit(p, pos, np, delta, s));
  }
  PM_TRY(fft_pass_rows_r2c(p, p->nb, delta, cbuf(p, 0), s));
  const bool fused = (st->flags & PM_STEP_DEPOSIT_NEXT) && gather_kdk_can_deposit(p, np);
  if (fused) PM_TRY(launch_fill(p, delta, n3 * p->nb, -1.0, s));
  PM_TRY(solve_from_c0(p, &st->solve, phi_state, force_scratch, s));
  if (!(st->flags & PM_STEP_DEPOSIT_NEXT))
    return launch_gather_kdk(p, force_scratch, pos, mom, np, st->kick, st->drift, nullptr, s);
  if (fused) {
    PM_TRY(launch_gather_kdk(p, force_scratch, pos, mom, np, st->kick, st->drift, delta, s));
  } else {
    PM_TRY(launch_fill(p, delta, n3 * p->nb, -1.0, s));
    PM_TRY(launch_gather_kdk(p, force_scratch, pos, mom, np, st->kick, st->drift, nullptr, s));
    PM_TRY(launch_deposit(p, pos, np, delta, s));
  }
  return PM_OK;
}

}  // namespace pm

extern "C" {

// Argument checks shared by pm_step_adjoint and its allocation-free variant.
static int check_step_adjoint(pm_plan* p, const void* pos, int64_t np, const pm_step_params* st, void* lam_pos,
                              void* lam_mom, const char* who) {
  PM_TRY(check_single(p, who));
  drop_density(p);
  if (np < 0) return set_error(PM_ERR_ARG, "%s: negative particle count", who);
  if (!st || (np > 0 && (!pos || !lam_pos || !lam_mom))) return set_error(PM_ERR_ARG, "%s: null pointer", who);
  if (st->solve.kind != PM_NEWTON) return set_error(PM_ERR_ARG, "%s: only the Newtonian step has an adjoint", who);
  return check_solve_params(&st->solve, nullptr, who);
}

// The adjoint cycle on `mesh_scratch` (3 N^3 reals, or 6 N^3 when force is null).
static int step_adjoint(pm_plan* p, const void* pos, int64_t np, const pm_step_params* st, const void* force,
                        void* mesh_scratch, void* lam_pos, void* lam_mom, hipStream_t s) {
  const int64_t n3 = (int64_t)p->n * p->n * p->n;
  const size_t mesh_bytes = (size_t)n3 * p->esize;
  char* g = static_cast<char*>(mesh_scratch);
  if (!force) {
    void* fs = g + 3 * mesh_bytes;
    void* delta = p->dens;
    PM_TRY(launch_fill(p, delta, n3, -1.0, s));
    PM_TRY(launch_deposit(p, pos, np, delta, s));
    PM_TRY(fft_pass_rows_r2c(p, 1, delta, cbuf(p, 0), s));
    PM_TRY(solve_from_c0(p, &st->solve, nullptr, fs, s));
    force = fs;
  }
  if (np == 0) return PM_OK;
  PM_TRY(launch_fill(p, g, 3 * n3, 0.0, s));
  PM_TRY(launch_adj_gather_kdk(p, force, pos, np, st->kick, st->drift, lam_pos, lam_mom, g, s));
  PM_TRY(fft3_r2c_n(p, 3, g, cbuf(p, 0), s));  // the three components in one set of launches
  PM_TRY(launch_div_newton(p, st->solve.grad, 1.5 * st->solve.omega_m / (double)n3, s));
  PM_TRY(fft3_c2r(p, 1, cbuf(p, 0), 0, g, s));
  return launch_grad_gather(p, g, pos, np, (double)n3 / (double)np, lam_pos, true, s);
}

int pm_step_adjoint(pm_plan* p, const void* pos, int64_t np, const pm_step_params* st, const void* force,
                    void* mesh_scratch, void* lam_pos, void* lam_mom, void* stream) {
  PM_TRY(check_step_adjoint(p, pos, np, st, lam_pos, lam_mom, "pm_step_adjoint"));
  if (!mesh_scratch) return set_error(PM_ERR_ARG, "pm_step_adjoint: null pointer");
  return step_adjoint(p, pos, np, st, force, mesh_scratch, lam_pos, lam_mom, static_cast<hipStream_t>(stream));
}

size_t pm_step_adjoint_noalloc_bytes(int n_mesh, int dtype, int with_force) {
  if (!mesh_supported(n_mesh) || (dtype != PM_F32 && dtype != PM_F64)) return 0;
  return (with_force ? 3 : 6) * (size_t)n_mesh * n_mesh * n_mesh * (dtype == PM_F32 ? 4 : 8);
}

int pm_step_adjoint_noalloc(pm_plan* p, const void* pos, int64_t np, const pm_step_params* st, const void* force,
                            void* lam_pos, void* lam_mom, void* stream) {
  PM_TRY(check_step_adjoint(p, pos, np, st, lam_pos, lam_mom, "pm_step_adjoint_noalloc"));
  const size_t need = pm_step_adjoint_noalloc_bytes(p->n, p->dtype, force != nullptr);
  if (need > kStaticScratchBytes)
    return set_error(PM_ERR_NOMEM,
                     "pm_step_adjoint_noalloc: N = %d (%s, force %s) needs %zu bytes of scratch, more than the "
                     "static %zu; use pm_step_adjoint with a caller workspace",
                     p->n, p->dtype == PM_F32 ? "FP32" : "FP64", force ? "given" : "recomputed", need,
                     kStaticScratchBytes);
  void* g = static_scratch(p->device);
  if (!g) return set_error(PM_ERR_STATE, "pm_step_adjoint_noalloc: no static scratch on device %d", p->device);
  return step_adjoint(p, pos, np, st, force, g, lam_pos, lam_mom, static_cast<hipStream_t>(stream));
}

int pk_adjoint(pm_plan* p, const void* pos, int64_t np, int n_bins, const double* dpk, void* lam_pos, void* stream) {
  PM_TRY(check_single(p, "pk_adjoint"));
  drop_density(p);
  if (np < 0) return set_error(PM_ERR_ARG, "pk_adjoint: negative particle count");
  if (!dpk || (np > 0 && (!pos || !lam_pos))) return set_error(PM_ERR_ARG, "pk_adjoint: null pointer");
  if (n_bins <= 0 || 3 * (size_t)n_bins > p->sums_cap || n_bins > 4 * p->n)
    return set_error(PM_ERR_ARG, "pk_adjoint: n_bins %d out of range", n_bins);
  if (np == 0) return PM_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n3 = (int64_t)p->n * p->n * p->n;
  void* delta = p->dens;
  PM_TRY(launch_fill(p, delta, n3, -1.0, s));
  PM_TRY(launch_deposit(p, pos, np, delta, s));
  PM_TRY(fft3_r2c(p, delta, cbuf(p, 0), s));
  PM_TRY(launch_zero_doubles(p->sums, 3 * (int64_t)n_bins, s));
  PM_TRY(launch_pk_reduce(p, cbuf(p, 0), n_bins, s));
  PM_TRY(launch_pk_adjoint_weight(p, cbuf(p, 0), n_bins, dpk, s));
  PM_TRY(fft3_c2r(p, 1, cbuf(p, 0), 0, delta, s));
  return launch_grad_gather(p, delta, pos, np, (double)n3 / (double)np, lam_pos, false, s);
}

int displacement_combine(const void* x_gr, const void* x_newton, int n_coarse, const void* x_fine, int n_fine,
                         int dtype, void* x_out, void* stream) {
  g_err[0] = 0;
  if (!x_gr || !x_newton || !x_fine || !x_out) return set_error(PM_ERR_ARG, "displacement_combine: null pointer");
  if (n_coarse <= 0 || n_fine <= 0 || n_fine % n_coarse != 0)
    return set_error(PM_ERR_ARG, "displacement_combine: n_fine (%d) must be a positive multiple of n_coarse (%d)",
                     n_fine, n_coarse);
  if (n_fine > 4096) return set_error(PM_ERR_SIZE, "displacement_combine: n_fine too large");
  if (dtype != PM_F32 && dtype != PM_F64) return set_error(PM_ERR_ARG, "displacement_combine: bad dtype");
  return launch_combine(x_gr, x_newton, n_coarse, x_fine, n_fine, dtype, x_out, static_cast<hipStream_t>(stream));
}

int displacement_add(const void* xi, int n_coarse, const void* x_fine, int n_fine, int dtype, void* x_out,
                     void* stream) {
  g_err[0] = 0;
  if (!xi || !x_fine || !x_out) return set_error(PM_ERR_ARG, "displacement_add: null pointer");
  if (n_coarse <= 0 || n_fine <= 0 || n_fine % n_coarse != 0)
    return set_error(PM_ERR_ARG, "displacement_add: n_fine (%d) must be a positive multiple of n_coarse (%d)", n_fine,
                     n_coarse);
  if (n_fine > 4096) return set_error(PM_ERR_SIZE, "displacement_add: n_fine too large");
  if (dtype != PM_F32 && dtype != PM_F64) return set_error(PM_ERR_ARG, "displacement_add: bad dtype");
  return launch_combine(xi, nullptr, n_coarse, x_fine, n_fine, dtype, x_out, static_cast<hipStream_t>(stream));
}

int pk_estimate(pm_plan* p, const void* delta, int n_bins, double* k_mean, double* pk, int64_t* n_modes,
                void* stream) {
  PM_TRY(check_plan(p));
  drop_density(p);
  if (!delta || !k_mean || !pk || !n_modes) return set_error(PM_ERR_ARG, "pk_estimate: null pointer");
  if (n_bins <= 0 || 3 * (size_t)n_bins * p->nb > p->sums_cap || n_bins > 4 * p->n)
    return set_error(PM_ERR_ARG, "pk_estimate: n_bins %d out of range", n_bins);
  hipStream_t s = static_cast<hipStream_t>(stream);
  PM_TRY(fft3_r2c(p, delta, cbuf(p, 0), s));
  PM_TRY(launch_zero_doubles(p->sums, 3 * (int64_t)n_bins * p->nb, s));
  PM_TRY(launch_pk_reduce(p, cbuf(p, 0), n_bins, s));
  return launch_pk_finalize(p, n_bins, k_mean, pk, n_modes, s);
}

int pk_cross_estimate(pm_plan* p, const void* delta_a, const void* delta_b, int n_bins, double* k_mean, double* pk,
                      int64_t* n_modes, void* stream) {
  PM_TRY(check_plan(p));
  drop_density(p);
  if (!delta_a || !delta_b || !k_mean || !pk || !n_modes) return set_error(PM_ERR_ARG, "pk_cross_estimate: null pointer");
  if (n_bins <= 0 || 3 * (size_t)n_bins * p->nb > p->sums_cap || n_bins > 4 * p->n)
    return set_error(PM_ERR_ARG, "pk_cross_estimate: n_bins %d out of range", n_bins);
  hipStream_t s = static_cast<hipStream_t>(stream);
  PM_TRY(fft3_r2c(p, delta_a, cbuf(p, 0), s));
  PM_TRY(fft3_r2c(p, delta_b, cbuf(p, 1), s));
  PM_TRY(launch_zero_doubles(p->sums, 3 * (int64_t)n_bins * p->nb, s));
  PM_TRY(launch_pk_reduce(p, cbuf(p, 0), n_bins, s, cbuf(p, 1)));
  return launch_pk_finalize(p, n_bins, k_mean, pk, n_modes, s);
}

int bias_fit(const double* k, const double* ratio, const int64_t* n_modes, int n_bins, double k_cut, double calh,
             int skip, int with_k2, double* coef) {
  g_err[0] = 0;
  if (!k || !ratio || !n_modes || !coef) return set_error(PM_ERR_ARG, "bias_fit: null pointer");
  if (n_bins <= 0 || skip < 0 || !(k_cut > 0.0)) return set_error(PM_ERR_ARG, "bias_fit: bad arguments");
  const int m = with_k2 ? 3 : 2;
  // weighted normal equations (weights: mode counts) over 0 < k < k_cut, after `skip` bins
  double a[3][3] = {{0}}, r[3] = {0};
  int used = 0, seen = 0;
  for (int b = 0; b < n_bins; ++b) {
    if (n_modes[b] <= 0 || !(k[b] > 0.0 && k[b] < k_cut)) continue;
    if (seen++ < skip) continue;
    const double x[3] = {1.0, calh * calh / (k[b] * k[b]), k[b] * k[b]};
    const double w = (double)n_modes[b];
    for (int i = 0; i < m; ++i) {
      r[i] += w * x[i] * ratio[b];
      for (int j = 0; j < m; ++j) a[i][j] += w * x[i] * x[j];
    }
    ++used;
  }
  if (used < m) return set_error(PM_ERR_ARG, "bias_fit: %d bins below k_cut after the skip, %d needed", used, m);
  // equilibrate to a unit diagonal (the columns differ by orders of magnitude), so that
  // a pivot below 1e-10 means linearly dependent columns
  double dsc[3];
  for (int i = 0; i < m; ++i) {
    if (!(a[i][i] > 0.0)) return set_error(PM_ERR_ARG, "bias_fit: singular system");
    dsc[i] = 1.0 / std::sqrt(a[i][i]);
  }
  for (int i = 0; i < m; ++i) {
    r[i] *= dsc[i];
    for (int j = 0; j < m; ++j) a[i][j] *= dsc[i] * dsc[j];
  }
  // Gaussian elimination with partial pivoting
  for (int c = 0; c < m; ++c) {
    int piv = c;
    for (int i = c + 1; i < m; ++i)
      if (std::fabs(a[i][c]) > std::fabs(a[piv][c])) piv = i;
    if (!(std::fabs(a[piv][c]) > 1e-10)) return set_error(PM_ERR_ARG, "bias_fit: singular system");
    if (piv != c) {
      for (int j = 0; j < m; ++j) std::swap(a[c][j], a[piv][j]);
      std::swap(r[c], r[piv]);
    }
    for (int i = c + 1; i < m; ++i) {
      const double f = a[i][c] / a[c][c];
      for (int j = c; j < m; ++j) a[i][j] -= f * a[c][j];
      r[i] -= f * r[c];
    }
  }
  double x[3] = {0.0, 0.0, 0.0};
  for (int i = m - 1; i >= 0; --i) {
    double v = r[i];
    for (int j = i + 1; j < m; ++j) v -= a[i][j] * x[j];
    x[i] = v / a[i][i];
  }
  for (int i = 0; i < 3; ++i) coef[i] = i < m ? x[i] * dsc[i] : 0.0;
  return PM_OK;
}

// Order in which the triangles of bk_estimate are evaluated: greedily, the next shell
// field to compute is the one that completes the most pending triangles together with
// the shells computed so far (ties: the shell used by more pending triangles, then the
// lower id), and each triangle follows the computation of its last shell.  For the
// usual sets (equilateral k, and squeezed k1 = k2 with a common k3) every shell is
// transformed once and each triangle directly follows its shells.
static std::vector<int> bk_triangle_order(int n_shells, const int32_t* tri, int n_tri) {
  std::vector<char> done(n_tri, 0), have(n_shells, 0);
  std::vector<int> order;
  order.reserve(n_tri);
  auto complete = [&](int t, int extra) {
    for (int j = 0; j < 3; ++j) {
      const int sh = tri[3 * t + j];
      if (!have[sh] && sh != extra) return false;
    }
    return true;
  };
  while ((int)order.size() < n_tri) {
    for (int t = 0; t < n_tri; ++t)
      if (!done[t] && complete(t, -1)) {
        done[t] = 1;
        order.push_back(t);
      }
    if ((int)order.size() == n_tri) break;
    std::vector<int> score(n_shells, 0), uses(n_shells, 0);
    for (int t = 0; t < n_tri; ++t) {
      if (done[t]) continue;
      for (int j = 0; j < 3; ++j) {
        const int sh = tri[3 * t + j];
        if (j > 0 && (sh == tri[3 * t] || (j == 2 && sh == tri[3 * t + 1]))) continue;
        uses[sh] += 1;
        if (!have[sh] && complete(t, sh)) score[sh] += 1;
      }
    }
    int best = -1;
    for (int sh = 0; sh < n_shells; ++sh) {
      if (have[sh] || uses[sh] == 0) continue;
      if (best < 0 || score[sh] > score[best] || (score[sh] == score[best] && uses[sh] > uses[best])) best = sh;
    }
    have[best] = 1;
  }
  return order;
}

int bk_estimate(pm_plan* p, const void* delta, int n_shells, const double* centre, double width, const int32_t* tri,
                int n_tri, double* bk, double* ntri_out, const double* ntri_known, void* shell_ws,
                size_t shell_ws_bytes, void* stream) {
  PM_TRY(check_single(p, "bk_estimate"));
  drop_density(p);
  if (!delta || !centre || !tri || !bk || !ntri_out || !shell_ws) return set_error(PM_ERR_ARG, "bk_estimate: null pointer");
  if (n_shells <= 0 || n_tri <= 0 || !(width > 0.0)) return set_error(PM_ERR_ARG, "bk_estimate: bad sizes");
  if (2 * (size_t)n_tri > p->sums_cap) return set_error(PM_ERR_ARG, "bk_estimate: too many triangles");
  for (int t = 0; t < 3 * n_tri; ++t)
    if (tri[t] < 0 || tri[t] >= n_shells) return set_error(PM_ERR_ARG, "bk_estimate: shell id out of range");
  const size_t fbytes = align256((size_t)p->n * p->n * p->n * p->esize);
  const int slots = (int)std::min<size_t>(shell_ws_bytes / fbytes, 1 << 20);
  if (slots < 3) return set_error(PM_ERR_NOMEM, "bk_estimate: shell workspace holds %d fields, 3 needed", slots);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const std::vector<int> order = bk_triangle_order(n_shells, tri, n_tri);
  PM_TRY(fft3_r2c(p, delta, cbuf(p, 0), s));
  PM_TRY(launch_zero_doubles(p->sums, 2 * (int64_t)n_tri, s));
  char* base = static_cast<char*>(shell_ws);
  const int passes = ntri_known ? 1 : 2;  // 0: the density's shells; 1: the shells' indicators
  for (int pass = 0; pass < passes; ++pass) {
    std::vector<int> slot_shell(slots, -1);
    TriPass tp{};  // triangles gathered for one pass over their fields
    auto flush = [&]() -> int {
      if (tp.nt == 0) return PM_OK;
      const int rc = launch_triple_multi(p, tp, s);
      tp = TriPass{};
      return rc;
    };
    auto pass_field = [&](int slot) {
      for (int f = 0; f < tp.nf; ++f)
        if (tp.field[f] == base + (size_t)slot * fbytes) return f;
      return -1;
    };
    for (int oi = 0; oi < n_tri; ++oi) {
      const int t = order[oi];
      // distinct shells of t: missing ones must be computed into slots that hold
      // neither t's other shells nor the fields of the gathered triangles
      int ts[3], nts = 0;
      for (int j = 0; j < 3; ++j) {
        const int sh = tri[3 * t + j];
        if (std::find(ts, ts + nts, sh) == ts + nts) ts[nts++] = sh;
      }
      int missing = 0, new_fields = 0, resident_outside = 0;
      for (int j = 0; j < nts; ++j) {
        const int k = (int)(std::find(slot_shell.begin(), slot_shell.end(), ts[j]) - slot_shell.begin());
        if (k == slots) {
          ++missing;
          ++new_fields;
        } else if (pass_field(k) < 0) {
          ++new_fields;
          ++resident_outside;
        }
      }
      if (tp.nt == kMaxTriPerPass || tp.nf + new_fields > kMaxFieldsPerPass ||
          slots - (tp.nf + resident_outside) < missing)
        PM_TRY(flush());
      int fidx[3];
      for (int j = 0; j < 3; ++j) {
        const int sh = tri[3 * t + j];
        int found = (int)(std::find(slot_shell.begin(), slot_shell.end(), sh) - slot_shell.begin());
        if (found == slots) {
          // evict the shell whose next use is farthest; never one of this triangle or of
          // the gathered triangles
          int best = -1;
          long best_next = -1;
          for (int k = 0; k < slots; ++k) {
            const int cs = slot_shell[k];
            if (cs < 0) {
              best = k;
              break;
            }
            if (cs == tri[3 * t] || cs == tri[3 * t + 1] || cs == tri[3 * t + 2] || pass_field(k) >= 0) continue;
            long next = (long)n_tri + 1;
            for (int u = oi + 1; u < n_tri && next > (long)n_tri; ++u) {
              const int tu = order[u];
              if (tri[3 * tu] == cs || tri[3 * tu + 1] == cs || tri[3 * tu + 2] == cs) next = u;
            }
            if (next > best_next) {
              best_next = next;
              best = k;
            }
          }
          if (best < 0) return set_error(PM_ERR_STATE, "bk_estimate: no shell slot to evict");
          const double c = centre[sh];
          const double lo = (2.0 * c - width) * (2.0 * c - width);
          const double hi = (2.0 * c + width) * (2.0 * c + width);
          PM_TRY(fft3_c2r_shell(p, pass == 0 ? cbuf(p, 0) : nullptr, cbuf(p, 1), base + (size_t)best * fbytes, lo, hi,
                                s));
          slot_shell[best] = sh;
          found = best;
        }
        int f = pass_field(found);
        if (f < 0) {
          f = tp.nf++;
          tp.field[f] = base + (size_t)found * fbytes;
        }
        fidx[j] = f;
      }
      for (int j = 0; j < 3; ++j) tp.idx[tp.nt][j] = fidx[j];
      tp.slot[tp.nt] = p->sums + (size_t)pass * n_tri + t;
      tp.nt += 1;
    }
    PM_TRY(flush());
  }
  return launch_bk_finalize(p, n_tri, p->sums, bk, ntri_out, ntri_known, s);
}

}  // extern "C"
