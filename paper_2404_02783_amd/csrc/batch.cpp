// C ABI of uneven ensembles (pm_batch_*): boxes of several mesh sizes advanced by
// grouped launches.  Boxes with equal mesh size and side form a size group with one
// internal batched plan; each call issues every kernel once per group, for all of the
// group's boxes, and the particle kernels find each box's arrays (and kick and drift)
// in the group's device table, which a small kernel refreshes at every call from
// values passed as kernel arguments (so the calls can be captured in a graph).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "pm_common.h"
#include "pm_plan.h"

#define PM_BATCH_TRY(expr)     \
  do {                         \
    const int rc_ = (expr);    \
    if (rc_ != PM_OK) return rc_; \
  } while (0)

namespace pm {
namespace {

constexpr int kTabChunk = 32;
struct TabChunk {
  BoxEntry e[kTabChunk];
  int offset, count;
};

__global__ void k_set_box_tab(BoxEntry* __restrict__ tab, TabChunk c) {
  const int i = threadIdx.x;
  if (i < c.count) tab[c.offset + i] = c.e[i];
}

}  // namespace
}  // namespace pm

struct pm_batch {
  struct Group {
    int n = 0;
    double box = 0.0;
    std::vector<int> boxes;     // batch indices of the group's boxes, in batch order
    pm_plan* plan = nullptr;    // batched plan of the group (box_tab = tab)
    pm::BoxEntry* tab = nullptr;  // device [boxes]
    void* force = nullptr;      // [3][boxes][N^3] force meshes (also the ICs' displacement)
    void* mesh = nullptr;       // [boxes][N^3] staging: noise copies, densities for P(k)
    double* kmean = nullptr;    // [boxes][4N] P(k) outputs of the group plan
    double* pk = nullptr;
    int64_t* nmodes = nullptr;
    hipStream_t stream = nullptr;  // PM_BATCH_CONCURRENT only
    hipEvent_t done = nullptr;
    bool dens_valid = false;
    std::vector<const void*> dens_pos;
  };
  int dtype = PM_F32;
  int flags = 0;
  int n_box = 0;
  std::vector<Group> groups;
  std::vector<int> box_group, box_slot;
  hipEvent_t fork = nullptr;
};

namespace pm {
namespace {

size_t esize_of(int dtype) { return dtype == PM_F32 ? 4 : 8; }

void free_group(pm_batch::Group& g) {
  if (g.plan) pm_plan_destroy(g.plan);
  if (g.tab) (void)hipFree(g.tab);
  if (g.force) (void)hipFree(g.force);
  if (g.mesh) (void)hipFree(g.mesh);
  if (g.kmean) (void)hipFree(g.kmean);
  if (g.pk) (void)hipFree(g.pk);
  if (g.nmodes) (void)hipFree(g.nmodes);
  if (g.done) (void)hipEventDestroy(g.done);
  if (g.stream) (void)hipStreamDestroy(g.stream);
  g = pm_batch::Group();
}

int hip_ok(hipError_t e, const char* what) {
  if (e == hipSuccess) return PM_OK;
  return set_error(PM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Writes the group's table: box j's entry from pos[box], mom[box] and kick/drift.
int set_table(const pm_batch::Group& g, void* const* pos, void* const* mom, const pm_step_params* per_box,
              hipStream_t s) {
  const int nb = (int)g.boxes.size();
  for (int o = 0; o < nb; o += kTabChunk) {
    TabChunk c;
    std::memset(&c, 0, sizeof(c));
    c.offset = o;
    c.count = std::min(kTabChunk, nb - o);
    for (int j = 0; j < c.count; ++j) {
      const int b = g.boxes[o + j];
      c.e[j].pos = pos[b];
      c.e[j].mom = mom ? mom[b] : nullptr;
      c.e[j].kick = per_box ? per_box[b].kick : 0.0;
      c.e[j].drift = per_box ? per_box[b].drift : 0.0;
    }
    hipLaunchKernelGGL(k_set_box_tab, dim3(1), dim3(kTabChunk), 0, s, g.tab, c);
  }
  return hip_ok(hipGetLastError(), "box table");
}

// Runs fn(group, stream) for every group: on the caller's stream, or (concurrent
// batches) on each group's stream, forked from and joined back into the caller's.
template <typename F>
int for_groups(pm_batch* b, hipStream_t s, F fn) {
  const bool conc = (b->flags & PM_BATCH_CONCURRENT) != 0;
  if (conc) {
    int rc = hip_ok(hipEventRecord(b->fork, s), "batch fork");
    if (rc) return rc;
  }
  for (auto& g : b->groups) {
    hipStream_t gs = s;
    if (conc) {
      gs = g.stream;
      int rc = hip_ok(hipStreamWaitEvent(gs, b->fork, 0), "batch fork wait");
      if (rc) return rc;
    }
    int rc = fn(g, gs);
    if (rc) return rc;
    if (conc) {
      rc = hip_ok(hipEventRecord(g.done, gs), "batch join");
      if (rc) return rc;
      rc = hip_ok(hipStreamWaitEvent(s, g.done, 0), "batch join wait");
      if (rc) return rc;
    }
  }
  return PM_OK;
}

bool same_solve(const pm_solve_params& a, const pm_solve_params& b) {
  return a.kind == b.kind && a.grad == b.grad && a.omega_m == b.omega_m && a.a == b.a && a.om_a == b.om_a &&
         a.calh == b.calh && a.c_g == b.c_g && a.inv_dtau == b.inv_dtau;
}

int check_ptrs(const pm_batch* b, void* const* a, const char* what, const char* who) {
  if (!a) return set_error(PM_ERR_ARG, "%s: null %s array", who, what);
  for (int i = 0; i < b->n_box; ++i)
    if (!a[i]) return set_error(PM_ERR_ARG, "%s: null %s pointer of box %d", who, what, i);
  return PM_OK;
}

}  // namespace
}  // namespace pm

extern "C" {

int pm_batch_create(pm_batch** out, int n_box, const int* n_mesh, const double* box_mpch, int dtype, int flags) {
  using namespace pm;
  if (!out) return set_error(PM_ERR_ARG, "pm_batch_create: null output pointer");
  *out = nullptr;
  if (n_box < 1 || !n_mesh || !box_mpch) return set_error(PM_ERR_ARG, "pm_batch_create: no boxes");
  if (dtype != PM_F32 && dtype != PM_F64) return set_error(PM_ERR_ARG, "pm_batch_create: bad dtype %d", dtype);
  if (flags & ~PM_BATCH_CONCURRENT) return set_error(PM_ERR_ARG, "pm_batch_create: bad flags");
  for (int i = 0; i < n_box; ++i) {
    if (pm_plan_workspace_bytes(n_mesh[i], dtype) == 0)
      return set_error(PM_ERR_SIZE, "pm_batch_create: unsupported mesh size %d (box %d)", n_mesh[i], i);
    if (!(box_mpch[i] > 0.0)) return set_error(PM_ERR_ARG, "pm_batch_create: box %d has no positive side", i);
  }
  pm_batch* b = new (std::nothrow) pm_batch();
  if (!b) return set_error(PM_ERR_NOMEM, "pm_batch_create: host allocation failed");
  b->dtype = dtype;
  b->flags = flags;
  b->n_box = n_box;
  b->box_group.assign(n_box, -1);
  b->box_slot.assign(n_box, -1);
  // size groups, largest meshes first
  std::vector<int> order(n_box);
  for (int i = 0; i < n_box; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    if (n_mesh[x] != n_mesh[y]) return n_mesh[x] > n_mesh[y];
    return box_mpch[x] < box_mpch[y];
  });
  for (int i : order) {
    if (b->groups.empty() || b->groups.back().n != n_mesh[i] || b->groups.back().box != box_mpch[i]) {
      b->groups.emplace_back();
      b->groups.back().n = n_mesh[i];
      b->groups.back().box = box_mpch[i];
    }
    b->box_group[i] = (int)b->groups.size() - 1;
    b->box_slot[i] = (int)b->groups.back().boxes.size();
    b->groups.back().boxes.push_back(i);
  }
  for (auto& bg : b->groups) std::sort(bg.boxes.begin(), bg.boxes.end());
  for (int gi = 0; gi < (int)b->groups.size(); ++gi)
    for (int j = 0; j < (int)b->groups[gi].boxes.size(); ++j) b->box_slot[b->groups[gi].boxes[j]] = j;
  int rc = PM_OK;
  const size_t es = esize_of(dtype);
  for (auto& g : b->groups) {
    const int nb = (int)g.boxes.size();
    const size_t n3 = (size_t)g.n * g.n * g.n;
    rc = pm_plan_create_batch(&g.plan, g.n, g.box, dtype, nb, nullptr, 0);
    if (rc) break;
    if (hipMalloc(&g.tab, nb * sizeof(BoxEntry)) != hipSuccess || hipMalloc(&g.force, 3 * nb * n3 * es) != hipSuccess ||
        hipMalloc(&g.mesh, nb * n3 * es) != hipSuccess ||
        hipMalloc(&g.kmean, (size_t)nb * 4 * g.n * sizeof(double)) != hipSuccess ||
        hipMalloc(&g.pk, (size_t)nb * 4 * g.n * sizeof(double)) != hipSuccess ||
        hipMalloc(&g.nmodes, (size_t)nb * 4 * g.n * sizeof(int64_t)) != hipSuccess) {
      rc = set_error(PM_ERR_NOMEM, "pm_batch_create: device allocation for the %d^3 group", g.n);
      break;
    }
    g.plan->box_tab = g.tab;
    if (flags & PM_BATCH_CONCURRENT) {
      // default priority (streams of other priorities are not used anywhere here)
      rc = hip_ok(hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking), "pm_batch_create: stream");
      if (rc) break;
      rc = hip_ok(hipEventCreateWithFlags(&g.done, hipEventDisableTiming), "pm_batch_create: event");
      if (rc) break;
    }
  }
  if (rc == PM_OK && (flags & PM_BATCH_CONCURRENT))
    rc = hip_ok(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming), "pm_batch_create: event");
  if (rc != PM_OK) {
    pm_batch_destroy(b);
    return rc;
  }
  *out = b;
  return PM_OK;
}

int pm_batch_destroy(pm_batch* b) {
  if (!b) return PM_OK;
  (void)hipDeviceSynchronize();
  for (auto& g : b->groups) pm::free_group(g);
  if (b->fork) (void)hipEventDestroy(b->fork);
  delete b;
  return PM_OK;
}

int pm_batch_num_groups(const pm_batch* b) { return b ? (int)b->groups.size() : 0; }

int pm_batch_group(const pm_batch* b, int group, int* n_mesh, double* box_mpch, int* n_boxes, pm_plan** plan) {
  using namespace pm;
  if (!b || group < 0 || group >= (int)b->groups.size()) return set_error(PM_ERR_ARG, "pm_batch_group: no such group");
  const auto& g = b->groups[group];
  if (n_mesh) *n_mesh = g.n;
  if (box_mpch) *box_mpch = g.box;
  if (n_boxes) *n_boxes = (int)g.boxes.size();
  if (plan) *plan = g.plan;
  return PM_OK;
}

int pm_batch_step(pm_batch* b, void* const* pos, void* const* mom, const pm_step_params* per_box, void* stream) {
  using namespace pm;
  if (!b) return set_error(PM_ERR_ARG, "pm_batch_step: null batch");
  PM_BATCH_TRY(check_ptrs(b, pos, "pos", "pm_batch_step"));
  PM_BATCH_TRY(check_ptrs(b, mom, "mom", "pm_batch_step"));
  if (!per_box) return set_error(PM_ERR_ARG, "pm_batch_step: null per-box parameters");
  for (auto& g : b->groups) {
    const pm_step_params& s0 = per_box[g.boxes[0]];
    if (s0.solve.kind != PM_NEWTON)
      return set_error(PM_ERR_ARG, "pm_batch_step: only Newtonian steps (the Poisson gauge carries a potential)");
    if (s0.flags & ~(PM_STEP_DEPOSIT_NEXT | PM_STEP_DENSITY_READY))
      return set_error(PM_ERR_ARG, "pm_batch_step: bad flags");
    for (int j : g.boxes) {
      if (per_box[j].flags != s0.flags || !same_solve(per_box[j].solve, s0.solve))
        return set_error(PM_ERR_ARG, "pm_batch_step: boxes %d and %d of the %d^3 group differ in flags or solve "
                                     "parameters", g.boxes[0], j, g.n);
      if (!(per_box[j].kick == per_box[j].kick) || !(per_box[j].drift == per_box[j].drift))
        return set_error(PM_ERR_ARG, "pm_batch_step: non-finite kick or drift of box %d", j);
    }
    if (s0.flags & PM_STEP_DENSITY_READY) {
      bool ok = g.dens_valid && g.dens_pos.size() == g.boxes.size();
      for (size_t j = 0; ok && j < g.boxes.size(); ++j) ok = g.dens_pos[j] == pos[g.boxes[j]];
      if (!ok) {
        for (auto& h : b->groups) h.dens_valid = false;
        return set_error(PM_ERR_STATE, "pm_batch_step: the %d^3 group holds no density of these positions", g.n);
      }
    }
  }
  for (auto& g : b->groups) {
    const int gr = per_box[g.boxes[0]].solve.grad;
    if (gr < PM_GRAD_SPECTRAL || gr > PM_GRAD_FD1) return set_error(PM_ERR_ARG, "pm_batch_step: bad gradient");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int rc = for_groups(b, s, [&](pm_batch::Group& g, hipStream_t gs) -> int {
    g.dens_valid = false;
    int r = set_table(g, pos, mom, per_box, gs);
    if (r) return r;
    const int64_t n3 = (int64_t)g.n * g.n * g.n;
    pm_step_params st = per_box[g.boxes[0]];
    r = step_cycle(g.plan, pos[g.boxes[0]], mom[g.boxes[0]], n3, &st, g.force, nullptr, gs);
    if (r) return r;
    if (st.flags & PM_STEP_DEPOSIT_NEXT) {
      g.dens_valid = true;
      g.dens_pos.resize(g.boxes.size());
      for (size_t j = 0; j < g.boxes.size(); ++j) g.dens_pos[j] = pos[g.boxes[j]];
    }
    return PM_OK;
  });
  if (rc)
    for (auto& g : b->groups) g.dens_valid = false;
  return rc;
}

int pm_batch_ic_zeldovich(pm_batch* b, const void* const* noise, const pm_ic_params* ic, void* const* pos,
                          void* const* mom, void* stream) {
  using namespace pm;
  if (!b) return set_error(PM_ERR_ARG, "pm_batch_ic_zeldovich: null batch");
  if (!ic) return set_error(PM_ERR_ARG, "pm_batch_ic_zeldovich: null IC parameters");
  PM_BATCH_TRY(check_ptrs(b, const_cast<void* const*>(noise), "noise", "pm_batch_ic_zeldovich"));
  PM_BATCH_TRY(check_ptrs(b, pos, "pos", "pm_batch_ic_zeldovich"));
  PM_BATCH_TRY(check_ptrs(b, mom, "mom", "pm_batch_ic_zeldovich"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t es = esize_of(b->dtype);
  return for_groups(b, s, [&](pm_batch::Group& g, hipStream_t gs) -> int {
    g.dens_valid = false;
    const size_t n3 = (size_t)g.n * g.n * g.n;
    for (size_t j = 0; j < g.boxes.size(); ++j) {
      const int r = hip_ok(hipMemcpyAsync(static_cast<char*>(g.mesh) + j * n3 * es, noise[g.boxes[j]], n3 * es,
                                          hipMemcpyDeviceToDevice, gs),
                           "pm_batch_ic_zeldovich: noise copy");
      if (r) return r;
    }
    const int r = set_table(g, pos, mom, nullptr, gs);
    if (r) return r;
    return pm_ic_zeldovich(g.plan, g.mesh, ic, g.force, pos[g.boxes[0]], mom[g.boxes[0]], gs);
  });
}

int pm_batch_pk_estimate(pm_batch* b, const void* const* pos, const int* n_bins, double* k_mean, double* pk,
                         int64_t* n_modes, void* stream) {
  using namespace pm;
  if (!b) return set_error(PM_ERR_ARG, "pm_batch_pk_estimate: null batch");
  PM_BATCH_TRY(check_ptrs(b, const_cast<void* const*>(pos), "pos", "pm_batch_pk_estimate"));
  if (!n_bins || !k_mean || !pk || !n_modes) return set_error(PM_ERR_ARG, "pm_batch_pk_estimate: null pointer");
  std::vector<int64_t> off(b->n_box + 1, 0);
  for (int i = 0; i < b->n_box; ++i) off[i + 1] = off[i] + n_bins[i];
  for (auto& g : b->groups)
    for (int j : g.boxes)
      if (n_bins[j] != n_bins[g.boxes[0]] || n_bins[j] <= 0 || n_bins[j] > 4 * g.n)
        return set_error(PM_ERR_ARG, "pm_batch_pk_estimate: bins of box %d (%d) must lie in [1, %d] and equal those "
                                     "of its size group", j, n_bins[j], 4 * g.n);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return for_groups(b, s, [&](pm_batch::Group& g, hipStream_t gs) -> int {
    g.dens_valid = false;
    const int64_t n3 = (int64_t)g.n * g.n * g.n;
    const int nb = (int)g.boxes.size(), bins = n_bins[g.boxes[0]];
    int r = set_table(g, const_cast<void* const*>(pos), nullptr, nullptr, gs);
    if (r) return r;
    r = launch_fill(g.plan, g.mesh, n3 * nb, -1.0, gs);
    if (r) return r;
    r = launch_deposit(g.plan, pos[g.boxes[0]], n3, g.mesh, gs);
    if (r) return r;
    r = pk_estimate(g.plan, g.mesh, bins, g.kmean, g.pk, g.nmodes, gs);
    if (r) return r;
    for (int j = 0; j < nb; ++j) {
      const int64_t o = off[g.boxes[j]];
      const size_t nbytes = (size_t)bins * 8;
      r = hip_ok(hipMemcpyAsync(k_mean + o, g.kmean + (size_t)j * bins, nbytes, hipMemcpyDeviceToDevice, gs), "copy");
      if (!r) r = hip_ok(hipMemcpyAsync(pk + o, g.pk + (size_t)j * bins, nbytes, hipMemcpyDeviceToDevice, gs), "copy");
      if (!r)
        r = hip_ok(hipMemcpyAsync(n_modes + o, g.nmodes + (size_t)j * bins, nbytes, hipMemcpyDeviceToDevice, gs),
                   "copy");
      if (r) return r;
    }
    return PM_OK;
  });
}

}  // extern "C"
