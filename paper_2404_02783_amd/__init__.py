"""pmhip: particle-mesh hot path of arXiv:2404.02783 as hand-written HIP kernels (gfx950).

Thin Python binding of the C ABI in ``include/pmhip.h`` (``libpmhip.so``): every
function below only marshals torch tensors (device memory) and the current HIP
stream into the library call of the same name.  There is no fallback: if the
library is missing or a call fails, a ``PMError`` is raised.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import torch

__all__ = [
    "PMError", "lib", "SolveParams", "StepParams", "Cosmology", "ICParams", "Plan",
    "pm_deposit", "pm_solve", "pm_gather", "pm_step", "displacement_combine", "displacement_add", "pm_xi_linear",
    "pk_estimate", "pk_cross_estimate", "bias_fit", "bk_estimate",
    "Batch", "pm_batch_step", "pm_batch_ic_zeldovich", "pm_batch_pk_estimate", "PM_BATCH_CONCURRENT",
    "pm_step_adjoint", "pm_step_adjoint_noalloc", "pm_step_adjoint_noalloc_bytes", "PM_STATIC_SCRATCH_BYTES",
    "pk_adjoint", "pm_ic_zeldovich_adjoint", "pm_noise_truncate",
    "pm_ic_zeldovich", "pm_ic_2lpt", "pm_ic_2lpt_adjoint", "pm_ic_gauge", "pm_noise_fix",
    "pm_plan_tuning_candidates", "pm_plan_get_tuning", "pm_plan_set_tuning", "pm_plan_autotune", "TUNING_SLOTS",
    "pm_check", "pm_profile_enable", "pm_profile_read", "kdk_factors", "gauge_params", "newton_params",
    "cosmo_hubble_e", "cosmo_omega_m_a", "cosmo_growth", "cosmo_growth_rate", "cosmo_kick", "cosmo_drift",
    "power_eh98_amplitude", "power_law_amplitude", "FIDUCIAL", "LIB_PATH", "log_steps", "leapfrog_factors",
    "pm_microbench_atomics", "build_info", "build_is_current",
    "PM_F32", "PM_F64", "PM_NEWTON", "PM_POISSON_GAUGE", "PM_GRAD_SPECTRAL", "PM_GRAD_FD2", "PM_GRAD_FD1",
    "PM_PK_POWERLAW", "PM_PK_EH98", "PM_STEP_DEPOSIT_NEXT", "PM_STEP_DENSITY_READY",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpmhip.so")

PM_OK, PM_ERR_ARG, PM_ERR_SIZE, PM_ERR_NOMEM, PM_ERR_HIP, PM_ERR_STATE = 0, -1, -2, -3, -4, -5
PM_F32, PM_F64 = 0, 1
PM_NEWTON, PM_POISSON_GAUGE = 0, 1
PM_GRAD_SPECTRAL, PM_GRAD_FD2, PM_GRAD_FD1 = 0, 1, 2
PM_PK_POWERLAW, PM_PK_EH98 = 0, 1
PM_STATIC_SCRATCH_BYTES = 64 << 20
PM_BATCH_CONCURRENT = 1

_c_int, _c_double, _c_void_p, _c_int64, _c_size_t = (
    ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t)


class PMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pmhip error {code}: {msg}")
        self.code = code


class SolveParams(ctypes.Structure):
    _fields_ = [("kind", _c_int), ("grad", _c_int), ("omega_m", _c_double), ("a", _c_double),
                ("om_a", _c_double), ("calh", _c_double), ("c_g", _c_double), ("inv_dtau", _c_double)]


PM_STEP_DEPOSIT_NEXT, PM_STEP_DENSITY_READY = 1, 2


class StepParams(ctypes.Structure):
    _fields_ = [("kick", _c_double), ("drift", _c_double), ("solve", SolveParams), ("flags", _c_int)]


class Cosmology(ctypes.Structure):
    _fields_ = [("omega_m", _c_double), ("omega_b", _c_double), ("h", _c_double), ("t_cmb", _c_double)]


class ICParams(ctypes.Structure):
    _fields_ = [("pk_kind", _c_int), ("amp", _c_double), ("index", _c_double), ("a_init", _c_double),
                ("a_norm", _c_double), ("cosmo", Cosmology)]


# Flat LCDM of the paper's simulation setup (Sec. 3), no radiation.
FIDUCIAL = Cosmology(omega_m=0.263771 + 0.0482754, omega_b=0.0482754, h=0.67556, t_cmb=2.7255)

_LIB = None


def _declare(l):
    P = ctypes.POINTER
    sig = {
        "pm_last_error": (ctypes.c_char_p, []),
        "pm_build_info": (ctypes.c_char_p, []),
        "pm_plan_workspace_bytes": (_c_size_t, [_c_int, _c_int]),
        "pm_plan_create": (_c_int, [P(_c_void_p), _c_int, _c_double, _c_int, _c_void_p, _c_size_t]),
        "pm_plan_workspace_bytes_batch": (_c_size_t, [_c_int, _c_int, _c_int]),
        "pm_plan_create_batch": (_c_int, [P(_c_void_p), _c_int, _c_double, _c_int, _c_int, _c_void_p, _c_size_t]),
        "pm_plan_destroy": (_c_int, [_c_void_p]),
        "pm_check": (_c_int, [_c_void_p, _c_void_p]),
        "pm_profile_enable": (_c_int, [_c_void_p, _c_int]),
        "pm_profile_read": (_c_int, [_c_void_p, _c_int, ctypes.c_char_p, P(_c_double), P(_c_int64)]),
        "pm_deposit": (_c_int, [_c_void_p, _c_void_p, _c_int64, _c_void_p, _c_void_p]),
        "pm_solve": (_c_int, [_c_void_p, _c_void_p, P(SolveParams), _c_void_p, _c_void_p, _c_void_p]),
        "pm_gather": (_c_int, [_c_void_p, _c_void_p, _c_void_p, _c_int64, _c_void_p, _c_void_p]),
        "pm_step": (_c_int, [_c_void_p, _c_void_p, _c_void_p, _c_int64, P(StepParams), _c_void_p, _c_void_p,
                             _c_void_p]),
        "displacement_combine": (_c_int, [_c_void_p, _c_void_p, _c_int, _c_void_p, _c_int, _c_int, _c_void_p,
                                          _c_void_p]),
        "displacement_add": (_c_int, [_c_void_p, _c_int, _c_void_p, _c_int, _c_int, _c_void_p, _c_void_p]),
        "pk_estimate": (_c_int, [_c_void_p, _c_void_p, _c_int, _c_void_p, _c_void_p, _c_void_p, _c_void_p]),
        "pk_cross_estimate": (_c_int, [_c_void_p, _c_void_p, _c_void_p, _c_int, _c_void_p, _c_void_p, _c_void_p,
                                       _c_void_p]),
        "bias_fit": (_c_int, [P(_c_double), P(_c_double), P(ctypes.c_int64), _c_int, _c_double, _c_double, _c_int,
                              _c_int, P(_c_double)]),
        "bk_estimate": (_c_int, [_c_void_p, _c_void_p, _c_int, P(_c_double), _c_double, P(ctypes.c_int32), _c_int,
                                 _c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_size_t, _c_void_p]),
        "pm_step_adjoint": (_c_int, [_c_void_p, _c_void_p, _c_int64, P(StepParams), _c_void_p, _c_void_p, _c_void_p,
                                     _c_void_p, _c_void_p]),
        "pm_batch_create": (_c_int, [P(_c_void_p), _c_int, P(_c_int), P(_c_double), _c_int, _c_int]),
        "pm_batch_destroy": (_c_int, [_c_void_p]),
        "pm_batch_num_groups": (_c_int, [_c_void_p]),
        "pm_batch_group": (_c_int, [_c_void_p, _c_int, P(_c_int), P(_c_double), P(_c_int), P(_c_void_p)]),
        "pm_batch_step": (_c_int, [_c_void_p, P(_c_void_p), P(_c_void_p), P(StepParams), _c_void_p]),
        "pm_batch_ic_zeldovich": (_c_int, [_c_void_p, P(_c_void_p), P(ICParams), P(_c_void_p), P(_c_void_p),
                                           _c_void_p]),
        "pm_batch_pk_estimate": (_c_int, [_c_void_p, P(_c_void_p), P(_c_int), _c_void_p, _c_void_p, _c_void_p,
                                          _c_void_p]),
        "pm_step_adjoint_noalloc": (_c_int, [_c_void_p, _c_void_p, _c_int64, P(StepParams), _c_void_p, _c_void_p,
                                             _c_void_p, _c_void_p]),
        "pm_step_adjoint_noalloc_bytes": (_c_size_t, [_c_int, _c_int, _c_int]),
        "pk_adjoint": (_c_int, [_c_void_p, _c_void_p, _c_int64, _c_int, _c_void_p, _c_void_p, _c_void_p]),
        "pm_ic_zeldovich": (_c_int, [_c_void_p, _c_void_p, P(ICParams), _c_void_p, _c_void_p, _c_void_p, _c_void_p]),
        "pm_ic_2lpt": (_c_int, [_c_void_p, _c_void_p, P(ICParams), _c_void_p, _c_void_p, _c_void_p, _c_void_p]),
        "pm_ic_2lpt_adjoint": (_c_int, [_c_void_p, _c_void_p, P(ICParams), _c_void_p, _c_void_p, _c_void_p,
                                        _c_void_p, _c_void_p]),
        "pm_noise_fix": (_c_int, [_c_void_p, _c_void_p, _c_int, _c_void_p, _c_void_p]),
        "pm_plan_tuning_candidates": (_c_int, [_c_void_p, _c_int, P(_c_int), _c_int]),
        "pm_plan_get_tuning": (_c_int, [_c_void_p, P(_c_int)]),
        "pm_plan_set_tuning": (_c_int, [_c_void_p, P(_c_int)]),
        "pm_plan_autotune": (_c_int, [_c_void_p, _c_void_p, _c_int, _c_int, P(_c_double), _c_void_p]),
        "pm_ic_zeldovich_adjoint": (_c_int, [_c_void_p, P(ICParams), _c_void_p, _c_void_p, _c_void_p, _c_void_p,
                                             _c_void_p]),
        "pm_noise_truncate": (_c_int, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p]),
        "pm_ic_gauge": (_c_int, [_c_void_p, _c_void_p, P(ICParams), _c_void_p, _c_void_p, _c_void_p, _c_void_p,
                                 _c_void_p, _c_void_p]),
        "pm_xi_linear": (_c_int, [_c_void_p, _c_void_p, P(ICParams), _c_double, _c_void_p, _c_void_p]),
        "pm_cosmo_hubble_e": (_c_double, [P(Cosmology), _c_double]),
        "pm_cosmo_omega_m_a": (_c_double, [P(Cosmology), _c_double]),
        "pm_cosmo_growth": (_c_double, [P(Cosmology), _c_double]),
        "pm_cosmo_growth_rate": (_c_double, [P(Cosmology), _c_double]),
        "pm_cosmo_kick": (_c_double, [P(Cosmology), _c_double, _c_double]),
        "pm_cosmo_drift": (_c_double, [P(Cosmology), _c_double, _c_double]),
        "pm_kdk_factors": (None, [P(Cosmology), _c_double, _c_double, P(_c_double)]),
        "pm_log_steps": (_c_int, [_c_double, _c_double, _c_int, P(_c_double)]),
        "pm_microbench_atomics": (_c_int, [_c_void_p, _c_int64, _c_int, _c_void_p]),
        "pm_leapfrog_factors": (_c_int, [P(Cosmology), P(_c_double), _c_int, P(_c_double), P(_c_double)]),
        "pm_gauge_params": (None, [P(Cosmology), _c_double, _c_int, _c_double, _c_double, P(SolveParams)]),
        "pm_power_eh98_amplitude": (_c_double, [P(Cosmology), _c_double, _c_double]),
        "pm_power_law_amplitude": (_c_double, [_c_int, _c_double, _c_double, _c_double]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(l, name)
        fn.restype = res
        fn.argtypes = args
    return l


def lib():
    """The loaded ``libpmhip.so`` (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise PMError(PM_ERR_ARG, f"{LIB_PATH} not built (run python -m paper_2404_02783_amd.build)")
        _LIB = _declare(ctypes.CDLL(LIB_PATH))
    return _LIB


def _check(rc: int):
    if rc != PM_OK:
        raise PMError(rc, lib().pm_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise PMError(PM_ERR_ARG, f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise PMError(PM_ERR_ARG, f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise PMError(PM_ERR_ARG, f"{name} has dtype {t.dtype}, expected {dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _need(t, numel: int, name: str):
    if t.numel() < numel:
        raise PMError(PM_ERR_ARG, f"{name} holds {t.numel()} elements, {numel} needed")


class Plan:
    """An N^3 mesh plan of ``batch`` equal boxes (default one); the spectrum
    workspace is a torch device buffer."""

    def __init__(self, n: int, box: float, dtype=torch.float32, device=None, batch: int = 1):
        self.n = int(n)
        self.box = float(box)
        self.dtype = dtype
        self.batch = int(batch)
        self.cdtype = PM_F32 if dtype == torch.float32 else PM_F64
        self.device = torch.device("cuda") if device is None else torch.device(device)
        nbytes = lib().pm_plan_workspace_bytes_batch(self.n, self.cdtype, self.batch)
        if nbytes == 0:
            raise PMError(PM_ERR_SIZE, f"unsupported mesh size {n} or batch {batch}")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = _c_void_p()
        _check(lib().pm_plan_create_batch(ctypes.byref(h), self.n, self.box, self.cdtype, self.batch,
                                          ctypes.c_void_p(self.workspace.data_ptr()), nbytes))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().pm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # allocation helpers (torch device memory)
    def mesh(self, ncomp: int = 0):
        """[N,N,N] ([batch,N,N,N] for a batch), or [ncomp, ...] of those."""
        shape = (self.n,) * 3 if self.batch == 1 else (self.batch,) + (self.n,) * 3
        if ncomp:
            shape = (ncomp,) + shape
        return torch.empty(shape, dtype=self.dtype, device=self.device)

    def particles(self):
        """Empty [3, N^3] ([batch, 3, N^3] for a batch) particle array."""
        shape = (3, self.n ** 3) if self.batch == 1 else (self.batch, 3, self.n ** 3)
        return torch.empty(shape, dtype=self.dtype, device=self.device)

    def spectrum(self):
        cd = torch.complex64 if self.dtype == torch.float32 else torch.complex128
        shape = (self.n, self.n, self.n // 2 + 1)
        if self.batch > 1:
            shape = (self.batch,) + shape
        return torch.zeros(shape, dtype=cd, device=self.device)


def pm_check(plan: Plan):
    _check(lib().pm_check(plan.handle, _stream()))


def pm_profile_enable(plan: Plan, on: bool = True):
    _check(lib().pm_profile_enable(plan.handle, int(bool(on))))


def pm_profile_read(plan: Plan):
    """{kernel kind: (total ms, launches)} since the last read."""
    nmax = 32
    names = ctypes.create_string_buffer(32 * nmax)
    ms = (ctypes.c_double * nmax)()
    cnt = (ctypes.c_int64 * nmax)()
    w = lib().pm_profile_read(plan.handle, nmax, names, ms, cnt)
    if w < 0:
        _check(w)
    raw = names.raw
    return {raw[32 * i:32 * (i + 1)].split(b"\0", 1)[0].decode(): (ms[i], cnt[i]) for i in range(w)}


def pm_deposit(plan: Plan, pos, delta=None):
    delta = plan.mesh() if delta is None else delta
    _need(delta, plan.batch * plan.n ** 3, "delta")
    _need(pos, plan.batch * 3 * pos.shape[-1], "pos")
    _check(lib().pm_deposit(plan.handle, _ptr(pos, plan.dtype, "pos"), pos.shape[-1], _ptr(delta, plan.dtype, "delta"),
                            _stream()))
    return delta


def pm_solve(plan: Plan, delta, sp: SolveParams, phi_state=None, force=None):
    force = plan.mesh(3) if force is None else force
    _need(delta, plan.batch * plan.n ** 3, "delta")
    _need(force, 3 * plan.batch * plan.n ** 3, "force")
    if phi_state is not None:
        _need(phi_state, plan.batch * plan.n ** 2 * (plan.n // 2 + 1), "phi_state")
    _check(lib().pm_solve(plan.handle, _ptr(delta, plan.dtype, "delta"), ctypes.byref(sp), _ptr(phi_state),
                          _ptr(force, plan.dtype, "force"), _stream()))
    return force


def pm_gather(plan: Plan, force, pos, acc=None):
    acc = torch.empty_like(pos) if acc is None else acc
    _check(lib().pm_gather(plan.handle, _ptr(force, plan.dtype, "force"), _ptr(pos, plan.dtype, "pos"), pos.shape[-1],
                           _ptr(acc, plan.dtype, "acc"), _stream()))
    return acc


def pm_step(plan: Plan, pos, mom, st: StepParams, force_scratch, phi_state=None):
    np_ = pos.shape[-1]
    _need(pos, plan.batch * 3 * np_, "pos")
    _need(mom, plan.batch * 3 * np_, "mom")
    _need(force_scratch, 3 * plan.batch * plan.n ** 3, "force_scratch")
    if phi_state is not None:
        _need(phi_state, plan.batch * plan.n ** 2 * (plan.n // 2 + 1), "phi_state")
    _check(lib().pm_step(plan.handle, _ptr(pos, plan.dtype, "pos"), _ptr(mom, plan.dtype, "mom"), pos.shape[-1],
                         ctypes.byref(st), _ptr(force_scratch, plan.dtype, "force_scratch"), _ptr(phi_state),
                         _stream()))


def pm_step_adjoint(plan: Plan, pos, st: StepParams, lam_pos, lam_mom, force=None, mesh_scratch=None):
    """Cotangents of one pm_step pulled back in place: (lam_pos, lam_mom) of the
    cycle's outputs -> those of its inputs.  ``pos`` are the positions the forward
    cycle started from; ``force`` the force meshes it used (or None to recompute)."""
    n3 = plan.n ** 3
    need = 3 * n3 if force is not None else 6 * n3
    if mesh_scratch is None:
        mesh_scratch = torch.empty(need, dtype=plan.dtype, device=plan.device)
    _need(mesh_scratch, need, "mesh_scratch")
    if force is not None:
        _need(force, 3 * n3, "force")
    np_ = pos.shape[-1]
    for t, nm in ((lam_pos, "lam_pos"), (lam_mom, "lam_mom")):
        _need(t, 3 * np_, nm)
    _check(lib().pm_step_adjoint(plan.handle, _ptr(pos, plan.dtype, "pos"), np_, ctypes.byref(st),
                                 _ptr(force, plan.dtype, "force"), _ptr(mesh_scratch, plan.dtype, "mesh_scratch"),
                                 _ptr(lam_pos, plan.dtype, "lam_pos"), _ptr(lam_mom, plan.dtype, "lam_mom"),
                                 _stream()))


class _GroupPlan:
    """The internal plan of one size group of a Batch, for the FFT launch-shape tuning
    calls and the profiler only (the batch owns it)."""

    def __init__(self, handle, n, box, dtype, batch, device):
        self.handle, self.n, self.box, self.dtype, self.batch, self.device = handle, n, box, dtype, batch, device

    def mesh(self, ncomp: int = 0):
        shape = (self.batch,) + (self.n,) * 3
        return torch.empty(((ncomp,) if ncomp else ()) + shape, dtype=self.dtype, device=self.device)


class Batch:
    """An uneven ensemble: box i has an n_mesh[i]^3 mesh and n_mesh[i]^3 particles in a
    periodic box of side box[i] (pm_batch_create).  Boxes of equal mesh size and side
    form a size group advanced by one launch per kernel."""

    def __init__(self, n_mesh, box, dtype=torch.float32, device=None, concurrent: bool = False):
        self.n_mesh = [int(v) for v in n_mesh]
        self.box = [float(v) for v in box]
        if len(self.n_mesh) != len(self.box) or not self.n_mesh:
            raise PMError(PM_ERR_ARG, "n_mesh and box must be non-empty lists of equal length")
        self.dtype = dtype
        self.cdtype = PM_F32 if dtype == torch.float32 else PM_F64
        self.device = torch.device("cuda") if device is None else torch.device(device)
        nb = len(self.n_mesh)
        h = _c_void_p()
        _check(lib().pm_batch_create(ctypes.byref(h), nb, (_c_int * nb)(*self.n_mesh), (_c_double * nb)(*self.box),
                                     self.cdtype, PM_BATCH_CONCURRENT if concurrent else 0))
        self.handle = h

    def __len__(self):
        return len(self.n_mesh)

    def groups(self):
        """[(n_mesh, box, boxes in the group, group plan view)] in the batch's group order."""
        out = []
        for g in range(lib().pm_batch_num_groups(self.handle)):
            n, box, cnt, ph = _c_int(), _c_double(), _c_int(), _c_void_p()
            _check(lib().pm_batch_group(self.handle, g, ctypes.byref(n), ctypes.byref(box), ctypes.byref(cnt),
                                        ctypes.byref(ph)))
            out.append((n.value, box.value, cnt.value,
                        _GroupPlan(ph, n.value, box.value, self.dtype, cnt.value, self.device)))
        return out

    def particles(self):
        """Empty [3, n^3] arrays, one per box."""
        return [torch.empty((3, n ** 3), dtype=self.dtype, device=self.device) for n in self.n_mesh]

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().pm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _box_ptrs(batch: Batch, arrays, per_box: int, name: str):
    if len(arrays) != len(batch):
        raise PMError(PM_ERR_ARG, f"{name}: {len(batch)} arrays expected")
    ptrs = []
    for i, (t, n) in enumerate(zip(arrays, batch.n_mesh)):
        _need(t, per_box * n ** 3, f"{name}[{i}]")
        ptrs.append(_ptr(t, batch.dtype, f"{name}[{i}]"))
    return (_c_void_p * len(ptrs))(*ptrs)


def pm_batch_step(batch: Batch, pos, mom, steps):
    """One force-kick-drift cycle of every box in place; ``steps`` is one StepParams for
    all boxes or one per box."""
    nb = len(batch)
    if isinstance(steps, StepParams):
        steps = [steps] * nb
    if len(steps) != nb:
        raise PMError(PM_ERR_ARG, f"{nb} step parameters expected")
    _check(lib().pm_batch_step(batch.handle, _box_ptrs(batch, pos, 3, "pos"), _box_ptrs(batch, mom, 3, "mom"),
                               (StepParams * nb)(*steps), _stream()))


def pm_batch_ic_zeldovich(batch: Batch, noise, ic: ICParams, pos, mom):
    _check(lib().pm_batch_ic_zeldovich(batch.handle, _box_ptrs(batch, noise, 1, "noise"), ctypes.byref(ic),
                                       _box_ptrs(batch, pos, 3, "pos"), _box_ptrs(batch, mom, 3, "mom"), _stream()))


def pm_batch_pk_estimate(batch: Batch, pos, n_bins=None, out=None):
    """P(k) of every box; ``n_bins`` per box (default N/2).  Returns [(k_mean, P,
    n_modes) per box], views of three flat device arrays (``out`` may supply them)."""
    nb = len(batch)
    bins = [n // 2 for n in batch.n_mesh] if n_bins is None else [int(v) for v in n_bins]
    total = sum(bins)
    if out is None:
        out = (torch.empty(total, dtype=torch.float64, device=batch.device),
               torch.empty(total, dtype=torch.float64, device=batch.device),
               torch.empty(total, dtype=torch.int64, device=batch.device))
    k, p, c = out
    for t, nm, dt in ((k, "k_mean", torch.float64), (p, "pk", torch.float64), (c, "n_modes", torch.int64)):
        _need(t, total, nm)
    _check(lib().pm_batch_pk_estimate(batch.handle, _box_ptrs(batch, pos, 3, "pos"), (_c_int * nb)(*bins),
                                      _ptr(k, torch.float64, "k_mean"), _ptr(p, torch.float64, "pk"),
                                      _ptr(c, torch.int64, "n_modes"), _stream()))
    res, o = [], 0
    for b in bins:
        res.append((k[o:o + b], p[o:o + b], c[o:o + b]))
        o += b
    return res


def pm_step_adjoint_noalloc_bytes(n: int, dtype, with_force: bool) -> int:
    """Scratch bytes pm_step_adjoint_noalloc takes from the library's static array."""
    cd = PM_F32 if dtype == torch.float32 else PM_F64
    return int(lib().pm_step_adjoint_noalloc_bytes(int(n), cd, 1 if with_force else 0))


def pm_step_adjoint_noalloc(plan: Plan, pos, st: StepParams, lam_pos, lam_mom, force=None):
    """pm_step_adjoint without a scratch argument: the library's static device scratch
    stands in for it, and the call allocates nothing (for graph capture or loops that
    must not allocate).  Calls that overlap in time on one GPU race."""
    n3 = plan.n ** 3
    if force is not None:
        _need(force, 3 * n3, "force")
    np_ = pos.shape[-1]
    for t, nm in ((lam_pos, "lam_pos"), (lam_mom, "lam_mom")):
        _need(t, 3 * np_, nm)
    _check(lib().pm_step_adjoint_noalloc(plan.handle, _ptr(pos, plan.dtype, "pos"), np_, ctypes.byref(st),
                                         _ptr(force, plan.dtype, "force"), _ptr(lam_pos, plan.dtype, "lam_pos"),
                                         _ptr(lam_mom, plan.dtype, "lam_mom"), _stream()))


def pk_adjoint(plan: Plan, pos, n_bins: int, dpk, lam_pos=None):
    """dL/dpos of a loss with cotangent ``dpk`` = dL/dP (device float64 [n_bins])
    through the CIC density and the P(k) estimator."""
    lam_pos = torch.empty_like(pos) if lam_pos is None else lam_pos
    _need(dpk, n_bins, "dpk")
    _check(lib().pk_adjoint(plan.handle, _ptr(pos, plan.dtype, "pos"), pos.shape[-1], int(n_bins),
                            _ptr(dpk, torch.float64, "dpk"), _ptr(lam_pos, plan.dtype, "lam_pos"), _stream()))
    return lam_pos


def displacement_combine(x_gr, x_newton, n_coarse: int, x_fine, n_fine: int, x_out=None):
    x_out = torch.empty_like(x_fine) if x_out is None else x_out
    dt = PM_F32 if x_fine.dtype == torch.float32 else PM_F64
    _check(lib().displacement_combine(_ptr(x_gr, x_fine.dtype, "x_gr"), _ptr(x_newton, x_fine.dtype, "x_newton"),
                                      int(n_coarse), _ptr(x_fine, x_fine.dtype, "x_fine"), int(n_fine), dt,
                                      _ptr(x_out, x_fine.dtype, "x_out"), _stream()))
    return x_out


def displacement_add(xi, n_coarse: int, x_fine, n_fine: int, x_out=None):
    """x_fine + (n_fine/n_coarse) xi interpolated to the fine lattice (wrapped)."""
    x_out = torch.empty_like(x_fine) if x_out is None else x_out
    dt = PM_F32 if x_fine.dtype == torch.float32 else PM_F64
    _need(xi, 3 * n_coarse ** 3, "xi")
    _need(x_fine, 3 * n_fine ** 3, "x_fine")
    _need(x_out, 3 * n_fine ** 3, "x_out")
    _check(lib().displacement_add(_ptr(xi, x_fine.dtype, "xi"), int(n_coarse), _ptr(x_fine, x_fine.dtype, "x_fine"),
                                  int(n_fine), dt, _ptr(x_out, x_fine.dtype, "x_out"), _stream()))
    return x_out


def pk_estimate(plan: Plan, delta, n_bins: int, out=None):
    """(k_mean, P, n_modes), each [n_bins] ([batch, n_bins] for a batch); ``out``:
    optional preallocated (k_mean, P, n_modes) device tensors to write."""
    shape = (n_bins,) if plan.batch == 1 else (plan.batch, n_bins)
    _need(delta, plan.batch * plan.n ** 3, "delta")
    if out is None:
        k = torch.empty(shape, dtype=torch.float64, device=plan.device)
        p = torch.empty(shape, dtype=torch.float64, device=plan.device)
        c = torch.empty(shape, dtype=torch.int64, device=plan.device)
    else:
        k, p, c = out
        for t, dt, nm in ((k, torch.float64, "k_mean"), (p, torch.float64, "pk"), (c, torch.int64, "n_modes")):
            if t.dtype != dt or t.numel() < plan.batch * n_bins or not t.is_contiguous():
                raise PMError(PM_ERR_ARG, f"pk_estimate: out {nm} must be a contiguous {dt} of {plan.batch * n_bins}")
    _check(lib().pk_estimate(plan.handle, _ptr(delta, plan.dtype, "delta"), int(n_bins), _ptr(k), _ptr(p), _ptr(c),
                             _stream()))
    return k, p, c


def pk_cross_estimate(plan: Plan, delta_a, delta_b, n_bins: int):
    """(k_mean, P_ab, n_modes), each [n_bins] ([batch, n_bins] for a batch)."""
    shape = (n_bins,) if plan.batch == 1 else (plan.batch, n_bins)
    _need(delta_a, plan.batch * plan.n ** 3, "delta_a")
    _need(delta_b, plan.batch * plan.n ** 3, "delta_b")
    k = torch.empty(shape, dtype=torch.float64, device=plan.device)
    p = torch.empty(shape, dtype=torch.float64, device=plan.device)
    c = torch.empty(shape, dtype=torch.int64, device=plan.device)
    _check(lib().pk_cross_estimate(plan.handle, _ptr(delta_a, plan.dtype, "delta_a"),
                                   _ptr(delta_b, plan.dtype, "delta_b"), int(n_bins), _ptr(k), _ptr(p), _ptr(c),
                                   _stream()))
    return k, p, c


def bias_fit(k, ratio, n_modes, k_cut: float, calh: float, skip: int = 2, with_k2: bool = True):
    """(b1, b1_GR, c2) of ratio(k) = b1 + b1_GR calh^2/k^2 (+ c2 k^2); host sequences."""
    k = [float(v) for v in k]
    ratio = [float(v) for v in ratio]
    n_modes = [int(v) for v in n_modes]
    nb = len(k)
    if len(ratio) != nb or len(n_modes) != nb:
        raise PMError(PM_ERR_ARG, "bias_fit: k, ratio and n_modes differ in length")
    coef = (ctypes.c_double * 3)()
    _check(lib().bias_fit((ctypes.c_double * nb)(*k), (ctypes.c_double * nb)(*ratio),
                          (ctypes.c_int64 * nb)(*n_modes), nb, float(k_cut), float(calh), int(skip),
                          int(bool(with_k2)), coef))
    return coef[0], coef[1], coef[2]


def bk_estimate(plan: Plan, delta, centres, width: float, triangles, shell_ws=None, ntri_known=None):
    cen = (ctypes.c_double * len(centres))(*[float(c) for c in centres])
    flat = [int(s) for t in triangles for s in t]
    tri = (ctypes.c_int32 * len(flat))(*flat)
    nt = len(triangles)
    if shell_ws is None:
        nsh = len({s for s in flat})
        shell_ws = torch.empty((max(3, nsh),) + (plan.n,) * 3, dtype=plan.dtype, device=plan.device)
    bk = torch.empty(nt, dtype=torch.float64, device=plan.device)
    ntri = torch.empty(nt, dtype=torch.float64, device=plan.device)
    _check(lib().bk_estimate(plan.handle, _ptr(delta, plan.dtype, "delta"), len(centres), cen, float(width), tri, nt,
                             _ptr(bk), _ptr(ntri), _ptr(ntri_known, torch.float64, "ntri_known"),
                             _ptr(shell_ws, plan.dtype, "shell_ws"), shell_ws.numel() * shell_ws.element_size(),
                             _stream()))
    return bk, ntri


def pm_ic_zeldovich(plan: Plan, noise, ic: ICParams, disp_scratch, pos, mom):
    n3 = plan.batch * plan.n ** 3
    _need(noise, n3, "noise")
    _need(disp_scratch, 3 * n3, "disp_scratch")
    _need(pos, 3 * n3, "pos")
    _need(mom, 3 * n3, "mom")
    _check(lib().pm_ic_zeldovich(plan.handle, _ptr(noise, plan.dtype, "noise"), ctypes.byref(ic),
                                 _ptr(disp_scratch, plan.dtype, "disp_scratch"), _ptr(pos, plan.dtype, "pos"),
                                 _ptr(mom, plan.dtype, "mom"), _stream()))


def pm_ic_2lpt(plan: Plan, noise, ic: ICParams, disp_scratch, pos, mom):
    """Second-order Lagrangian Newtonian set (single-box plans)."""
    n3 = plan.n ** 3
    _need(noise, n3, "noise")
    _need(disp_scratch, 3 * n3, "disp_scratch")
    _need(pos, 3 * n3, "pos")
    _need(mom, 3 * n3, "mom")
    _check(lib().pm_ic_2lpt(plan.handle, _ptr(noise, plan.dtype, "noise"), ctypes.byref(ic),
                            _ptr(disp_scratch, plan.dtype, "disp_scratch"), _ptr(pos, plan.dtype, "pos"),
                            _ptr(mom, plan.dtype, "mom"), _stream()))


TUNING_SLOTS = ("cols", "solve", "r2c_rows", "c2r_rows")


def pm_plan_tuning_candidates(plan: Plan, kind: int):
    buf = (_c_int * 16)()
    n = lib().pm_plan_tuning_candidates(plan.handle, int(kind), buf, 16)
    if n < 0:
        _check(n)
    return [buf[i] for i in range(min(n, 16))]


def pm_plan_get_tuning(plan: Plan):
    buf = (_c_int * 4)()
    _check(lib().pm_plan_get_tuning(plan.handle, buf))
    return [buf[i] for i in range(4)]


def pm_plan_set_tuning(plan: Plan, shapes):
    vals = [int(v) for v in shapes]
    if len(vals) != 4:
        raise PMError(PM_ERR_ARG, "four tuning shapes expected")
    _check(lib().pm_plan_set_tuning(plan.handle, (_c_int * 4)(*vals)))


def pm_plan_autotune(plan: Plan, reps: int = 3, use_cache: bool = True, mesh_scratch=None):
    """Times every allowed launch shape of the plan's FFT passes and keeps the fastest;
    returns (shapes, best ms per launch or -1 where taken from the process cache)."""
    mesh_scratch = plan.mesh() if mesh_scratch is None else mesh_scratch
    _need(mesh_scratch, plan.batch * plan.n ** 3, "mesh_scratch")
    ms = (_c_double * 4)()
    _check(lib().pm_plan_autotune(plan.handle, _ptr(mesh_scratch, plan.dtype, "mesh_scratch"), int(reps),
                                  int(bool(use_cache)), ms, _stream()))
    return pm_plan_get_tuning(plan), [ms[i] for i in range(4)]


def pm_ic_2lpt_adjoint(plan: Plan, noise, ic: ICParams, lam_pos, lam_mom, scratch=None, lam_noise=None):
    """dL/dnoise from the cotangents of the second-order (pos, mom)."""
    n3 = plan.n ** 3
    scratch = plan.mesh(9) if scratch is None else scratch
    lam_noise = plan.mesh() if lam_noise is None else lam_noise
    _need(noise, n3, "noise")
    _need(scratch, 9 * n3, "scratch")
    _need(lam_noise, n3, "lam_noise")
    _need(lam_pos, 3 * n3, "lam_pos")
    _need(lam_mom, 3 * n3, "lam_mom")
    _check(lib().pm_ic_2lpt_adjoint(plan.handle, _ptr(noise, plan.dtype, "noise"), ctypes.byref(ic),
                                    _ptr(lam_pos, plan.dtype, "lam_pos"), _ptr(lam_mom, plan.dtype, "lam_mom"),
                                    _ptr(scratch, plan.dtype, "scratch"), _ptr(lam_noise, plan.dtype, "lam_noise"),
                                    _stream()))
    return lam_noise


def pm_noise_fix(plan: Plan, noise, pair_mode: int = 0, out=None):
    """Paired-and-fixed noise: 0 fixed, 1 fixed and negated, 2 odd boxes of a batch
    negated (pairs of boxes)."""
    out = torch.empty_like(noise) if out is None else out
    n3 = plan.batch * plan.n ** 3
    _need(noise, n3, "noise")
    _need(out, n3, "out")
    _check(lib().pm_noise_fix(plan.handle, _ptr(noise, plan.dtype, "noise"), int(pair_mode),
                              _ptr(out, plan.dtype, "out"), _stream()))
    return out


def pm_ic_zeldovich_adjoint(plan: Plan, ic: ICParams, lam_pos, lam_mom, disp_scratch=None, lam_noise=None):
    """dL/dnoise from the cotangents of the Zel'dovich (pos, mom)."""
    n3 = plan.n ** 3
    disp_scratch = plan.mesh(3) if disp_scratch is None else disp_scratch
    lam_noise = plan.mesh() if lam_noise is None else lam_noise
    _need(disp_scratch, 3 * n3, "disp_scratch")
    _need(lam_noise, n3, "lam_noise")
    _need(lam_pos, 3 * n3, "lam_pos")
    _need(lam_mom, 3 * n3, "lam_mom")
    _check(lib().pm_ic_zeldovich_adjoint(plan.handle, ctypes.byref(ic), _ptr(lam_pos, plan.dtype, "lam_pos"),
                                         _ptr(lam_mom, plan.dtype, "lam_mom"),
                                         _ptr(disp_scratch, plan.dtype, "disp_scratch"),
                                         _ptr(lam_noise, plan.dtype, "lam_noise"), _stream()))
    return lam_noise


def pm_noise_truncate(fine: Plan, noise_fine, coarse: Plan, noise_coarse=None):
    """Coarse white noise sharing the fine noise's phases on the shared modes."""
    noise_coarse = coarse.mesh() if noise_coarse is None else noise_coarse
    _need(noise_fine, fine.n ** 3, "noise_fine")
    _need(noise_coarse, coarse.n ** 3, "noise_coarse")
    _check(lib().pm_noise_truncate(fine.handle, _ptr(noise_fine, fine.dtype, "noise_fine"), coarse.handle,
                                   _ptr(noise_coarse, coarse.dtype, "noise_coarse"), _stream()))
    return noise_coarse


def pm_ic_gauge(plan: Plan, noise, ic: ICParams, disp_scratch, pos_n, mom_n, pos_gr, mom_gr):
    _check(lib().pm_ic_gauge(plan.handle, _ptr(noise, plan.dtype, "noise"), ctypes.byref(ic),
                             _ptr(disp_scratch, plan.dtype, "disp_scratch"), _ptr(pos_n, plan.dtype, "pos_n"),
                             _ptr(mom_n, plan.dtype, "mom_n"), _ptr(pos_gr, plan.dtype, "pos_gr"),
                             _ptr(mom_gr, plan.dtype, "mom_gr"), _stream()))


def pm_xi_linear(plan: Plan, noise, ic: ICParams, a: float, xi=None):
    """Linear Poisson-gauge displacement xi_lin(a) [3, N^3] (cells) from the noise."""
    n3 = plan.n ** 3
    xi = plan.mesh(3) if xi is None else xi
    _need(noise, n3, "noise")
    _need(xi, 3 * n3, "xi")
    _check(lib().pm_xi_linear(plan.handle, _ptr(noise, plan.dtype, "noise"), ctypes.byref(ic), float(a),
                              _ptr(xi, plan.dtype, "xi"), _stream()))
    return xi


# ------------------------------------------------------------ host cosmology --

def cosmo_hubble_e(a, c=FIDUCIAL): return lib().pm_cosmo_hubble_e(ctypes.byref(c), a)
def cosmo_omega_m_a(a, c=FIDUCIAL): return lib().pm_cosmo_omega_m_a(ctypes.byref(c), a)
def cosmo_growth(a, c=FIDUCIAL): return lib().pm_cosmo_growth(ctypes.byref(c), a)
def cosmo_growth_rate(a, c=FIDUCIAL): return lib().pm_cosmo_growth_rate(ctypes.byref(c), a)
def cosmo_kick(a0, a1, c=FIDUCIAL): return lib().pm_cosmo_kick(ctypes.byref(c), a0, a1)
def cosmo_drift(a0, a1, c=FIDUCIAL): return lib().pm_cosmo_drift(ctypes.byref(c), a0, a1)


def kdk_factors(a0, a1, c=FIDUCIAL):
    out = (ctypes.c_double * 3)()
    lib().pm_kdk_factors(ctypes.byref(c), a0, a1, out)
    return out[0], out[1], out[2]


def pm_microbench_atomics(buf, passes: int = 1):
    """Unreturned float atomics (+1.0 each) over every element of the float32 device
    tensor ``buf``, ``passes`` times, on the current stream (reference rate for the
    deposits' global atomics)."""
    if buf.dtype != torch.float32 or not buf.is_cuda or not buf.is_contiguous():
        raise PMError(PM_ERR_ARG, "buf must be a contiguous float32 device tensor")
    _check(lib().pm_microbench_atomics(_c_void_p(buf.data_ptr()), buf.numel(), int(passes), _stream()))


def build_info() -> str:
    """The loaded library's build record: "pmhip <arch> sources <sha256>"."""
    return lib().pm_build_info().decode()


def build_is_current() -> bool:
    """Whether the loaded library was compiled from the sources in this tree."""
    from .build import source_digest
    return build_info().endswith(" sources " + source_digest())


def log_steps(a_start: float, a_end: float, n_steps: int):
    """n_steps + 1 scale factors equally spaced in ln a (pm_log_steps)."""
    out = (ctypes.c_double * (int(n_steps) + 1))()
    _check(lib().pm_log_steps(float(a_start), float(a_end), int(n_steps), out))
    return list(out)


def leapfrog_factors(a_steps, c=FIDUCIAL):
    """(kick, drift) of the chain of pm_step cycles that runs the kick-drift-kick
    leapfrog over a_steps: cycle j < n kicks by K2(step j-1) + K1(step j) and drifts by
    Dr(step j); the closing cycle n kicks by K2(step n-1) with drift 0
    (pm_leapfrog_factors)."""
    n = len(a_steps) - 1
    a = (ctypes.c_double * (n + 1))(*[float(x) for x in a_steps])
    kick, drift = (ctypes.c_double * (n + 1))(), (ctypes.c_double * (n + 1))()
    _check(lib().pm_leapfrog_factors(ctypes.byref(c), a, n, kick, drift))
    return list(kick), list(drift)


def gauge_params(box, n, a, a_prev=0.0, c=FIDUCIAL) -> SolveParams:
    sp = SolveParams()
    lib().pm_gauge_params(ctypes.byref(c), float(box), int(n), float(a), float(a_prev), ctypes.byref(sp))
    return sp


def newton_params(c=FIDUCIAL, grad=PM_GRAD_SPECTRAL) -> SolveParams:
    return SolveParams(kind=PM_NEWTON, grad=grad, omega_m=c.omega_m)


def power_eh98_amplitude(n_s, sigma8, c=FIDUCIAL):
    return lib().pm_power_eh98_amplitude(ctypes.byref(c), n_s, sigma8)


def power_law_amplitude(n, box, rms, index=-2.0):
    return lib().pm_power_law_amplitude(int(n), float(box), float(rms), float(index))


from . import sim  # noqa: E402,F401
