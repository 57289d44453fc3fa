"""Benchmark of the PM hot path on one MI355X.

Workload (default): the fine Newtonian run of the displacement-combination
configuration -- 1024^3 particles on a 1024^3 mesh, periodic box L = 4000 Mpc/h,
seeded Gaussian white noise, Eisenstein-Hu no-wiggle LCDM spectrum (n_s = 0.965,
sigma_8 = 0.81) with second-order (2LPT) initial conditions at a = 0.02, 50 steps log-spaced
in a to a = 1, FP32.  A "step" is one force-kick-drift cycle of the leapfrog: CIC
deposit -> r2c FFT -> fused k-space Poisson solve and gradient -> three inverse
FFTs -> CIC gather fused with kick and drift.  The W warmup steps are the first W
steps of the schedule; the K timed steps follow them; the rest of the schedule then
runs to a = 1 untimed, and its last ten cycles (the most clustered) are reported as a
late-time sample beside the average over all cycles.

Prints one JSON line with particle-updates/s, the roofline of the dominant kernel
(per-kernel HIP event timing on the library's stream during the timed region) and
the FP64 CPU oracle timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "PM particle-updates/s at 1024^3 mesh + % HBM roofline; adjoint/forward time ratio"


def algorithmic_bytes(n: int, np_: int, es: int = 4):
    """Minimum HBM bytes per launch of each kernel kind (FP32 unless es = 8)."""
    n3 = n ** 3
    c = n * n * (n // 2 + 1)          # complex elements of one spectrum
    cs = 2 * es                       # bytes per complex
    return {
        "fill": es * n3,
        "deposit": 3 * es * np_ + es * n3,                  # read positions, write the mesh once
        "fft_r2c_rows": es * n3 + cs * c,
        "fft_cols_fwd_axis1": 2 * cs * c,
        "fft_solve_axis0": cs * c + 2 * cs * c,             # read delta_hat, write F_x and G spectra
        "fft_cols_inv_axis1": 2 * cs * c + 3 * cs * c,      # read F_x, G; write F_x, D_y G, G (y-transformed)
        "fft_c2r_rows": 3 * cs * c + 3 * es * n3,
        "gather_kick_drift": 12 * es * np_ + 3 * es * n3,   # x, p read and written; force read once
        # the same plus the next cycle's density written once (positions still in registers)
        "gather_kick_drift_deposit": 12 * es * np_ + 3 * es * n3 + es * n3,
    }


# Source files that define each timed kernel (its translation unit and the headers it includes).
_PARTICLE_SOURCES = ["paper_2404_02783_amd/csrc/particles.hip", "paper_2404_02783_amd/csrc/pm_particles.h",
                     "paper_2404_02783_amd/csrc/pm_common.h", "paper_2404_02783_amd/csrc/pm_plan.h", "include/pmhip.h"]
KERNEL_SOURCES = {"gather_kick_drift": _PARTICLE_SOURCES, "gather_kick_drift_deposit": _PARTICLE_SOURCES}


def kernel_source_digest(kernel: str = "gather_kick_drift") -> str:
    """sha256 over the sources that define ``kernel`` (any change to them alters it)."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read())
    return h.hexdigest()


def profile_values(kernel: str, n: int):
    """The `- key: value` lines of the committed counter summary of ``kernel`` at mesh
    n, or {} when there is none or the kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{kernel}_{n}.md")
    if kernel not in KERNEL_SOURCES or not os.path.exists(path):
        return {}
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    return vals if vals.get("source_sha256") == kernel_source_digest(kernel) else {}


def measured_traffic(kernel: str, n: int):
    """HBM bytes per launch of ``kernel`` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes, each scaled by the same counter's reading for
    a plain device copy), or None when there is none for this kernel and mesh or the
    kernel sources changed since the counters were taken."""
    vals = profile_values(kernel, n)
    try:
        return int(float(vals["fetch_bytes_per_launch"]) + float(vals["write_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def l2_atomic_rate(pm, n: int = 1 << 28, passes: int = 4, reps: int = 3) -> float:
    """Unreturned float atomics per second (G/s) of pm_microbench_atomics on n distinct
    consecutive cells (the deposits' flush pattern), best of reps launches."""
    import torch
    buf = torch.zeros(n, dtype=torch.float32, device="cuda")
    pm.pm_microbench_atomics(buf, passes=1)  # warm
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = None
    for _ in range(reps):
        e0.record()
        pm.pm_microbench_atomics(buf, passes=passes)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del buf
    return n * passes / (best / 1000.0) / 1e9


def cpu_baseline(n_sample: int, seed: int = 5, min_seconds: float = 10.0, max_cycles: int = 4):
    """Force-kick-drift cycles of the FP64 oracle on n_sample^3 particles, repeated
    until about ``min_seconds`` of CPU work (at most ``max_cycles``)."""
    import torch
    import synth_inputs as si
    from oracle import integrate
    x = torch.from_numpy(si.lattice_jitter_particles(n_sample, seed, 0.8))
    v = torch.zeros_like(x)
    force = integrate.NewtonForce(n_sample)
    cycles = 0
    t0 = time.perf_counter()
    while cycles < max_cycles and (cycles == 0 or time.perf_counter() - t0 < min_seconds):
        x, v = integrate.force_then_kick_drift(x, v, 0.01, 0.01, force, 0.5, n_sample)
        cycles += 1
    dt = time.perf_counter() - t0
    return {"value": cycles * n_sample ** 3 / dt, "unit": "particle-updates/s", "cores": torch.get_num_threads(),
            "kind": "oracle", "host": host_description(),
            "sample": f"{cycles} force-kick-drift cycles of the FP64 CPU oracle (plain PyTorch) on {n_sample}^3 "
                      f"particles and a {n_sample}^3 mesh ({dt:.1f} s), scaled per particle-update"}


def host_description():
    """CPU model, logical CPUs this process may use, and RAM of the host (Linux /proc)."""
    model, mem_kib = None, None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal:"):
                    mem_kib = int(line.split()[1])
                    break
    except OSError:
        pass
    return {"cpu_model": model, "cpus_available": len(os.sched_getaffinity(0)),
            "ram_GiB": round(mem_kib / 2 ** 20, 1) if mem_kib else None}


def adjoint_ratio(pm, plan, noise, icp, n_cycles: int, ckpt: int, n_bins: int):
    """Times the differentiable forward model (ICs, n_cycles leapfrog cycles of the
    schedule's start, deposit, P(k)) and its reverse pass (P(k) adjoint, checkpoint
    recomputation, adjoint cycles, IC adjoint) on the same plan.  Returns
    (forward s, backward s, per-kernel profile of the reverse pass)."""
    import torch
    from paper_2404_02783_amd import diff
    a_s = pm.sim.log_steps(0.02, 1.0, 50)
    dpk = torch.linspace(-1.0, 1.0, n_bins, dtype=torch.float64, device=plan.device)
    # warm the adjoint kernels once on a single cycle
    _, tape = diff.forward(plan, noise, icp, diff.Schedule(a_s[:2]), n_bins, 1)
    diff.backward(tape, dpk)
    del tape
    torch.cuda.synchronize()
    sched = diff.Schedule(a_s[:n_cycles + 1])
    t0 = time.perf_counter()
    _, tape = diff.forward(plan, noise, icp, sched, n_bins, ckpt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pm.pm_profile_enable(plan, True)
    g = diff.backward(tape, dpk)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    prof = pm.pm_profile_read(plan)
    pm.pm_profile_enable(plan, False)
    del tape, g
    return t1 - t0, t2 - t1, prof


def estimators_and_combination(pm, plan, pos, fine_noise, a_end, n_bins=256):
    """Timings of the estimator and combination calls of the displacement-combination
    configuration on the final 1024^3 positions: deposit + P(k) in 256 bins, B(k)
    on 64 triangles (32 equilateral k = m*16 k_f, 32 squeezed with k3 = 4 k_f; shell
    width 2 k_f), the combination of a 256^3 pair into the 1024^3 run, and the
    combination with the linear shift at 256^3 in place of the pair; then P(k) and
    B(k) of the two combinations against each other and against the Newtonian run
    (the comparison of the paper's power-spectrum and bispectrum figures)."""
    import torch
    import synth_inputs as si
    out = {}
    n = plan.n
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    delta = pm.pm_deposit(plan, pos)
    k, pk, cnt = pm.pk_estimate(plan, delta, n_bins)
    torch.cuda.synchronize()
    out["deposit_pk_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    # B(k): shells m*16 k_f (m = 1..32) and the squeezed shell at 4 k_f
    centres = [16.0 * m for m in range(1, 33)] + [4.0]
    tris = [(m, m, m) for m in range(32)] + [(m, m, 32) for m in range(32)]
    shell_ws = torch.empty((8,) + (n,) * 3, dtype=plan.dtype, device=plan.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bk, ntri = pm.bk_estimate(plan, delta, centres, 2.0, tris, shell_ws=shell_ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    bk2, _ = pm.bk_estimate(plan, delta, centres, 2.0, tris, shell_ws=shell_ws, ntri_known=ntri)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out["bk_first_call_ms"] = round((t1 - t0) * 1e3, 1)
    out["bk_cached_counts_ms"] = round((t2 - t1) * 1e3, 1)
    del bk
    # combination: a coarse 256^3 Newtonian/Poisson-gauge pair (L = 4000 Mpc/h, 50 log steps)
    nc = 256
    cplan = pm.Plan(nc, plan.box, plan.dtype, plan.device)
    noise = pm.pm_noise_truncate(plan, fine_noise, cplan)  # same phases as the fine run
    icp = pm.ICParams(pk_kind=pm.PM_PK_EH98, amp=pm.power_eh98_amplitude(0.965, 0.81), index=0.965, a_init=0.02,
                      a_norm=1.0, cosmo=pm.FIDUCIAL)
    xn, pn, xg, pg = (torch.empty((3, nc ** 3), dtype=plan.dtype, device=plan.device) for _ in range(4))
    disp = cplan.mesh(3)
    pm.pm_ic_2lpt(cplan, noise, icp, disp, xn, pn)   # second-order start (Sec. 3), as the fine run
    pm.pm_ic_gauge(cplan, noise, icp, disp, xn, pn, xg, pg)
    a_s = pm.sim.log_steps(0.02, 1.0, 50)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pm.sim.Run(cplan, xn, pn).leapfrog(a_s, close=False)
    pm.sim.Run(cplan, xg, pg, gauge=True).leapfrog(a_s, close=False)
    torch.cuda.synchronize()
    out["coarse_pair_256_50steps_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
    x_out = torch.empty_like(pos)
    pm.displacement_combine(xg, xn, nc, pos, n, x_out)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pm.displacement_combine(xg, xn, nc, pos, n, x_out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["combine_ms"] = round(dt * 1e3, 2)
    out["combine_GBps_alg"] = round(24 * n ** 3 / dt / 1e9, 1)  # read x_fine, write x_out
    stats = {"newton": (pk, bk2)}

    def statistics(x):
        d = pm.pm_deposit(plan, x)
        p = pm.pk_estimate(plan, d, n_bins)[1]
        b, _ = pm.bk_estimate(plan, d, centres, 2.0, tris, shell_ws=shell_ws, ntri_known=ntri)
        return p, b
    stats["combined"] = statistics(x_out)
    # combination with linear theory: the linear Poisson-gauge shift at a = 1 from the
    # coarse noise (one k-space pass and its inverse transform), added to the fine run
    xi = cplan.mesh(3)
    pm.pm_xi_linear(cplan, noise, icp, 1.0, xi)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pm.pm_xi_linear(cplan, noise, icp, 1.0, xi)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pm.displacement_add(xi, nc, pos, n, x_out)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out["xi_linear_256_ms"] = round((t1 - t0) * 1e3, 2)
    out["add_linear_shift_ms"] = round((t2 - t1) * 1e3, 2)
    del xi
    stats["combined_1lpt"] = statistics(x_out)
    pb = [0, 1, 2, 3, 5, 8, 16, 64]
    tb = [0, 1, 3, 7, 32, 33, 35, 39]   # equilateral m = 1, 2, 4, 8 and squeezed m = 1, 2, 4, 8

    def rel(a, b, idx):
        return [round(float(a[i] / b[i] - 1.0), 5) for i in idx]
    (p_n, b_n), (p_c, b_c), (p_l, b_l) = stats["newton"], stats["combined"], stats["combined_1lpt"]
    out["combined_vs_linear"] = {
        "a_end": round(a_end, 4),
        "k_h_per_Mpc": [round(float(k[i]), 5) for i in pb],
        "pk_combined_over_newton_minus_1": rel(p_c, p_n, pb),
        "pk_combined_1lpt_over_combined_minus_1": rel(p_l, p_c, pb),
        "bk_triangles": ["equilateral 16,32,64,128 k_f", "squeezed k1=k2=16,32,64,128 k_f, k3=4 k_f"],
        "bk_combined_over_newton_minus_1": rel(b_c, b_n, tb),
        "bk_combined_1lpt_over_combined_minus_1": rel(b_l, b_c, tb)}
    del stats, shell_ws, bk2, ntri
    # cross spectrum of the combined field with the fine run's (256 bins)
    delta_c = pm.pm_deposit(plan, x_out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pm.pk_cross_estimate(plan, delta_c, delta, n_bins)
    torch.cuda.synchronize()
    out["pk_cross_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    del delta_c
    out["note"] = ("coarse noise is the Fourier truncation of the fine noise (shared phases); B(k) keeps 8 shell "
                   "fields resident and recomputes evicted shells")
    del x_out, xn, pn, xg, pg, disp, cplan, delta
    return out


def ic_leg(pm, plan, noise, icp):
    """Wall time of the Zel'dovich and second-order (2LPT) initial conditions at the
    plan's size (one call each after a warm call; not part of the timed step)."""
    import torch
    out = {}
    disp = plan.mesh(3)
    pos, mom = plan.particles(), plan.particles()
    for name, fn in (("zeldovich", pm.pm_ic_zeldovich), ("2lpt", pm.pm_ic_2lpt)):
        fn(plan, noise, icp, disp, pos, mom)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn(plan, noise, icp, disp, pos, mom)
        torch.cuda.synchronize()
        out[f"{name}_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    del disp, pos, mom
    return out


def gradient_study(pm, n=256, box=2000.0, steps=50, n_bins=128):
    """Gradient-order study on the 256^3 configuration (EH98 ICs at a = 0.02, 50 log
    steps to a = 1): P(k) of the Newtonian and Poisson-gauge runs with the first- and
    second-order finite-difference gradients relative to the spectral runs, and of the
    spectral Newtonian run combined with each variant's xi relative to the spectral
    Poisson-gauge run, at selected bins."""
    import torch
    import synth_inputs as si
    plan = pm.Plan(n, box, torch.float32)
    noise = torch.from_numpy(si.white_noise(n, 11, dtype=np.float32)).to(plan.device)
    icp = pm.ICParams(pk_kind=pm.PM_PK_EH98, amp=pm.power_eh98_amplitude(0.965, 0.81), index=0.965, a_init=0.02,
                      a_norm=1.0, cosmo=pm.FIDUCIAL)
    disp = plan.mesh(3)
    a_s = pm.sim.log_steps(0.02, 1.0, steps)
    pk, runs = {}, {}
    for name, g in (("spectral", pm.PM_GRAD_SPECTRAL), ("fd2", pm.PM_GRAD_FD2), ("fd1", pm.PM_GRAD_FD1)):
        pos, mom, pg, mg = (plan.particles() for _ in range(4))
        pm.pm_ic_zeldovich(plan, noise, icp, disp, pos, mom)
        pm.pm_ic_gauge(plan, noise, icp, disp, pos, mom, pg, mg)
        pm.sim.Run(plan, pos, mom, grad=g).leapfrog(a_s)
        pm.sim.Run(plan, pg, mg, gauge=True, grad=g).leapfrog(a_s)
        runs[name] = (pos, pg)
        for tag, x in (("N", pos), ("GR", pg)):
            k, p, _ = pm.pk_estimate(plan, pm.pm_deposit(plan, x), n_bins)
            pk[name, tag] = p.cpu()
    for name in ("fd2", "fd1"):
        comb = pm.displacement_combine(runs[name][1], runs[name][0], n, runs["spectral"][0], n)
        _, p, _ = pm.pk_estimate(plan, pm.pm_deposit(plan, comb), n_bins)
        pk[name, "comb"] = p.cpu()
    torch.cuda.synchronize()
    sel = [0, 2, 5, 12, 20, 40, 60, n_bins - 1]
    kk = k.cpu()
    out = {"workload": f"{n}^3, L={box:g} Mpc/h, EH98 ICs a=0.02, {steps} log steps to a=1, P(k) in {n_bins} bins",
           "k_h_per_Mpc": [round(float(kk[i]), 4) for i in sel]}
    for name in ("fd1", "fd2"):
        for tag, ref in (("N", ("spectral", "N")), ("GR", ("spectral", "GR")), ("comb", ("spectral", "GR"))):
            r = pk[name, tag] / pk[ref] - 1.0
            out[f"{name}_{tag}_rel"] = [round(float(r[i]), 4) for i in sel]
    del runs, plan
    return out


def adjoint_small(pm, n=128, box=1000.0, n_steps=20, ckpt=5, n_bins=64):
    """Adjoint/forward time of the differentiable configuration: 128^3, L = 1000 Mpc/h,
    20 log steps a = 0.05 -> 1, P(k) in 64 bins, checkpoints every 5 cycles."""
    import torch
    import synth_inputs as si
    from paper_2404_02783_amd import diff
    dev = torch.device("cuda:0")
    plan = pm.Plan(n, box, torch.float32, dev)
    noise = torch.from_numpy(si.white_noise(n, 5, dtype=np.float32)).to(dev)
    icp = pm.ICParams(pk_kind=pm.PM_PK_EH98, amp=pm.power_eh98_amplitude(0.965, 0.81), index=0.965, a_init=0.05,
                      a_norm=1.0, cosmo=pm.FIDUCIAL)
    sched = diff.Schedule(pm.sim.log_steps(0.05, 1.0, n_steps))
    dpk = torch.linspace(-1.0, 1.0, n_bins, dtype=torch.float64, device=dev)
    best = None
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, tape = diff.forward(plan, noise, icp, sched, n_bins, ckpt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        diff.backward(tape, dpk)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if best is None or (t2 - t1) + (t1 - t0) < best[0] + best[1]:
            best = (t1 - t0, t2 - t1)
    gm = diff.GraphedModel(plan, icp, sched, n_bins, ckpt).capture()
    gbest = None
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gm.forward(noise)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gm.backward(dpk)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if gbest is None or (t2 - t0) < gbest[0] + gbest[1]:
            gbest = (t1 - t0, t2 - t1)
    del gm
    # the same with the second-order (2LPT) start, graph-captured
    g2 = diff.GraphedModel(plan, icp, diff.Schedule(sched.a_steps, lpt_order=2), n_bins, ckpt).capture()
    g2best = None
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g2.forward(noise)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g2.backward(dpk)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if g2best is None or (t2 - t0) < g2best[0] + g2best[1]:
            g2best = (t1 - t0, t2 - t1)
    return {"workload": f"{n}^3, L={box:g} Mpc/h, {n_steps} log steps a=0.05->1, P(k) in {n_bins} bins, "
                        f"checkpoints every {ckpt}",
            "eager": {"forward_ms": round(best[0] * 1e3, 2), "backward_ms": round(best[1] * 1e3, 2),
                      "ratio": round(best[1] / best[0], 3)},
            "graphed": {"forward_ms": round(gbest[0] * 1e3, 2), "backward_ms": round(gbest[1] * 1e3, 2),
                        "ratio": round(gbest[1] / gbest[0], 3)},
            "graphed_2lpt_start": {"forward_ms": round(g2best[0] * 1e3, 2),
                                   "backward_ms": round(g2best[1] * 1e3, 2),
                                   "ratio": round(g2best[1] / g2best[0], 3)}}


def ensemble_leg(pm):
    """64-box ensemble (16 x 64^3, 24 x 128^3, 16 x 192^3, 8 x 256^3; 30 log steps
    a = 0.02 -> 1; per-box P(k)) as one pm_batch: one captured graph of the batch calls
    (one launch per kernel and size group; FFT launch shapes autotuned per group; also
    timed with the built-in shapes and with the groups on concurrent streams) vs the
    same boxes run one by one on single-box plans (also autotuned) with eager launches;
    plus the ensemble's HBM roofline fraction."""
    import torch
    import synth_inputs as si
    from paper_2404_02783_amd import ensemble
    dev = torch.device("cuda:0")
    groups = ensemble.default_groups()
    noise_fn = lambda n, s: si.white_noise(n, s)  # noqa: E731
    from paper_2404_02783_amd import tuning
    # the graph with the built-in FFT launch shapes, then with autotuned ones
    ens = ensemble.Ensemble(groups, noise_fn, 0.02, 1.0, 30, torch.float32, dev)
    ens.capture()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.replay()
    torch.cuda.synchronize()
    t_graph_builtin = time.perf_counter() - t0
    del ens
    # the groups on streams of their own inside the graph (their kernels may overlap)
    ens = ensemble.Ensemble(groups, noise_fn, 0.02, 1.0, 30, torch.float32, dev, autotune=True, concurrent=True)
    ens.capture()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.replay()
    torch.cuda.synchronize()
    t_graph_conc = time.perf_counter() - t0
    pk_conc = [o[1].clone() for o in ens.power_spectra()]
    del ens
    ens = ensemble.Ensemble(groups, noise_fn, 0.02, 1.0, 30, torch.float32, dev, autotune=True)
    shapes = {f"{n}^3 x {cnt}": t[0] for (n, _, cnt), t in ens.group_tuning}
    ens.capture()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.replay()
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    t0 = time.perf_counter()
    ens.run()
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - t0
    pk_batched = [o[1].clone() for o in ens.power_spectra()]
    plans = {(g.n, g.box): pm.Plan(g.n, g.box, torch.float32, dev) for g in groups}
    for pl in plans.values():
        tuning.tune(pl)
    noises = {s: st.noise[i] for st in ens.states for i, s in enumerate(st.group.seeds)}
    one = [ensemble.Group(g.n, g.box, g.seeds[:1]) for g in groups]
    ensemble.run_sequential(one, noise_fn, 0.02, 1.0, 30, torch.float32, dev, plans, noises)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pk_seq = ensemble.run_sequential(groups, noise_fn, 0.02, 1.0, 30, torch.float32, dev, plans, noises)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    worst = max(float(((a - b).abs() / b.abs().clamp_min(1e-30)).max()) for a, b in zip(pk_batched, pk_seq))
    worst_conc = max(float(((a - b).abs() / b.abs().clamp_min(1e-30)).max()) for a, b in zip(pk_conc, pk_batched))
    # HBM roofline of the ensemble: algorithmic bytes of the 30 cycles of every box (the
    # kernels of one pm_step cycle with the handed-over density) over the graph replay,
    # which also holds the ICs and the final P(k)
    cyc_bytes = 0
    for g in groups:
        a = algorithmic_bytes(g.n, g.n ** 3)
        per_cycle = sum(a[k] for k in ("fill", "fft_r2c_rows", "fft_cols_fwd_axis1", "fft_solve_axis0",
                                       "fft_cols_inv_axis1", "fft_c2r_rows", "gather_kick_drift_deposit"))
        cyc_bytes += 30 * per_cycle * len(g.seeds)
    out = {"boxes": sum(len(g.seeds) for g in groups),
           "particle_updates_per_s_graph": round(30 * sum(len(g.seeds) * g.n ** 3 for g in groups) / t_graph, 1),
           "hbm_roofline_graph": {"alg_bytes_30_cycles": cyc_bytes, "achieved_GBps": round(cyc_bytes / t_graph / 1e9, 1),
                                  "frac": round(cyc_bytes / t_graph / 1e9 / HBM_PEAK_GBS, 4),
                                  "note": "graph time includes the ICs and the final P(k)"},
           "graph_s": round(t_graph, 4),
           "graph_builtin_fft_shapes_s": round(t_graph_builtin, 4), "fft_shapes_autotuned": shapes,
           "graph_concurrent_groups_s": round(t_graph_conc, 4),
           "speedup_concurrent_graph_vs_sequential": round(t_seq / t_graph_conc, 2),
           "max_rel_pk_diff_concurrent_vs_serial": worst_conc,
           "batched_eager_s": round(t_eager, 4), "sequential_s": round(t_seq, 4),
           "speedup_graph_vs_sequential": round(t_seq / t_graph, 2),
           "max_rel_pk_diff_batched_vs_sequential": worst}
    del ens, plans, noises
    # the same comparison for 64 small boxes only (64^3, L = 500 Mpc/h), where launches dominate
    small = [ensemble.Group(64, 500.0, list(range(200, 264)))]
    ens = ensemble.Ensemble(small, noise_fn, 0.02, 1.0, 30, torch.float32, dev, autotune=True)
    ens.capture()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.replay()
    torch.cuda.synchronize()
    ts_graph = time.perf_counter() - t0
    plans = {(64, 500.0): pm.Plan(64, 500.0, torch.float32, dev)}
    tuning.tune(plans[(64, 500.0)])
    noises = {s: ens.states[0].noise[i] for i, s in enumerate(small[0].seeds)}
    ensemble.run_sequential([ensemble.Group(64, 500.0, [200])], noise_fn, 0.02, 1.0, 30, torch.float32, dev, plans,
                            noises)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ensemble.run_sequential(small, noise_fn, 0.02, 1.0, 30, torch.float32, dev, plans, noises)
    torch.cuda.synchronize()
    ts_seq = time.perf_counter() - t0
    out["small_boxes_64x64^3"] = {"graph_s": round(ts_graph, 4), "sequential_s": round(ts_seq, 4),
                                  "speedup_graph_vs_sequential": round(ts_seq / ts_graph, 2)}
    return out


# Legs that need only the library (their own inputs and plans).  Each runs in a child
# process of its own, started before this process touches the GPU (a process that has
# initialised the GPU starts no programs) and released, one at a time, once the 1024^3
# legs have freed their memory: a failure in one is recorded in its entry and costs
# neither the other legs nor the headline line.
CHILD_LEGS = ("gradient_order_study", "adjoint_128", "ensemble")
CHILD_LEG_TIMEOUT_S = 600


def start_child_leg(name: str):
    return subprocess.Popen([sys.executable, "-u", os.path.abspath(__file__), "--leg", name], cwd=ROOT,
                            stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True)


def finish_child_leg(proc, name: str) -> dict:
    """Release a waiting child leg and collect the JSON line it prints."""
    print(f"[bench] {name} (child process {proc.pid})", file=sys.stderr, flush=True)
    try:
        out, _ = proc.communicate("go\n", timeout=CHILD_LEG_TIMEOUT_S)
    except subprocess.TimeoutExpired:
        proc.kill()
        proc.communicate()
        return {"error": f"no result within {CHILD_LEG_TIMEOUT_S} s (killed)"}
    lines = [ln for ln in out.splitlines() if ln.startswith("{")]
    if proc.returncode == 0 and lines:
        return json.loads(lines[-1])
    return {"error": f"child process ended with status {proc.returncode} before its result"}


def run_child_leg(name: str) -> None:
    """Body of a child leg: wait for the parent's go (end of input: the parent is gone),
    then run the leg on cuda:0 and print its result as one JSON line."""
    import torch  # noqa: F401  (loaded while waiting; the GPU is not touched before the go)
    if sys.stdin.readline().strip() != "go":
        return
    import paper_2404_02783_amd as pm
    torch.cuda.set_device(torch.device("cuda:0"))
    leg = {"gradient_order_study": gradient_study, "adjoint_128": adjoint_small, "ensemble": ensemble_leg}[name]
    print(json.dumps(leg(pm)), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--box", type=float, default=4000.0)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--adjoint-cycles", type=int, default=4,
                    help="leapfrog cycles of the differentiable run timed for the adjoint/forward ratio (0: skip)")
    ap.add_argument("--adjoint-ckpt", type=int, default=2)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the estimator/combination timings, the 128^3 adjoint and the ensemble legs")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the FFT launch shapes of the 1024^3 plan (per pass; measured slower for the "
                         "whole step than the built-in shapes, so off by default)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 1 GiB device copy first (reference for hardware byte counters)")
    ap.add_argument("--legs", default=",".join(CHILD_LEGS),
                    help="comma-separated child-process legs to run (of %s; ignored with --no-extras)"
                         % ", ".join(CHILD_LEGS))
    ap.add_argument("--leg", choices=CHILD_LEGS, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.leg:
        run_child_leg(args.leg)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the multi-GPU (sharded) path is not implemented",
              file=sys.stderr)
        sys.exit(2)
    legs = [] if args.no_extras else [x for x in args.legs.split(",") if x]
    for x in legs:
        if x not in CHILD_LEGS:
            ap.error(f"unknown leg {x!r}")
    children = {x: start_child_leg(x) for x in legs}   # before this process touches the GPU

    import numpy as np
    import torch
    import paper_2404_02783_amd as pm
    import synth_inputs as si

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n, box = args.n, args.box
    t_setup = time.perf_counter()
    plan = pm.Plan(n, box, torch.float32, dev)
    pos = torch.empty((3, n ** 3), dtype=torch.float32, device=dev)
    mom = torch.empty_like(pos)
    disp = plan.mesh(3)
    noise = torch.from_numpy(si.white_noise(n, args.seed, dtype=np.float32)).to(dev)
    print(f"[bench] noise {n}^3 ready in {time.perf_counter() - t_setup:.1f}s", file=sys.stderr, flush=True)
    icp = pm.ICParams(pk_kind=pm.PM_PK_EH98, amp=pm.power_eh98_amplitude(0.965, 0.81), index=0.965,
                      a_init=0.02, a_norm=1.0, cosmo=pm.FIDUCIAL)
    pm.pm_ic_2lpt(plan, noise, icp, disp, pos, mom)   # second-order Lagrangian ICs (Sec. 3)
    del disp
    torch.cuda.synchronize()
    print(f"[bench] initial conditions ready in {time.perf_counter() - t_setup:.1f}s", file=sys.stderr, flush=True)

    # FFT launch shapes of the 1024^3 plan: built-in, or measured once before the run
    # (setup, untimed) with --autotune
    if not args.autotune:
        tuned, tuned_ms = pm.pm_plan_get_tuning(plan), [-1.0] * 4
    else:
        scratch = plan.mesh()
        tuned, tuned_ms = pm.pm_plan_autotune(plan, reps=3, use_cache=False, mesh_scratch=scratch)
        del scratch
    print(f"[bench] FFT launch shapes {tuned} ({[round(m, 3) for m in tuned_ms]} ms)", file=sys.stderr, flush=True)

    total = max(50, args.warmup + args.steps)
    a_s = pm.sim.log_steps(0.02, 1.0, total)
    run = pm.sim.Run(plan, pos, mom)
    kicks, drifts = pm.leapfrog_factors(a_s)

    def cycle(j):
        run.cycle(a_s[j], kicks[j], drifts[j])

    # every cycle of the schedule is profiled (HIP events around each launch on the
    # library's stream); windows: warm-up, timed, the rest, and the late-time sample
    # of the last ten cycles (a -> 1, the most clustered and slowest)
    pm.pm_profile_enable(plan, True)
    for j in range(args.warmup):
        cycle(j)
    torch.cuda.synchronize()
    prof_warm = pm.pm_profile_read(plan)
    t0 = time.perf_counter()
    for j in range(args.warmup, args.warmup + args.steps):
        cycle(j)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = pm.pm_profile_read(plan)
    pm.pm_check(plan)
    print(f"[bench] timed {args.steps} steps in {t1 - t0:.3f}s", file=sys.stderr, flush=True)
    late0 = max(args.warmup + args.steps, total - 10)
    for j in range(args.warmup + args.steps, late0):
        cycle(j)
    torch.cuda.synchronize()
    prof_mid = pm.pm_profile_read(plan)
    t2 = time.perf_counter()
    for j in range(late0, total):
        cycle(j)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    prof_late = pm.pm_profile_read(plan)
    pm.pm_profile_enable(plan, False)
    pm.pm_check(plan)
    print(f"[bench] cycles {late0}..{total - 1} in {t3 - t2:.3f}s (schedule done, a = 1)", file=sys.stderr,
          flush=True)

    ms_step = (t1 - t0) * 1000.0 / args.steps
    value = n ** 3 / (ms_step / 1000.0)
    alg = algorithmic_bytes(n, n ** 3)
    kernels = {}
    for name, (ms, cnt) in prof.items():
        avg = ms / cnt
        b = alg.get(name)
        kernels[name] = {"avg_ms": round(avg, 4), "launches": cnt,
                         "alg_GBps": round(b / (avg / 1000.0) / 1e9, 1) if b else None}
    dom = max(prof.items(), key=lambda kv: kv[1][0])[0]
    dom_avg = prof[dom][0] / prof[dom][1]
    dom_gbs = alg[dom] / (dom_avg / 1000.0) / 1e9
    # algorithmic bytes of the kernels the timed steps actually launched, per step
    step_bytes = sum(alg[k] * cnt for k, (_, cnt) in prof.items() if k in alg) // args.steps
    step_gbs = step_bytes / (ms_step / 1000.0) / 1e9

    def window(pr, cycles, wall_s=None):
        ms, cnt = pr.get(dom, (0.0, 0))
        w = {"cycles": cycles, "dominant_avg_ms": round(ms / cnt, 4) if cnt else None,
             "dominant_frac": round(alg[dom] / (ms / cnt / 1000.0) / 1e9 / HBM_PEAK_GBS, 4) if cnt else None}
        if wall_s is not None and total > late0:
            w["ms_per_step"] = round(wall_s * 1000.0 / (total - late0), 3)
        return w
    whole = {}
    for pr in (prof_warm, prof, prof_mid, prof_late):
        for k, (ms, cnt) in pr.items():
            a, b = whole.get(k, (0.0, 0))
            whole[k] = (a + ms, b + cnt)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Gaussian white noise -> 2LPT ICs)",
        "config": {"workload": f"Newtonian PM run, {n}^3 particles on a {n}^3 mesh, L={box:g} Mpc/h, EH98 no-wiggle "
                               f"LCDM 2LPT ICs at a=0.02, {total} log steps to a=1 (steps {args.warmup}..."
                               f"{args.warmup + args.steps - 1} timed)",
                   "n_mesh": n, "n_particles": n ** 3, "box_mpch": box, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(dom_gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(dom_gbs / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom, n), "alg_bytes_per_launch": alg[dom]},
        "step_roofline": {"alg_bytes_per_step": step_bytes, "achieved_GBps": round(step_gbs, 1),
                          "frac": round(step_gbs / HBM_PEAK_GBS, 4),
                          "late_sample": window(prof_late, f"{late0}..{total - 1}", t3 - t2),
                          "whole_run": window(whole, f"0..{total - 1}")},
        "kernels": kernels,
        "fft_tuning": {"slots": list(pm.TUNING_SLOTS), "shapes": tuned, "autotuned": bool(args.autotune),
                       "best_ms": [round(m, 4) for m in tuned_ms]},
        "adjoint_forward_ratio": None,
    }
    # the deposit part's global atomics against the L2 atomic rate (microbenchmark on
    # the flush pattern); the fused kernel's atomic requests per launch and the
    # microbenchmark's requests per atomic come from the committed counter summary
    rate = l2_atomic_rate(pm)
    vals = profile_values(dom, n)
    atom = {"l2_atomic_rate_G_per_s": round(rate, 1), "kernel": dom}
    try:
        req = float(vals["atomic_requests_per_launch"])
        per_atomic = float(vals["microbench_requests_per_atomic"])
        atom["atomic_requests_per_launch"] = int(req)
        atom["atomics_per_launch_equiv"] = int(req / per_atomic)
        atom["atomics_G_per_s_equiv"] = round(req / per_atomic / (dom_avg / 1000.0) / 1e9, 1)
        atom["frac_of_l2_atomic_rate"] = round(atom["atomics_G_per_s_equiv"] / rate, 3)
    except (KeyError, ValueError, ZeroDivisionError):
        atom["atomic_requests_per_launch"] = None
    out["deposit_atomics"] = atom
    if not args.no_extras:
        print("[bench] estimators and combination at 1024^3", file=sys.stderr, flush=True)
        a_end = float(a_s[total])
        out["estimators_combination_1024"] = estimators_and_combination(pm, plan, pos, noise, a_end)
        print("[bench] initial conditions at 1024^3", file=sys.stderr, flush=True)
        out["initial_conditions_1024"] = ic_leg(pm, plan, noise, icp)
    del run, pos, mom
    if args.adjoint_cycles > 0:
        torch.cuda.synchronize()
        print(f"[bench] adjoint: {args.adjoint_cycles} cycles, checkpoint every {args.adjoint_ckpt}",
              file=sys.stderr, flush=True)
        t_fwd, t_bwd, aprof = adjoint_ratio(pm, plan, noise, icp, args.adjoint_cycles, args.adjoint_ckpt, 256)
        out["adjoint_forward_ratio"] = round(t_bwd / t_fwd, 3)
        out["adjoint"] = {
            "workload": f"d loss/d noise through Zel'dovich ICs, {args.adjoint_cycles} leapfrog cycles (a=0.02 start of "
                        f"the same schedule), CIC deposit and P(k) in 256 bins at {n}^3; checkpoints every "
                        f"{args.adjoint_ckpt} cycles",
            "forward_s": round(t_fwd, 4), "backward_s": round(t_bwd, 4),
            "kernels": {k: {"avg_ms": round(ms / c, 4), "launches": c} for k, (ms, c) in aprof.items()}}
    del noise, plan
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    for x, proc in children.items():
        out[x] = finish_child_leg(proc, x)
    if not args.no_cpu_baseline:
        print(f"[bench] CPU oracle baseline at {args.cpu_sample}^3 ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
