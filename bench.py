"""Benchmark of the PM hot path on one MI355X.

Workload (default): the fine Newtonian run of the displacement-combination
configuration -- 1024^3 particles on a 1024^3 mesh, periodic box L = 4000 Mpc/h,
seeded Gaussian white noise, Eisenstein-Hu no-wiggle LCDM spectrum (n_s = 0.965,
sigma_8 = 0.81) with Zel'dovich initial conditions at a = 0.02, 50 steps log-spaced
in a to a = 1, FP32.  A "step" is one force-kick-drift cycle of the leapfrog: CIC
deposit -> r2c FFT -> fused k-space Poisson solve and gradient -> three inverse
FFTs -> CIC gather fused with kick and drift.  The W warmup steps are the first W
steps of the schedule; the K timed steps follow them.

Prints one JSON line with particle-updates/s, the roofline of the dominant kernel
(per-kernel HIP event timing on the library's stream during the timed region) and
the FP64 CPU oracle timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

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
        "fft_solve_axis0": cs * c + 3 * cs * c,             # read delta_hat, write 3 force spectra
        "fft_cols_inv_axis1": 3 * 2 * cs * c,
        "fft_c2r_rows": 3 * cs * c + 3 * es * n3,
        "gather_kick_drift": 12 * es * np_ + 3 * es * n3,   # x, p read and written; force read once
    }


def kernel_source_digest() -> str:
    """sha256 over the HIP/C++ sources of the library (any kernel change alters it)."""
    import hashlib
    d = os.path.join(ROOT, "paper_2404_02783_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(kernel: str, n: int):
    """HBM bytes per launch of ``kernel`` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes, each scaled by the same counter's reading for
    a plain device copy), or None when there is none for this kernel and mesh or the
    kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{kernel}_{n}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != kernel_source_digest():
        return None
    try:
        return int(float(vals["fetch_bytes_per_launch"]) + float(vals["write_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


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
            "kind": "oracle",
            "sample": f"{cycles} force-kick-drift cycles of the FP64 CPU oracle (plain PyTorch) on {n_sample}^3 "
                      f"particles and a {n_sample}^3 mesh ({dt:.1f} s), scaled per particle-update"}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=48)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--box", type=float, default=4000.0)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--adjoint-cycles", type=int, default=4,
                    help="leapfrog cycles of the differentiable run timed for the adjoint/forward ratio (0: skip)")
    ap.add_argument("--adjoint-ckpt", type=int, default=2)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 1 GiB device copy first (reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (see DESIGN.md, sharding)",
              file=sys.stderr)
        sys.exit(2)

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
    pm.pm_ic_zeldovich(plan, noise, icp, disp, pos, mom)
    del disp
    torch.cuda.synchronize()
    print(f"[bench] initial conditions ready in {time.perf_counter() - t_setup:.1f}s", file=sys.stderr, flush=True)

    total = max(50, args.warmup + args.steps)
    a_s = pm.sim.log_steps(0.02, 1.0, total)
    run = pm.sim.Run(plan, pos, mom)
    k2_prev = 0.0

    def cycle(j):
        nonlocal k2_prev
        k1, dr, k2 = pm.kdk_factors(a_s[j], a_s[j + 1])
        run.cycle(a_s[j], k2_prev + k1, dr)
        k2_prev = k2

    for j in range(args.warmup):
        cycle(j)
    torch.cuda.synchronize()
    pm.pm_profile_enable(plan, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(args.warmup, args.warmup + args.steps):
        cycle(j)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = pm.pm_profile_read(plan)
    pm.pm_profile_enable(plan, False)
    pm.pm_check(plan)
    print(f"[bench] timed {args.steps} steps in {t1 - t0:.3f}s", file=sys.stderr, flush=True)

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
    step_bytes = sum(alg.values())
    step_gbs = step_bytes / (ms_step / 1000.0) / 1e9
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
        "data": "synthetic (seeded Gaussian white noise -> Zel'dovich ICs)",
        "config": {"workload": f"Newtonian PM run, {n}^3 particles on a {n}^3 mesh, L={box:g} Mpc/h, EH98 no-wiggle "
                               f"LCDM ICs at a=0.02, {total} log steps to a=1 (steps {args.warmup}..."
                               f"{args.warmup + args.steps - 1} timed)",
                   "n_mesh": n, "n_particles": n ** 3, "box_mpch": box, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(dom_gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(dom_gbs / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom, n), "alg_bytes_per_launch": alg[dom]},
        "step_roofline": {"alg_bytes_per_step": step_bytes, "achieved_GBps": round(step_gbs, 1),
                          "frac": round(step_gbs / HBM_PEAK_GBS, 4)},
        "kernels": kernels,
        "adjoint_forward_ratio": None,
    }
    if args.adjoint_cycles > 0:
        del run, pos, mom
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
    del noise
    if not args.no_cpu_baseline:
        print(f"[bench] CPU oracle baseline at {args.cpu_sample}^3 ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
