"""FFT launch shapes per plan: measured by ``pm_plan_autotune`` in the library and
kept in an optional JSON file keyed by device, mesh size, dtype and batch, so that
later processes reuse a measurement instead of repeating it.

Host plumbing only: the measurement and the launches run in the library."""
from __future__ import annotations

import json
import os

import torch

from . import Plan, pm_plan_autotune, pm_plan_set_tuning

__all__ = ["tuning_key", "tune"]


def tuning_key(plan: Plan) -> str:
    name = torch.cuda.get_device_name(plan.device)
    dt = "f32" if plan.dtype == torch.float32 else "f64"
    return f"{name}|n={plan.n}|{dt}|boxes={plan.batch}"


def tune(plan: Plan, cache_path: str | None = None, reps: int = 3, mesh_scratch=None):
    """Applies the shapes recorded for this plan's key in ``cache_path`` if there are
    any, else measures them (``pm_plan_autotune``) and records them there.  Returns
    (shapes, source) with source "file", "process" (library cache) or "measured"."""
    key = tuning_key(plan)
    table = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            table = json.load(f)
        if key in table:
            pm_plan_set_tuning(plan, table[key]["shapes"])
            return list(table[key]["shapes"]), "file"
    shapes, ms = pm_plan_autotune(plan, reps=reps, use_cache=True, mesh_scratch=mesh_scratch)
    source = "process" if all(m < 0 for m in ms) else "measured"
    if cache_path:
        table[key] = {"shapes": shapes, "best_ms": ms}
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return shapes, source
