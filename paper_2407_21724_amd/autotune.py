"""Autotuner of the product's tile shapes.

It times, with the library's dispatch-timed profiling of real products:
the row tiles per block of the two matrix-core GEMM launches (near field +
projection, receive: 1, 2 or 4 tiles of 16 rows), then for every level the
aggregation and the disaggregation with each candidate row chunk (rows of
a pattern per streaming wave), and keeps the fastest of each.  A tile shape
or chunk changes only how the kernels divide the work, not any output value
(each output is computed by the same arithmetic in the same order), so the
tuned product is bitwise identical to the default one.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import mlfma

# rows per chunk of the streamed interpolation (0: the planner's chunks)
CANDIDATES = (0, 8, 16, 32, 64, 128, 100000)


def _stage_times(ctx, x, y, reps):
    ctx.profile(True)
    for _ in range(reps):
        ctx.matvec(x, out=y)
    st = ctx.profile_read()
    ctx.profile(False)
    return {s["name"]: s["total_ms"] / s["launches"] for s in st}


def _level_time(st, kind, l):
    """Time of one level's aggregation or disaggregation."""
    return st.get(f"{kind}_l{l}", float("inf"))


def autotune(ctx: "mlfma.Context", R: int = 1, reps: int = 4, candidates=CANDIDATES, log=None):
    """Tune ctx in place for products with R right-hand sides.  Returns
    {"default": (agg, dis), "tuned": (agg, dis), "stage_us": {...}}."""
    import torch
    L = ctx.info()["n_levels"]
    if L < 2:
        return {"default": ctx.get_tuning(), "tuned": ctx.get_tuning(), "gemm_rows": ctx.get_gemm_tiles(),
                "default_gemm_rows": ctx.get_gemm_tiles(), "stage_us": {}}
    n = 2 * ctx.n_modes
    rng = np.random.default_rng(0)
    x = torch.as_tensor(rng.standard_normal((R, ctx.n_particles, n)) + 1j * rng.standard_normal(
        (R, ctx.n_particles, n))).to("cuda", ctx.dtype).contiguous()
    y = torch.empty_like(x)
    default = ctx.get_tuning()
    agg, dis = [list(v) for v in default]
    ctx.matvec(x, out=y)
    report = {}
    gemm = list(ctx.get_gemm_tiles())
    default_gemm = tuple(gemm)
    if ctx.params.precision in (mlfma.C64, mlfma.C64_BF16):
        for gi, names in ((0, ("near+project", "near", "project")), (1, ("receive",))):
            times = {}
            for rt in (1, 2, 4):
                trial = list(gemm)
                trial[gi] = rt
                ctx.set_tuning(agg, dis, trial)
                st = _stage_times(ctx, x, y, reps)
                times[rt] = sum(st.get(nm, 0.0) for nm in names)
            best = min(times, key=times.get)
            gemm[gi] = best
            ctx.set_tuning(agg, dis, gemm)
            report["gemm_" + names[0]] = {"rows": best, "tried_us": {k: round(1e3 * v, 2) for k, v in times.items()}}
            if log:
                log(f"gemm {names[0]}: {1e3 * times[default_gemm[gi]]:.1f} us -> {1e3 * times[best]:.1f} us "
                    f"({best} row tiles)")
    base = _stage_times(ctx, x, y, reps)
    for kind, idx_range in (("aggregate", range(1, L)), ("disaggregate", range(0, L - 1))):
        for l in idx_range:
            name = f"{kind}_l{l}"
            cur = agg if kind == "aggregate" else dis
            best_h, best_t = cur[l], _level_time(base, kind, l)
            tried = {cur[l]: best_t}
            for h in candidates:
                if h in tried:
                    continue
                trial = list(cur)
                trial[l] = h
                try:
                    if kind == "aggregate":
                        ctx.set_tuning(trial, dis)
                    else:
                        ctx.set_tuning(agg, trial)
                except mlfma.MlfmaError:
                    continue           # tile does not fit (or taller than the level)
                t = _level_time(_stage_times(ctx, x, y, reps), kind, l)
                tried[h] = t
                if t < best_t:
                    best_h, best_t = h, t
            cur[l] = best_h
            ctx.set_tuning(agg, dis)
            report[name] = {"default_us": 1e3 * _level_time(base, kind, l), "tuned_us": 1e3 * best_t,
                            "rows": best_h, "tried_us": {int(k): round(1e3 * v, 2) for k, v in tried.items()}}
            if log:
                log(f"{name}: {report[name]['default_us']:.1f} us -> {report[name]['tuned_us']:.1f} us "
                    f"({best_h} rows)")
    ctx.set_tuning(agg, dis)
    return {"default": default, "tuned": (agg, dis), "gemm_rows": tuple(gemm), "default_gemm_rows": default_gemm,
            "stage_us": report}


TUNING_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning")


def tuning_file(workload: str, R: int) -> str:
    return os.path.join(TUNING_DIR, f"{workload}_r{R}.json")


def save(path, ctx, report, meta: dict):
    """Write the context's current tile shapes (after autotune) to path."""
    agg, dis = ctx.get_tuning()
    rec = dict(meta, agg_rows=agg, dis_rows=dis, gemm_rows=list(ctx.get_gemm_tiles()),
               stage_us=report.get("stage_us", {}))
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)


def apply(path, ctx):
    """Apply the tile shapes of a tuning file written by save()."""
    with open(path) as f:
        rec = json.load(f)
    ctx.set_tuning(rec["agg_rows"], rec["dis_rows"], tuple(rec["gemm_rows"]))
    return rec
