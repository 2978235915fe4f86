"""MLFMA-SMR matrix-vector throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c5] [--rhs 16]

Workload (default): the 200 x 200 metalens of dielectric cylinders (height
0.6, eps 6.25, pitch 0.5 wavelengths, 32 diameter classes on the hyperbolic
focusing profile of focal length 50, 600-triangle jittered meshes, 15 + 15
static modes per current: 2,400,000 unknowns, 7 translation levels), FP32
complex product, 16 seeded random right-hand sides resident in HBM.  A step
is one full product Y = Z X for the 16 columns (near blocks, leaf
projection, aggregation, translation, disaggregation, receive).  Beside it:
GMRES time to a 1e-4 true relative residual on the same lens for one
normal-incidence plane wave, from zero and from the learned initial guess;
the 64-RHS product of the 40 x 40 array; and the 80 x 80 lens solved for 16
incidences in one batched GMRES.

Prints one JSON line.  The cpu_baseline leg times the FP64 oracle on a
bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
FP32_MFMA_PEAK = 157.3e12   # MI355X dense FP32 matrix-core peak
FP32_VALU_PEAK = 157.3e12   # MI355X FP32 vector peak
ENGINE_SRC = os.path.join(ROOT, "paper_2407_21724_amd", "csrc", "engine.hip")

# product stages (as named by mlfma_profile_read) -> kernel symbol prefix and
# the roofline that bounds it (FP32 product; the GEMM stages are named by
# kernel_of from the dispatch rules of the engine)
KERNELS = [
    ("aggregate_l", "k_agg_stream", "hbm"),
    ("translate", "k_translate_reg", "hbm"),          # FP32: every level in one launch, tiles in registers
    ("disaggregate_l", "k_dis_stream", "hbm"),
    ("near_sum", "k_near_sum", "hbm"),
]


def kernel_of(stage, gemm_rows=(4, 4), R=1, multi_class=True):
    """Kernel symbol and roofline bound of a product stage of the FP32
    product.  The GEMM stages follow the engine's dispatch: the LDS-staged
    kernel k_gemm_lds<mode, waves, column tiles, tag> when R is a multiple
    of 4 and both jobs of the launch take the same mode (mode 0: K fits one
    chunk; mode 1: M does), else k_gemm_stream<row tiles, column tiles, tag,
    8> with 4 column tiles when R is a multiple of 4, 2 when even, else 1.
    The near job of a single-class array (nine blocks side by side, mode 1)
    and the projection (mode 0) share a launch, so that launch stays on
    k_gemm_stream."""
    rn, rr = gemm_rows
    ct = 4 if R % 4 == 0 else 2 if R % 2 == 0 else 1
    lds = R % 4 == 0 and os.environ.get("MLFMA_GEMM") != "stream"
    w0, c0 = (8, 2) if R % 16 == 0 else (8, 1) if R % 8 == 0 else (4, 1)   # mode 0
    w1 = 8 if R % 8 == 0 else 4                                            # mode 1
    near_mode = 0 if multi_class else 1
    gemm = {
        "near+project": f"k_gemm_lds<0, {w0}, {c0}, 0>" if lds and multi_class else f"k_gemm_stream<{rn}, {ct}, 0, 8>",
        "near": (f"k_gemm_lds<0, {w0}, {c0}, 1>" if near_mode == 0 else f"k_gemm_lds<1, {w1}, 1, 1>") if lds
        else f"k_gemm_stream<{rn}, {ct}, 1, 8>",
        "project": f"k_gemm_lds<0, {w0}, {c0}, 2>" if lds else f"k_gemm_stream<{rn}, {ct}, 2, 8>",
        "receive": f"k_gemm_lds<1, {w1}, 1, 3>" if lds else f"k_gemm_stream<{rr}, {ct}, 3, 8>"}
    if stage in gemm:
        return gemm[stage], "mfma"
    for prefix, sym, bound in KERNELS:
        if stage == prefix or (prefix.endswith("_l") and stage.startswith(prefix)):
            return sym, bound
    return stage, "hbm"


def source_digest():
    import hashlib
    with open(ENGINE_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def kernel_table(stages, gemm_rows=(4, 4), R=1, multi_class=True):
    """Group per-stage event timings by the symbol of the kernel each stage
    launched (the unit rocprofv3 reports, template arguments included, as
    the library records it): total time, launches, algorithmic bytes and
    flops.  Stages without a recorded symbol fall back to kernel_of."""
    groups = {}
    for s in stages:
        fsym, bound = kernel_of(s["name"], gemm_rows, R, multi_class)
        sym = s.get("kernel") or fsym
        bound = "mfma" if sym.startswith("k_gemm") else bound
        g = groups.setdefault(sym, {"kernel": sym, "bound": bound, "total_ms": 0.0, "launches": 0,
                                    "bytes": 0.0, "flops": 0.0, "stages": []})
        g["total_ms"] += s["total_ms"]
        g["launches"] += s["launches"]
        g["bytes"] += s["bytes_per_launch"] * s["launches"]
        g["flops"] += s["flops_per_launch"] * s["launches"]
        g["stages"].append(s["name"])
    return groups


def kernel_roofline(g):
    """Achieved rate of one kernel group against the peak that bounds it."""
    secs = g["total_ms"] * 1e-3
    if secs <= 0:
        return None
    if g["bound"] == "mfma":
        a = g["flops"] / secs / 1e12
        return {"bound": "mfma", "achieved": round(a, 2), "unit": "TFLOP/s",
                "frac": round(a * 1e12 / FP32_MFMA_PEAK, 4)}
    a = g["bytes"] / secs / 1e9
    return {"bound": "hbm", "achieved": round(a, 1), "unit": "GB/s", "frac": round(a / HBM_PEAK_GBS, 4)}


def measured_traffic(sym, workload, R):
    """HBM bytes per launch of kernel `sym` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE runs of this workload, or None when they are
    missing or were taken on another version of the kernel source."""
    try:
        with open(traffic_file(workload, R)) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != source_digest():
        return None
    ks = rec.get("kernels", {})
    # counter files name template kernels with their arguments (k_agg_stream<float, 6, 32>)
    k = ks.get(sym) or next((v for n, v in ks.items() if n.startswith(sym + "<float")), None)
    return None if k is None else k["traffic_bytes_per_launch"]


def pmc_digest(fetch_csv, write_csv, copy_mib, out_path, label):
    """Turn two rocprofv3 --pmc counter CSVs (FETCH_SIZE, WRITE_SIZE; KiB per
    dispatch) into HBM bytes per launch per kernel symbol.  Each counter is
    scaled by the ratio of known bytes to its reading on the plain copy
    kernel of the calibration (the runtime's device copy of copy_mib MiB that
    --copy-calibration makes, the largest copy dispatch of the run)."""
    import csv
    from collections import defaultdict

    def read(path, counter):
        per = defaultdict(list)
        with open(path) as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                per[row["Kernel_Name"]].append(float(row["Counter_Value"]))
        return per

    fetch, write = read(fetch_csv, "FETCH_SIZE"), read(write_csv, "WRITE_SIZE")
    copy_bytes = copy_mib * 2 ** 20

    def calib(per):   # the largest dispatch of the runtime's device-to-device copy kernel
        vals = [max(v) for k, v in per.items() if "copyBuffer" in k]
        if not vals:
            raise RuntimeError("no copy kernel in the counter file (run bench.py with --copy-calibration)")
        return max(vals) * 1024.0

    cal_f, cal_w = calib(fetch), calib(write)
    sf, sw = copy_bytes / cal_f, copy_bytes / cal_w
    kernels = {}
    for name in fetch:
        sym = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "").replace("mlfma::", "")
        if not sym.startswith("k_"):
            continue
        fb = sum(fetch[name]) / len(fetch[name]) * 1024.0 * sf
        wb = sum(write.get(name, [0.0])) / max(1, len(write.get(name, []))) * 1024.0 * sw
        kernels[sym] = {"fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                        "traffic_bytes_per_launch": fb + wb, "dispatches": len(fetch[name])}
    rec = {"workload": label, "source_sha256": source_digest(),
           "calibration": {"copy_bytes": copy_bytes, "fetch_KiB": cal_f / 1024, "write_KiB": cal_w / 1024,
                           "fetch_scale": sf, "write_scale": sw},
           "kernels": kernels}
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    print(json.dumps(rec, indent=1))


_T0 = time.perf_counter()


def progress(msg):
    """One line on stderr per finished leg (the JSON result goes to stdout)."""
    print(f"bench [{time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def _limit_blas(n):
    try:
        from threadpoolctl import threadpool_limits
        return threadpool_limits(n)
    except Exception:                    # threadpoolctl missing: no limit
        import contextlib
        return contextlib.nullcontext()


def cpu_baseline_lens(R, Ms):
    """The oracle on a 10 x 10 lens of the full-scale recipe (6,000 unknowns,
    the subarray the oracle can solve), on the host cores, with the one-off
    block assembly and the dense product Z X timed separately:
      - assembly: a bounded sample of distinct pair blocks by direct
        quadrature on all cores (forked workers), and the blocks the whole
        subarray needs, counted;
      - product: the dense 6,000 x 6,000 product with R columns, the oracle's
        own dense() + matmul, with the block cache filled from the sampled
        blocks (the product's cost does not depend on the values), on all
        cores and on one.
    value = unknowns * R / product time (all cores)."""
    import numpy as np

    import workloads as w
    from oracle.pmchwt import DenseProblem, ParticleClass
    cores = len(os.sched_getaffinity(0))
    wl = w.workload("c5", 10, 10)
    used = sorted(set(wl.class_id.tolist()))
    t0 = time.perf_counter()
    pcs = []
    for c in used:   # the static-mode basis both sides are given
        v, t, e = wl.meshes[c]
        pcs.append(ParticleClass(v, t, e, wl.n_perp, wl.n_par, wl.eps_r, M=Ms[c]))
    modes_s = time.perf_counter() - t0
    compact = np.array([used.index(c) for c in wl.class_id])
    prob = DenseProblem(pcs, wl.centers, compact)
    P = wl.n_particles
    keys = {}
    for mu in range(P):
        for nu in range(P):
            keys.setdefault(prob._key(mu, nu), (mu, nu))
    pairs = [v for v in keys.values() if v[0] != v[1]]
    S = min(len(pairs), 2 * cores)
    t0 = time.perf_counter()
    prob.prefetch(pairs[:S], workers=cores)
    asm_s = time.perf_counter() - t0
    sample = [prob.block(*pr) for pr in pairs[:S]]
    for i, k in enumerate(keys):
        if k not in prob._cache:
            prob._cache[k] = sample[i % len(sample)]
    X = w.random_complex((P * pcs[0].n, R), 1)
    t0 = time.perf_counter()
    Z = prob.dense()
    dense_s = time.perf_counter() - t0

    def timed(nrep):
        t0 = time.perf_counter()
        for _ in range(nrep):
            Z @ X
        return (time.perf_counter() - t0) / nrep

    timed(1)
    t_all = timed(5)
    with _limit_blas(1):
        t_one = timed(2)
    n = P * pcs[0].n
    return {"value": n * R / t_all, "unit": "unknowns*RHS/s", "cores": cores, "kind": "oracle",
            "sample": (f"10x10 lens of the full-scale recipe ({n} unknowns, {len(used)} classes), dense product "
                       f"Z X with {R} columns: {t_all * 1e3:.1f} ms on {cores} cores, {t_one * 1e3:.1f} ms on 1; "
                       f"assembly timed apart: {S} distinct pair blocks by direct quadrature in {asm_s:.1f} s on "
                       f"{cores} processes, {len(keys)} distinct blocks needed"),
            "product_s": t_all, "product_1thread_s": t_one, "unknowns": n, "rhs": R,
            "assembly": {"blocks_sampled": S, "wall_s": asm_s, "blocks_needed": len(keys),
                         "extrapolated_wall_s": asm_s / S * len(keys), "class_setup_s": modes_s,
                         "dense_fill_s": dense_s}}


def cpu_baseline_c2(wl, M, R):
    """The oracle on the 40 x 40 array: a bounded sample of distinct pair
    blocks by direct quadrature (all cores) and block products (the dense
    product's work unit, one core and all), extrapolated to the product with
    R columns; assembly reported apart, not charged to the product."""
    from oracle.pmchwt import DenseProblem, ParticleClass
    cores = len(os.sched_getaffinity(0))
    v, t, e = wl.meshes[0]
    pc = ParticleClass(v, t, e, wl.n_perp, wl.n_par, wl.eps_r, M=M)
    prob = DenseProblem([pc], wl.centers, wl.class_id)
    P = wl.n_particles
    S = 2 * cores
    row = 20 * 40 + 20
    pairs = [(row, q) for q in range(P) if q != row][:S]
    t0 = time.perf_counter()
    prob.prefetch(pairs, workers=cores)
    t_block = (time.perf_counter() - t0) / S
    blocks = [prob.block(a, b) for a, b in pairs]
    import workloads as w
    X = w.random_complex((pc.n, R), 3)
    nrep = 400

    def timed():
        t0 = time.perf_counter()
        for i in range(nrep):
            blocks[i % S] @ X
        return (time.perf_counter() - t0) / nrep

    t_all = timed()
    with _limit_blas(1):
        t_one = timed()
    T = P * P * t_all
    return {"value": wl.n_unknowns * R / T, "unit": "unknowns*RHS/s", "cores": cores, "kind": "oracle",
            "sample": (f"{nrep} block products ({pc.n}x{pc.n} by {pc.n}x{R}) of the 40x40 array, "
                       f"{t_all * 1e6:.1f} us each ({t_one * 1e6:.1f} us on 1 core), times {P * P} block "
                       f"products = {T:.2f} s per product; assembly timed apart: {S} distinct pair blocks in "
                       f"{t_block * S:.1f} s on {cores} processes"),
            "product_s": T, "product_1thread_s": P * P * t_one,
            "assembly": {"blocks_sampled": S, "wall_s_per_block": t_block, "blocks_needed": (2 * 40 - 1) ** 2}}


def focal_field(ctx, wl, x, inc, focal, torch, n=200, half=10.0):
    """Field of the lens solution x on an n x n grid in the focal plane
    (z = focal length above the array, +-half wavelengths about the axis),
    by mlfma_fields; the focal spot's peak and its width along x."""
    import numpy as np
    c = wl.centers.mean(0)
    g = np.linspace(-half, half, n)
    X, Y = np.meshgrid(g, g)
    pts = np.stack([c[0] + X.ravel(), c[1] + Y.ravel(), np.full(X.size, c[2] + focal)], -1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E = ctx.fields(x, pts)[0].cpu().numpy()
    dt = time.perf_counter() - t0
    k = 2 * np.pi
    Einc = np.asarray(inc.pol)[None, :] * np.exp(-1j * k * (pts @ np.asarray(inc.khat)))[:, None]
    I_s = np.sum(np.abs(E) ** 2, 1).reshape(n, n)
    I_t = np.sum(np.abs(E + Einc) ** 2, 1).reshape(n, n)
    iy, ix = np.unravel_index(np.argmax(I_t), I_t.shape)
    row = I_t[iy]
    above = np.nonzero(row >= 0.5 * row[ix])[0]
    return {"grid": f"{n}x{n} points, plane z = {focal:g} above the array, +-{half:g} wavelengths about the axis",
            "time_s": dt, "pairs": int(len(pts) * wl.n_particles),
            "peak_total_intensity": float(I_t[iy, ix]), "incident_intensity": 1.0,
            "peak_at_wavelengths": [float(g[ix]), float(g[iy])],
            "fwhm_x_wavelengths": float((above.max() - above.min() + 1) * (g[1] - g[0])),
            "peak_scattered_intensity": float(I_s.max())}


def lens_gmres(torch, w, mlfma):
    """80 x 80 metalens (32 diameter classes, 384,000 unknowns, FP32 product):
    GMRES(300) time to a 1e-4 true residual from zero and from the learned
    initial guess of the committed checkpoint; then 16 incidences batched."""
    import numpy as np

    from paper_2407_21724_amd import learned
    ckpt = os.path.join(ROOT, "paper_2407_21724_amd", "checkpoints", "lens_guess.npz")
    wl = w.workload("c4")
    t0 = time.perf_counter()
    ctx = mlfma.Context(wl.centers, wl.class_id, len(wl.meshes), mlfma.default_params(precision=mlfma.C64))
    for c in sorted(set(wl.class_id.tolist())):
        v, t, e = wl.meshes[c]
        M, _ = mlfma.static_modes(v, t, e, wl.n_perp, wl.n_par)
        ctx.set_static_modes(c, v, t, e, wl.n_perp, wl.n_par, M, wl.eps_r)
    ctx.prepare()
    setup_s = time.perf_counter() - t0
    from paper_2407_21724_amd import autotune
    tfile = autotune.tuning_file("c4", 1)
    if os.path.exists(tfile):
        autotune.apply(tfile, ctx)
    inc = wl.incidences[0]
    b = ctx.plane_wave_rhs(inc.khat[None], inc.pol[None])
    res = {"workload": "80x80 metalens, 32 classes, 384000 unknowns, normal incidence, FP32 product",
           "restart": 300, "setup_s": setup_s,
           "tuning": os.path.relpath(tfile, ROOT) if os.path.exists(tfile) else "default tile shapes"}
    # a short solve first allocates the Krylov basis and loads the kernels,
    # so that neither timed solve pays for them
    ctx.gmres_solve(b, rtol=1e-4, max_iter=20, restart=300)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st, _ = ctx.gmres_solve(b, rtol=1e-4, max_iter=4000, restart=300)
    torch.cuda.synchronize()
    progress("80x80 lens: gmres from zero done")
    res["plain"] = {"time_to_1e-4_s": time.perf_counter() - t0, "iterations": st[0]["iterations"],
                    "true_rel_res": st[0]["true_rel_res"], "converged": st[0]["converged"]}
    if os.path.exists(ckpt):
        net, dia, scale, meta = learned.load(ckpt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x0 = ctx.learned_guess(net, dia, scale, inc.khat[None])
        _, st, _ = ctx.gmres_solve(b, x=x0, rtol=1e-4, max_iter=4000, restart=300, use_x0=True)
        torch.cuda.synchronize()
        res["learned"] = {"time_to_1e-4_s": time.perf_counter() - t0, "iterations": st[0]["iterations"],
                          "true_rel_res": st[0]["true_rel_res"], "converged": st[0]["converged"],
                          "includes": "feature build + network inference + GMRES",
                          "checkpoint": {k: meta[k] for k in ("patches", "patch_side", "samples")}}
    # 16 incidences in one batched GMRES (one product launch per iteration for
    # all of them), from zero and from the learned guess, against the plain
    # single-RHS solve above
    incs = w.tilted_incidences(16, 20.0)
    kh = np.array([i.khat for i in incs])
    bb = ctx.plane_wave_rhs(kh, np.array([i.pol for i in incs]))
    for name, guess in (("batched_16", False), ("batched_16_learned", True)):
        if guess and not os.path.exists(ckpt):
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if guess:
            x0 = ctx.learned_guess(net, dia, scale, kh)
            xb, st, _ = ctx.gmres_solve(bb, x=x0, rtol=1e-4, max_iter=4000, restart=300, use_x0=True)
        else:
            xb, st, _ = ctx.gmres_solve(bb, rtol=1e-4, max_iter=4000, restart=300)
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        its = [s["iterations"] for s in st]
        progress(f"80x80 lens: {name} done in {T:.1f} s")
        res[name] = {"rhs": 16, "incidences": "x-polarised, polar angle 0..20 deg in the xz plane",
                     "time_to_1e-4_s": T, "per_rhs_s": T / 16, "iterations_min": min(its),
                     "iterations_max": max(its), "true_rel_res_max": max(s["true_rel_res"] for s in st),
                     "converged": all(s["converged"] for s in st),
                     "per_rhs_speedup_vs_plain_single": res["plain"]["time_to_1e-4_s"] / (T / 16)}
        del xb
    ctx.close()
    return res


WORKLOADS = {
    "c2": "40x40 dielectric cylinders D0.3 H0.6 eps6.25 pitch0.5, 600-tri mesh, 15+15 static modes, "
          "96000 unknowns, FP32 matvec",
    "c4": "80x80 metalens of cylinders (H0.6, eps6.25, pitch0.5, 32 diameter classes on the focusing profile "
          "of focal length 20), 384000 unknowns, FP32 matvec",
    "c5": "200x200 metalens of cylinders (H0.6, eps6.25, pitch0.5, 32 diameter classes on the focusing profile "
          "of focal length 50, 600-tri meshes, 15+15 static modes), 2400000 unknowns, 7 translation levels, "
          "FP32 matvec",
}
DEFAULT_RHS = {"c2": 1, "c4": 1, "c5": 16}


def traffic_file(workload, R):
    return os.path.join(ROOT, "profiles", f"pmc_traffic_{workload}_r{R}.json")


def gmres_pair(ctx, wl, torch, restart, max_iter, learned_ok=True, fp32_basis=False):
    """One normal-incidence solve from zero and one from the learned initial
    guess of the committed checkpoint (its time includes the feature build
    and the network), each after a 20-iteration warm-up solve that allocates
    the Krylov basis and loads the kernels."""
    import numpy as np

    from paper_2407_21724_amd import learned
    ckpt = os.path.join(ROOT, "paper_2407_21724_amd", "checkpoints", "lens_guess.npz")
    inc = wl.incidences[0]
    b = ctx.plane_wave_rhs(np.asarray(inc.khat)[None], np.asarray(inc.pol)[None])
    ctx.gmres_solve(b, rtol=1e-4, max_iter=20, restart=restart, fp32_basis=fp32_basis)
    torch.cuda.synchronize()
    out = {"restart": restart, "rhs": 1, "krylov_basis": "fp32" if fp32_basis else "fp64",
           "incidence": "normal, x-polarised"}
    t0 = time.perf_counter()
    xs, st, _ = ctx.gmres_solve(b, rtol=1e-4, max_iter=max_iter, restart=restart, fp32_basis=fp32_basis)
    torch.cuda.synchronize()
    out["plain"] = {"time_to_1e-4_s": time.perf_counter() - t0, "iterations": st[0]["iterations"],
                    "true_rel_res": st[0]["true_rel_res"], "converged": st[0]["converged"],
                    "cycles": st[0]["cycles"]}
    progress(f"gmres from zero: {out['plain']['iterations']} iterations, {out['plain']['time_to_1e-4_s']:.1f} s")
    if learned_ok and os.path.exists(ckpt):
        net, dia, scale, meta = learned.load(ckpt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x0 = ctx.learned_guess(net, dia, scale, np.asarray(inc.khat)[None])
        _, st, _ = ctx.gmres_solve(b, x=x0, rtol=1e-4, max_iter=max_iter, restart=restart, use_x0=True,
                                   fp32_basis=fp32_basis)
        torch.cuda.synchronize()
        out["learned"] = {"time_to_1e-4_s": time.perf_counter() - t0, "iterations": st[0]["iterations"],
                          "true_rel_res": st[0]["true_rel_res"], "converged": st[0]["converged"],
                          "includes": "feature build + network inference + GMRES"}
        out["learned_speedup"] = out["plain"]["time_to_1e-4_s"] / out["learned"]["time_to_1e-4_s"]
    return out, xs


def c3_batched(torch, w, mlfma, ctx=None):
    """The 40 x 40 array with the 64 incidences of the batched configuration
    as one 64-column product (FP32)."""
    wl = w.workload("c2")
    if ctx is None:
        v, t, e = wl.meshes[0]
        M, _ = mlfma.static_modes(v, t, e, wl.n_perp, wl.n_par)
        ctx = mlfma.Context(wl.centers, wl.class_id, 1, mlfma.default_params(precision=mlfma.C64))
        ctx.set_static_modes(0, v, t, e, wl.n_perp, wl.n_par, M, wl.eps_r)
        ctx.prepare()
    P, n = wl.n_particles, 2 * (wl.n_perp + wl.n_par)
    xb = torch.as_tensor(w.random_complex((64, P, n), 2)).to("cuda", torch.complex64).contiguous()
    yb = torch.empty_like(xb)
    for _ in range(2):
        ctx.matvec(xb, out=yb)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        ctx.matvec(xb, out=yb)
    e1.record()
    torch.cuda.synchronize()
    msb = e0.elapsed_time(e1) / 10
    return {"workload": WORKLOADS["c2"], "rhs": 64, "ms_per_product": msb,
            "unknowns_rhs_per_s": wl.n_unknowns * 64 / (msb * 1e-3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rhs", type=int, default=0, help="right-hand sides per product (default 16 for c5, else 1)")
    ap.add_argument("--workload", choices=("c2", "c4", "c5"), default="c5",
                    help="c5: the 200x200 metalens (the headline); c2: 40x40 cylinders; c4: 80x80 metalens")
    ap.add_argument("--restart", type=int, default=0, help="GMRES restart (default 100 for c2, 300 otherwise)")
    ap.add_argument("--max-iter", type=int, default=None,
                    help="GMRES iteration cap (default 4000; 10000 for the 200 x 200 lens)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gmres", action="store_true")
    ap.add_argument("--no-tuning", action="store_true", help="ignore the tuning file: default tile shapes")
    ap.add_argument("--autotune", action="store_true",
                    help="run the autotuner and write the tuning file that later runs apply")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-RHS product of the 40x40 array")
    ap.add_argument("--no-lens", action="store_true",
                    help="skip the 80 x 80 metalens batched GMRES (16 incidences, zero and learned starts)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--pmc-digest", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="digest two rocprofv3 counter CSVs into the traffic record of --workload/--rhs and exit")
    args = ap.parse_args()
    R = args.rhs or DEFAULT_RHS[args.workload]
    if args.pmc_digest:
        pmc_digest(args.pmc_digest[0], args.pmc_digest[1], args.copy_calibration or 256,
                   traffic_file(args.workload, R), f"{WORKLOADS[args.workload]}, R = {R}")
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the product is computed on a single MI355X; "
              "multi-GPU sharding is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as w
    from paper_2407_21724_amd import mlfma

    wl = w.workload(args.workload)
    used = sorted(set(wl.class_id.tolist()))
    t0 = time.perf_counter()
    Ms = {}
    for c in used:                                                # host-only calls
        v, t, e = wl.meshes[c]
        Ms[c], _ = mlfma.static_modes(v, t, e, wl.n_perp, wl.n_par)
    modes_s = time.perf_counter() - t0
    # the oracle leg runs first, before this process touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_lens(R, Ms) if args.workload in ("c4", "c5") else cpu_baseline_c2(wl, Ms[0], R)
        progress(f"oracle baseline: {cpu['value']:.3e} {cpu['unit']}")

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration * 2 ** 18, device="cuda", dtype=torch.float32)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t0 = time.perf_counter()
    ctx = mlfma.Context(wl.centers, wl.class_id, len(wl.meshes), mlfma.default_params(precision=mlfma.C64))
    for c in used:
        v, t, e = wl.meshes[c]
        ctx.set_static_modes(c, v, t, e, wl.n_perp, wl.n_par, Ms[c], wl.eps_r)
    ctx.prepare()
    setup_s = time.perf_counter() - t0 + modes_s
    info = ctx.info()
    progress(f"setup of {args.workload}: {setup_s:.1f} s")
    from paper_2407_21724_amd import autotune
    tfile = autotune.tuning_file(args.workload, R)
    tuning = {"source": "default tile shapes"}
    if args.autotune:
        t0 = time.perf_counter()
        rep = autotune.autotune(ctx, R=R, reps=5)
        autotune.save(tfile, ctx, rep, {"workload": args.workload, "rhs": R})
        tuning = {"source": "autotuned now (written to the tuning file)", "seconds": time.perf_counter() - t0}
    elif not args.no_tuning and os.path.exists(tfile):
        autotune.apply(tfile, ctx)
        tuning = {"source": os.path.relpath(tfile, ROOT)}
    agg, dis = ctx.get_tuning()
    tuning.update({"agg_rows": agg, "dis_rows": dis, "gemm_row_tiles": list(ctx.get_gemm_tiles())})
    P, n = wl.n_particles, 2 * (wl.n_perp + wl.n_par)
    x = torch.as_tensor(w.random_complex((R, P, n), 1)).to("cuda", torch.complex64).contiguous()
    y = torch.empty_like(x)
    stream = torch.cuda.Stream()          # default priority
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            ctx.matvec(x, out=y)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(args.steps):
            ctx.matvec(x, out=y)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        # second pass over the same steps, launched directly (not from the
        # cached graph) with per-kernel HIP events recorded on the stream
        ctx.profile(True)
        for _ in range(args.steps):
            ctx.matvec(x, out=y)
        torch.cuda.synchronize()
        stages = ctx.profile_read()
        ctx.profile(False)
    value = wl.n_unknowns * R / (ms * 1e-3)
    del x, y
    progress(f"product: {ms:.3f} ms for {R} RHS, {value:.3e} unknowns*RHS/s")

    # roofline of the dominant kernel (largest share of the product's time)
    gemm_rows = ctx.get_gemm_tiles()
    groups = kernel_table(stages, gemm_rows, R, len(set(wl.class_id.tolist())) > 1)
    dom = max(groups.values(), key=lambda g: g["total_ms"])
    avg_s = dom["total_ms"] / dom["launches"] * 1e-3
    if dom["bound"] == "hbm":
        achieved = dom["bytes"] / dom["launches"] / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS}
    else:
        achieved = dom["flops"] / dom["launches"] / avg_s / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": FP32_MFMA_PEAK / 1e12, "unit": "TFLOP/s",
                "frac": achieved * 1e12 / FP32_MFMA_PEAK}
    roof["traffic"] = measured_traffic(dom["kernel"], args.workload, R)
    roof["kernel"] = dom["kernel"]
    roof["stages"] = dom["stages"]
    roof["avg_launch_us"] = avg_s * 1e6
    roof["algorithmic_bytes_per_launch"] = dom["bytes"] / dom["launches"]
    roof["algorithmic_flops_per_launch"] = dom["flops"] / dom["launches"]

    out = {
        "metric": "MLFMA-SMR matvec throughput (unknowns*RHS/s); GMRES time-to-1e-4, learned vs plain, beside it",
        "value": value, "unit": "unknowns*RHS/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "rhs": R, "levels": info["n_levels"], "L": info["L"],
                   "K": info["K"]},
        "roofline": roof,
        "hbm_roofline_product_ms": None,
        "stages_us": {s_["name"]: round(1e3 * s_["total_ms"] / s_["launches"], 2) for s_ in stages},
        "kernels_us": {g["kernel"]: round(1e3 * g["total_ms"] / g["launches"], 2) for g in groups.values()},
        # every kernel against its own roofline (algorithmic bytes or flops over its event time)
        "kernel_rooflines": {g["kernel"]: kernel_roofline(g) for g in groups.values()},
        "setup_s": setup_s,
        "tuning": tuning,
    }
    # whole-product algorithmic bytes at 8 TB/s (the product's own roofline)
    tot_bytes = sum(g["bytes"] for g in groups.values()) / args.steps
    out["hbm_roofline_product_ms"] = tot_bytes / (HBM_PEAK_GBS * 1e9) * 1e3
    if not args.no_gmres:
        restart = args.restart or (100 if args.workload == "c2" else 300)
        max_iter = args.max_iter or (10000 if args.workload == "c5" else 4000)
        out["gmres"], xs = gmres_pair(ctx, wl, torch, restart, max_iter, learned_ok=args.workload != "c2")
        progress("gmres: " + json.dumps({k: v for k, v in out["gmres"].items() if k in ("plain", "learned")}))
        if args.workload in ("c4", "c5"):   # field of the zero-start solution in the focal plane
            out["focal_field"] = focal_field(ctx, wl, xs[:1].contiguous(), wl.incidences[0],
                                             20.0 if args.workload == "c4" else 50.0, torch)
        del xs
    if not args.no_batched:
        out["batched_64_rhs"] = c3_batched(torch, w, mlfma, ctx if args.workload == "c2" else None)
        progress(f"64-RHS product of the 40x40 array: {out['batched_64_rhs']['ms_per_product']:.3f} ms")
    ctx.close()
    if not args.no_gmres and not args.no_lens:
        out["gmres_lens_80x80"] = lens_gmres(torch, w, mlfma)
        progress("80x80 lens gmres done")
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
