"""Write the oracle's expected values used by the GPU parity tests.

Calls only ``oracle`` and the shared seeded input generators in
``workloads``; nothing here touches the library.

    python tests/golden/make_golden.py [c2_6x6 c2_12x12 c2_40x40_rows ...]

Each file holds the oracle's static modes M of the cylinder class (the basis
both sides are given), the workload description and the dense products
y = Z x for the seeded x = workloads.random_complex((P, 2N), seed=1):
  c2_6x6.npz        all 36 particles (two translation levels)
  c2_12x12.npz      all 144 particles (three translation levels)
  c2_40x40_rows.npz rows of 4 interior particles of the full 40 x 40
                    array (the bench workload; all six levels contribute)
  c4_8x8.npz        all 64 particles of an 8 x 8 metalens of the c4 recipe
                    (several diameter classes; M holds each used class's
                    modes, `classes` their class ids)
  c5_10x10_fields.npz  a 10 x 10 lens of the c5 recipe solved densely for the
                    normal-incidence x-polarised wave: the solution, the
                    scattered near field on the plane z = 1 over the array
                    (21 x 21 points) and the far-field amplitude on a
                    16 x 32 sphere grid
  c5_sparse.npz     all 18 particles of the sparse full-extent lens
                    (workloads c5_sparse: pairs at every level of the
                    200 x 200 tree), full product and near part
  c3_40x40_rows.npz rows of the 4 interior particles of the 40 x 40 array
                    for 64 seeded right-hand sides (seed 2)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as w  # noqa: E402
from oracle.pmchwt import DenseProblem, ParticleClass  # noqa: E402

SEED = 1


def _cylinder_class(wl):
    v, t, e = wl.meshes[0]
    return ParticleClass(v, t, e, wl.n_perp, wl.n_par, wl.eps_r)


def make_lens(name: str):
    t0 = time.time()
    nx = int(name.split("_")[1].split("x")[0])
    wl = w.workload("c4", nx, nx)
    used = sorted(set(wl.class_id.tolist()))
    pcs = []
    for c in used:
        v, t, e = wl.meshes[c]
        pcs.append(ParticleClass(v, t, e, wl.n_perp, wl.n_par, wl.eps_r))
    compact = np.array([used.index(c) for c in wl.class_id], np.int32)
    prob = DenseProblem(pcs, wl.centers, compact)
    P, n = wl.n_particles, pcs[0].n
    x = w.random_complex((P, n), SEED)
    rows = np.arange(P)
    prob.prefetch([(mu, nu) for mu in rows for nu in range(P)])
    y = prob.matvec_rows(x, rows)
    out = os.path.join(HERE, name + ".npz")
    np.savez_compressed(out, M=np.stack([pc.M for pc in pcs]), classes=np.array(used, np.int32), rows=rows, y=y,
                        seed=SEED, eps_r=wl.eps_r, n_perp=wl.n_perp, n_par=wl.n_par, nx=nx, ny=nx)
    print(f"{name}: {P} rows, classes {used} in {time.time() - t0:.1f} s -> {out}", flush=True)


def make_lens_fields(name: str):
    from oracle.fields import far_amplitude, near_field, sphere_grid
    from oracle.pmchwt import solve_dense
    t0 = time.time()
    wl = w.workload("c5", 10, 10)
    used = sorted(set(wl.class_id.tolist()))
    pcs = []
    for c in used:
        v, t, e = wl.meshes[c]
        pcs.append(ParticleClass(v, t, e, wl.n_perp, wl.n_par, wl.eps_r))
    compact = np.array([used.index(c) for c in wl.class_id], np.int32)
    prob = DenseProblem(pcs, wl.centers, compact)
    P = wl.n_particles
    prob.prefetch([(mu, nu) for mu in range(P) for nu in range(P)])
    inc = wl.incidences[0]
    V = prob.rhs(inc.khat, inc.pol)
    J = solve_dense(prob, V)
    g = np.linspace(-0.5, 5.0, 21)
    X, Y = np.meshgrid(g, g)
    pts = np.stack([X.ravel(), Y.ravel(), np.full(X.size, 1.0)], -1)
    near = near_field(prob, J, pts)
    rhat, _ = sphere_grid(16, 32)
    far = far_amplitude(prob, J, rhat)
    out = os.path.join(HERE, name + ".npz")
    np.savez_compressed(out, M=np.stack([pc.M for pc in pcs]), classes=np.array(used, np.int32), J=J, V=V,
                        pts=pts, near=near, rhat=rhat, far=far, khat=inc.khat, pol=inc.pol, eps_r=wl.eps_r,
                        n_perp=wl.n_perp, n_par=wl.n_par, nx=10, ny=10)
    print(f"{name}: classes {used}, solved and fields in {time.time() - t0:.1f} s -> {out}", flush=True)


def make_sparse(name: str):
    """All rows of the sparse full-extent lens (18 particles, 13 classes):
    the full product and its near part (self + adjacent sites)."""
    t0 = time.time()
    wl = w.workload("c5_sparse")
    used = sorted(set(wl.class_id.tolist()))
    pcs = []
    for c in used:
        v, t, e = wl.meshes[c]
        pcs.append(ParticleClass(v, t, e, wl.n_perp, wl.n_par, wl.eps_r))
    compact = np.array([used.index(c) for c in wl.class_id], np.int32)
    prob = DenseProblem(pcs, wl.centers, compact)
    P, n = wl.n_particles, pcs[0].n
    x = w.random_complex((P, n), SEED)
    rows = np.arange(P)
    prob.prefetch([(mu, nu) for mu in rows for nu in range(P)])
    y = prob.matvec_rows(x, rows)
    site = np.round(wl.centers[:, :2] / 0.5).astype(int)
    ynear = np.array([sum(prob.block(mu, nu) @ x[nu] for nu in range(P)
                          if np.abs(site[nu] - site[mu]).max() <= 1) for mu in rows])
    out = os.path.join(HERE, name + ".npz")
    np.savez_compressed(out, M=np.stack([pc.M for pc in pcs]), classes=np.array(used, np.int32), rows=rows, y=y,
                        ynear=ynear, seed=SEED, eps_r=wl.eps_r, n_perp=wl.n_perp, n_par=wl.n_par)
    print(f"{name}: {P} rows, classes {used} in {time.time() - t0:.1f} s -> {out}", flush=True)


def make_batched_rows(name: str):
    """Rows of 4 interior particles of the 40 x 40 array for 64 seeded
    right-hand sides (x = random_complex((64, P, 2N), seed=2)): y [4][2N][64]."""
    t0 = time.time()
    wl = w.workload("c2")
    rows = np.array([19 * 40 + 19, 19 * 40 + 20, 20 * 40 + 19, 20 * 40 + 20])
    pc = _cylinder_class(wl)
    prob = DenseProblem([pc], wl.centers, wl.class_id)
    P, n = wl.n_particles, pc.n
    X = w.random_complex((64, P, n), 2)
    prob.prefetch([(mu, nu) for mu in rows for nu in range(P)])
    y = prob.matvec_rows(np.transpose(X, (1, 2, 0)), rows)
    out = os.path.join(HERE, name + ".npz")
    np.savez_compressed(out, M=pc.M, rows=rows, y=y, seed=2, rhs=64, eps_r=wl.eps_r, n_perp=wl.n_perp,
                        n_par=wl.n_par, nx=40, ny=40)
    print(f"{name}: {len(rows)} rows x 64 RHS in {time.time() - t0:.1f} s -> {out}", flush=True)


def make(name: str):
    if name == "c5_10x10_fields":
        return make_lens_fields(name)
    if name == "c5_sparse":
        return make_sparse(name)
    if name == "c3_40x40_rows":
        return make_batched_rows(name)
    if name.startswith("c4_"):
        return make_lens(name)
    t0 = time.time()
    if name in ("c2_6x6", "c2_12x12"):
        nx = 6 if name == "c2_6x6" else 12
        wl = w.workload("c2", nx, nx)
        rows = np.arange(wl.n_particles)
    elif name == "c2_40x40_rows":
        wl = w.workload("c2")
        rows = np.array([19 * 40 + 19, 19 * 40 + 20, 20 * 40 + 19, 20 * 40 + 20])
    else:
        raise ValueError(name)
    pc = _cylinder_class(wl)
    prob = DenseProblem([pc], wl.centers, wl.class_id)
    P, n = wl.n_particles, pc.n
    x = w.random_complex((P, n), SEED)
    prob.prefetch([(mu, nu) for mu in rows for nu in range(P)])
    y = prob.matvec_rows(x, rows)
    # near-field part (self + 8 neighbours) for the same rows
    ix, iy = np.round(wl.centers[:, 0] / 0.5).astype(int), np.round(wl.centers[:, 1] / 0.5).astype(int)
    ynear = []
    for mu in rows:
        acc = np.zeros(n, complex)
        for nu in range(P):
            if abs(ix[nu] - ix[mu]) <= 1 and abs(iy[nu] - iy[mu]) <= 1:
                acc += prob.block(mu, nu) @ x[nu]
        ynear.append(acc)
    out = os.path.join(HERE, name + ".npz")
    np.savez_compressed(out, M=pc.M, rows=rows, y=y, ynear=np.array(ynear), seed=SEED,
                        eps_r=wl.eps_r, n_perp=wl.n_perp, n_par=wl.n_par, nx=int(ix.max() + 1),
                        ny=int(iy.max() + 1))
    print(f"{name}: {len(rows)} rows in {time.time() - t0:.1f} s -> {out}", flush=True)


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["c2_6x6", "c2_12x12", "c2_40x40_rows"]:
        make(nm)
