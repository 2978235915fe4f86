"""Learned initial guess for GMRES (network kernels in libmlfma).

A fully connected ReLU network (C + 11 -> 256 -> 256 -> 256 -> 4N) maps a
particle's class (one-hot: each class has its own static-mode basis), its
eight neighbours' diameters (0 where a site is empty), the incidence
direction (khat_x, khat_y) and its distance to the array edge (capped at 6
sites) to its static-mode coefficients with the incident
phase exp(-j k khat . r_p) removed (mlfma_guess_features /
mlfma_learned_guess).  It is trained on solutions the method itself
produces: nx x nx patches of the particle classes, each solved by GPU GMRES,
for plane waves in the xz plane (polar angle up to theta_max, E along
theta-hat, i.e. x-polarised at normal incidence).  A quarter of the patches
draw every site's class at random; the rest vary slowly around a random
base class (a random gradient plus +-1 class of noise), like a lens.  The
training runs on the GPU through the library's own forward, backward and
Adam kernels; this module only moves arrays.
"""
from __future__ import annotations

import json
import math
import time

import numpy as np

from . import mlfma

HIDDEN = (256, 256, 256)


def sizes(n_classes: int, n_unknowns: int):
    """Layer sizes for C classes and 2N unknowns per particle."""
    return (n_classes + 11,) + HIDDEN + (2 * n_unknowns,)


def patch_classes(rng, nx, n_classes):
    """Class map of one training patch (see the module docstring)."""
    if rng.random() < 0.25:
        return rng.integers(0, n_classes, nx * nx)
    base = rng.integers(0, n_classes)
    gx, gy = rng.uniform(-1.0, 1.0, 2) * (6.0 / nx)
    iy, ix = np.meshgrid(np.arange(nx), np.arange(nx), indexing="ij")
    c = base + gx * (ix - nx / 2) + gy * (iy - nx / 2) + rng.uniform(-1, 1, (nx, nx))
    return np.clip(np.rint(c), 0, n_classes - 1).astype(np.int64).ravel()


def incidence(theta: float):
    """Plane wave in the xz plane at polar angle theta, E along theta-hat."""
    st, ct = math.sin(theta), math.cos(theta)
    return np.array([st, 0.0, ct]), np.array([ct, 0.0, -st], complex)


def _lattice(nx, ny, pitch=0.5):
    iy, ix = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([ix.ravel() * pitch, iy.ravel() * pitch, np.zeros(nx * ny)], -1)


def targets(x, centers, khat):
    """x [P][2N] complex -> [P][4N] float: (re, im) of x_p exp(+j k khat . r_p)."""
    t = x * np.exp(1j * 2 * np.pi * (centers @ khat))[:, None]
    return np.stack([t.real, t.imag], -1).reshape(len(x), -1).astype(np.float32)


def solve_patches(lib_ctx, class_param, scale, n_classes, n_patches, seed=0, nx=6, theta_max_deg=20.0,
                  rtol=1e-4, params=None, log=None):
    """Solve n_patches random nx x nx patches (classes uniform over
    0..n_classes-1, all set in lib_ctx) and return features X [S][11],
    targets T [S][4N] and the patch index of every sample."""
    rng = np.random.default_rng(seed)
    centers = _lattice(nx, nx)
    Xs, Ts, pid = [], [], []
    t0 = time.perf_counter()
    iters = []
    for i in range(n_patches):
        cls = patch_classes(rng, nx, n_classes).astype(np.int32)
        theta = math.radians(theta_max_deg) * rng.random()
        khat, pol = incidence(theta)
        ctx = mlfma.Context(centers, cls, n_classes, params or mlfma.default_params())
        ctx.share_setup(lib_ctx)
        ctx.prepare()
        b = ctx.plane_wave_rhs(khat[None], pol[None])
        x, st, rc = ctx.gmres_solve(b, rtol=rtol, max_iter=3000, restart=300)
        if rc != mlfma.OK and not st[0]["true_rel_res"] < 10 * rtol:
            if log:
                log(f"patch {i} skipped: {st[0]}")
            ctx.close()
            continue
        iters.append(st[0]["iterations"])
        Xs.append(ctx.guess_features(class_param, scale, khat)[0])
        Ts.append(targets(x.cpu().numpy()[0].astype(complex), centers, khat))
        pid.append(np.full(nx * nx, i, np.int32))
        ctx.close()
        if log and (i + 1) % max(1, n_patches // 10) == 0:
            log(f"patches {i + 1}/{n_patches}: {time.perf_counter() - t0:.1f} s, mean GMRES iterations "
                f"{np.mean(iters):.1f}")
    return np.concatenate(Xs), np.concatenate(Ts), np.concatenate(pid)


def train(net: "mlfma.Mlp", X, T, epochs=200, batch=256, lr=1e-3, seed=0, val_frac=0.1, log=None):
    """Adam on 0.5 * mean |net(X) - T / s|^2 with s the targets' RMS, then s
    folded into the last layer so that the network predicts T itself.
    Returns a history dict (train / validation loss, relative errors)."""
    import torch
    rng = np.random.default_rng(seed)
    S = len(X)
    perm = rng.permutation(S)
    nval = int(val_frac * S)
    val, tr = perm[:nval], perm[nval:]
    s = float(np.sqrt(np.mean(T[tr] ** 2)))
    Xd = torch.as_tensor(X, device="cuda")
    Td = torch.as_tensor(T / s, device="cuda")
    hist = {"epoch": [], "train_loss": [], "val_rel_err": [], "scale": s}
    steps = 0
    for ep in range(epochs):
        order = torch.as_tensor(rng.permutation(tr), device="cuda")
        lr_ep = lr * 0.5 * (1 + math.cos(math.pi * ep / epochs))       # cosine schedule
        tot = 0.0
        nb = 0
        for b0 in range(0, len(order), batch):
            idx = order[b0:b0 + batch]
            tot += net.train_step(Xd[idx].contiguous(), Td[idx].contiguous(), lr_ep)
            nb += 1
            steps += 1
        if ep % max(1, epochs // 10) == 0 or ep == epochs - 1:
            vi = torch.as_tensor(val, device="cuda")
            pred = net.forward(Xd[vi].contiguous()).cpu().numpy()
            ref = T[val] / s
            rel = float(np.linalg.norm(pred - ref) / np.linalg.norm(ref))
            hist["epoch"].append(ep)
            hist["train_loss"].append(tot / nb)
            hist["val_rel_err"].append(rel)
            if log:
                log(f"epoch {ep}: train loss {tot / nb:.4e}, validation relative error {rel:.3f}")
    hist["steps"] = steps
    # fold the target scale into the last layer
    p = net.get_params()
    (W, b) = net.layers(p)[-1]
    W *= s
    b *= s
    net.set_params(p)
    return hist


def save(path, net: "mlfma.Mlp", class_param, scale, meta: dict):
    np.savez_compressed(path, sizes=np.array(net.sizes, np.int32), params=net.get_params(),
                        class_param=np.asarray(class_param, np.float64), scale=float(scale),
                        meta=json.dumps(meta))


def load(path):
    """-> (net, class_param, scale, meta)"""
    d = np.load(path, allow_pickle=False)
    net = mlfma.Mlp([int(v) for v in d["sizes"]])
    net.set_params(d["params"])
    return net, d["class_param"], float(d["scale"]), json.loads(str(d["meta"]))
