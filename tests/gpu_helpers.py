"""Shared set-up for the GPU parity tests: builds library contexts and oracle
problems on the same seeded workloads (the basis M comes from the oracle and
is passed to both sides, as mlfma_set_static_modes takes it as input)."""
from __future__ import annotations

import sys

import numpy as np

import workloads as w


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def make_ctx(wl, M, precision, **params):
    """M: one basis for every class, a list per class, or a dict {class: M}
    for the classes in use (the others stay unset)."""
    from paper_2407_21724_amd import mlfma
    tp = mlfma.default_params(precision=precision, **params)
    ctx = mlfma.Context(wl.centers, wl.class_id, len(wl.meshes), tp)
    for c, (v, t, e) in enumerate(wl.meshes):
        if isinstance(M, dict):
            if c not in M:
                continue
            Mc = M[c]
        else:
            Mc = M[c] if isinstance(M, list) else M
        ctx.set_static_modes(c, v, t, e, wl.n_perp, wl.n_par, Mc, wl.eps_r)
    return ctx


def to_dev(x, ctx):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=ctx.dtype).contiguous()


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()
