"""GPU assembly of the blocks between neighbouring particles (FP64 MFMA
quadrature) against the library's host quadrature of the same Galerkin
entries (which the CPU tests pin to the oracle's pair blocks)."""
import time

import numpy as np
import pytest

import workloads as w
from gpu_helpers import note

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2407_21724_amd import mlfma  # noqa: E402


def _ctx_with_classes(wl, classes):
    ctx = mlfma.Context(wl.centers, wl.class_id, len(wl.meshes), mlfma.default_params())
    for c in classes:
        v, t, e = wl.meshes[c]
        M, _ = mlfma.static_modes(v, t, e, wl.n_perp, wl.n_par)
        ctx.set_static_modes(c, v, t, e, wl.n_perp, wl.n_par, M, wl.eps_r)
    return ctx


@pytest.mark.parametrize("case", ["same_class", "two_classes"])
def test_device_pair_blocks_match_host(case):
    if case == "same_class":
        wl = w.workload("c2", 3, 3)
        pairs = [(0, 0, 1, 0), (0, 0, 1, 1), (0, 0, 0, -1), (0, 0, -1, 1)]
        classes = [0]
    else:
        wl = w.workload("c4", 6, 6)
        used = sorted(set(wl.class_id.tolist()))
        a, b = used[0], used[-1]
        pairs = [(a, b, 1, 0), (b, a, -1, 0), (a, a, 0, 1), (b, a, 1, -1)]
        classes = [a, b]
    ctx = _ctx_with_classes(wl, classes)
    for cp, cq, dx, dy in pairs:
        t0 = time.perf_counter()
        Zd = ctx.debug_pair_block_device(cp, cq, dx, dy)
        td = time.perf_counter() - t0
        Zh = ctx.debug_near_block(cp, cq, dx, dy)
        err = np.abs(Zd - Zh).max() / np.abs(Zh).max()
        note(f"pair ({cp},{cq},{dx},{dy}): device vs host max rel {err:.2e} ({td * 1e3:.1f} ms)")
        assert err < 1e-11
