"""The autotuner changes only how the kernels divide the work (row chunks
of the streamed interpolation, row tiles of the GEMMs): the tuned product
is bitwise identical to the default one, and invalid shapes are
rejected."""
import numpy as np
import pytest

import workloads as w
from gpu_helpers import make_ctx, note

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2407_21724_amd import autotune, mlfma  # noqa: E402


def test_tuned_product_is_bitwise_identical():
    wl = w.workload("c2", 16, 16)
    v, t, e = wl.meshes[0]
    M, _ = mlfma.static_modes(v, t, e, wl.n_perp, wl.n_par)
    ctx = make_ctx(wl, M, mlfma.C64)
    x = torch.as_tensor(w.random_complex((2, wl.n_particles, 60), 3)).to("cuda", torch.complex64).contiguous()
    y0 = ctx.matvec(x).cpu().numpy()
    rep = autotune.autotune(ctx, R=2, reps=2, candidates=(0, 4, 8, 32, 100000))
    note(f"tuned {rep['tuned']} from {rep['default']}")
    y1 = ctx.matvec(x).cpu().numpy()
    assert np.array_equal(y0, y1)
    agg, dis = ctx.get_tuning()
    with pytest.raises(mlfma.MlfmaError):
        ctx.set_tuning([-1 for a in agg], dis)             # a chunk needs at least one row
    with pytest.raises(mlfma.MlfmaError):
        ctx.set_tuning(agg, dis, (3, 4))                    # row tiles must be 1, 2 or 4
    ctx.set_tuning([0] * len(agg), [0] * len(dis), (0, 0))
    assert ctx.get_tuning() == rep["default"] and ctx.get_gemm_tiles() == (4, 4)
    assert np.array_equal(ctx.matvec(x).cpu().numpy(), y0)
