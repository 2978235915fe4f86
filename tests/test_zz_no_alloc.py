"""The no-allocation product (mlfma_matvec_noalloc): its pattern buffers live
in the library's static device scratch.  Checked through the C ABI against
mlfma_matvec on the same context, on two calls in a row, the second with a
smaller input, on arrays with empty sites (the leaf buffer must read zero
there) and with several particle classes (the class-pair near partials)."""
import numpy as np
import pytest

import workloads as w
from gpu_helpers import make_ctx, note, rel_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2407_21724_amd import mlfma  # noqa: E402


def _cylinders_with_holes():
    wl = w.workload("c2", 9, 7)
    keep = np.ones(wl.n_particles, bool)
    keep[[3, 10, 24, 40, 50]] = False
    return w.Workload("holes", wl.centers[keep], wl.class_id[keep], wl.meshes, wl.eps_r, wl.n_perp, wl.n_par)


def _lens():
    return w.workload("c4", 6, 5)


def _basis(wl):
    Ms = {}
    for c in sorted(set(wl.class_id.tolist())):
        v, t, e = wl.meshes[c]
        Ms[c], _ = mlfma.static_modes(v, t, e, wl.n_perp, wl.n_par)
    return Ms


@pytest.mark.parametrize("case,prec,ra,rb", [("holes", mlfma.C64, 3, 1), ("holes", mlfma.C128, 3, 1),
                                             ("lens", mlfma.C64, 3, 1), ("lens", mlfma.C64_BF16, 3, 1),
                                             ("lens", mlfma.C64, 16, 4)])
def test_noalloc_matches_matvec_two_calls(case, prec, ra, rb):
    """ra then rb right-hand sides; 16 and 4 RHS take the LDS-staged GEMMs
    (class-pair near partials in the scratch)."""
    wl = _cylinders_with_holes() if case == "holes" else _lens()
    ctx = make_ctx(wl, _basis(wl), prec)
    ctx.prepare()
    n = 2 * (wl.n_perp + wl.n_par)
    xa = to_dev(w.random_complex((ra, wl.n_particles, n), 11), ctx)
    xb = to_dev(w.random_complex((rb, wl.n_particles, n), 12), ctx)
    ya_ref, yb_ref = ctx.matvec(xa), ctx.matvec(xb)
    ya, yb = torch.empty_like(xa), torch.empty_like(xb)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ctx.matvec_noalloc(xa, ya)            # ra RHS
    ctx.matvec_noalloc(xb, yb)            # then rb RHS in the same scratch
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    ea = rel_err(ya.cpu().numpy(), ya_ref.cpu().numpy())
    eb = rel_err(yb.cpu().numpy(), yb_ref.cpu().numpy())
    note(f"{case} precision={prec}: rel. difference to mlfma_matvec {ea:.1e} ({ra} RHS), {eb:.1e} ({rb} RHS); "
         f"free device memory {free0} -> {free1}")
    # the same kernels on the same inputs in the same order: equal bit for bit
    assert torch.equal(ya, ya_ref) and torch.equal(yb, yb_ref)
    assert free1 == free0


def test_noalloc_limits():
    # an unprepared context is refused (preparing allocates)
    wl = _cylinders_with_holes()
    ctx = make_ctx(wl, _basis(wl), mlfma.C64)
    x = to_dev(w.random_complex((1, wl.n_particles, 60), 1), ctx)
    with pytest.raises(mlfma.MlfmaError) as ei:
        ctx.matvec_noalloc(x, torch.empty_like(x))
    assert ei.value.code == mlfma.ENOTREADY
    # two particles at the corners of a 120 x 120 lattice: the leaf pattern
    # buffers alone (14,400 boxes x 2 x 242 samples x 8 B, twice) exceed the
    # 64 MiB scratch
    cen = np.array([[0.0, 0.0, 0.0], [59.5, 59.5, 0.0]])
    big = w.Workload("corners", cen, np.zeros(2, np.int32), wl.meshes, wl.eps_r, wl.n_perp, wl.n_par)
    ctx2 = make_ctx(big, _basis(wl), mlfma.C64)
    ctx2.prepare()
    x2 = to_dev(w.random_complex((1, 2, 60), 1), ctx2)
    with pytest.raises(mlfma.MlfmaError) as ei:
        ctx2.matvec_noalloc(x2, torch.empty_like(x2))
    assert ei.value.code == mlfma.EINVAL
