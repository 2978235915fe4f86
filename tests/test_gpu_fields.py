"""GPU field evaluation (mlfma_fields): each particle's field expanded about
its centre from its leaf radiation pattern and the translation operator
taken to the observation point, against the oracle's direct quadrature of
the same currents (scattered E at exterior points)."""
import os

import numpy as np
import pytest

import workloads as w
from gpu_helpers import make_ctx, note, rel_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle.fields import near_field  # noqa: E402
from oracle.pmchwt import DenseProblem, ParticleClass, solve_dense  # noqa: E402
from paper_2407_21724_amd import mlfma  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_10x10_fields.npz")


@pytest.fixture(scope="module")
def c1():
    wl = w.workload("c1")
    v, t, e = wl.meshes[0]
    pc = ParticleClass(v, t, e, wl.n_perp, wl.n_par, wl.eps_r)
    prob = DenseProblem([pc], wl.centers, wl.class_id)
    P = wl.n_particles
    prob.prefetch([(a, b) for a in range(P) for b in range(P)])
    inc = wl.incidences[0]
    J = solve_dense(prob, prob.rhs(inc.khat, inc.pol))
    return wl, pc, prob, J


@pytest.mark.parametrize("prec", [mlfma.C128, mlfma.C64])
def test_c1_fields_of_dense_solution(c1, prec):
    """4 x 4 spheres, the oracle's dense solution as currents: planes z = 0.6
    and z = 2 over the array, and points beside it in the array plane."""
    wl, pc, prob, J = c1
    ctx = make_ctx(wl, pc.M, prec)
    g = np.linspace(-0.5, 2.0, 7)
    X, Y = np.meshgrid(g, g)
    pts = np.concatenate([np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], -1) for z in (0.6, 2.0)]
                         + [np.array([[-1.0, 0.7, 0.0], [2.6, 0.2, 0.0], [0.75, -1.2, 0.0]])])
    E = ctx.fields(to_dev(J[None], ctx), pts).cpu().numpy()[0]
    ref = near_field(prob, J, pts)
    err = rel_err(E, ref)
    worst = float(np.max(np.linalg.norm(E - ref, axis=1)) / np.max(np.linalg.norm(ref, axis=1)))
    note(f"C1 fields precision={prec}: rel 2-norm error {err:.2e}, worst point {worst:.2e}")
    assert err < 1e-3 and worst < 1e-3


def test_lens_subarray_fields():
    """10 x 10 lens of the full-scale recipe (four classes), plane z = 1:
    the field of the oracle's solution (parity of the field evaluation), and
    the field of the GPU GMRES solution against the oracle's field of its own
    dense solution (the full path, bar 1e-2)."""
    if not os.path.exists(GOLDEN):
        pytest.skip("golden not generated")
    g = np.load(GOLDEN)
    wl = w.workload("c5", 10, 10)
    classes = [int(c) for c in g["classes"]]
    M = {c: g["M"][i] for i, c in enumerate(classes)}
    ctx = make_ctx(wl, M, mlfma.C64)
    E_or = ctx.fields(to_dev(g["J"][None], ctx), g["pts"]).cpu().numpy()[0]
    e1 = rel_err(E_or, g["near"])
    b = ctx.plane_wave_rhs(g["khat"][None], g["pol"][None])
    x, stats, rc = ctx.gmres_solve(b, rtol=1e-5, max_iter=2000, restart=300)
    assert rc == mlfma.OK
    E = ctx.fields(x, g["pts"]).cpu().numpy()[0]
    e2 = rel_err(E, g["near"])
    note(f"lens 10x10 fields: of the oracle solution {e1:.2e}, of the GPU solution {e2:.2e}")
    assert e1 < 1e-3 and e2 < 1e-2


def test_fields_batched_and_guarded(c1):
    """Two RHS in one call equal two single calls; a point inside a
    particle's leaf box is rejected."""
    wl, pc, prob, J = c1
    ctx = make_ctx(wl, pc.M, mlfma.C64)
    x2 = np.stack([J, w.random_complex(J.shape, 9)])
    pts = np.array([[0.25, 0.25, 1.5], [3.0, -1.0, 0.8]])
    E2 = ctx.fields(to_dev(x2, ctx), pts).cpu().numpy()
    for r in range(2):
        E1 = ctx.fields(to_dev(x2[r:r + 1], ctx), pts).cpu().numpy()[0]
        assert np.array_equal(E1, E2[r])
    with pytest.raises(mlfma.MlfmaError):
        ctx.fields(to_dev(J[None], ctx), np.array([[0.5, 0.5, 0.1]]))
