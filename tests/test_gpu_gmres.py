"""GPU GMRES (right block-diagonal preconditioner, FP64 Arnoldi) against the
oracle's dense solve; solutions compared in the unknowns and in the
scattered far and near fields (tolerance 1e-2 in the fields)."""
import numpy as np
import pytest

import workloads as w
from gpu_helpers import make_ctx, note, rel_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle.fields import far_amplitude, near_field, scattering_cross_section, sphere_grid  # noqa: E402
from oracle.pmchwt import DenseProblem, ParticleClass, solve_dense  # noqa: E402
from paper_2407_21724_amd import mlfma  # noqa: E402


@pytest.fixture(scope="module")
def c1_solution():
    wl = w.workload("c1")
    v, t, e = wl.meshes[0]
    pc = ParticleClass(v, t, e, wl.n_perp, wl.n_par, wl.eps_r)
    prob = DenseProblem([pc], wl.centers, wl.class_id)
    P = wl.n_particles
    prob.prefetch([(a, b) for a in range(P) for b in range(P)])
    inc = wl.incidences[0]
    V = prob.rhs(inc.khat, inc.pol)
    J = solve_dense(prob, V)
    return wl, pc, prob, V, J


def _fields(prob, x):
    rhat, _ = sphere_grid(32, 64)
    far = far_amplitude(prob, x, rhat)
    g = np.linspace(-0.25, 1.75, 9)
    X, Y = np.meshgrid(g, g)
    pts = np.stack([X.ravel(), Y.ravel(), np.full(X.size, 0.4)], -1)   # plane z = 0.4 above C1
    near = near_field(prob, x, pts)
    return far, near


@pytest.mark.parametrize("prec,rtol", [(mlfma.C128, 1e-6), (mlfma.C64, 1e-4)])
def test_c1_gmres_vs_dense_solve(c1_solution, prec, rtol):
    wl, pc, prob, V, J = c1_solution
    note(f"c1 gmres precision={prec} rtol={rtol}")
    ctx = make_ctx(wl, pc.M, prec)
    inc = wl.incidences[0]
    b = ctx.plane_wave_rhs(inc.khat[None], inc.pol[None])
    x, stats, rc = ctx.gmres_solve(b, rtol=rtol, max_iter=200, restart=50)
    note(f"  {stats[0]}")
    assert rc == mlfma.OK and stats[0]["converged"]
    assert stats[0]["true_rel_res"] <= rtol
    xs = x.cpu().numpy()[0]
    # true residual with the oracle's dense operator
    Z = prob.dense()
    r_or = np.linalg.norm(Z @ xs.reshape(-1) - V.reshape(-1)) / np.linalg.norm(V)
    note(f"  oracle residual {r_or:.3e}, unknowns err {rel_err(xs, J):.3e}")
    assert r_or < 10 * rtol
    far_g, near_g = _fields(prob, xs)
    far_o, near_o = _fields(prob, J)
    ef, en = rel_err(far_g, far_o), rel_err(near_g, near_o)
    note(f"  far-field err {ef:.3e} near-field err {en:.3e}")
    assert ef < 1e-2 and en < 1e-2
    cs_g, cs_o = scattering_cross_section(prob, xs), scattering_cross_section(prob, J)
    assert abs(cs_g / cs_o - 1) < 1e-2


def test_gmres_initial_guess_and_zero_rhs(c1_solution):
    wl, pc, prob, V, J = c1_solution
    ctx = make_ctx(wl, pc.M, mlfma.C128)
    inc = wl.incidences[0]
    b = ctx.plane_wave_rhs(inc.khat[None], inc.pol[None])
    # exact initial guess: converges with no iterations
    x0 = to_dev(J[None], ctx)
    x, stats, rc = ctx.gmres_solve(b, x=x0.clone(), rtol=1e-6, max_iter=50, restart=20, use_x0=True)
    assert rc == mlfma.OK and stats[0]["iterations"] == 0
    # the guess is scaled by the complex factor that minimises its residual:
    # a multiple of the solution needs no iteration ...
    x, stats, rc = ctx.gmres_solve(b, x=((1.5 - 2.0j) * x0).contiguous(), rtol=1e-6, max_iter=50, restart=20,
                                   use_x0=True)
    assert rc == mlfma.OK and stats[0]["iterations"] == 0
    # ... and a guess unrelated to it is scaled towards zero
    bad = to_dev(1e3 * w.random_complex(J[None].shape, 4), ctx)
    x, stats, rc = ctx.gmres_solve(b, x=bad, rtol=1e-6, max_iter=200, restart=50, use_x0=True)
    assert rc == mlfma.OK and stats[0]["true_rel_res"] <= 1e-6
    # zero right-hand side -> zero solution
    z = torch.zeros_like(b)
    x, stats, rc = ctx.gmres_solve(z, rtol=1e-6, max_iter=10, restart=5)
    assert rc == mlfma.OK and float(x.abs().max()) == 0.0
    # not converged within max_iter -> warning status, best iterate returned
    x, stats, rc = ctx.gmres_solve(b, rtol=1e-14, max_iter=3, restart=3)
    assert rc == mlfma.NOT_CONVERGED and not stats[0]["converged"]
    assert stats[0]["true_rel_res"] < 1.0
    # NaN or Inf in the right-hand side or in the guess: rejected with
    # ENONFINITE before any product
    bn = b.clone()
    bn[0, 3, 5] = complex(float("nan"), 0.0)
    with pytest.raises(mlfma.MlfmaError) as ei:
        ctx.gmres_solve(bn, rtol=1e-6, max_iter=10, restart=5)
    assert ei.value.code == mlfma.ENONFINITE
    xi = torch.zeros_like(b)
    xi[0, 1, 2] = complex(float("inf"), 0.0)
    with pytest.raises(mlfma.MlfmaError) as ei:
        ctx.gmres_solve(b, x=xi, rtol=1e-6, max_iter=10, restart=5, use_x0=True)
    assert ei.value.code == mlfma.ENONFINITE


def test_lens_subarray_fields_vs_oracle():
    """A 10 x 10 lens of the full-scale recipe (four diameter classes): FP32
    product GMRES against the oracle's dense solve, in the unknowns and in
    the scattered near field (plane z = 1 over the array) and far field."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_10x10_fields.npz")
    if not os.path.exists(path):
        pytest.skip("golden not generated")
    g = np.load(path)
    wl = w.workload("c5", 10, 10)
    classes = [int(c) for c in g["classes"]]
    M = {c: g["M"][i] for i, c in enumerate(classes)}
    ctx = make_ctx(wl, M, mlfma.C64)
    b = ctx.plane_wave_rhs(g["khat"][None], g["pol"][None])
    x, stats, rc = ctx.gmres_solve(b, rtol=1e-5, max_iter=2000, restart=300)   # FP32 product: floor ~1e-6
    note(f"lens 10x10 gmres: {stats[0]}")
    assert rc == mlfma.OK
    xs = x.cpu().numpy()[0]
    # oracle's field evaluation on the GPU solution (same static-mode basis)
    pcs = []
    for c in classes:
        v, t, e = wl.meshes[c]
        pcs.append(ParticleClass(v, t, e, wl.n_perp, wl.n_par, wl.eps_r, M=M[c]))
    compact = np.array([classes.index(c) for c in wl.class_id], np.int32)
    prob = DenseProblem(pcs, wl.centers, compact)
    near = near_field(prob, xs, g["pts"])
    far = far_amplitude(prob, xs, g["rhat"])
    ex, en, ef = rel_err(xs, g["J"]), rel_err(near, g["near"]), rel_err(far, g["far"])
    note(f"  unknowns {ex:.3e}, near field {en:.3e}, far field {ef:.3e}")
    assert en < 1e-2 and ef < 1e-2


@pytest.mark.parametrize("prec", [mlfma.C64, mlfma.C64_BF16])
def test_c3_batched_64_incidences(prec):
    """64 incidences (polar 5i deg x azimuth 45j deg, TE/TM alternating) on a
    12 x 12 subarray of the cylinders, solved in one batched GMRES with FP32
    or BF16-split products: every RHS reaches its own true residual, the
    batched product agrees with the single-RHS products to FP32 rounding
    (with 64 RHS the FP32 receive GEMM runs on the LDS-staged kernel, which
    sums its 968 terms in another order than the one-RHS launch), and two
    RHS agree with their single solves."""
    wl = w.workload("c3", 12, 12)
    v, t, e = wl.meshes[0]
    M, _ = mlfma.static_modes(v, t, e, wl.n_perp, wl.n_par)
    ctx = make_ctx(wl, M, prec)
    kh = np.array([i.khat for i in wl.incidences])
    pol = np.array([i.pol for i in wl.incidences])
    b = ctx.plane_wave_rhs(kh, pol)
    assert b.shape[0] == 64
    yb = ctx.matvec(b)
    for r in (0, 17, 63):
        y1 = ctx.matvec(b[r:r + 1].contiguous())
        assert float(torch.linalg.vector_norm(y1 - yb[r:r + 1]) / torch.linalg.vector_norm(y1)) < 2e-6
    x, stats, rc = ctx.gmres_solve(b, rtol=1e-4, max_iter=2000, restart=200)
    res = [s["true_rel_res"] for s in stats]
    its = [s["iterations"] for s in stats]
    note(f"c3 64 RHS precision={prec}: iterations {min(its)}..{max(its)}, true residual max {max(res):.2e}")
    assert rc == mlfma.OK and max(res) <= 1e-4
    for r in (5, 40):
        xs, st, rc1 = ctx.gmres_solve(b[r:r + 1].contiguous(), rtol=1e-4, max_iter=2000, restart=200)
        assert rc1 == mlfma.OK
        d = rel_err(x[r].cpu().numpy(), xs[0].cpu().numpy())
        note(f"  RHS {r}: batched vs single solve {d:.2e}")
        assert d < 1e-3


def test_fp32_krylov_basis():
    """GMRES with the Krylov basis stored in FP32 (FP64 arithmetic) reaches
    the same true residual as with the FP64 basis, in about as many
    iterations, on a 12 x 12 subarray of the cylinders."""
    wl = w.workload("c2", 12, 12)
    v, t, e = wl.meshes[0]
    M, _ = mlfma.static_modes(v, t, e, wl.n_perp, wl.n_par)
    ctx = make_ctx(wl, M, mlfma.C64)
    inc = wl.incidences[0]
    b = ctx.plane_wave_rhs(inc.khat[None], inc.pol[None])
    x64, s64, rc64 = ctx.gmres_solve(b, rtol=1e-4, max_iter=2000, restart=100)
    x32, s32, rc32 = ctx.gmres_solve(b, rtol=1e-4, max_iter=2000, restart=100, fp32_basis=True)
    note(f"FP64 basis {s64[0]['iterations']} it, FP32 basis {s32[0]['iterations']} it, "
         f"solutions differ by {rel_err(x32.cpu().numpy(), x64.cpu().numpy()):.2e}")
    assert rc64 == mlfma.OK and rc32 == mlfma.OK
    assert s32[0]["true_rel_res"] <= 1e-4
    assert abs(s32[0]["iterations"] - s64[0]["iterations"]) <= 0.1 * s64[0]["iterations"] + 2
    assert rel_err(x32.cpu().numpy(), x64.cpu().numpy()) < 1e-3


@pytest.mark.parametrize("fp32_basis", [False, True])
def test_graph_replayed_arnoldi_steps_match_direct_launches(monkeypatch, fp32_basis):
    """With MLFMA_GMRES_GRAPHS, the product and the Arnoldi step are replayed
    captured graphs (the step index read from the device); they give the
    same iterates, bit for bit, as the default direct launches: several restart cycles, one and then two
    right-hand sides, with the host's own work and synchronisations between
    the replays."""
    wl = w.workload("c2", 12, 12)
    v, t, e = wl.meshes[0]
    M, _ = mlfma.static_modes(v, t, e, wl.n_perp, wl.n_par)
    res = {}
    rhs = None
    for mode in ("graph", "direct"):
        if mode == "graph":
            monkeypatch.setenv("MLFMA_GMRES_GRAPHS", "1")
        else:
            monkeypatch.delenv("MLFMA_GMRES_GRAPHS", raising=False)
        ctx = make_ctx(wl, M, mlfma.C64)
        ctx.prepare()
        if rhs is None:
            kh = np.array([i.khat for i in wl.incidences[:2]])
            pol = np.array([i.pol for i in wl.incidences[:2]])
            b2 = ctx.plane_wave_rhs(kh, pol)
            rhs = (b2[:1].contiguous(), b2)
        out = []
        for b in rhs:
            x, st, rc = ctx.gmres_solve(b, rtol=1e-4, max_iter=600, restart=30, fp32_basis=fp32_basis)
            out.append((x.cpu(), [s["iterations"] for s in st], [s["true_rel_res"] for s in st], rc))
        res[mode] = out
    for (xg, ig, rg, cg), (xd, idd, rd, cd) in zip(res["graph"], res["direct"]):
        note(f"graph-replayed steps (fp32 basis {fp32_basis}): iterations {ig}, true residual {rg}")
        assert min(ig) > 60  # at least three restart cycles
        assert ig == idd and rg == rd and cg == cd
        assert torch.equal(xg, xd)


def test_c5_full_scale_batched_restarted_gmres():
    """The full-scale lens (200 x 200 cylinders, 32 classes, 2.4 M unknowns):
    two incidences in one restarted GMRES (restart 100, 150 steps, so one
    restart with its true-residual product) take the same steps as each
    incidence alone, bit for bit, since the batched product and Arnoldi keep
    every right-hand side separate."""
    wl = w.workload("c5")
    M = {}
    for c in sorted(set(wl.class_id.tolist())):
        v, t, e = wl.meshes[c]
        M[c], _ = mlfma.static_modes(v, t, e, wl.n_perp, wl.n_par)
    ctx = make_ctx(wl, M, mlfma.C64)
    kh = np.array([i.khat for i in wl.incidences[:2]])
    pol = np.array([i.pol for i in wl.incidences[:2]])
    b = ctx.plane_wave_rhs(kh, pol)
    x2, st2, _ = ctx.gmres_solve(b, rtol=1e-8, max_iter=150, restart=100)
    assert [s["iterations"] for s in st2] == [150, 150]
    for r in range(2):
        x1, st1, _ = ctx.gmres_solve(b[r:r + 1].contiguous(), rtol=1e-8, max_iter=150, restart=100)
        note(f"C5 RHS {r}: 150 steps, true residual {st1[0]['true_rel_res']:.3e} alone, "
             f"{st2[r]['true_rel_res']:.3e} batched")
        assert st1[0]["iterations"] == 150 and st1[0]["cycles"] == st2[r]["cycles"] == 2
        assert st1[0]["true_rel_res"] == st2[r]["true_rel_res"]
        assert torch.equal(x1[0], x2[r])
