"""Node-by-node parity of the FP32 iteration's residual pass as it runs (the residual form: FP64
displacement, FP32 residual-sized fields; tiled kernel, and its fallback for node planes wider
than 2048 tiles) through fftc_stage_residual_form, against quantities formed from the oracle:
p after proj_P (Algorithm 1), K0 delta = -2^b div_D(R0 : grad_D delta) (eq 3), R = p + K0 delta - e,
dR = R - R_prev, dY = p - p_prev + K0 delta.  At DOFs held at 0 by a Dirichlet face p is 0 and the
transforms drop the entries; R, dR, dY there are compared with K0 delta from the symmetric image,
the stencil the pass applies (the oracle's reference term has no equation there)."""
import numpy as np
import pytest

import workloads as W
from oracle import tetra2
from oracle.solver import Solver as OSolver

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2607_26082_amd as F
    F.load()
    return F


def _box(xs, ys, zs):
    g = np.stack(np.meshgrid(np.asarray(xs), np.asarray(ys), np.asarray(zs), indexing="ij"), -1)
    return g.reshape(-1, 3)


# grids straddling the 31 x 7 node tiles of the tiled pass (ragged last tiles in x and y),
# periodic axes, and a thin wide grid whose node plane needs more than 2048 tiles (fallback)
SHAPES = [((40, 15, 9), None, False), ((30, 15, 6), 0, False), ((45, 20, 8), 1, False), ((32, 12, 10), 2, False),
          ((40, 15, 9), None, True), ((30, 15, 6), 0, True), ((720, 720, 3), None, False)]


def _case(seed, n, per):
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    lam = rng.uniform(0.4, 2.5, (nz, ny, nx)); mu = rng.uniform(0.3, 1.8, (nz, ny, nx))
    lam[0, 0, :3] = 0.0; mu[0, 0, :3] = 0.0
    bc = rng.integers(0, 2, (3, 3, 2)).astype(np.int8)
    bc[:, 2, 0] = W.BC_D
    bc[0, 2, 1] = W.BC_N          # the strong DOF below sits on the top face
    if per is not None:
        bc[:, per, :] = W.BC_P
    strong = [W.Strong(np.array([[2, 2, nz if per != 2 else nz - 1]]), np.array([0], np.int8), np.array([0.01]))]
    avg = [W.Average(_box([4, 5], [3, 4], [1, 2])[None], np.array([1], np.int8), np.array([0.01]), set_id=1)]
    return lam, mu, bc, strong, avg


@pytest.mark.parametrize("idx", range(len(SHAPES)))
@pytest.mark.parametrize("il", [0, 1, 3])
@pytest.mark.parametrize("fp64_stress", [0, 1])
def test_stage_residual_form(idx, il, fp64_stress):
    """fp64_stress = 1: the pass the FP32 form takes below the refinement threshold (stresses
    formed in FP64, every field FP32): then the bar is 2e-6, FP32 rounding of the outputs and
    of the FP32 inputs (delta, e, p_prev, R_prev) only."""
    F = _lib()
    n, per, fs = SHAPES[idx]
    if n[0] == 720 and il != 3:
        pytest.skip("the wide grid runs once (every output formed at il = 3)")
    print(f"[residual form] n={n} periodic={per} finite_strain={fs} il={il} fp64_stress={fp64_stress}", flush=True)
    lam, mu, bc, strong, avg = _case(70 + idx, n, per)
    o = OSolver(n, lam, mu, bc, strong, avg, r0_factor=1.3, finite_strain=fs)
    g = F.Solver(n, lam, mu, bc, strong, avg, r0_factor=1.3, precision="fp32", finite_strain=fs)
    rng = np.random.default_rng(idx + 10 * il)
    shape = o.zeros().shape
    A = o.plan.amask
    u = rng.standard_normal(shape) * (5e-2 if fs else 1e-2)
    u[A] = 0.0
    o.cons.proj_U(u)
    fields = []
    for sc in (1e-3, 2e-2, 2e-2, 2e-2):
        f = rng.standard_normal(shape) * sc
        f[A] = 0.0
        fields.append(f)
    delta, e, p_prev, R_prev = fields
    p, R, dR, dY, sums = g.stage_residual_form(u, delta, e, p_prev, R_prev, il, fp64_stress=fp64_stress)
    parts = o.iterate_parts(u)
    k0d = -o.reference_term(tetra2.tet_gradients(delta, o.plan))
    tol = 2e-6 if fp64_stress else 2e-5
    pe = parts["p"]
    assert np.abs(p - pe).max() <= tol * np.abs(pe).max()
    assert abs(sums[0] - parts["pnorm2"]) <= 10 * tol * parts["pnorm2"]
    assert abs(sums[1] - parts["sig2"]) <= 10 * tol * parts["sig2"]
    if il >= 1:
        Re = pe + k0d - e
        free = ~A
        assert np.abs(R - Re)[free].max() <= tol * np.abs(Re).max()
        if il >= 2:
            dRe = Re - R_prev
            dYe = pe - p_prev + k0d
            assert np.abs(dR - dRe)[free].max() <= tol * np.abs(dRe).max()
            assert np.abs(dY - dYe)[free].max() <= tol * np.abs(dYe).max()


@pytest.mark.parametrize("idx", range(6))
def test_mean_stress_of_returned_iterate(idx):
    """The FP32 form reports the mean stress of the iterate it returns, formed once at the end:
    compared with the oracle's volume average of the stress (PK1 in finite strain) of that same
    FP64 displacement, on heterogeneous cells with and without a periodic axis.  The solve is
    cut after a few iterations so that the field is far from any closed form."""
    F = _lib()
    n, per, fs = SHAPES[idx]
    print(f"[mean stress] n={n} periodic={per} finite_strain={fs}", flush=True)
    lam, mu, bc, strong, avg = _case(70 + idx, n, per)
    g = F.Solver(n, lam, mu, bc, strong, avg, r0_factor=1.3, precision="fp32", finite_strain=fs, max_iter=12)
    rc, rep = g.solve()
    assert rep.iterations <= 12 and np.isfinite(rep.residual)
    o = OSolver(n, lam, mu, bc, strong, avg, r0_factor=1.3, finite_strain=fs)
    u = g.u.cpu().numpy().reshape(o.zeros().shape)
    sig = o.iterate_parts(u)["sig"]
    M = tetra2.mean_stress(sig)
    want = np.array([M[0, 0], M[1, 1], M[2, 2], M[1, 2], M[0, 2], M[0, 1]])
    scale = np.abs(sig).mean()
    assert np.abs(np.array(rep.mean_stress) - want).max() <= 2e-6 * scale


@pytest.mark.parametrize("idx", [0, 1, 2, 3])
@pytest.mark.parametrize("dscale", [2e-2, 1e-7])
def test_stage_residual_form_incremental(idx, dscale):
    """The incremental pass (small strain, no obstacle, singular modes or relations): p = p_prev +
    the divergence term of the stresses of delta, u not read.  With p_prev = the oracle's p of
    u - delta (eq 3), p must equal the oracle's p of u, and dY = p(u) - p(u - delta) + K0 delta,
    R = p + K0 delta - e as in the pass from u.  dscale 1e-7: an update far below u, as when the
    iteration stagnates; there dY is held to 2e-6 of its own size, which the pass from u (p_i -
    p_{i-1} of two FP32 fields of size |p|) cannot meet (printed for comparison)."""
    F = _lib()
    n, per, fs = SHAPES[idx]
    assert not fs
    print(f"[residual form, incremental] n={n} periodic={per} delta scale={dscale}", flush=True)
    lam, mu, bc, strong, _ = _case(70 + idx, n, per)
    o = OSolver(n, lam, mu, bc, strong, (), r0_factor=1.3)
    g = F.Solver(n, lam, mu, bc, strong, (), r0_factor=1.3, precision="fp32")
    rng = np.random.default_rng(100 + idx)
    shape = o.zeros().shape
    A = o.plan.amask
    u = rng.standard_normal(shape) * 1e-2
    u[A] = 0.0
    o.cons.proj_U(u)
    delta = rng.standard_normal(shape) * dscale
    delta[A] = 0.0
    e = rng.standard_normal(shape) * 2e-2
    e[A] = 0.0
    R_prev = rng.standard_normal(shape) * 2e-2
    R_prev[A] = 0.0
    p_prev = o.iterate_parts(u - delta)["p"]
    pe = o.iterate_parts(u)["p"]
    k0d = -o.reference_term(tetra2.tet_gradients(delta, o.plan))
    free = ~A
    dYe = pe - p_prev + k0d
    Re = pe + k0d - e
    p, R, dR, dY, sums = g.stage_residual_form(u, delta, e, p_prev, R_prev, 3, incremental=True)
    assert np.abs(p - pe).max() <= 2e-5 * np.abs(pe).max()
    assert abs(sums[0] - np.sum(pe[free] ** 2)) <= 2e-4 * np.sum(pe[free] ** 2)
    assert sums[1] == 0.0
    err_inc = np.abs(dY - dYe)[free].max() / np.abs(dYe).max()
    _, _, _, dY_u, _ = g.stage_residual_form(u, delta, e, p_prev, R_prev, 3)
    err_u = np.abs(dY_u - dYe)[free].max() / np.abs(dYe).max()
    print(f"[residual form, incremental] dY error / |dY|: incremental {err_inc:.2e}, from u {err_u:.2e}", flush=True)
    assert err_inc <= 2e-6
    assert np.abs(R - Re)[free].max() <= 2e-5 * np.abs(Re).max()
    assert np.abs(dR - (Re - R_prev))[free].max() <= 2e-5 * np.abs(Re - R_prev).max()


@pytest.mark.parametrize("n", [(40, 36, 28), (128, 128, 128)])
def test_incremental_solve_matches_pass_from_u(n):
    """Whole FP32 solves of a two-phase cell (strong patch, fixed base) with the incremental pass
    (a pass from u every 16th iteration, the default) and with the pass from u every iteration:
    both within 1e-5 (rel-L2) of the FP64 solution at tol 1e-10.  At 128^3 the incremental pass
    runs on its own tile grid (four blocks per CU, 13-plane segments), the pass from u on the
    smaller one, and the control step sums the larger count of partial rows."""
    F = _lib()
    prob = W.m256_metric(n=n)
    print(f"[residual form] incremental vs from-u solves, {n}", flush=True)
    ref = F.Solver.from_problem(prob, precision="fp64", tol=1e-10, max_iter=4000)
    rc, rep = ref.solve()
    assert rc == 0
    u64 = ref.u.cpu().numpy()
    for ae in (16, 0):
        g = F.Solver.from_problem(prob, precision="fp32", tol=1e-6, max_iter=4000, anchor_every=ae)
        rc, rep = g.solve()
        assert rc == 0, (ae, rep.iterations)
        err = np.linalg.norm(g.u.cpu().numpy() - u64) / np.linalg.norm(u64)
        print(f"[residual form] anchor_every={ae}: {rep.iterations} iterations, rel-L2 to FP64 {err:.2e}", flush=True)
        assert err <= 1e-5


def test_stall_triggered_refinement_high_contrast_cell():
    """A held-out indentation cell of contrast 90 (64^3, rigid sphere, d/R 0.028): with FP32
    stresses to the end its residual stalls above 1e-6 (the FP32 noise floor of this cell lies
    above ten times the tolerance, so the threshold alone never starts the refinement); the
    refinement started by the stall (no halving in 100 iterations below 1e-2) takes it to 1e-6,
    within 5e-5 (rel-L2) of the FP64 solution at 1e-10."""
    F = _lib()
    prob = W.nn_case_build(W.nn_case_spec(W.NN_EVAL_SEED + 5))
    assert prob.meta["kind"] == "indent" and prob.meta["contrast"] > 80
    print(f"[residual form] stall refinement, contrast {prob.meta['contrast']:.1f}", flush=True)
    g0 = F.Solver.from_problem(prob, precision="fp32", tol=1e-6, max_iter=4000, refine_below=0.0)
    rc0, rep0 = g0.solve()
    print(f"[residual form] FP32 stresses throughout: rc {rc0}, {rep0.iterations} iterations, residual "
          f"{rep0.residual:.2e}", flush=True)
    g = F.Solver.from_problem(prob, precision="fp32", tol=1e-6, max_iter=4000)
    rc, rep = g.solve()
    print(f"[residual form] default refinement: {rep.iterations} iterations", flush=True)
    assert rc == 0
    # the trajectory depends on the rounding: the stall shows as no convergence or a far longer solve
    assert rc0 != 0 or rep0.iterations > 1.5 * rep.iterations
    ref = F.Solver.from_problem(prob, precision="fp64", tol=1e-10, max_iter=20000)
    assert ref.solve()[0] == 0
    u64 = ref.u.cpu().numpy()
    err = np.linalg.norm(g.u.cpu().numpy() - u64) / np.linalg.norm(u64)
    print(f"[residual form] rel-L2 to FP64 {err:.2e}", flush=True)
    assert err <= 5e-5
