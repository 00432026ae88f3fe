"""Pins of the oracle's Algorithm 1: direct KKT solves, exact fields, reactions, projections."""
import numpy as np
import pytest

import workloads as W
from oracle import kkt, tetra2
from oracle.solver import Anderson, Constraints, Solver
from oracle.plan import Plan


def _box_nodes(xs, ys, zs):
    g = np.stack(np.meshgrid(np.asarray(xs), np.asarray(ys), np.asarray(zs), indexing="ij"), -1)
    return g.reshape(-1, 3)


CASES = [
    # (n, extra Dirichlet faces (comp, axis, face), with weak 8-node, with weak 4-node face support)
    ((4, 5, 4), [], True, False),
    ((5, 4, 6), [(0, 0, 1), (1, 1, 0)], True, True),
    ((6, 4, 4), [(0, 0, 0), (1, 1, 1), (0, 1, 0)], False, True),
    ((4, 4, 5), [(1, 0, 1)], False, False),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_fixed_point_equals_dense_kkt(case):
    """Eq (18)-(22): the converged fixed point solves the saddle-point system; reactions = multipliers."""
    n, extra, weak8, weak4 = CASES[case]
    rng = np.random.default_rng(100 + case)
    nx, ny, nz = n
    lam = rng.uniform(0.2, 3, (nz, ny, nx)); mu = rng.uniform(0.3, 2, (nz, ny, nx))
    lam[0, 0, 0] = mu[0, 0, 0] = 0.0                 # one void voxel
    bc = W.bc_table(W.BC_N); bc[:, 2, 0] = W.BC_D
    for c, a, f in extra:
        bc[c, a, f] = W.BC_D
    strong = [W.Strong(np.array([[2, 2, nz], [1, 2, nz], [2, 3, 2]]), np.array([2, 2, 0], np.int8),
                       np.array([-0.1, -0.05, 0.02]))]
    avg = []
    if weak8:
        avg.append(W.Average(_box_nodes([1, 2], [1, 2], [1, 2])[None], np.array([1], np.int8),
                             np.array([0.03]), set_id=1))
    if weak4:
        avg.append(W.Average(_box_nodes([2, 3], [2, 3], [nz])[None], np.array([0], np.int8),
                             np.array([-0.02]), set_id=2))
    s = Solver(n, lam, mu, bc, strong, avg, r0_factor=1.0)
    out = s.solve(tol=1e-13, max_iter=5000)
    assert out["converged"]
    d = kkt.dense_kkt(n, lam, mu, bc, strong, avg)
    ui = kkt.project_off(out["u"], d["Z"]); ud = kkt.project_off(d["u"], d["Z"])
    assert np.linalg.norm(ui - ud) <= 1e-9 * np.linalg.norm(ud)
    f = np.concatenate([out["f_strong"], out["f_weak"]])
    assert np.abs(f - d["reaction"]).max() <= 1e-9 * np.abs(d["reaction"]).max()
    # constraints hold exactly at the returned field
    uf = out["u"].reshape(3, -1)
    cons = s.cons
    assert np.abs(uf[cons.s_comp, cons.s_node] - cons.s_val).max() < 1e-15
    for rel in cons.rel:
        assert abs(uf[rel.comp, rel.nodes].mean() - rel.value) < 1e-15


def test_uniaxial_strain_exact_linear_field():
    """Homogeneous block, lateral rollers, top pressed: u_z = delta z / L exactly, sigma_zz = (lam+2mu) delta/L."""
    n = (4, 4, 6)
    nx, ny, nz = n
    lam0, mu0 = 1.2, 0.8
    lam = np.full((nz, ny, nx), lam0); mu = np.full((nz, ny, nx), mu0)
    bc = W.bc_table(W.BC_N)
    bc[0, 0, :] = W.BC_D; bc[1, 1, :] = W.BC_D; bc[2, 2, 0] = W.BC_D
    delta = 0.03
    top = _box_nodes(range(nx + 1), range(ny + 1), [nz])
    strong = [W.Strong(top, np.full(len(top), 2, np.int8), np.full(len(top), delta))]
    s = Solver(n, lam, mu, bc, strong, r0_factor=1.0)
    Nx, Ny, Nz = s.plan.N
    exact = s.zeros()
    exact[2] = delta * np.arange(Nz)[:, None, None] / nz * np.ones((Nz, Ny, Nx))
    parts = s.iterate_parts(exact)
    assert np.sqrt(parts["pnorm2"]) < 1e-14 * np.sqrt(parts["sig2"])
    out = s.solve(tol=1e-12, max_iter=2000)
    assert np.abs(out["u"] - exact).max() < 1e-12
    szz = (lam0 + 2 * mu0) * delta / nz
    assert abs(out["totals"][0, 2] - szz * nx * ny) < 1e-12
    assert np.allclose(out["mean_stress"], np.diag([lam0, lam0, lam0 + 2 * mu0]) * delta / nz, atol=1e-14)


def test_uniaxial_stress_with_pins():
    """Traction-free sides: u_x = -nu eps (x - L/2), u_z = eps z; sigma_zz = E eps."""
    n = (4, 4, 4)
    E, nu = 2.0, 0.25
    lam_v, mu_v = W.lame(E, nu)
    lam = np.full((4, 4, 4), float(lam_v)); mu = np.full((4, 4, 4), float(mu_v))
    bc = W.bc_table(W.BC_N); bc[2, 2, 0] = W.BC_D
    eps = 0.01
    top = _box_nodes(range(5), range(5), [4])
    strong = [W.Strong(top, np.full(len(top), 2, np.int8), np.full(len(top), eps * 4)),
              W.Strong(np.array([[2, 2, 0], [2, 2, 0], [4, 2, 0], [2, 4, 0]]), np.array([0, 1, 1, 0], np.int8),
                       np.zeros(4), set_id=1)]
    s = Solver(n, lam, mu, bc, strong, r0_factor=1.0)
    out = s.solve(tol=1e-12, max_iter=3000)
    z, y, x = np.meshgrid(np.arange(5), np.arange(5), np.arange(5), indexing="ij")
    ex = np.stack([-nu * eps * (x - 2.0), -nu * eps * (y - 2.0), eps * z]).astype(float)
    assert np.abs(out["u"] - ex).max() < 1e-11
    assert abs(out["totals"][0, 2] - E * eps * 16) < 1e-11
    assert np.abs(out["totals"][1]).max() < 1e-12


def test_c1_pin_reactions_vanish_and_acceleration_trend():
    prob = W.c1_inclusion_patch()
    s = Solver.from_problem(prob)
    res = {}
    for acv, per in (("P", 2), ("P", 3), ("U", 2)):
        out = s.solve(tol=1e-8, acv=acv, period=per)
        assert out["converged"]
        res[(acv, per)] = out["iterations"]
        assert np.abs(out["totals"][1]).max() < 1e-10 * abs(out["totals"][0, 2])
        assert out["totals"][0, 2] < 0
    # Table 1b trend: ACV_P beats ACV_U, period 2 beats period 3 (counts: parity unpinned)
    assert res[("P", 2)] <= res[("P", 3)] and res[("P", 2)] <= res[("U", 2)]


def test_strong_single_node_loads_one_sublattice():
    """Section 4.2.3: with TETRA2 a strong single-node load moves only nodes of its parity."""
    n = (6, 6, 6)
    lam = np.ones((6, 6, 6)); mu = np.ones((6, 6, 6))
    bc = W.bc_table(W.BC_D)
    s = Solver(n, lam, mu, bc, [W.Strong(np.array([[3, 3, 3]]), np.array([2], np.int8), np.array([0.1]))])
    out = s.solve(tol=1e-12)
    z, y, x = np.meshgrid(np.arange(7), np.arange(7), np.arange(7), indexing="ij")
    same = (x + y + z) % 2 == (3 + 3 + 3) % 2
    assert np.abs(out["u"][:, ~same]).max() < 1e-13
    assert np.abs(out["u"][:, same & ((x + y + z) != 9)]).max() > 1e-3


def test_projections_are_exact():
    plan = Plan((4, 4, 4), np.zeros((3, 3, 2), np.int8))
    sup = _box_nodes([1, 2], [1, 2], [4])
    cons = Constraints(plan, [W.Strong(np.array([[0, 0, 0]]), np.array([1], np.int8), np.array([0.5]))],
                       [W.Average(sup[None], np.array([2], np.int8), np.array([0.25]))])
    rng = np.random.default_rng(2)
    u = rng.standard_normal((3, 5, 5, 5))
    cons.proj_U(u)
    flat = sup[:, 0] + 5 * (sup[:, 1] + 5 * sup[:, 2])
    assert abs(u.reshape(3, -1)[2, flat].mean() - 0.25) < 1e-15 and u[1, 0, 0, 0] == 0.5
    p = rng.standard_normal((3, 5, 5, 5))
    p0 = p.copy()
    fs, fw = cons.proj_P(p)
    phys = p.reshape(3, -1)[2, flat] / plan.w2b.ravel()[flat]
    assert abs(phys.sum()) < 1e-14 and p[1, 0, 0, 0] == 0.0
    assert fs[0] == -p0[1, 0, 0, 0] / 8.0
    assert abs(fw[0] + np.sum(p0.reshape(3, -1)[2, flat] / plan.w2b.ravel()[flat])) < 1e-14


def test_anderson_reduces_to_secant_on_linear_map():
    """Affine map on R^3: the affine hull of four stored iterates is the whole space, so the
    constrained least squares zeroes the combined residual and lands on the fixed point."""
    rng = np.random.default_rng(4)
    A = rng.standard_normal((3, 3)) * 0.3
    b = rng.standard_normal(3)
    xs = np.linalg.solve(np.eye(3) - A, b)
    acc = Anderson(4, 2, reg=0.0)
    x = np.zeros(3)
    for i in range(5):
        x = acc.step(i, x)
        if i == 4:
            assert acc.last_alpha is not None
            break
        x = A @ x + b
    assert np.linalg.norm(x - xs) < 1e-8 * np.linalg.norm(xs)


def test_too_soft_reference_medium_diverges():
    """With the reference medium far softer than the stiffest phase the fixed-point map is no
    contraction and the iterate grows without bound.  The solve must report divergence
    (an undefined equilibrium measure), never convergence, also when the stress norm
    overflows before the residual norm (their quotient alone would read 0)."""
    p = W.c1_inclusion_patch()
    with np.errstate(over="ignore", invalid="ignore"):
        o = Solver(p.n, p.lam, p.mu, p.bc, p.strong, p.average, r0_factor=0.02).solve(tol=p.tol, max_iter=3000)
    assert not o["converged"] and not np.isfinite(o["residual"]) and o["iterations"] < 3000
    assert np.isnan(Solver.residual(1e307, np.inf)) and np.isnan(Solver.residual(np.inf, 1.0))
    assert Solver.residual(0.0, 0.0) == 0.0


def test_c2_golden_reactions_balance():
    """The stored FP64 oracle reactions of the C2 plate (tests/golden/c2_reactions.txt) satisfy
    global equilibrium: the y reactions of the two pin sets are equal and opposite (no other
    condition acts along y), and nothing acts along x or z on them."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_reactions.txt")
    rows = {}
    for line in open(path):
        if line.startswith("set"):
            k, v = line.split(":", 1)
            rows[int(k[3:])] = np.array([float(x) for x in v.split()])
    r0, r1 = rows[0], rows[1]
    assert r0[1] > 0 and abs(r0[1] + r1[1]) <= 1e-8 * r0[1]
    assert r0[0] == r0[2] == r1[0] == r1[2] == 0.0
