"""Pins of the HEX1 scheme and of the isotropic reference medium (Section 3.1.2, eq 4, Section
3.2.3-3.2.4; hourglass modes of Section 4.2.3)."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import hex1, kkt, tetra2
from oracle.green import Green
from oracle.plan import Plan
from oracle.solver import Solver


def _coords(plan):
    Nx, Ny, Nz = plan.N
    z, y, x = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    return np.stack([x, y, z]).astype(np.float64)


def test_centre_gradient_reproduces_linear_fields_and_weights():
    plan = Plan((3, 4, 2), np.zeros((3, 3, 2), np.int8))
    rng = np.random.default_rng(0)
    A = rng.standard_normal((3, 3))
    u = np.einsum("ij,jzyx->izyx", A, _coords(plan)) + rng.standard_normal(3)[:, None, None, None]
    G = hex1.gradients(u, plan)
    assert np.abs(G[0] - A[:, :, None, None, None]).max() < 1e-13
    # B weights: (2a - 1) / 4 per corner; they sum to 0 and each has |B_j| = 1/4
    assert np.abs(hex1.B.sum(axis=0)).max() == 0.0 and np.all(np.abs(hex1.B) == 0.25)


PERIODIC = np.full((3, 3, 2), 2, np.int8)


def test_hourglass_null_space():
    """A periodic 4^3 HEX1 block has 3 translations and the hourglass modes: every frequency
    with two of its three angles equal to pi, 10 of them on 4^3, times 3 components = 33.
    The mode u_x = (-1)^(j + k) is one of them; TETRA2 gives it energy."""
    plan = Plan((4, 4, 4), PERIODIC)
    one = np.ones((4, 4, 4))
    K = hex1.assemble_dense(plan, lambda *_: tetra2.element_tensor_iso(1.3, 0.7))
    ev = np.linalg.eigvalsh(K)
    count = sum(1 for t in itertools.product(range(4), repeat=3) if t == (0, 0, 0) or sum(v == 2 for v in t) >= 2)
    assert count == 11
    assert int(np.sum(np.abs(ev) < 1e-10 * np.abs(ev).max())) == 3 * count
    k, j, i = np.meshgrid(range(4), range(4), range(4), indexing="ij")
    u = np.zeros((3, 4, 4, 4)); u[0] = (-1.0) ** (j + k)
    assert np.abs(K @ u.ravel()).max() < 1e-12
    K2 = tetra2.assemble_dense(plan, lambda *_: tetra2.element_tensor_iso(1.3, 0.7))
    assert np.abs(K2 @ u.ravel()).max() > 0.1


def _null_projector(K, free):
    Kr = K[np.ix_(free, free)]
    w, V = np.linalg.eigh(Kr)
    Z = V[:, np.abs(w) < 1e-10 * np.abs(w).max()]
    return Z


@pytest.mark.parametrize("bc_kind", ["periodic", "mixed"])
def test_paux_green_inverts_the_assembled_hex1_reference(bc_kind):
    """Green.apply(2^b K0 u) = u off the null space, K0 assembled from HEX1 element matrices
    with the Paux tensor; the Green operator reads its symbol from a separate 4^3 assembly."""
    rng = np.random.default_rng(1)
    n = (4, 5, 6)
    if bc_kind == "periodic":
        bc = PERIODIC
    else:
        bc = rng.integers(0, 2, (3, 3, 2)).astype(np.int8)
    plan = Plan(n, bc)
    lam0, mu0 = 1.4, 0.9
    K0 = hex1.assemble_dense(plan, lambda *_: tetra2.element_tensor_paux(lam0, mu0))
    free = np.flatnonzero(~plan.amask.ravel())
    Z = _null_projector(K0, free)
    u = np.zeros(3 * int(np.prod(plan.N)))
    ur = rng.standard_normal(len(free))
    ur -= Z @ (Z.T @ ur)
    u[free] = ur
    v = (K0 @ u) * np.tile(plan.w2b.ravel(), 3)
    v[~np.isin(np.arange(len(u)), free)] = 0.0
    g = Green(plan, lam0, mu0, scheme="hex1")
    out = g.apply(v.reshape(3, *plan.w2b.shape))
    assert np.abs(out.ravel() - u).max() < 1e-10 * np.abs(u).max()


def test_iso_green_inverts_the_assembled_isotropic_reference():
    rng = np.random.default_rng(2)
    plan = Plan((4, 6, 5), PERIODIC)
    lam0, mu0 = 1.4, 0.9
    K0 = hex1.assemble_dense(plan, lambda *_: hex1.element_tensor_iso0(lam0, mu0))
    free = np.arange(K0.shape[0])
    Z = _null_projector(K0, free)
    u = rng.standard_normal(K0.shape[0])
    u -= Z @ (Z.T @ u)
    g = hex1.IsoGreenPeriodic(plan, lam0, mu0)
    out = g.apply((K0 @ u).reshape(3, *plan.w2b.shape))
    assert np.abs(out.ravel() - u).max() < 1e-10 * np.abs(u).max()
    # the isotropic medium couples the components; the Paux medium does not
    assert np.abs(K0[0:plan.w2b.size, plan.w2b.size:2 * plan.w2b.size]).max() > 0.1


def test_uniaxial_strain_exact_hex1():
    n = (4, 4, 6)
    nx, ny, nz = n
    lam = np.full((nz, ny, nx), 1.2); mu = np.full((nz, ny, nx), 0.8)
    bc = W.bc_table(W.BC_N)
    bc[0, 0, :] = W.BC_D; bc[1, 1, :] = W.BC_D; bc[2, 2, 0] = W.BC_D
    delta = 0.03
    top = np.stack(np.meshgrid(range(nx + 1), range(ny + 1), [nz], indexing="ij"), -1).reshape(-1, 3)
    strong = [W.Strong(top, np.full(len(top), 2, np.int8), np.full(len(top), delta))]
    s = Solver(n, lam, mu, bc, strong, r0_factor=1.0, scheme="hex1")
    out = s.solve(tol=1e-12, max_iter=3000)
    assert out["converged"]
    exact = s.zeros()
    exact[2] = delta * np.arange(nz + 1)[:, None, None] / nz
    # hourglass components are not fixed by these conditions: compare the centre gradients
    G = hex1.gradients(out["u"], s.plan)
    Ge = hex1.gradients(exact, s.plan)
    assert np.abs(G - Ge).max() < 1e-12
    szz = (1.2 + 1.6) * delta / nz
    assert abs(out["totals"][0, 2] - szz * nx * ny) < 1e-10 * szz * nx * ny


def _kkt_hex1(n, lam, mu, bc, strong, avg):
    """Dense eq (18)-(22) with the HEX1 stiffness."""
    plan = Plan(n, bc)
    K = hex1.assemble_dense(plan, lambda vx, vy, vz: tetra2.element_tensor_iso(lam[vz, vy, vx], mu[vz, vy, vx]))
    Nx, Ny, Nz = plan.N
    Nn = Nx * Ny * Nz
    free = np.flatnonzero(~plan.amask.ravel())
    pos = -np.ones(3 * Nn, np.int64); pos[free] = np.arange(len(free))
    rows, rhs = [], []
    for st in strong:
        for (i, j, k), c, v in zip(st.node, st.comp, st.value):
            r = np.zeros(len(free)); r[pos[int(c) * Nn + i + Nx * (j + Ny * k)]] = 1.0
            rows.append(r); rhs.append(v)
    for av in avg:
        for sup, c, v in zip(av.support, av.comp, av.value):
            r = np.zeros(len(free))
            for (i, j, k) in sup:
                r[pos[int(c) * Nn + i + Nx * (j + Ny * k)]] += 1.0 / len(sup)
            rows.append(r); rhs.append(v)
    A = np.array(rows)
    Kr = K[np.ix_(free, free)]
    m = len(rows)
    KKT = np.block([[Kr, A.T], [A, np.zeros((m, m))]])
    sol, *_ = np.linalg.lstsq(KKT, np.concatenate([np.zeros(len(free)), rhs]), rcond=1e-12)
    M = np.vstack([Kr, A])
    _, sv, Vt = np.linalg.svd(M)
    Zr = Vt[np.sum(sv > sv.max() * 1e-10):].T
    u = np.zeros(3 * Nn); u[free] = sol[:len(free)]
    Z = np.zeros((3 * Nn, Zr.shape[1])); Z[free] = Zr
    return u, Z


def _hex1_case():
    n = (4, 5, 4)
    rng = np.random.default_rng(4)
    nx, ny, nz = n
    lam = rng.uniform(0.5, 2, (nz, ny, nx)); mu = rng.uniform(0.4, 1.5, (nz, ny, nx))
    bc = W.bc_table(W.BC_N); bc[:, 2, 0] = W.BC_D
    strong = [W.Strong(np.array([[2, 2, nz], [1, 3, nz]]), np.array([2, 0], np.int8), np.array([-0.05, 0.02]))]
    sup = np.stack(np.meshgrid([1, 2], [1, 2], [1, 2], indexing="ij"), -1).reshape(1, 8, 3)
    face = np.stack(np.meshgrid([2, 3], [1, 2], [nz], indexing="ij"), -1).reshape(1, 4, 3)
    avg = [W.Average(sup, np.array([1], np.int8), np.array([0.03])),
           W.Average(face, np.array([2], np.int8), np.array([-0.04]), set_id=1)]
    return n, lam, mu, bc, strong, avg


def test_hex1_strong_point_conditions_stall_weak_conditions_converge():
    """Section 4.2.3: with HEX1, displacements applied strongly to single nodes excite
    hourglass modes and the iteration does not converge; applied weakly (voxel and face
    averages) it does."""
    n, lam, mu, bc, strong, avg = _hex1_case()
    out = Solver(n, lam, mu, bc, strong, [], r0_factor=1.0, scheme="hex1").solve(tol=1e-8, max_iter=1500)
    assert not out["converged"] and out["residual"] > 1e-3
    out = Solver(n, lam, mu, bc, [], avg, r0_factor=1.0, scheme="hex1").solve(tol=1e-8, max_iter=1500)
    assert out["converged"]
    # TETRA2 converges with the same strong conditions
    out = Solver(n, lam, mu, bc, strong, [], r0_factor=1.0).solve(tol=1e-8, max_iter=1500)
    assert out["converged"]


def test_fixed_point_hex1_equals_dense_kkt():
    """Average constraints with HEX1 (Section 4.2.3 applies weak conditions with HEX1): the
    converged fixed point solves eq (20) modulo the hourglass modes the constraints leave
    free."""
    n, lam, mu, bc, _, avg = _hex1_case()
    strong = []
    s = Solver(n, lam, mu, bc, strong, avg, r0_factor=1.0, scheme="hex1")
    out = s.solve(tol=1e-12, max_iter=6000)
    assert out["converged"]
    ud, Z = _kkt_hex1(n, lam, mu, bc, strong, avg)
    ui = kkt.project_off(out["u"], Z); ud = kkt.project_off(ud, Z)
    assert np.linalg.norm(ui - ud) <= 1e-9 * np.linalg.norm(ud)


def test_isotropic_and_paux_media_reach_the_same_solution():
    """The reference medium preconditions the iteration and does not move its fixed point: a
    periodic HEX1 cell (centrosymmetric, so that the solution has no component at the
    frequencies the Green operator drops), isotropic vs Paux medium."""
    outs = {}
    for ref in ("paux", "iso"):
        prob = W.periodic_centrosymmetric(n=(6, 6, 6), reference=ref)
        s = Solver.from_problem(prob)
        outs[ref] = s.solve(tol=1e-11, max_iter=3000)
        assert outs[ref]["converged"]
    Ga = hex1.gradients(outs["paux"]["u"], s.plan); Gb = hex1.gradients(outs["iso"]["u"], s.plan)
    assert np.abs(Ga - Gb).max() < 1e-8 * np.abs(Ga).max()
    assert np.abs(outs["paux"]["f_weak"] - outs["iso"]["f_weak"]).max() < 1e-8 * np.abs(outs["iso"]["f_weak"]).max()
    # the isotropic medium needs fewer iterations here (19 against 29 when measured)
    assert outs["iso"]["iterations"] < outs["paux"]["iterations"]


# -- isotropic medium under normal-mixed DTT boundaries ------------------------------------

def _normal_mixed_bc(normal):
    """normal[J][f]: the normal component's condition on face f of axis J (0 Neumann,
    1 Dirichlet); the two tangential components take the other one."""
    bc = np.zeros((3, 3, 2), np.int8)
    for J in range(3):
        for f in range(2):
            for c in range(3):
                bc[c, J, f] = normal[J][f] if c == J else 1 - normal[J][f]
    return bc


def _spectral_iso_green(plan, lam0, mu0, p):
    """An independent evaluation of the same Green operator: each component transformed by
    its own DTT (scipy), coefficients aligned on a common frequency index per axis, and per
    frequency the 3x3 symbol of the periodic medium, mu0 |d|^2 I + (lam0 + mu0) d d^T with
    d_J = 2 sin(theta_J / 2) prod_{K != J} cos(theta_K / 2), conjugated by the sign s_J = +1
    (normal component sine-type on axis J) or -1 (cosine-type): derivatives turn a cosine of
    the tangential components into a sine of the normal one with a minus sign, and back with a
    plus sign, so the coupling term of components i and j carries s_i s_j."""
    from oracle.green import forward_dt, inverse_dt
    n = plan.n
    kinds = [plan.types[J][J] for J in range(3)]
    th = [np.pi * np.arange(n[J] + 1) / n[J] if kinds[J] in ("DCT1", "DST1")
          else np.pi * (np.arange(n[J] + 1) + 0.5) / n[J] for J in range(3)]
    sgn = np.array([1.0 if kinds[J].startswith("DST") else -1.0 for J in range(3)])
    shape = tuple(n[J] + 1 for J in (2, 1, 0))
    X = np.zeros((3,) + shape)
    pos = []
    for c in range(3):
        coef = forward_dt(p[c], plan, c)
        sl = tuple(slice(1, n[J]) if plan.types[c][J] == "DST1" else slice(0, coef.shape[2 - J])
                   for J in (2, 1, 0))
        X[(c,) + sl] = coef
        pos.append(sl)
    tz, ty, tx = np.meshgrid(th[2], th[1], th[0], indexing="ij")
    t = [tx, ty, tz]
    d = np.stack([2 * np.sin(t[J] / 2) * np.prod([np.cos(t[K] / 2) for K in range(3) if K != J], axis=0)
                  for J in range(3)])
    d2 = (d * d).sum(0)
    Xs = sgn[:, None, None, None] * X
    dX = (d * Xs).sum(0)
    with np.errstate(divide="ignore", invalid="ignore"):
        U = (Xs - (lam0 + mu0) / (lam0 + 2 * mu0) * d * dX / d2) / (mu0 * d2)
    U[:, d2 < 1e-12] = 0.0
    U *= sgn[:, None, None, None]
    return np.stack([inverse_dt(U[(c,) + pos[c]], plan, c) for c in range(3)])


NM_INVERTIBLE = [[[1, 0], [0, 1], [1, 0]], [[0, 1], [1, 0], [1, 1]], [[1, 0], [1, 0], [0, 1]]]
NM_SINGULAR = [[[1, 1], [1, 1], [1, 1]], [[0, 0], [1, 1], [0, 0]]]


@pytest.mark.parametrize("normal", NM_INVERTIBLE)
def test_iso_green_dtt_matches_the_spectral_solve(normal):
    """Where the boundary-weighted operator is invertible (no hourglass line reaches the stored
    frequencies), its dense inverse and the transform-space solve agree to rounding (a missing
    sign conjugation fails here)."""
    plan = Plan((5, 4, 6), _normal_mixed_bc(normal))
    assert hex1.normal_mixed(plan)
    g = hex1.IsoGreenDTT(plan, 1.3, 0.7)
    assert np.linalg.matrix_rank(g.K) == g.K.shape[0]
    p = np.random.default_rng(5).standard_normal(g.shape)
    p[plan.amask] = 0.0
    a, b = g.apply(p), _spectral_iso_green(plan, 1.3, 0.7, p)
    assert np.abs(a - b).max() <= 1e-11 * np.abs(a).max()
    # the dense operator is the weighted reference term of the solver, not a transposed copy
    v = np.random.default_rng(6).standard_normal(g.shape); v[plan.amask] = 0.0
    s = Solver((5, 4, 6), np.ones((6, 4, 5)), np.ones((6, 4, 5)), _normal_mixed_bc(normal), scheme="hex1",
               reference="iso", lam0=1.3, mu0=0.7)
    q = -s.reference_term(hex1.gradients(v, plan))
    assert np.abs(g.K @ v.ravel()[g.idx] - q.ravel()[g.idx]).max() <= 1e-12 * np.abs(q).max()


@pytest.mark.parametrize("normal", NM_SINGULAR)
def test_iso_green_dtt_singular_boundaries_solve_in_the_range(normal):
    """With DCT1/DST1 axes the hourglass lines reach stored frequencies and the operator is
    singular; for a load in its range both solves satisfy K0 u = p."""
    plan = Plan((5, 4, 6), _normal_mixed_bc(normal))
    g = hex1.IsoGreenDTT(plan, 1.3, 0.7)
    assert np.linalg.matrix_rank(g.K) < g.K.shape[0]
    v = np.random.default_rng(7).standard_normal(g.idx.size)
    pf = g.K @ v
    p = np.zeros(g.shape); p.ravel()[g.idx] = pf
    for u in (g.apply(p), _spectral_iso_green(plan, 1.3, 0.7, p)):
        assert np.abs(g.K @ u.ravel()[g.idx] - pf).max() <= 1e-10 * np.abs(pf).max()


def test_normal_mixed_detection():
    assert not hex1.normal_mixed(Plan((4, 4, 4), PERIODIC))
    bc = _normal_mixed_bc([[1, 1], [1, 1], [1, 1]])
    assert hex1.normal_mixed(Plan((4, 4, 4), bc))
    bc[1, 0, 0] = 1                       # a tangential component fixed with the normal one
    assert not hex1.normal_mixed(Plan((4, 4, 4), bc))
