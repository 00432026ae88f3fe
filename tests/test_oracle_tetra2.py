"""Pins of the TETRA2 reading and of the reference-medium symbol."""
import numpy as np
import pytest

from oracle import dtt, green, kkt, tetra2
from oracle.plan import Plan


def test_p1_gradients_reproduce_linear_fields():
    rng = np.random.default_rng(0)
    plan = Plan((3, 4, 2), np.zeros((3, 3, 2), np.int8))
    A = rng.standard_normal((3, 3))
    b = rng.standard_normal(3)
    Nx, Ny, Nz = plan.N
    z, y, x = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    X = np.stack([x, y, z])
    u = np.einsum("ij,jzyx->izyx", A, X) + b[:, None, None, None]
    G = tetra2.tet_gradients(u, plan)
    for t in range(2):
        assert np.abs(G[t] - A[:, :, None, None, None]).max() < 1e-13


def test_tets_are_the_two_parity_classes_and_fill_a_third_of_the_voxel():
    for tet in tetra2.TETS:
        parity = {int(c.sum()) % 2 for c in tet}
        assert len(parity) == 1
        V = np.array([c for c in tet], float)
        vol = abs(np.linalg.det(V[1:] - V[0])) / 6.0
        assert abs(vol - 1.0 / 3.0) < 1e-14


def test_null_space_has_twelve_rigid_sublattice_modes():
    assert kkt.sublattice_nullity((3, 3, 3)) == 12
    assert kkt.sublattice_nullity((2, 3, 4)) == 12


def test_symbol_zeros_only_at_0_and_pi():
    st = green.stencil(1.3, 0.9)
    th = np.linspace(0, np.pi, 25)
    for c in range(3):
        M = green.symbol(st[c], th, th, th)
        zero = M < 1e-10 * M.max()
        idx = np.argwhere(zero)
        assert {tuple(i) for i in idx} == {(0, 0, 0), (24, 24, 24)}


def test_symbol_continuum_limit():
    """M_i(theta) ~ sum_j c_ij theta_j^2 with c_ij = 2 mu0 + lam0 delta_ij (Paux medium)."""
    lam0, mu0 = 1.7, 0.6
    st = green.stencil(lam0, mu0)
    rng = np.random.default_rng(3)
    for c in range(3):
        for _ in range(5):
            d = rng.standard_normal(3)
            eps = 1e-3
            t = eps * d
            M = green.symbol(st[c], [t[0]], [t[1]], [t[2]])[0, 0, 0]
            cj = np.array([2 * mu0 + lam0 * (j == c) for j in range(3)])
            assert abs(M / eps ** 2 - np.sum(cj * d * d)) < 1e-4 * np.sum(cj * d * d)


@pytest.mark.parametrize("seed", range(8))
def test_transform_diagonalises_boundary_weighted_operator(seed):
    """DT(2^b K0 u) = M DT(u) for random boundary mixes (the 2^b reading of eq 6)."""
    rng = np.random.default_rng(seed)
    n = tuple(int(v) for v in rng.integers(3, 7, 3))
    bc = rng.integers(0, 2, (3, 3, 2)).astype(np.int8)
    if seed == 0:
        bc[:, 1, :] = 2
    plan = Plan(n, bc)
    lam0, mu0 = rng.uniform(0.5, 2, 2)
    u = rng.standard_normal((3,) + tuple(plan.N[J] for J in (2, 1, 0)))
    u[plan.amask] = 0.0
    G = tetra2.tet_gradients(u, plan)
    K0u = -plan.w2b[None] * tetra2.divergence(tetra2.paux(G, lam0, mu0), plan)
    K0u[plan.amask] = 0.0
    st = green.stencil(lam0, mu0)
    for c in range(3):
        th = [dtt.thetas(plan.types[c][J], plan.n[J]) for J in range(3)]
        M = green.symbol(st[c], *th)
        lhs = green.forward_dt(K0u[c], plan, c)
        rhs = M * green.forward_dt(u[c], plan, c)
        assert np.abs(lhs - rhs).max() < 1e-13 * np.abs(rhs).max()


def test_divergence_matches_dense_assembly():
    """-div_D(C:grad u) from the stress path equals K u from element-matrix assembly."""
    rng = np.random.default_rng(11)
    n = (3, 4, 3)
    bc = rng.integers(0, 3, (3, 3, 2)).astype(np.int8)
    bc[:, 1, :] = 2
    bc[:, 0, :] = np.where(bc[:, 0, :] == 2, 0, bc[:, 0, :])
    bc[:, 2, :] = np.where(bc[:, 2, :] == 2, 1, bc[:, 2, :])
    plan = Plan(n, bc)
    nx, ny, nz = n
    lam = rng.uniform(0, 2, (nz, ny, nx)); mu = rng.uniform(0.1, 2, (nz, ny, nx))
    u = rng.standard_normal((3,) + tuple(plan.N[J] for J in (2, 1, 0)))
    F = -tetra2.divergence(tetra2.stress(tetra2.tet_gradients(u, plan), lam, mu), plan)
    K = kkt.assemble_physical(plan, lam, mu)
    assert np.abs(F.ravel() - K @ u.ravel()).max() < 1e-12 * np.abs(F).max()


def test_uniform_stress_gives_face_traction_times_area():
    """Nodal forces of a uniform sigma_zz on the top face sum to sigma_zz * area."""
    plan = Plan((4, 3, 2), np.zeros((3, 3, 2), np.int8))
    s = np.zeros((2, 3, 3, 2, 3, 4)); s[:, 2, 2] = 1.7
    F = -tetra2.divergence(s, plan)
    assert abs(F[2, -1].sum() - 1.7 * 12) < 1e-13
    assert abs(F[2].sum()) < 1e-13
