"""Pins of the finite-strain form (Section 5.2, eq 29, Algorithm 3; Saint-Venant-Kirchhoff law
of Section 5.4): objectivity, an exact homogeneous stretch worked out by hand, consistency
of the nodal forces with the stored energy, the small-strain limit, and contact."""
import numpy as np
import pytest

import workloads as W
from oracle import tetra2
from oracle.contact import ContactSolver
from oracle.solver import Solver

LAM, MU = 2.0, 3.0


def _block(n, bc=None, lam=LAM, mu=MU):
    nz, ny, nx = n[2], n[1], n[0]
    return (np.full((nz, ny, nx), lam), np.full((nz, ny, nx), mu),
            np.zeros((3, 3, 2), np.int8) if bc is None else bc)


def _coords(s):
    Nx, Ny, Nz = s.plan.N
    z, y, x = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    return np.stack([x, y, z]).astype(np.float64)


def test_rigid_rotation_is_stress_free():
    """A finite rigid rotation (30 degrees about a skew axis) has F = R, E = 0: no stress and no
    nodal force, where the small-strain law sees a large strain."""
    n = (4, 3, 5)
    lam, mu, bc = _block(n)
    a = np.array([1.0, 2.0, 2.0]) / 3.0
    th = np.pi / 6
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    R = np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K
    fs = Solver(n, lam, mu, bc, finite_strain=True)
    u = np.einsum("ij,jzyx->izyx", R - np.eye(3), _coords(fs))
    parts = fs.iterate_parts(u)
    assert parts["sig2"] < 1e-26 and parts["pnorm2"] < 1e-24
    ss = Solver(n, lam, mu, bc).iterate_parts(u)
    assert ss["sig2"] > 1.0


# Uniaxial strain F = diag(1, 1, 1 + e), e = 0.1, lam = 2, mu = 3:
#   E = diag(0, 0, e + e^2/2) = diag(0, 0, 0.105);  S = lam tr(E) I + 2 mu E
#   S_xx = S_yy = 2 * 0.105 = 0.21,  S_zz = (2 + 6) * 0.105 = 0.84
#   PK1 = F S:  P_xx = P_yy = 0.21,  P_zz = 1.1 * 0.84 = 0.924
P_XX, P_ZZ = 0.21, 0.924


def test_uniaxial_stretch_exact_solution():
    """Lateral rollers, bottom fixed, top nodes moved by e L: the homogeneous stretch is the
    exact discrete solution of the finite-strain problem, and the top reaction is P_zz per unit
    area (the hand values above)."""
    n = (3, 4, 5)
    nx, ny, nz = n
    bc = W.bc_table(W.BC_N)
    bc[0, 0, :] = W.BC_D; bc[1, 1, :] = W.BC_D; bc[2, 2, 0] = W.BC_D
    lam, mu, _ = _block(n)
    e = 0.1
    top = np.stack(np.meshgrid(range(nx + 1), range(ny + 1), [nz], indexing="ij"), -1).reshape(-1, 3)
    strong = [W.Strong(top, np.full(len(top), 2, np.int8), np.full(len(top), e * nz))]
    s = Solver(n, lam, mu, bc, strong, r0_factor=10.0, finite_strain=True)
    exact = s.zeros()
    exact[2] = e * np.arange(nz + 1)[:, None, None] * np.ones((nz + 1, ny + 1, nx + 1))
    parts = s.iterate_parts(exact)
    assert np.sqrt(parts["pnorm2"]) < 1e-13 * np.sqrt(parts["sig2"])
    ms = tetra2.mean_stress(parts["sig"])
    assert abs(ms[0, 0] - P_XX) < 1e-14 and abs(ms[1, 1] - P_XX) < 1e-14 and abs(ms[2, 2] - P_ZZ) < 1e-14
    out = s.solve(tol=1e-12, max_iter=3000)
    assert out["converged"]
    assert np.abs(out["u"] - exact).max() < 1e-11
    assert abs(out["totals"][0, 2] - P_ZZ * nx * ny) < 1e-10 * P_ZZ * nx * ny


def test_nodal_forces_are_minus_the_energy_gradient():
    """p / 2^b = -dW/du with W the Saint-Venant-Kirchhoff energy (central differences): pins the
    PK1 formula, its transposition and the divergence of a non-symmetric stress."""
    n = (2, 3, 2)
    rng = np.random.default_rng(5)
    nz, ny, nx = n[2], n[1], n[0]
    lam = rng.uniform(0.5, 2.0, (nz, ny, nx)); mu = rng.uniform(0.5, 2.0, (nz, ny, nx))
    s = Solver(n, lam, mu, np.zeros((3, 3, 2), np.int8), finite_strain=True)
    u = 0.2 * rng.standard_normal(s.zeros().shape)
    p = s.iterate_parts(u)["p"] / s.plan.w2b[None]

    def W_of(v):
        return tetra2.svk_energy(tetra2.tet_gradients(v, s.plan), lam, mu)

    h = 1e-6
    for idx in [(0, 0, 0, 0), (1, 1, 2, 1), (2, 2, 1, 2), (0, 1, 3, 2), (2, 0, 0, 1)]:
        up, um = u.copy(), u.copy()
        up[idx] += h; um[idx] -= h
        g = (W_of(up) - W_of(um)) / (2 * h)
        assert abs(p[idx] + g) < 1e-7 * max(1.0, abs(g))


def test_small_strain_limit():
    """PK1 of eps u over eps tends to the linear stress of u (F -> I)."""
    n = (3, 3, 3)
    rng = np.random.default_rng(6)
    lam, mu, bc = _block(n)
    fs = Solver(n, lam, mu, bc, finite_strain=True)
    ss = Solver(n, lam, mu, bc)
    u = rng.standard_normal(fs.zeros().shape)
    p_ss = ss.iterate_parts(u)["p"]
    for eps, bound in ((1e-3, 2e-2), (1e-5, 2e-4)):
        p_fs = fs.iterate_parts(eps * u)["p"] / eps
        assert np.abs(p_fs - p_ss).max() <= bound * np.abs(p_ss).max()


def test_finite_and_small_strain_contact_agree_at_small_depth():
    """Section 5.4: the two forms agree at small indentation depth and part as d/R grows.  The
    relative gap of the forces grows like the contact strain a/R = sqrt(d/R): measured 1.8 %
    at d/R = 0.002 and 12 % at 0.05 on this grid."""
    n = (24, 24, 12); R = 12.0
    prob = W.c3_indentation(n=n, R=R)
    out = {}
    for fs in (False, True):
        cs = ContactSolver(n, prob.lam, prob.mu, prob.bc, face=5, radius=R, r0_factor=10.0 if fs else 5.0,
                           finite_strain=fs)
        u = None
        forces = []
        for d_over_R in (0.002, 0.05):
            c = np.array([12.0, 12.0, 12 + R - d_over_R * R])
            o = cs.solve_increment(u, c, tol=1e-8, max_iter=4000)
            assert o["converged"]
            # contact KKT signs hold in both forms
            assert np.all(o["gap"][~o["C"]] >= -1e-9) and np.all(o["f_nc"][o["C"]] <= 1e-12)
            forces.append(o["force_mean_stress"])
            u = o["u"]
        out[fs] = forces
    small = abs(out[True][0] / out[False][0] - 1)
    large = abs(out[True][1] / out[False][1] - 1)
    assert small < 0.03
    assert large > 3 * small
