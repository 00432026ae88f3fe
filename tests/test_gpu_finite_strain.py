"""GPU parity of the finite-strain form (Section 5.2, eq 29, Algorithm 3; Saint-Venant-Kirchhoff
PK1 of Section 5.4) through the C ABI, against the FP64 oracle pinned in
tests/test_oracle_finite_strain.py."""
import numpy as np
import pytest

import workloads as W
from oracle.contact import ContactSolver
from oracle.solver import Solver as OSolver
from test_oracle_finite_strain import P_ZZ

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2607_26082_amd as F
    F.load()
    return F


SHAPES = [((6, 5, 9), None), ((16, 12, 10), 1), ((32, 48, 6), None), ((24, 20, 18), 0)]


@pytest.mark.parametrize("idx", range(len(SHAPES)))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_stage_residual_finite_strain(idx, prec):
    F = _lib()
    n, per = SHAPES[idx]
    print(f"[fs stage] n={n} periodic={per} {prec}", flush=True)
    rng = np.random.default_rng(80 + idx)
    nx, ny, nz = n
    lam = rng.uniform(0.3, 3, (nz, ny, nx)); mu = rng.uniform(0.2, 2, (nz, ny, nx))
    bc = rng.integers(0, 2, (3, 3, 2)).astype(np.int8)
    if per is not None:
        bc[:, per, :] = 2
    o = OSolver(n, lam, mu, bc, r0_factor=1.3, finite_strain=True)
    g = F.Solver(n, lam, mu, bc, r0_factor=1.3, precision=prec, finite_strain=True)
    u = rng.standard_normal(o.zeros().shape) * 0.1          # gradients of order 0.2: nonlinear
    u[o.plan.amask] = 0.0
    parts = o.iterate_parts(u)
    p, pt, sums = g.stage_residual(u)
    tol = 1e-12 if prec == "fp64" else 2e-5
    assert np.abs(p - parts["p"]).max() <= tol * np.abs(parts["p"]).max()
    assert np.abs(pt - parts["ptil"]).max() <= tol * np.abs(parts["ptil"]).max()
    assert abs(sums[0] - parts["pnorm2"]) <= 10 * tol * parts["pnorm2"]
    assert abs(sums[1] - parts["sig2"]) <= 10 * tol * parts["sig2"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_uniaxial_stretch_finite_strain(prec):
    """The homogeneous stretch e = 0.1 is the exact solution; the top reaction is P_zz per
    unit area (hand value 0.924 for lam = 2, mu = 3)."""
    F = _lib()
    n = (6, 8, 10)
    nx, ny, nz = n
    print(f"[fs stretch] {prec}", flush=True)
    bc = W.bc_table(W.BC_N)
    bc[0, 0, :] = W.BC_D; bc[1, 1, :] = W.BC_D; bc[2, 2, 0] = W.BC_D
    lam = np.full((nz, ny, nx), 2.0); mu = np.full((nz, ny, nx), 3.0)
    e = 0.1
    top = np.stack(np.meshgrid(range(nx + 1), range(ny + 1), [nz], indexing="ij"), -1).reshape(-1, 3)
    strong = [W.Strong(top, np.full(len(top), 2, np.int8), np.full(len(top), e * nz))]
    g = F.Solver(n, lam, mu, bc, strong, r0_factor=10.0, precision=prec, tol=1e-12 if prec == "fp64" else 1e-6,
                 max_iter=4000, finite_strain=True)
    rc, rep = g.solve()
    assert rc == 0
    exact = np.zeros((3, nz + 1, ny + 1, nx + 1))
    exact[2] = e * np.arange(nz + 1)[:, None, None]
    tol = 1e-11 if prec == "fp64" else 1e-5
    u = g.u.cpu().numpy()
    assert np.abs(u - exact).max() <= tol * e * nz
    _, _, tot = g.reactions()
    assert abs(tot[0, 2] - P_ZZ * nx * ny) <= tol * 10 * P_ZZ * nx * ny
    assert abs(rep.mean_stress[2] - P_ZZ) <= tol * 10 * P_ZZ


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_contact_increments_finite_strain(prec):
    """Algorithm 3 on the top face, three warm-started increments up to d/R = 0.03: active sets
    bit-exact, displacements (FP64 1e-10 at tol 1e-12; FP32 at 1e-6 against the oracle at
    1e-11: 1e-5) and the contact force against the oracle."""
    F = _lib()
    n = (32, 32, 16); R = 12.0
    print(f"[fs contact] {prec}", flush=True)
    prob = W.c3_indentation(n=n, R=R, finite_strain=True)
    cs = ContactSolver(n, prob.lam, prob.mu, prob.bc, face=5, radius=R, r0_factor=10.0, finite_strain=True)
    sph = W.Sphere(np.array([16.0, 16.0, 16 + R]), R, 5)
    g = F.Solver(n, prob.lam, prob.mu, prob.bc, sphere=sph, r0_factor=10.0, precision=prec,
                 tol=1e-6 if prec == "fp32" else 1e-12, max_iter=4000, finite_strain=True)
    u_o = None
    for k, dr in enumerate((0.01, 0.02, 0.03)):
        c = np.array([16.0, 16.0, 16 + R - dr * R])
        o = cs.solve_increment(u_o, c, tol=1e-12 if prec == "fp64" else 1e-11, max_iter=4000)
        assert o["converged"]
        u_o = o["u"]
        g.move_sphere(c)
        rc, rep = g.solve(zero_start=(k == 0))
        assert rc == 0
        mask, fnc, gap = g.contact()
        assert np.array_equal(mask.reshape(-1).astype(bool), o["C"])
        u = g.u.cpu().numpy()
        tol = 1e-10 if prec == "fp64" else 1e-5
        err = np.linalg.norm(u - o["u"]) / np.linalg.norm(o["u"])
        print(f"[fs contact] d/R {dr} iterations {rep.iterations} (oracle {o['iterations']}) rel-L2 {err:.2e}",
              flush=True)
        assert err <= tol
        assert abs(rep.force_mean_stress - o["force_mean_stress"]) <= (1e-8 if prec == "fp64" else 1e-4) * abs(
            o["force_mean_stress"])
        assert abs(rep.force_contact - rep.force_mean_stress) <= 1e-3 * abs(rep.force_mean_stress)


def test_rigid_rotation_stress_free_on_gpu():
    F = _lib()
    n = (8, 6, 5)
    nx, ny, nz = n
    lam = np.full((nz, ny, nx), 2.0); mu = np.full((nz, ny, nx), 3.0)
    g = F.Solver(n, lam, mu, np.zeros((3, 3, 2), np.int8), precision="fp64", finite_strain=True)
    th = 0.4
    R = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    z, y, x = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    u = np.einsum("ij,jzyx->izyx", R - np.eye(3), np.stack([x, y, z]).astype(np.float64))
    p, _, sums = g.stage_residual(u)
    assert np.abs(p).max() < 1e-13 and sums[1] < 1e-26
