"""Pins of the oracle's Algorithm 2 (unilateral contact): KKT conditions, fixed-zone solve, force identity."""
import numpy as np
import pytest
from scipy.optimize import least_squares

import workloads as W
from oracle import kkt
from oracle.contact import ContactSolver, hertz_force, hertz_radius


def _small(n=(8, 8, 4), R=5.0, d=0.15):
    prob = W.c3_indentation(n=n, R=R)
    cs = ContactSolver(n, prob.lam, prob.mu, prob.bc, face=5, radius=R, r0_factor=5.0)
    center = np.array([n[0] / 2, n[1] / 2, n[2] + R - d])
    return prob, cs, center


def test_contact_kkt_conditions_and_force_identity():
    prob, cs, center = _small()
    out = cs.solve_increment(None, center, tol=1e-11, max_iter=4000)
    assert out["converged"] and out["contact_nodes"] > 0
    C, g, f = out["C"], out["gap"], out["f_nc"]
    R = cs.radius
    assert np.abs(g[C]).max() < 1e-12 * R              # g = 0 on C
    assert g[~C].min() >= 0.0                           # g >= 0 off C
    assert f[C].max() <= 0.0                            # compressive reactions on C
    # eq (33) complementarity: no force off C (free nodes balanced to the tolerance)
    p, sig, s2, _ = cs.stress_residual(out["u"])
    pface = p.reshape(3, -1)[:, cs.face_nodes]
    assert np.abs(pface[:, ~C]).max() < 1e-9 * np.abs(pface[:, C]).max()
    # Section 5.4: F = A0 <sigma_zz> equals the sum of contact reactions
    assert abs(out["force_mean_stress"] - out["force_contact"]) < 1e-9 * out["force_contact"]


def test_fixed_zone_matches_direct_nonlinear_solve():
    """With the converged active set fixed, solve eq (27) directly: equilibrium off C,
    zero tangential force and zero gap on C (dense least squares on the assembled K)."""
    prob, cs, center = _small(n=(6, 6, 3), R=4.0, d=0.2)
    out = cs.solve_increment(None, center, tol=1e-12, max_iter=4000)
    assert out["converged"]
    C = out["C"]
    plan = cs.plan
    K = kkt.assemble_physical(plan, prob.lam, prob.mu)
    free = np.flatnonzero(~plan.amask.reshape(-1))
    Nn = np.prod(plan.N)
    cnodes = cs.face_nodes[C]
    Xc = cs.X[C]
    cdofs = np.concatenate([c * Nn + cnodes for c in range(3)])
    other = np.setdiff1d(free, cdofs)

    def resid(x):
        u = np.zeros(3 * Nn); u[free] = x
        F = K @ u
        U = u.reshape(3, -1)[:, cnodes].T
        dvec = Xc + U - center
        r = np.linalg.norm(dvec, axis=1)
        nc = -dvec / r[:, None]
        Fc = F.reshape(3, -1)[:, cnodes].T
        tang = Fc - np.sum(Fc * nc, 1)[:, None] * nc
        return np.concatenate([F[other], tang.ravel(), r - cs.radius])

    sol = least_squares(resid, np.zeros(len(free)), xtol=1e-15, ftol=1e-15, gtol=1e-15)
    u_direct = np.zeros(3 * Nn); u_direct[free] = sol.x
    assert np.abs(resid(sol.x)).max() < 1e-12
    assert np.linalg.norm(out["u"].ravel() - u_direct) < 1e-8 * np.linalg.norm(u_direct)


def test_hertz_closed_form_values():
    """Eq (30) with E* = E/(1-nu^2): spot values for R = 96 (E = 1, nu = 0.3)."""
    R = 96.0
    for dR, F, a in [(0.002, 1.20777, 4.2933), (0.010, 13.50330, 9.6000), (0.020, 38.19309, 13.5765)]:
        d = dR * R
        assert abs(hertz_force(1.0, 0.3, R, d) - F) < 1e-4
        assert abs(hertz_radius(R, d) - a) < 1e-4


@pytest.mark.slow
def test_small_indentation_tracks_hertz():
    n = (48, 48, 24); R = 18.0
    prob = W.c3_indentation(n=n, R=R)
    cs = ContactSolver(n, prob.lam, prob.mu, prob.bc, face=5, radius=R, r0_factor=5.0)
    u = None
    for k in (1, 2):
        d = 0.01 * k * R
        out = cs.solve_increment(u, np.array([24.0, 24.0, 24 + R - d]), tol=1e-6)
        u = out["u"]
        assert out["converged"]
        assert abs(out["force_contact"] / hertz_force(1.0, 0.3, R, d) - 1) < 0.2
