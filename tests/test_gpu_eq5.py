"""The GPU's equilibrium sums (eq 5) against the hand-derived closed forms of the oracle pins.

sums[0] = ||p||^2 (boundary-weighted residual after proj_P), sums[1] = sum over voxels and
both integration points of (1/2) sigma:sigma; expected values are the paper-and-pencil ones of
tests/test_oracle_eq5.py (no oracle call)."""
import numpy as np
import pytest

import workloads as W
from test_oracle_eq5 import CORNER_P, EPS, LAM, MU, SIG, SIG_SIG, _uniform_p2

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2607_26082_amd as F
    F.load()
    return F


def _block(F, n, prec, bc=None, strong=()):
    nz, ny, nx = n[2], n[1], n[0]
    lam = np.full((nz, ny, nx), LAM)
    mu = np.full((nz, ny, nx), MU)
    return F.Solver(n, lam, mu, np.zeros((3, 3, 2), np.int8) if bc is None else bc, strong, precision=prec)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-6)])
def test_uniform_strain_sums(prec, tol):
    F = _lib()
    n = (4, 3, 5)
    print(f"[eq5] uniform strain {n} {prec}", flush=True)
    g = _block(F, n, prec)
    Nx, Ny, Nz = g.N
    z, y, x = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    u = np.einsum("ij,jzyx->izyx", EPS, np.stack([x, y, z]).astype(np.float64))
    p, _, sums = g.stage_residual(u)
    assert abs(sums[1] - 60 * SIG_SIG) <= tol * 60 * SIG_SIG
    p2 = _uniform_p2(n, SIG)
    assert abs(sums[0] - p2) <= tol * p2
    assert np.abs(p[:, 5, 1, 1] + 2.0 * SIG[:, 2]).max() <= tol * np.abs(SIG).max()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-6)])
def test_corner_perturbation_sums(prec, tol):
    F = _lib()
    n = (3, 3, 3)
    print(f"[eq5] corner perturbation {n} {prec}", flush=True)
    g = _block(F, n, prec)
    u = np.zeros((3, 4, 4, 4))
    u[0, 0, 0, 0] = 1.0
    p, _, sums = g.stage_residual(u)
    assert abs(sums[1] - 13.5) <= tol * 13.5
    assert abs(sums[0] - 257.625) <= tol * 257.625
    for (i, j, k), val in CORNER_P.items():
        assert np.abs(p[:, k, j, i] - np.array(val)).max() <= tol * 14.0
    # strong DOF at the moved node: its p leaves the norm (proj_P before the test)
    g = _block(F, n, prec, strong=[W.Strong(np.array([[0, 0, 0]]), np.array([0], np.int8), np.array([1.0]))])
    _, _, sums = g.stage_residual(u)
    assert abs(sums[0] - (257.625 - 196.0)) <= tol * 257.625
