"""Pins of the equilibrium measure of eq (5) against values worked out by hand.

The measure is h ||div_D sigma|| / ||sigma|| with (reading of eq 5 and Section 3.1.2):
  ||sigma||^2 = sum over voxels and their two TETRA2 integration points of (1/2) sigma:sigma,
                sigma:sigma = sum_ij sigma_ij^2 (shear terms counted twice),
  ||div_D sigma||^2 = sum over free DOFs of p^2, p = 2^b x (nodal force summed over the
                in-cell voxels), b = number of non-periodic faces through the node.
Every expected number below was derived on paper from the definitions (P1 gradients of the
two tetrahedra, isotropic Hooke law, nodal force -(1/2) B^T sigma per tetrahedron); none is
produced by the oracle.  A change of the 1/2 integration-point weight, of the factor 2 on
the shear terms or of the 2^b boundary weight changes every one of them.
"""
import numpy as np
import pytest

from oracle.solver import Solver

LAM, MU = 2.0, 3.0


def _solver(n, bc=None):
    nz, ny, nx = n[2], n[1], n[0]
    lam = np.full((nz, ny, nx), LAM)
    mu = np.full((nz, ny, nx), MU)
    return Solver(n, lam, mu, np.zeros((3, 3, 2), np.int8) if bc is None else bc)


def _coords(s):
    Nx, Ny, Nz = s.plan.N
    z, y, x = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    return np.stack([x, y, z]).astype(np.float64)


# Uniform strain eps (symmetric, with a shear term) on a free 4x3x5 block:
#   tr = -0.5e-3;  sigma = lam tr I + 2 mu eps
#   sigma_xx = -1e-3 + 6e-3 = 5e-3,  sigma_yy = -1e-3 - 12e-3 = -13e-3,
#   sigma_zz = -1e-3 + 3e-3 = 2e-3,  sigma_xy = 6 * 0.7e-3 = 4.2e-3
#   sigma:sigma = (25 + 169 + 4 + 2 * 17.64) e-6 = 233.28e-6
EPS = np.array([[1.0e-3, 0.7e-3, 0.0], [0.7e-3, -2.0e-3, 0.0], [0.0, 0.0, 0.5e-3]])
SIG = np.array([[5.0e-3, 4.2e-3, 0.0], [4.2e-3, -13.0e-3, 0.0], [0.0, 0.0, 2.0e-3]])
SIG_SIG = 233.28e-6


def _uniform_p2(n, sig):
    """||p||^2 of a uniform stress on a free block: a boundary node's p is -2 sum over the
    faces through it of sigma.n_face (its 2^b weight times the in-cell nodal force); interior
    nodes carry none.  Summed by counting the nodes on each face, edge and corner."""
    total = 0.0
    nx, ny, nz = n
    for sx in (-1, 0, 1):
        for sy in (-1, 0, 1):
            for sz in (-1, 0, 1):
                if sx == sy == sz == 0:
                    continue
                cnt = (1 if sx else nx - 1) * (1 if sy else ny - 1) * (1 if sz else nz - 1)
                t = -2.0 * (sx * sig[:, 0] + sy * sig[:, 1] + sz * sig[:, 2])
                total += cnt * float(t @ t)
    return total


def test_uniform_strain_stress_norm_counts_both_points_with_weight_half_and_shear_twice():
    n = (4, 3, 5)
    s = _solver(n)
    u = np.einsum("ij,jzyx->izyx", EPS, _coords(s))
    parts = s.iterate_parts(u)
    assert abs(parts["sig2"] - 60 * SIG_SIG) <= 1e-15 * 60 * SIG_SIG * 10
    assert np.abs(SIG - (LAM * np.trace(EPS) * np.eye(3) + 2 * MU * EPS)).max() < 1e-16


def test_uniform_strain_residual_norm_carries_the_boundary_weight():
    n = (4, 3, 5)
    s = _solver(n)
    u = np.einsum("ij,jzyx->izyx", EPS, _coords(s))
    parts = s.iterate_parts(u)
    p2 = _uniform_p2(n, SIG)
    assert abs(parts["pnorm2"] - p2) <= 1e-12 * p2
    # a face node of the top face: p = -2 sigma.e_z, so the component x of the node (1,1,5)
    assert abs(parts["p"][:, 5, 1, 1] - (-2.0 * SIG[:, 2])).max() < 1e-17
    # an edge node (x = 4, y = 0): p = -2 (sigma.e_x - sigma.e_y)
    assert np.abs(parts["p"][:, 2, 0, 4] + 2.0 * (SIG[:, 0] - SIG[:, 1])).max() < 1e-17
    res = Solver.residual(parts["pnorm2"], parts["sig2"])
    assert abs(res - np.sqrt(p2) / np.sqrt(60 * SIG_SIG)) <= 1e-12 * res


# One corner node moved by delta = 1 along x on a free 3x3x3 block (lam = 2, mu = 3).
# Only tetrahedron T1 = {000, 110, 101, 011} of voxel 0 deforms; P1 gradients of its
# vertices: 000 (-1,-1,-1)/2, 110 (1,1,-1)/2, 101 (1,-1,1)/2, 011 (-1,1,1)/2.
#   grad u = e_x (x) (-1,-1,-1)/2;  eps_xx = -1/2, eps_xy = eps_xz = -1/4;  tr = -1/2
#   sigma = [[-4, -1.5, -1.5], [-1.5, -1, 0], [-1.5, 0, -1]];  sigma:sigma = 16+1+1+4*2.25 = 27
#   ||sigma||^2 = (1/2) 27 = 13.5 (one tetrahedron, weight 1/2)
# Nodal forces F_k = -(1/2) sigma grad(phi_k):
#   000: (-1.75, -0.625, -0.625)  corner, b = 3, p = 8 F = (-14, -5, -5)
#   110: ( 1,     0.625,  0.125)  face z = 0, b = 1, p = (2, 1.25, 0.25)
#   101: ( 1,     0.125,  0.625)  face y = 0, b = 1, p = (2, 0.25, 1.25)
#   011: (-0.25, -0.125, -0.125)  face x = 0, b = 1, p = (-0.5, -0.25, -0.25)
#   ||p||^2 = 246 + 5.625 + 5.625 + 0.375 = 257.625
CORNER_P = {(0, 0, 0): (-14.0, -5.0, -5.0), (1, 1, 0): (2.0, 1.25, 0.25),
            (1, 0, 1): (2.0, 0.25, 1.25), (0, 1, 1): (-0.5, -0.25, -0.25)}


def test_single_corner_node_perturbation_hand_values():
    n = (3, 3, 3)
    s = _solver(n)
    u = s.zeros()
    u[0, 0, 0, 0] = 1.0
    parts = s.iterate_parts(u)
    assert abs(parts["sig2"] - 13.5) < 1e-13
    assert abs(parts["pnorm2"] - 257.625) < 1e-12
    p = parts["p"]
    nz_nodes = {(i, j, k) for k, j, i in zip(*np.nonzero(np.abs(p).sum(axis=0) > 1e-14))}
    assert nz_nodes == set(CORNER_P)
    for (i, j, k), val in CORNER_P.items():
        assert np.abs(p[:, k, j, i] - np.array(val)).max() < 1e-14
    assert abs(Solver.residual(parts["pnorm2"], parts["sig2"]) - np.sqrt(257.625 / 13.5)) < 1e-13


def test_strong_constraint_and_dirichlet_face_leave_the_norm():
    """proj_P zeroes a constrained DOF before the norm (Algorithm 1 order), and a DOF held at
    0 by a Dirichlet face (antisymmetric extension) carries no equation: both drop out of
    ||p||^2 of the corner perturbation above."""
    from workloads import Strong
    n = (3, 3, 3)
    s = _solver(n)
    u = s.zeros()
    u[0, 0, 0, 0] = 1.0
    s2 = Solver(n, s.lam, s.mu, np.zeros((3, 3, 2), np.int8),
                strong=[Strong(node=np.array([[0, 0, 0]]), comp=np.array([0]), value=np.array([1.0]))])
    parts = s2.iterate_parts(u)
    assert abs(parts["pnorm2"] - (257.625 - 14.0 ** 2)) < 1e-12
    assert abs(parts["f_strong"][0] - 14.0 / 8.0) < 1e-14     # reaction -2^-b p = 1.75
    # u_y Dirichlet on the face z = 0: node 110 (b = 1 on z = 0) loses its y equation
    bc = np.zeros((3, 3, 2), np.int8)
    bc[1, 2, 0] = 1
    s3 = Solver(n, s.lam, s.mu, bc)
    parts = s3.iterate_parts(u)
    assert abs(parts["pnorm2"] - (257.625 - 1.25 ** 2 - 5.0 ** 2)) < 1e-12
