"""TETRA2 finite-difference scheme: per-voxel gradients at two integration points.

Paper, Section 3.1.1 and Figure 1: every voxel carries two integration points
at its centre; at each one the displacement gradient is the gradient of the
linear interpolant on one of the two tetrahedra formed by voxel corners.
The scheme itself is deferred by the paper to other work; the reading used
here (the paper's "two symmetric tetrahedra", "two decoupled sub-grids",
Section 4.2.3) is:

  T1 = corners {000, 110, 101, 011},  T2 = corners {100, 010, 001, 111}

(corner abc = offset (a, b, c) from the voxel origin), each tetrahedron with
the P1 (linear) gradient, integration weight 1/2 each, h = 1.  Each
tetrahedron only links nodes of equal parity i+j+k, which yields the two
decoupled sub-grids the paper describes.

The nodal divergence of an element stress field is minus the transpose of the
gradient: div_D(s)[node] = - sum over voxels, tets containing the node of
(1/2) * B_t[node]^T s_t.  With unit voxels this is the nodal force balance of
the paper's eq (3), and gives nodal forces whose sum over a face equals the
traction times the face area.
"""
from __future__ import annotations

import itertools

import numpy as np

CORNERS = [np.array(c) for c in itertools.product((0, 1), repeat=3)]   # (a, b, c) = (dx, dy, dz)
T1 = [c for c in CORNERS if c.sum() % 2 == 0]
T2 = [c for c in CORNERS if c.sum() % 2 == 1]
TETS = (T1, T2)
IP_WEIGHT = 0.5


def p1_gradients(vertices):
    """Gradients of the four linear basis functions of a tetrahedron.

    Solves [1 x y z] a = e_k for each vertex k; the gradient of basis k is
    (a_1, a_2, a_3).  Returns B with B[k] = grad(phi_k)."""
    V = np.array([[1.0, *v] for v in vertices])
    coef = np.linalg.inv(V)            # column k: coefficients of phi_k
    return coef[1:, :].T.copy()        # [4, 3]


TET_B = [p1_gradients(t) for t in TETS]


def _padded(u, plan):
    """Node field [..., Nz, Ny, Nx] -> array with n_J + 1 entries on every axis
    (periodic axes get a copy of node 0 appended), so voxel v has corners v and v+1."""
    out = u
    for J in range(3):
        if plan.periodic[J]:
            ax = u.ndim - 1 - J
            first = np.take(out, [0], axis=ax)
            out = np.concatenate([out, first], axis=ax)
    return out


def _fold(F, plan):
    """Inverse of _padded for accumulated nodal sums: add the appended plane to node 0."""
    for J in range(3):
        if plan.periodic[J]:
            ax = F.ndim - 1 - J
            n = plan.n[J]
            sl_last = [slice(None)] * F.ndim
            sl_last[ax] = slice(n, n + 1)
            sl_first = [slice(None)] * F.ndim
            sl_first[ax] = slice(0, 1)
            F[tuple(sl_first)] += F[tuple(sl_last)]
            keep = [slice(None)] * F.ndim
            keep[ax] = slice(0, n)
            F = F[tuple(keep)]
    return F


def corner_view(up, corner, plan):
    a, b, c = corner
    nx, ny, nz = plan.n
    return up[..., c:c + nz, b:b + ny, a:a + nx]


def tet_gradients(u, plan):
    """Displacement gradients G[t][i][j] = d u_i / d x_j on every voxel, t in {T1, T2}.
    Returns an array [2, 3, 3, nz, ny, nx]."""
    up = _padded(u, plan)
    nx, ny, nz = plan.n
    G = np.zeros((2, 3, 3, nz, ny, nx))
    for t, tet in enumerate(TETS):
        B = TET_B[t]
        for k, corner in enumerate(tet):
            uc = corner_view(up, corner, plan)          # [3, nz, ny, nx]
            for j in range(3):
                if B[k, j] != 0.0:
                    G[t, :, j] += B[k, j] * uc
    return G


def divergence(s, plan):
    """Nodal divergence of an element field s[t][i][j] (2 IPs per voxel), summed
    over the voxels inside the cell only: returns -sum (1/2) B^T s, shape [3, Nz, Ny, Nx]."""
    nx, ny, nz = plan.n
    shp = tuple(plan.n[J] + 1 for J in (2, 1, 0))
    F = np.zeros((3,) + shp)
    for t, tet in enumerate(TETS):
        B = TET_B[t]
        for k, corner in enumerate(tet):
            a, b, c = corner
            contrib = np.zeros((3, nz, ny, nx))
            for j in range(3):
                if B[k, j] != 0.0:
                    contrib += B[k, j] * s[t, :, j]
            F[:, c:c + nz, b:b + ny, a:a + nx] += IP_WEIGHT * contrib
    return -_fold(F, plan)


def stress(G, lam, mu):
    """Isotropic linear elasticity at each IP: sigma = lam tr(eps) I + 2 mu eps, eps = sym(G)."""
    eps = 0.5 * (G + np.swapaxes(G, 1, 2))
    tr = eps[:, 0, 0] + eps[:, 1, 1] + eps[:, 2, 2]
    sig = 2.0 * mu[None, None, None] * eps
    for i in range(3):
        sig[:, i, i] += lam[None] * tr
    return sig


def stress_svk(G, lam, mu):
    """Finite strain (Section 5.2, eq 29; the example law of Section 5.4): first Piola-Kirchhoff
    stress PK1 = F S of the Saint-Venant-Kirchhoff law at each IP, with F = I + grad u,
    Green-Lagrange strain E = (F^T F - I) / 2 and S = lam tr(E) I + 2 mu E.
    Returns the non-symmetric PK1[t][i][J] (row i: component, column J: material direction),
    the layout `divergence` takes."""
    I = np.eye(3)[None, :, :, None, None, None]
    F = I + G
    E = 0.5 * (np.einsum("tkaxyz,tkbxyz->tabxyz", F, F) - I)
    tr = E[:, 0, 0] + E[:, 1, 1] + E[:, 2, 2]
    S = 2.0 * mu[None, None, None] * E
    for i in range(3):
        S[:, i, i] += lam[None] * tr
    return np.einsum("tikxyz,tkjxyz->tijxyz", F, S)


def svk_energy(G, lam, mu):
    """Stored energy of the Saint-Venant-Kirchhoff law summed over voxels and both IPs with
    weight 1/2: W = sum (1/2) (lam/2 tr(E)^2 + mu E:E).  Its derivative with respect to the
    nodal displacements is minus the nodal force of PK1 (used to pin stress_svk)."""
    I = np.eye(3)[None, :, :, None, None, None]
    F = I + G
    E = 0.5 * (np.einsum("tkaxyz,tkbxyz->tabxyz", F, F) - I)
    tr = E[:, 0, 0] + E[:, 1, 1] + E[:, 2, 2]
    w = 0.5 * lam[None] * tr ** 2 + mu[None] * np.sum(E * E, axis=(1, 2))
    return float(IP_WEIGHT * np.sum(w))


def paux(G, lam0, mu0):
    """Reference-medium flux of Paux et al. (Section 3.2.3): R0:grad u = lam0 (grad u o I) + 2 mu0 grad u,
    with o the entrywise product, on the full (non-symmetric) gradient."""
    out = 2.0 * mu0 * G
    for i in range(3):
        out[:, i, i] += lam0 * G[:, i, i]
    return out


def stress_norm2(sig):
    """sum over voxels and IPs of (1/2) sigma:sigma (h = 1); the same measure of PK1 in the
    finite-strain form (all nine components)."""
    return float(IP_WEIGHT * np.sum(sig * sig))


def mean_stress(sig):
    """Volume average <sigma> over the cell, [3, 3]."""
    nvox = sig[0, 0, 0].size
    return IP_WEIGHT * sig.sum(axis=(0, 3, 4, 5)) / nvox


# ---------------------------------------------------------------------------
# Independent element-matrix assembly (used for the direct KKT solves and the symbol)
# ---------------------------------------------------------------------------

def element_tensor_iso(lam, mu):
    """C_{iajb} of isotropic elasticity (acts on full gradients, symmetrised by construction)."""
    d = np.eye(3)
    return (lam * np.einsum("ia,jb->iajb", d, d)
            + mu * (np.einsum("ij,ab->iajb", d, d) + np.einsum("ib,aj->iajb", d, d)))


def element_tensor_paux(lam0, mu0):
    """R0_{iajb} of the Paux reference medium: (lam0 delta_ia + 2 mu0) delta_ij delta_ab."""
    d = np.eye(3)
    return np.einsum("ij,ab->iajb", d, d) * (2.0 * mu0 + lam0 * d)[:, :, None, None]


def assemble_dense(plan, tensor_of_voxel):
    """Dense stiffness over all 3*Nnode DOFs (DOF = comp * Nnode + node):
    K = sum_v sum_t (1/2) B_t^T C_v B_t.  `tensor_of_voxel(vx, vy, vz)` returns C_{iajb}."""
    nx, ny, nz = plan.n
    Nx, Ny, Nz = plan.N
    Nn = Nx * Ny * Nz
    K = np.zeros((3 * Nn, 3 * Nn))
    for vz in range(nz):
        for vy in range(ny):
            for vx in range(nx):
                C = tensor_of_voxel(vx, vy, vz)
                for t, tet in enumerate(TETS):
                    B = TET_B[t]
                    nodes = [((vx + c[0]) % Nx) + Nx * (((vy + c[1]) % Ny) + Ny * ((vz + c[2]) % Nz))
                             for c in tet]
                    Ke = IP_WEIGHT * np.einsum("ka,iajb,lb->kilj", B, C, B)   # [4,3,4,3]
                    for k in range(4):
                        for l in range(4):
                            for i in range(3):
                                K[i * Nn + nodes[k], np.arange(3) * Nn + nodes[l]] += Ke[k, i, l, :]
    return K
