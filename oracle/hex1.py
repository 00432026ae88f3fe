"""HEX1 scheme and the isotropic reference medium with its coupled Green operator.

Paper, Section 3.1.2 (discrete operators: the HEX1 scheme evaluates the gradient of the
trilinear interpolant at the voxel centre, one integration point of weight 1 per voxel),
eq (4) and Section 3.2.3 (the Green operator of a reference medium; an isotropic medium
couples the three components, so its symbol is a full 3x3 matrix per frequency), Section
3.2.4 (periodic axes with complex transforms), and Section 4.2.3 (HEX1 has hourglass modes:
displacement fields with zero centre gradient in every voxel).

  gradient at the centre:  G = sum over the 8 corners of u_corner (x) B_corner,
                           B_(a,b,c) = (2a - 1, 2b - 1, 2c - 1) / 4   (h = 1)
  nodal force:             F_node = - sum over the voxels around it of B^T sigma
  isotropic medium:        sigma0 = lam0 tr(G) I + mu0 (G + G^T)

The isotropic Green operator is built here only for cells periodic on all three axes, with
numpy's complex FFT (a library primitive) and, per frequency, the pseudo-inverse of the 3x3
symbol M_ij(theta) = sum_delta c^ij_delta e^{i theta . delta} read off the assembled K0 (no
closed form).  Frequencies where M is singular (theta = 0 and the hourglass lines) get 0.
"""
from __future__ import annotations

import itertools

import numpy as np

from .plan import Plan

CORNERS = [np.array(c) for c in itertools.product((0, 1), repeat=3)]
B = np.array([(2 * c - 1) / 4.0 for c in CORNERS])      # [8, 3]


def _padded(u, plan):
    out = u
    for J in range(3):
        if plan.periodic[J]:
            ax = u.ndim - 1 - J
            out = np.concatenate([out, np.take(out, [0], axis=ax)], axis=ax)
    return out


def _fold(F, plan):
    for J in range(3):
        if plan.periodic[J]:
            ax = F.ndim - 1 - J
            n = plan.n[J]
            last = [slice(None)] * F.ndim
            last[ax] = slice(n, n + 1)
            first = [slice(None)] * F.ndim
            first[ax] = slice(0, 1)
            F[tuple(first)] += F[tuple(last)]
            keep = [slice(None)] * F.ndim
            keep[ax] = slice(0, n)
            F = F[tuple(keep)]
    return F


def gradients(u, plan):
    """Centre gradient G[i][j] = d u_i / d x_j of every voxel, shape [1, 3, 3, nz, ny, nx] (one
    integration point; the leading axis keeps the layout of the two-point scheme)."""
    up = _padded(u, plan)
    nx, ny, nz = plan.n
    G = np.zeros((1, 3, 3, nz, ny, nx))
    for k, (a, b, c) in enumerate(CORNERS):
        uc = up[..., c:c + nz, b:b + ny, a:a + nx]
        for j in range(3):
            G[0, :, j] += B[k, j] * uc
    return G


def divergence(s, plan):
    """Nodal divergence -sum B^T s over the voxels inside the cell, [3, Nz, Ny, Nx]."""
    nx, ny, nz = plan.n
    F = np.zeros((3,) + tuple(plan.n[J] + 1 for J in (2, 1, 0)))
    for k, (a, b, c) in enumerate(CORNERS):
        contrib = np.zeros((3, nz, ny, nx))
        for j in range(3):
            contrib += B[k, j] * s[0, :, j]
        F[:, c:c + nz, b:b + ny, a:a + nx] += contrib
    return -_fold(F, plan)


def stress_norm2(sig):
    """sum over voxels of sigma:sigma (one integration point of weight 1)."""
    return float(np.sum(sig * sig))


def mean_stress(sig):
    return sig.sum(axis=(0, 3, 4, 5)) / sig[0, 0, 0].size


def iso(G, lam0, mu0):
    """Isotropic reference flux lam0 tr(G) I + mu0 (G + G^T)."""
    out = mu0 * (G + np.swapaxes(G, 1, 2))
    tr = G[:, 0, 0] + G[:, 1, 1] + G[:, 2, 2]
    for i in range(3):
        out[:, i, i] += lam0 * tr
    return out


def assemble_dense(plan, tensor_of_voxel):
    """Dense HEX1 stiffness over all 3 Nnode DOFs: K = sum_v B^T C_v B (weight 1)."""
    nx, ny, nz = plan.n
    Nx, Ny, Nz = plan.N
    Nn = Nx * Ny * Nz
    K = np.zeros((3 * Nn, 3 * Nn))
    for vz in range(nz):
        for vy in range(ny):
            for vx in range(nx):
                C = tensor_of_voxel(vx, vy, vz)
                nodes = [((vx + c[0]) % Nx) + Nx * (((vy + c[1]) % Ny) + Ny * ((vz + c[2]) % Nz)) for c in CORNERS]
                Ke = np.einsum("ka,iajb,lb->kilj", B, C, B)
                for k in range(8):
                    for l in range(8):
                        for i in range(3):
                            K[i * Nn + nodes[k], np.arange(3) * Nn + nodes[l]] += Ke[k, i, l, :]
    return K


def element_tensor_iso0(lam0, mu0):
    d = np.eye(3)
    return (lam0 * np.einsum("ia,jb->iajb", d, d)
            + mu0 * (np.einsum("ij,ab->iajb", d, d) + np.einsum("ib,aj->iajb", d, d)))


def iso_stencil(lam0, mu0):
    """c[delta][i][j]: row of node 0 of the assembled isotropic HEX1 K0 on a 4^3 periodic grid."""
    plan = Plan((4, 4, 4), np.full((3, 3, 2), 2, np.int8))
    K = assemble_dense(plan, lambda *_: element_tensor_iso0(lam0, mu0))
    Nn = 64
    st = {}
    for node in range(Nn):
        blk = np.array([[K[i * Nn + 0, j * Nn + node] for j in range(3)] for i in range(3)])
        if np.abs(blk).max() > 0.0:
            i, j, k = node % 4, (node // 4) % 4, node // 16
            st[tuple(v if v < 2 else v - 4 for v in (i, j, k))] = blk
    return st


def normal_mixed(plan):
    """True when no axis is periodic and on every face the normal displacement component and
    the two tangential ones have opposite symmetries (one held at 0, the others free): then
    the transform of each component (Table 2) also diagonalises the coupled isotropic operator
    (Section 3.2.3), frequency by frequency."""
    if any(plan.periodic):
        return False
    for J in range(3):
        for f in range(2):
            for c in range(3):
                if c != J and plan.sym[c, J, f] == plan.sym[J, J, f]:
                    return False
    return True


class IsoGreenDTT:
    """Green operator of the isotropic HEX1 reference medium under normal-mixed boundaries,
    taken from its definition: K0 = 2^b times the in-cell isotropic HEX1 stiffness on the DOFs
    that are not held at 0 (the boundary-weighted reference operator of eq 3), assembled as a
    dense matrix column by column, and its pseudo-inverse (the operator vanishes on the
    hourglass lines).  Small grids only (dense)."""

    def __init__(self, plan, lam0, mu0):
        if not normal_mixed(plan):
            raise ValueError("the isotropic Green operator needs periodic or normal-mixed boundaries")
        self.plan = plan
        self.shape = (3,) + tuple(plan.N[J] for J in (2, 1, 0))
        self.idx = np.flatnonzero(~plan.amask.ravel())
        K = np.zeros((self.idx.size, self.idx.size))
        for col, e in enumerate(self.idx):
            u = np.zeros(self.shape)
            u.ravel()[e] = 1.0
            q = -plan.w2b[None] * divergence(iso(gradients(u, plan), lam0, mu0), plan)
            K[:, col] = q.ravel()[self.idx]
        self.K = K
        self.Kinv = np.linalg.pinv(K, rcond=1e-11)

    def apply(self, p):
        u = np.zeros(self.shape)
        u.ravel()[self.idx] = self.Kinv @ p.ravel()[self.idx]
        return u


class IsoGreenPeriodic:
    """u_hat = M(theta)^+ p_hat per frequency, complex FFT over a fully periodic cell."""

    def __init__(self, plan, lam0, mu0):
        if not all(plan.periodic):
            raise ValueError("the isotropic Green operator needs periodic axes")
        self.plan = plan
        nx, ny, nz = plan.n
        st = iso_stencil(lam0, mu0)
        tz, ty, tx = np.meshgrid(2 * np.pi * np.fft.fftfreq(nz), 2 * np.pi * np.fft.fftfreq(ny),
                                 2 * np.pi * np.fft.fftfreq(nx), indexing="ij")
        M = np.zeros(tz.shape + (3, 3), complex)
        for (dx, dy, dz), blk in st.items():
            M += np.exp(1j * (dx * tx + dy * ty + dz * tz))[..., None, None] * blk
        w, V = np.linalg.eigh(M)
        scale = np.abs(w).max()
        winv = np.where(w > 1e-12 * scale, 1.0 / np.where(w > 1e-12 * scale, w, 1.0), 0.0)
        self.Minv = np.einsum("...ik,...k,...jk->...ij", V, winv, V.conj())

    def apply(self, p):
        ph = np.stack([np.fft.fftn(p[c]) for c in range(3)], -1)
        uh = np.einsum("...ij,...j->...i", self.Minv, ph)
        return np.stack([np.fft.ifftn(uh[..., c]).real for c in range(3)])
