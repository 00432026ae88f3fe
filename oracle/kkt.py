"""Direct solves of the constrained minimisation problems (plain definitions).

Paper, Section 4.3, eq (18)-(23): the converged fixed point solves
min 1/2 u^T K u subject to A u = U, i.e. the saddle-point system
[K A^T; A 0][u; f] = [0; U], where K is assembled over the voxels of the
cell, u holds every DOF not eliminated by an antisymmetric extension, A holds
unit rows for strong constraints (eq 21) and 1/k rows for average relations
(eq 22).  Smoothly applied conditions (eq 23) replace A^T by a distribution
matrix B: the system [K B; A 0] is no longer symmetric.  Section 5.5, eq
(31)-(33) adds unilateral contact.

Sign convention: `reaction` returned here is the force the constraint applies
to the body, K u = B f (the paper's eq 8 convention, f = -lambda of eq 19),
reported per constraint as the total force sum(B column) f.  Remaining free modes of [K; A] (rigid sub-lattice motions left free
by the boundary conditions) are reported as an orthonormal basis Z so that a
caller can compare displacements modulo that span.
"""
from __future__ import annotations

import numpy as np

from .plan import Plan
from .relations import relations_from
from .tetra2 import assemble_dense, element_tensor_iso


def assemble_physical(plan, lam, mu):
    return assemble_dense(plan, lambda vx, vy, vz: element_tensor_iso(lam[vz, vy, vx], mu[vz, vy, vx]))


def dense_kkt(n, lam, mu, bc, strong=(), average=(), smooth=()):
    plan = Plan(n, bc)
    Nx, Ny, Nz = plan.N
    Nn = Nx * Ny * Nz
    K = assemble_physical(plan, np.asarray(lam), np.asarray(mu))
    free = ~plan.amask.reshape(-1)                # DOF = comp * Nn + node
    fidx = np.flatnonzero(free)
    pos = -np.ones(3 * Nn, np.int64)
    pos[fidx] = np.arange(len(fidx))
    Kr = K[np.ix_(fidx, fidx)]
    rows, cols, rhs = [], [], []
    for s in strong:
        node = np.asarray(s.node, np.int64).reshape(-1, 3)
        for (i, j, k), c, v in zip(node, s.comp, s.value):
            dof = int(c) * Nn + i + Nx * (j + Ny * k)
            if pos[dof] < 0:
                continue                           # eliminated DOF with value 0
            r = np.zeros(len(fidx)); r[pos[dof]] = 1.0
            rows.append(r); cols.append(r); rhs.append(float(v))
    for rel in relations_from(plan, average, smooth):
        r = np.zeros(len(fidx)); bcol = np.zeros(len(fidx))
        for node, wa, wb in zip(rel.nodes, rel.a, rel.b):
            r[pos[rel.comp * Nn + int(node)]] += wa
            bcol[pos[rel.comp * Nn + int(node)]] += wb
        rows.append(r); cols.append(bcol); rhs.append(rel.value)
    A = np.array(rows).reshape(-1, len(fidx))
    B = np.array(cols).reshape(-1, len(fidx)).T
    U = np.array(rhs)
    m = A.shape[0]
    KKT = np.block([[Kr, B], [A, np.zeros((m, m))]])
    b = np.concatenate([np.zeros(len(fidx)), U])
    sol, *_ = np.linalg.lstsq(KKT, b, rcond=1e-13)
    ur, lam_mult = sol[:len(fidx)], sol[len(fidx):]
    total = B.sum(axis=0) if m else np.zeros(0)
    # free modes: null space of [Kr; A]
    M = np.vstack([Kr, A]) if m else Kr
    _, sv, Vt = np.linalg.svd(M)
    tolz = sv.max() * 1e-10
    Zr = Vt[np.sum(sv > tolz):].T
    u = np.zeros(3 * Nn)
    u[fidx] = ur
    Z = np.zeros((3 * Nn, Zr.shape[1]))
    Z[fidx] = Zr
    return dict(u=u.reshape(3, Nz, Ny, Nx), reaction=-lam_mult * total, Z=Z, K=K, plan=plan,
                residual=np.abs(KKT @ sol - b).max())


def project_off(u, Z):
    """Remove the components of u along the orthonormal columns of Z."""
    v = u.reshape(-1)
    if Z.shape[1] == 0:
        return v.copy()
    return v - Z @ (Z.T @ v)


def sublattice_nullity(n, lam=1.0, mu=1.0):
    """Dimension of the null space of K on a free block (all faces Neumann)."""
    plan = Plan(n, np.zeros((3, 3, 2), np.int8))
    nx, ny, nz = plan.n
    K = assemble_physical(plan, np.full((nz, ny, nx), lam), np.full((nz, ny, nx), mu))
    ev = np.linalg.eigvalsh(K)
    return int(np.sum(np.abs(ev) < 1e-9 * np.abs(ev).max()))
