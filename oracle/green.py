"""Reference medium, its discrete symbol, and the Green solve of eq (3)/(4).

Paper, eq (3): the new displacement solves div_D(R0 : grad_D u) = -p, i.e.
K0 u = p with K0 the (positive) stiffness of the homogeneous reference medium.
Section 3.2.3: for non-periodic boundaries the reference medium of Paux et al.
is used; it acts on each displacement component separately, so its symbol is
a diagonal 3x3 matrix M(theta) per frequency, and Section 3.2.3 applies the
Green operator only at the frequencies selected by eq (7).

Reading of eq (4) (sign and normalisation garbled in the extraction):
u_hat = M(theta)^-1 p_hat, where M is the symbol of K0.  M is computed here
independently of any closed form: K0 is assembled from element matrices on a
small periodic grid, the row of one node is read off as a stencil c_delta,
and M(theta) = sum_delta c_delta cos(theta . delta).  Where M vanishes
(theta = 0 and theta = (pi, pi, pi) for components transformed by DCT1/DFT on
all three axes) the Green operator is set to 0 (the paper assumes enough
Dirichlet conditions for these modes not to be excited).
"""
from __future__ import annotations

import numpy as np

from . import dtt, hex1, tetra2
from .plan import Plan
from .tetra2 import element_tensor_paux


def reference_from_factor(lam, mu, factor):
    """Reading for heterogeneous media: (lam0, mu0) = factor * (max lam, max mu)."""
    return factor * float(np.max(lam)), factor * float(np.max(mu))


def stencil(lam0, mu0, scheme="tetra2"):
    """Stencil {delta: coefficient} of each component of the assembled Paux K0 of a scheme."""
    plan = Plan((4, 4, 4), np.full((3, 3, 2), 2, np.int8))       # 4^3 periodic
    assemble = tetra2.assemble_dense if scheme == "tetra2" else hex1.assemble_dense
    K = assemble(plan, lambda *_: element_tensor_paux(lam0, mu0))
    Nn = 64
    out = []
    for c in range(3):
        row = K[c * Nn + 0]
        # no coupling between components for this reference medium
        for c2 in range(3):
            if c2 != c:
                assert np.abs(row[c2 * Nn:(c2 + 1) * Nn]).max() < 1e-12 * np.abs(row).max()
        st = {}
        r = row[c * Nn:(c + 1) * Nn]
        for node in range(Nn):
            if r[node] != 0.0:
                i, j, k = node % 4, (node // 4) % 4, node // 16
                d = tuple(v if v < 2 else v - 4 for v in (i, j, k))
                st[d] = r[node]
        out.append(st)
    return out


def symbol(st, th_x, th_y, th_z):
    """M(theta) = sum_delta c_delta cos(theta . delta) on the grid th_z x th_y x th_x.

    The stencil rows sum to zero (rigid translations are in the null space of K0), so the
    same value is evaluated as -2 sum_delta c_delta sin^2(theta . delta / 2), which avoids
    the cancellation of the O(1) terms at low frequencies."""
    tz, ty, tx = np.meshgrid(th_z, th_y, th_x, indexing="ij")
    M = np.zeros(tz.shape)
    for (dx, dy, dz), cval in st.items():
        if (dx, dy, dz) == (0, 0, 0):
            continue
        M -= 2.0 * cval * np.sin(0.5 * (dx * tx + dy * ty + dz * tz)) ** 2
    return M


def forward_dt(field_c, plan, c):
    """Forward transform of one component: select S_R on each axis, transform x, y, z."""
    sel = plan.selection_slices(c)
    a = field_c[np.ix_(sel[2], sel[1], sel[0])]
    for J in range(3):
        a = dtt.forward(a, plan.types[c][J], 2 - J, plan.n[J])
    return a


def inverse_dt(coef, plan, c):
    """Inverse transform of one component back onto the node grid (eliminated nodes = 0)."""
    a = coef
    for J in (2, 1, 0):
        a = dtt.inverse(a, plan.types[c][J], 2 - J, plan.n[J])
    out = np.zeros(tuple(plan.N[J] for J in (2, 1, 0)))
    sel = plan.selection_slices(c)
    out[np.ix_(sel[2], sel[1], sel[0])] = a
    return out


class Green:
    def __init__(self, plan, lam0, mu0, scheme="tetra2"):
        self.plan = plan
        st = stencil(lam0, mu0, scheme)
        self.Minv = []
        for c in range(3):
            th = [dtt.thetas(plan.types[c][J], plan.n[J]) for J in range(3)]
            M = symbol(st[c], th[0], th[1], th[2])
            scale = np.abs(M).max()
            Minv = np.zeros_like(M)
            nz = M > 1e-12 * scale
            Minv[nz] = 1.0 / M[nz]
            self.Minv.append(Minv)
        self.stencils = st

    def apply(self, p):
        """u = DT^-1( M^-1 DT(p) ) per component (eq 3, right part)."""
        u = np.zeros_like(p)
        for c in range(3):
            u[c] = inverse_dt(forward_dt(p[c], self.plan, c) * self.Minv[c], self.plan, c)
        return u
