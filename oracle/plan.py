"""Boundary table -> symmetries, transform types, eliminated DOFs, boundary weights.

Paper, Section 3.2.1, Table 1: for component i on face S_J^alpha a Dirichlet
condition extends u_i antisymmetrically (A, so u_i vanishes on the face), a
Neumann condition extends it symmetrically (S), periodicity (P) pairs the two
faces.  Table 2 then gives the transform of each (component, axis).

Reading used for the residual at boundary nodes (paper eq 6 puts
sigma = C:eps only inside the cell and extends sigma by the symmetries of
Table 1): the divergence of the extended stress at a node that lies on b
non-periodic faces equals 2^b times the sum over the voxels inside the cell,
for every component that is not eliminated there.  Components with an A
extension on a face through the node are eliminated (held at 0, no equation).
"""
from __future__ import annotations

import numpy as np

from .dtt import SYM_TO_TYPE

BC_N, BC_D, BC_P = 0, 1, 2


class Plan:
    def __init__(self, n, bc):
        self.n = tuple(int(v) for v in n)
        bc = np.asarray(bc, dtype=np.int8).reshape(3, 3, 2)
        self.bc = bc
        self.periodic = []
        for J in range(3):
            isp = bc[:, J, :] == BC_P
            if isp.any() and not isp.all():
                raise ValueError(f"axis {J}: periodicity must hold on both faces for all components")
            self.periodic.append(bool(isp.all()))
        # node counts per axis (x, y, z)
        self.N = tuple(self.n[J] + (0 if self.periodic[J] else 1) for J in range(3))
        self.sym = np.empty((3, 3, 2), dtype="<U1")
        for c in range(3):
            for J in range(3):
                for f in range(2):
                    self.sym[c, J, f] = {BC_N: "S", BC_D: "A", BC_P: "P"}[int(bc[c, J, f])]
        self.types = [[SYM_TO_TYPE[(self.sym[c, J, 0], self.sym[c, J, 1])] for J in range(3)]
                      for c in range(3)]
        Nx, Ny, Nz = self.N
        # eliminated (A) DOFs, shape [3, Nz, Ny, Nx]
        self.amask = np.zeros((3, Nz, Ny, Nx), dtype=bool)
        for c in range(3):
            for J in range(3):
                if self.periodic[J]:
                    continue
                for f in range(2):
                    if self.sym[c, J, f] == "A":
                        idx = [slice(None)] * 3
                        idx[2 - J] = 0 if f == 0 else self.n[J]
                        self.amask[(c,) + tuple(idx)] = True
        # number of non-periodic faces through each node
        self.b = np.zeros((Nz, Ny, Nx), dtype=np.int64)
        for J in range(3):
            if self.periodic[J]:
                continue
            for f in range(2):
                idx = [slice(None)] * 3
                idx[2 - J] = 0 if f == 0 else self.n[J]
                self.b[tuple(idx)] += 1
        self.w2b = 2.0 ** self.b            # boundary weight 2^b

    def node_index(self, ijk):
        """Flat node index i + Nx (j + Ny k) of integer triples [..., 3]."""
        ijk = np.asarray(ijk, dtype=np.int64)
        Nx, Ny, _ = self.N
        return ijk[..., 0] + Nx * (ijk[..., 1] + Ny * ijk[..., 2])

    def selection_slices(self, c):
        """Per axis (x, y, z), the node index range kept by the transform of component c."""
        from .dtt import selection
        return [selection(self.types[c][J], self.n[J]) for J in range(3)]
