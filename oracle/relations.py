"""Kinematic relations on several nodes: averages and smoothly applied conditions.

Paper, Section 4.2.1 (eq 10-14: a displacement prescribed to the mean of the 8 corners of a
voxel or the 4 corners of a face; Section 4.2.3 uses the same equations on V*, the 44 nodes of
a line of ten voxels), Section 4.2.2 (eq 15-17, Table 2: a displacement prescribed at one node
whose reaction is spread over the neighbouring nodes) and Section 4.3 (eq 22-23: both are
linear equality constraints, the second with a force-distribution matrix B that differs from
the transpose of the constraint matrix A).

A relation on component c has a support S (a list of nodes) and three weight vectors on S:
  a  its kinematic row:             a . u_S = U                         (eq 10, eq 15)
  b  the distribution of its multiplier onto nodal forces (a column of B in eq 23; A^T for
     an average)                                                          (eq 12, eq 16)
  d  the direction along which proj_U moves u_S to satisfy the row
Average over k nodes: a = 1/k, b = d = 1.  Smooth condition at node i0: a = d = e_i0 and
b = 1 at i0, the Table 2 weight at each neighbour.
  proj_U:  u_S += d (U - a . u_S) / (a . d)                             (eq 11, eq 15)
  proj_P:  on the physical residual q = 2^-b p:  f = (a . q) / (a . b),  q_S -= b f
           (eq 14: f is the mean and is removed from every node; eq 17: f = q_i0, which
           zeroes q_i0 and adds w (-f) at each neighbour)
The reaction reported for a relation is the total force it applies, -f sum(b): for an average
minus the sum of the support's residuals, for a smooth condition (1 + sum w) times the node's
multiplier -q_i0, i.e. 8 (volume) or 4 (surface) times it (Section 4.2.2).

Reading where the paper is silent: a smooth condition is defined for a node on no
non-periodic face (volume, 26 neighbours) or on exactly one (surface, the 8 neighbours in the
face plane); a node on an edge or corner of the cell is rejected, and so is a support that
reaches a DOF held at 0 by a Dirichlet face or that overlaps another constraint.
"""
from __future__ import annotations

import itertools

import numpy as np

# Table 2 weights, keyed by the number of non-zero offsets of the neighbour from i0
VOLUME_WEIGHTS = {1: 0.5, 2: 0.25, 3: 0.125}     # middle of faces, middle of edges, corners
SURFACE_WEIGHTS = {1: 0.5, 2: 0.25}              # middle of edges, corners (in the face plane)


class Relation:
    __slots__ = ("comp", "nodes", "a", "b", "d", "value", "set_id")

    def __init__(self, comp, nodes, a, b, d, value, set_id):
        self.comp = int(comp)
        self.nodes = np.asarray(nodes, np.int64)
        self.a = np.asarray(a, np.float64)
        self.b = np.asarray(b, np.float64)
        self.d = np.asarray(d, np.float64)
        self.value = float(value)
        self.set_id = int(set_id)


def average_relation(plan, support_ijk, comp, value, set_id=0):
    """Mean of u[comp] over the support nodes equals value (eq 10; V* of Section 4.2.3)."""
    flat = plan.node_index(np.asarray(support_ijk, np.int64).reshape(-1, 3))
    k = len(flat)
    return Relation(comp, flat, np.full(k, 1.0 / k), np.ones(k), np.ones(k), value, set_id)


def smooth_support(plan, ijk):
    """Neighbours of node ijk and their Table 2 weights: ([(i, j, k)], [w]), centre excluded.
    Volume node: the 26 nodes of the 2x2x2-voxel cell around it; surface node (one
    non-periodic face): the 8 nodes of the 2x2 face cell around it in the face plane."""
    ijk = [int(v) for v in ijk]
    faces = [J for J in range(3) if not plan.periodic[J] and ijk[J] in (0, plan.n[J])]
    if len(faces) > 1:
        raise ValueError("smooth condition on an edge or corner node of the cell")
    axes = [J for J in range(3) if J not in faces]
    weights = VOLUME_WEIGHTS if not faces else SURFACE_WEIGHTS
    nbr, w = [], []
    for off in itertools.product((-1, 0, 1), repeat=len(axes)):
        nz = sum(o != 0 for o in off)
        if nz == 0:
            continue
        q = list(ijk)
        for J, o in zip(axes, off):
            x = q[J] + o
            if plan.periodic[J]:
                x %= plan.N[J]
            elif x < 0 or x > plan.n[J]:
                raise ValueError("smooth support leaves the cell")
            q[J] = x
        nbr.append(tuple(q))
        w.append(weights[nz])
    return nbr, w


def smooth_relation(plan, ijk, comp, value, set_id=0):
    """Displacement value prescribed at node ijk, reaction spread by Table 2 (eq 15-17)."""
    nbr, w = smooth_support(plan, ijk)
    nodes = plan.node_index(np.array([tuple(int(v) for v in ijk)] + nbr, np.int64))
    k = len(nodes)
    a = np.zeros(k)
    a[0] = 1.0
    b = np.concatenate([[1.0], w])
    return Relation(comp, nodes, a, b, a.copy(), value, set_id)


def relations_from(plan, average=(), smooth=()):
    rel = []
    for av in average:
        sup = np.asarray(av.support, np.int64).reshape(len(av.comp), -1, 3)
        for r in range(sup.shape[0]):
            rel.append(average_relation(plan, sup[r], av.comp[r], av.value[r], av.set_id))
    for sm in smooth:
        node = np.asarray(sm.node, np.int64).reshape(-1, 3)
        for r in range(node.shape[0]):
            rel.append(smooth_relation(plan, node[r], sm.comp[r], sm.value[r], sm.set_id))
    return rel


def check_relations(plan, rel, strong_keys=()):
    """Raises on a support DOF held at 0 by a Dirichlet face, or on DOFs shared by two
    constraints (the projections are exact only for disjoint supports)."""
    amask = plan.amask.reshape(3, -1)
    used = set(int(k) for k in strong_keys)
    Nn = amask.shape[1]
    for r in rel:
        if amask[r.comp, r.nodes].any():
            raise ValueError("relation support holds a DOF eliminated by a Dirichlet face")
        keys = {r.comp * Nn + int(n) for n in r.nodes}
        if len(keys) != len(r.nodes) or used & keys:
            raise ValueError("overlapping constraint supports")
        used |= keys


def proj_U(u, rel):
    uf = u.reshape(3, -1)
    for r in rel:
        cur = uf[r.comp, r.nodes]
        uf[r.comp, r.nodes] = cur + r.d * (r.value - r.a @ cur) / (r.a @ r.d)
    return u


def proj_P(p, rel, w2b):
    """Projects p in place; returns the total reaction of every relation."""
    pf = p.reshape(3, -1)
    out = np.zeros(len(rel))
    for k, r in enumerate(rel):
        wb = w2b[r.nodes]
        q = pf[r.comp, r.nodes] / wb
        f = (r.a @ q) / (r.a @ r.b)
        pf[r.comp, r.nodes] = (q - r.b * f) * wb
        out[k] = -f * r.b.sum()
    return out
