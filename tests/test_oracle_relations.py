"""Pins of the relations on several nodes: smoothly applied conditions (Section 4.2.2, eq 15-17,
Table 2), averages over a line of voxels (Section 4.2.3) and the non-symmetric saddle-point
system of eq (23)."""
import numpy as np
import pytest

import workloads as W
from oracle import kkt, relations
from oracle.plan import Plan
from oracle.solver import Solver


def _box(xs, ys, zs):
    g = np.stack(np.meshgrid(np.asarray(xs), np.asarray(ys), np.asarray(zs), indexing="ij"), -1)
    return g.reshape(-1, 3)


def test_table2_weights_and_totals():
    """Table 2: volume w_ME = 1/4, w_MF = 1/2, w_Co = 1/8 over 12 + 6 + 8 neighbours; surface
    w_ME = 1/2, w_Co = 1/4 over 4 + 4; total reaction 8 f and 4 f (Section 4.2.2)."""
    plan = Plan((4, 4, 4), np.zeros((3, 3, 2), np.int8))
    nbr, w = relations.smooth_support(plan, (2, 2, 2))
    assert len(nbr) == 26
    for q, wq in zip(nbr, w):
        nz = sum(int(q[J] != 2) for J in range(3))
        assert wq == {1: 0.5, 2: 0.25, 3: 0.125}[nz]
    assert sorted(w).count(0.25) == 12 and sorted(w).count(0.5) == 6 and sorted(w).count(0.125) == 8
    assert 1.0 + sum(w) == 8.0
    nbr, w = relations.smooth_support(plan, (2, 1, 4))          # top face z = 4
    assert len(nbr) == 8 and all(q[2] == 4 for q in nbr)
    assert sorted(w) == [0.25] * 4 + [0.5] * 4
    assert 1.0 + sum(w) == 4.0
    with pytest.raises(ValueError):
        relations.smooth_support(plan, (0, 2, 4))                # edge node
    # periodic axis: the support wraps, the node on x = 0 is a volume node
    bc = np.zeros((3, 3, 2), np.int8); bc[:, 0, :] = 2
    plan = Plan((4, 4, 4), bc)
    nbr, w = relations.smooth_support(plan, (0, 2, 2))
    assert len(nbr) == 26 and {q[0] for q in nbr} == {0, 1, 3}


def _problem(n, seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    lam = rng.uniform(0.5, 2.5, (nz, ny, nx)); mu = rng.uniform(0.4, 1.6, (nz, ny, nx))
    bc = W.bc_table(W.BC_N); bc[:, 2, 0] = W.BC_D                 # bottom face fixed
    return lam, mu, bc


RCASES = {
    "smooth_volume": dict(smooth=[W.Smooth(np.array([[2, 2, 3]]), np.array([2], np.int8), np.array([-0.05]))]),
    "smooth_surface": dict(smooth=[W.Smooth(np.array([[2, 3, 5]]), np.array([2], np.int8), np.array([-0.04]))],
                           strong=[W.Strong(np.array([[1, 1, 2]]), np.array([0], np.int8), np.array([0.01]))]),
    "smooth_two_comps": dict(smooth=[W.Smooth(np.array([[2, 2, 3], [4, 2, 3]]), np.array([0, 1], np.int8),
                                              np.array([0.03, -0.02]), set_id=1)]),
    "line_of_voxels": dict(average=[W.Average(_box(range(0, 6), [2, 3], [3, 4])[None], np.array([2], np.int8),
                                              np.array([-0.03]))]),
    "mixed": dict(average=[W.Average(_box([1, 2], [1, 2], [1, 2])[None], np.array([1], np.int8), np.array([0.02]))],
                  smooth=[W.Smooth(np.array([[3, 3, 5]]), np.array([2], np.int8), np.array([-0.03]), set_id=1)]),
}


@pytest.mark.parametrize("name", sorted(RCASES))
def test_fixed_point_solves_eq23(name):
    """The converged iteration of Algorithm 1 with the projections of eq 11/14/15/17 solves the
    saddle-point system with B != A^T (eq 23); the reported reactions are its total forces."""
    n = (5, 5, 5) if name != "line_of_voxels" else (5, 5, 6)
    lam, mu, bc = _problem(n, 7)
    kw = RCASES[name]
    strong, avg, sm = kw.get("strong", []), kw.get("average", []), kw.get("smooth", [])
    s = Solver(n, lam, mu, bc, strong, avg, r0_factor=1.0, smooth=sm)
    out = s.solve(tol=1e-13, max_iter=6000)
    assert out["converged"]
    d = kkt.dense_kkt(n, lam, mu, bc, strong, avg, sm)
    assert d["Z"].shape[1] == 0
    assert np.linalg.norm(out["u"] - d["u"]) <= 1e-9 * np.linalg.norm(d["u"])
    f = np.concatenate([out["f_strong"], out["f_weak"]])
    assert np.abs(f - d["reaction"]).max() <= 1e-9 * np.abs(d["reaction"]).max()
    uf = out["u"].reshape(3, -1)
    for rel in s.cons.rel:
        assert abs(rel.a @ uf[rel.comp, rel.nodes] - rel.value) < 1e-15


def test_line_of_voxels_is_one_mean_over_44_nodes():
    """Section 4.2.3: the ten voxels (0.5:9.5, 24.5, 24.5) of the CT-like specimen hold 44 nodes;
    the reading is one relation, the mean over those 44 nodes."""
    plan = Plan((10, 50, 50), np.zeros((3, 3, 2), np.int8))
    sup = _box(range(0, 11), [24, 25], [24, 25])
    rel = relations.average_relation(plan, sup, 1, -0.1)
    assert len(rel.nodes) == 44 and len(set(rel.nodes.tolist())) == 44
    assert np.allclose(rel.a, 1 / 44) and np.all(rel.b == 1.0)


def test_smooth_condition_loads_both_sublattices():
    """A strong condition on one node loads one TETRA2 sub-lattice only (Section 4.2.3, Figure 5
    right); spreading its reaction over the 26 neighbours (eq 16) loads both."""
    n = (8, 8, 8)
    nx, ny, nz = n
    lam = np.full((nz, ny, nx), 1.0); mu = np.full((nz, ny, nx), 1.0)
    bc = W.bc_table(W.BC_N); bc[:, 2, 0] = W.BC_D
    node = np.array([[4, 4, 4]])
    runs = {}
    for kind in ("strong", "smooth"):
        kw = {"strong": [W.Strong(node, np.array([2], np.int8), np.array([0.1]))]} if kind == "strong" else \
             {"smooth": [W.Smooth(node, np.array([2], np.int8), np.array([0.1]))]}
        s = Solver(n, lam, mu, bc, kw.get("strong", []), r0_factor=1.0, smooth=kw.get("smooth", []))
        runs[kind] = s.solve(tol=1e-10, max_iter=4000)["u"]
    k, j, i = np.meshgrid(range(9), range(9), range(9), indexing="ij")
    par = (i + j + k) % 2 == 0
    for kind, u in runs.items():
        same = np.abs(u[2][par]).max()
        other = np.abs(u[2][~par]).max()
        if kind == "strong":
            assert other < 1e-8 * same
        else:
            assert other > 0.3 * same


def test_smooth_and_weak_give_similar_iteration_counts():
    """Section 4.2.3 reports the same iteration count (332) for a condition applied smoothly at a
    node and weakly at the centre of the voxel next to it (a trend, checked within 25 %)."""
    n = (10, 10, 10)
    lam, mu, bc = _problem(n, 3)
    sm = [W.Smooth(np.array([[4, 4, 5]]), np.array([2], np.int8), np.array([-0.05]))]
    av = [W.Average(_box([4, 5], [4, 5], [5, 6])[None], np.array([2], np.int8), np.array([-0.05]))]
    a = Solver(n, lam, mu, bc, r0_factor=1.0, smooth=sm).solve(tol=1e-8, max_iter=4000)
    b = Solver(n, lam, mu, bc, average=av, r0_factor=1.0).solve(tol=1e-8, max_iter=4000)
    assert a["converged"] and b["converged"]
    assert abs(a["iterations"] - b["iterations"]) <= 0.25 * b["iterations"]


def test_relation_validation():
    n = (5, 5, 5)
    lam, mu, bc = _problem(n, 1)
    sm = W.Smooth(np.array([[2, 2, 1]]), np.array([0], np.int8), np.array([0.01]))
    with pytest.raises(ValueError):    # support reaches z = 0, where every component is held at 0
        Solver(n, lam, mu, bc, smooth=[sm])
    sm = W.Smooth(np.array([[2, 2, 3]]), np.array([0], np.int8), np.array([0.01]))
    st = W.Strong(np.array([[3, 3, 4]]), np.array([0], np.int8), np.array([0.0]))
    with pytest.raises(ValueError):    # overlaps a strong DOF
        Solver(n, lam, mu, bc, strong=[st], smooth=[sm])
