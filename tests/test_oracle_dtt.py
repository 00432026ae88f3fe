"""Pins of the oracle's transforms: defining sums, library routine, eq (7), Tables 1-3."""
import os

import numpy as np
import pytest

from oracle import dtt
from oracle.plan import Plan

GOLD = os.path.join(os.path.dirname(__file__), "golden")
KINDS = ("DCT1", "DCT3", "DST1", "DST3")


@pytest.mark.parametrize("n", [2, 3, 5, 7, 8, 13, 15, 16, 22, 48])
@pytest.mark.parametrize("kind", KINDS + ("DFT",))
def test_scipy_matches_defining_sums(kind, n):
    rng = np.random.default_rng(n)
    m = len(dtt.selection(kind, n))
    x = rng.standard_normal((m, 3))
    X = dtt.forward(x, kind, 0, n)
    Xd = dtt.forward_matrix(kind, n) @ x
    assert np.abs(X - Xd).max() <= 1e-13 * max(1.0, np.abs(Xd).max())
    back = dtt.inverse(X, kind, 0, n)
    assert np.abs(back - x).max() < 1e-13
    assert np.abs(dtt.inverse_matrix(kind, n) @ Xd - x).max() < 1e-12


@pytest.mark.parametrize("n", [3, 4, 7, 16])
@pytest.mark.parametrize("kind", KINDS)
def test_eq7_dft_of_4n_extension(kind, n):
    """Eq (7): S_4F(DFT(q4)) = alpha * DTT(S_R(q)), with q4 built from the symmetries."""
    rng = np.random.default_rng(7 * n)
    q = rng.standard_normal(n + 1)
    q4 = dtt.extension_4n(q, kind, n)
    idx, alpha = dtt.s4f(kind, n)
    F = np.fft.fft(q4)
    sel = dtt.selection(kind, n)
    assert np.abs(F[idx] - alpha * dtt.forward(q[sel], kind, 0, n)).max() < 1e-12
    # the other parity class of DFT indices vanishes (period 2n vs anti-period 2n)
    other = np.arange(1 if kind in ("DCT1", "DST1") else 0, 4 * n, 2)
    assert np.abs(F[other]).max() < 1e-11
    # theta of a stored coefficient equals 2 pi k / 4n at its DFT index
    assert np.allclose(dtt.thetas(kind, n), 2 * np.pi * idx / (4 * n))


def test_table3_fixture():
    rows = [l.split() for l in open(os.path.join(GOLD, "table3_selection.txt")) if l.strip() and l[0] != "#"]
    n = 9
    for kind, first, last, _, count, alpha in rows:
        sel = dtt.selection(kind, n)
        ev = lambda s: eval(s, {"n": n})
        assert sel[0] == ev(first) and sel[-1] == ev(last) and len(sel) == ev(count)
        idx, a = dtt.s4f(kind, n)
        assert len(idx) == ev(count)
        assert a == (2.0 if alpha == "2" else -2.0j)


def test_table1_and_table2_fixtures():
    t1 = {l.split()[0]: l.split()[1] for l in open(os.path.join(GOLD, "table1_bc_symmetry.txt"))
          if l.strip() and l[0] != "#"}
    t2 = {l.split()[0]: l.split()[1] for l in open(os.path.join(GOLD, "table2_sym_dtt.txt"))
          if l.strip() and l[0] != "#"}
    code = {"Neumann": 0, "Dirichlet": 1}
    for f0 in ("Neumann", "Dirichlet"):
        for f1 in ("Neumann", "Dirichlet"):
            bc = np.zeros((3, 3, 2), np.int8)
            bc[1, 2, 0], bc[1, 2, 1] = code[f0], code[f1]
            plan = Plan((4, 4, 4), bc)
            assert plan.sym[1, 2, 0] == t1[f0] and plan.sym[1, 2, 1] == t1[f1]
            assert plan.types[1][2] == t2[t1[f0] + t1[f1]]
    bc = np.full((3, 3, 2), 2, np.int8)
    plan = Plan((4, 4, 4), bc)
    assert plan.sym[0, 0, 0] == t1["Periodic"] and plan.types[0][0] == "DFT"


def test_plan_eliminated_dofs_and_weights():
    bc = np.zeros((3, 3, 2), np.int8)
    bc[2, 2, 0] = 1          # u_z Dirichlet on z = 0
    bc[0, 0, 1] = 1          # u_x Dirichlet on x = n
    plan = Plan((3, 4, 5), bc)
    assert plan.amask[2, 0].all() and not plan.amask[2, 1:].any()
    assert plan.amask[0, :, :, 3].all() and plan.amask[0].sum() == 6 * 5
    assert plan.b[0, 0, 0] == 3 and plan.b[2, 2, 1] == 0 and plan.b[0, 2, 1] == 1 and plan.b[0, 0, 1] == 2
    with pytest.raises(ValueError):
        bad = np.zeros((3, 3, 2), np.int8); bad[0, 1, 0] = 2
        Plan((3, 3, 3), bad)
