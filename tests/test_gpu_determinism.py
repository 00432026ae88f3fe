"""Repeat-solve determinism: the same problem solved again on the same handle, and on a fresh
handle, gives bitwise the same displacement, iteration count, residual, reactions, mean stress
and (with an obstacle) active set and contact force.  Every reduction of the library has a
fixed order (block partial rows summed in index order), so this holds by construction; the
test guards it against atomics or launch-dependent partitions slipping in."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2607_26082_amd as F
    F.load()
    return F


def _record(g, rep, contact=False):
    _, _, tot = g.reactions()
    out = dict(u=g.u.cpu().numpy().copy(), it=rep.iterations, res=rep.residual, tot=np.array(tot),
               ms=np.array(rep.mean_stress))
    if contact:
        mask, fnc, gap = g.contact()
        out.update(mask=np.array(mask), fnc=np.array(fnc), F=rep.force_contact)
    return out


def _same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_repeat_solve_bitwise(prec):
    F = _lib()
    prob = W.c1_inclusion_patch()
    print(f"[determinism] C1 {prec}", flush=True)
    g = F.Solver.from_problem(prob, precision=prec, tol=1e-10 if prec == "fp64" else 1e-6)
    rc, rep = g.solve()
    assert rc == 0
    first = _record(g, rep)
    rc, rep = g.solve()
    _same(first, _record(g, rep))
    g2 = F.Solver.from_problem(prob, precision=prec, tol=1e-10 if prec == "fp64" else 1e-6)
    rc, rep = g2.solve()
    _same(first, _record(g2, rep))


def test_repeat_contact_solve_bitwise():
    F = _lib()
    n = (32, 32, 16)
    prob = W.c3_indentation(n=n, R=12.0, d_over_R=0.03)
    print("[determinism] indentation fp32", flush=True)
    runs = []
    for _ in range(2):
        g = F.Solver.from_problem(prob, precision="fp32", tol=1e-6)
        rc, rep = g.solve()
        assert rc == 0 and rep.contact_nodes > 0
        runs.append(_record(g, rep, contact=True))
    _same(runs[0], runs[1])


def test_repeat_batch_bitwise():
    F = _lib()
    cells = [W.c1_inclusion_patch(), W.c2_compact_tension(n=(30, 30, 6), notch_len=8, notch_h=2, radius=2.0,
                                                         offset=6)]
    print("[determinism] batch of 2 fp32", flush=True)
    outs = []
    for _ in range(2):
        solvers = [F.Solver.from_problem(p, precision="fp32", tol=1e-6, max_iter=3000) for p in cells]
        rc, reps = F.Batch(solvers).solve()
        assert rc == 0
        outs.append([(s.u.cpu().numpy().copy(), r.iterations, r.residual) for s, r in zip(solvers, reps)])
    for (u0, i0, r0), (u1, i1, r1) in zip(*outs):
        assert i0 == i1 and r0 == r1 and np.array_equal(u0, u1)
