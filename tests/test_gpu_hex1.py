"""GPU parity of the HEX1 scheme and of the isotropic reference medium (Section 3.1.2, eq 4,
Section 3.2.3-3.2.4) through the C ABI, FP64, against the oracle pinned in
tests/test_oracle_hex1.py.  HEX1 displacements are compared through their centre gradients
and reactions where hourglass modes are left free by the conditions."""
import numpy as np
import pytest

import workloads as W
from oracle import hex1
from oracle.solver import Solver as OSolver
from test_oracle_hex1 import NM_INVERTIBLE, NM_SINGULAR, _hex1_case, _normal_mixed_bc

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2607_26082_amd as F
    F.load()
    return F


SHAPES = [((6, 5, 9), None), ((10, 12, 15), 1), ((16, 16, 16), None), ((24, 20, 18), 0), ((32, 48, 6), None),
          ((8, 6, 10), "all")]


def _stiff(rng, n):
    nx, ny, nz = n
    lam = rng.uniform(0.3, 3, (nz, ny, nx)); mu = rng.uniform(0.2, 2, (nz, ny, nx))
    return lam, mu


@pytest.mark.parametrize("idx", range(len(SHAPES)))
def test_stage_residual_hex1(idx):
    F = _lib()
    n, per = SHAPES[idx]
    print(f"[hex1 stage residual] n={n} periodic={per}", flush=True)
    rng = np.random.default_rng(90 + idx)
    lam, mu = _stiff(rng, n)
    bc = rng.integers(0, 2, (3, 3, 2)).astype(np.int8)
    ref = "paux"
    if per == "all":
        bc[:] = 2
        ref = "iso"
    elif per is not None:
        bc[:, per, :] = 2
    o = OSolver(n, lam, mu, bc, r0_factor=1.3, scheme="hex1", reference=ref)
    g = F.Solver(n, lam, mu, bc, r0_factor=1.3, precision="fp64", scheme="hex1", reference=ref)
    u = rng.standard_normal(o.zeros().shape) * 1e-2
    u[o.plan.amask] = 0.0
    parts = o.iterate_parts(u)
    p, pt, sums = g.stage_residual(u)
    assert np.abs(p - parts["p"]).max() <= 1e-12 * np.abs(parts["p"]).max()
    assert np.abs(pt - parts["ptil"]).max() <= 1e-12 * np.abs(parts["ptil"]).max()
    assert abs(sums[0] - parts["pnorm2"]) <= 1e-11 * parts["pnorm2"]
    assert abs(sums[1] - parts["sig2"]) <= 1e-11 * parts["sig2"]


@pytest.mark.parametrize("idx", range(len(SHAPES)))
def test_stage_green_hex1(idx):
    F = _lib()
    n, per = SHAPES[idx]
    print(f"[hex1 stage green] n={n} periodic={per}", flush=True)
    rng = np.random.default_rng(95 + idx)
    lam, mu = _stiff(rng, n)
    bc = rng.integers(0, 2, (3, 3, 2)).astype(np.int8)
    ref = "paux"
    if per == "all":
        bc[:] = 2
        ref = "iso"
    elif per is not None:
        bc[:, per, :] = 2
    o = OSolver(n, lam, mu, bc, r0_factor=0.8, scheme="hex1", reference=ref)
    g = F.Solver(n, lam, mu, bc, r0_factor=0.8, precision="fp64", scheme="hex1", reference=ref)
    p = rng.standard_normal(o.zeros().shape)
    p[o.plan.amask] = 0.0
    ref_u = o.green.apply(p)
    out = g.stage_green(p)
    # The HEX1 symbol tends to 0 towards the hourglass lines, so a random input's output is
    # dominated by those frequencies and their rounding is amplified by the symbol's condition
    # number (largest over smallest non-zero value): the bar is 50 ulps of it.
    if ref == "iso":     # eigenvalues mu0 |d|^2 (twice) and (lam0 + 2 mu0) |d|^2 of the 3x3 symbol
        w = np.linalg.eigvalsh(np.linalg.pinv(o.green.Minv.reshape(-1, 3, 3), hermitian=True))
        w = np.abs(w[np.abs(w) > 1e-12 * np.abs(w).max()])
    else:
        w = 1.0 / np.concatenate([np.ravel(m)[np.ravel(m) != 0] for m in o.green.Minv])
    cond = np.abs(w).max() / np.abs(w).min()
    tol = max(1e-12, 50 * 2.2e-16 * cond)
    print(f"[hex1 stage green] symbol condition {cond:.2e}, bar {tol:.1e}", flush=True)
    assert np.abs(out - ref_u).max() <= tol * np.abs(ref_u).max()


def test_solve_hex1_weak_conditions():
    """Voxel and face averages with HEX1, both sides converged to 1e-12: centre gradients and
    reactions to 1e-10 (the displacement itself is fixed only up to free hourglass modes)."""
    F = _lib()
    n, lam, mu, bc, _, avg = _hex1_case()
    print("[hex1 solve weak]", flush=True)
    o = OSolver(n, lam, mu, bc, [], avg, r0_factor=1.0, scheme="hex1").solve(tol=1e-12, max_iter=6000)
    assert o["converged"]
    g = F.Solver(n, lam, mu, bc, [], avg, r0_factor=1.0, precision="fp64", tol=1e-12, max_iter=6000, scheme="hex1")
    rc, rep = g.solve()
    assert rc == 0
    plan = OSolver(n, lam, mu, bc, scheme="hex1").plan
    Gg = hex1.gradients(g.u.cpu().numpy(), plan); Go = hex1.gradients(o["u"], plan)
    assert np.abs(Gg - Go).max() <= 1e-10 * np.abs(Go).max()
    _, rel, tot = g.reactions()
    assert np.abs(rel - o["f_weak"]).max() <= 1e-10 * np.abs(o["f_weak"]).max()


@pytest.mark.parametrize("ref", ["paux", "iso"])
def test_solve_periodic_hex1(ref):
    """The centrosymmetric periodic cell: same iteration count as the oracle at 1e-8 and the
    converged (1e-12) centre gradients and reactions to 1e-10, with the Paux and the
    isotropic medium."""
    F = _lib()
    prob = W.periodic_centrosymmetric(n=(12, 10, 8), reference=ref)
    print(f"[hex1 periodic] {ref}", flush=True)
    o = OSolver.from_problem(prob).solve(tol=1e-8, max_iter=3000)
    g = F.Solver.from_problem(prob, precision="fp64", tol=1e-8, max_iter=3000)
    rc, rep = g.solve()
    assert rc == 0 and rep.iterations == o["iterations"]
    o = OSolver.from_problem(prob).solve(tol=1e-12, max_iter=3000)
    g = F.Solver.from_problem(prob, precision="fp64", tol=1e-12, max_iter=3000)
    rc, rep = g.solve()
    assert rc == 0
    plan = OSolver.from_problem(prob).plan
    Gg = hex1.gradients(g.u.cpu().numpy(), plan); Go = hex1.gradients(o["u"], plan)
    assert np.abs(Gg - Go).max() <= 1e-10 * np.abs(Go).max()
    _, rel, _ = g.reactions()
    assert np.abs(rel - o["f_weak"]).max() <= 1e-10 * np.abs(o["f_weak"]).max()


# -- isotropic medium under normal-mixed DTT faces ------------------------------------------

NM_SHAPES = [(5, 4, 6), (9, 8, 6), (6, 10, 5)]


@pytest.mark.parametrize("i", range(len(NM_SHAPES)))
def test_stage_green_iso_normal_mixed(i):
    """Green stage of the isotropic medium on normal-mixed faces (every transform type on some
    axis) against the oracle's dense inverse of the weighted reference operator, to 50 ulps of
    that operator's condition number."""
    F = _lib()
    n = NM_SHAPES[i]
    bc = _normal_mixed_bc(NM_INVERTIBLE[i])
    print(f"[iso normal-mixed green] n={n} normal={NM_INVERTIBLE[i]}", flush=True)
    rng = np.random.default_rng(140 + i)
    lam, mu = _stiff(rng, n)
    o = OSolver(n, lam, mu, bc, r0_factor=0.8, scheme="hex1", reference="iso")
    g = F.Solver(n, lam, mu, bc, r0_factor=0.8, precision="fp64", scheme="hex1", reference="iso")
    p = rng.standard_normal(o.zeros().shape)
    p[o.plan.amask] = 0.0
    ref_u = o.green.apply(p)
    out = g.stage_green(p)
    tol = max(1e-12, 50 * 2.2e-16 * np.linalg.cond(o.green.K))
    assert np.abs(out - ref_u).max() <= tol * np.abs(ref_u).max()


@pytest.mark.parametrize("normal", NM_SINGULAR)
def test_stage_green_iso_normal_mixed_singular(normal):
    """DCT1/DST1 faces: hourglass lines reach stored frequencies, the operator is singular;
    for a load in its range the GPU output solves K0 u = p (it differs from the oracle's
    minimum-norm solution by a null vector)."""
    F = _lib()
    n = (5, 4, 6)
    bc = _normal_mixed_bc(normal)
    print(f"[iso normal-mixed green singular] normal={normal}", flush=True)
    rng = np.random.default_rng(150)
    lam, mu = _stiff(rng, n)
    o = OSolver(n, lam, mu, bc, r0_factor=0.8, scheme="hex1", reference="iso")
    g = F.Solver(n, lam, mu, bc, r0_factor=0.8, precision="fp64", scheme="hex1", reference="iso")
    K, idx = o.green.K, o.green.idx
    pf = K @ rng.standard_normal(idx.size)
    p = np.zeros(o.zeros().shape); p.ravel()[idx] = pf
    out = g.stage_green(p)
    assert np.abs(K @ out.ravel()[idx] - pf).max() <= 1e-10 * np.abs(pf).max()


def test_solve_iso_normal_mixed():
    """A heterogeneous HEX1 cell on normal-mixed faces with half-frequency transforms (no
    hourglass line is stored, so a strong condition is well posed) plus a face average: same
    iteration count as the oracle at 1e-8, and the converged (1e-12) displacement and
    reactions to 1e-10."""
    F = _lib()
    n = (6, 5, 7)
    nx, ny, nz = n
    bc = _normal_mixed_bc([[1, 0], [0, 1], [1, 0]])
    rng = np.random.default_rng(160)
    lam, mu = _stiff(rng, n)
    strong = [W.Strong(np.array([[3, 2, 3]]), np.array([0], np.int8), np.array([0.02]))]
    face = np.stack(np.meshgrid([2, 3], [1, 2], [2], indexing="ij"), -1).reshape(1, 4, 3)
    avg = [W.Average(face, np.array([2], np.int8), np.array([-0.03]), set_id=1)]
    print("[iso normal-mixed solve]", flush=True)
    kw = dict(r0_factor=1.0, scheme="hex1", reference="iso")
    o = OSolver(n, lam, mu, bc, strong, avg, **kw).solve(tol=1e-8, max_iter=4000)
    g = F.Solver(n, lam, mu, bc, strong, avg, precision="fp64", tol=1e-8, max_iter=4000, **kw)
    rc, rep = g.solve()
    assert o["converged"] and rc == 0 and rep.iterations == o["iterations"]
    o = OSolver(n, lam, mu, bc, strong, avg, **kw).solve(tol=1e-12, max_iter=4000)
    g = F.Solver(n, lam, mu, bc, strong, avg, precision="fp64", tol=1e-12, max_iter=4000, **kw)
    rc, rep = g.solve()
    assert rc == 0
    u = g.u.cpu().numpy()
    assert np.linalg.norm(u - o["u"]) <= 1e-10 * np.linalg.norm(o["u"])
    _, rel, tot = g.reactions()
    assert np.abs(tot - o["totals"]).max() <= 1e-10 * np.abs(o["totals"]).max()
