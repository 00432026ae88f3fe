"""The boundary's conventions on the GPU: voxel size h (lengths in the unit of h, forces in
stress times its square), stiffness given as FP32 arrays or as (E, nu), constraint arrays in
device memory, contact force and area, and the learned start's training-target kernel."""
import numpy as np
import pytest

import workloads as W
from oracle.contact import ContactSolver

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2607_26082_amd as F
    F.load()
    return F


def test_voxel_size_scales_lengths_and_forces():
    """The same problem in voxel units and with h = 0.25 (prescribed values and displacements
    times h, forces times h^2): the internal problem is identical, so the results scale exactly."""
    F = _lib()
    prob = W.c1_inclusion_patch()
    print("[abi] voxel size", flush=True)
    a = F.Solver.from_problem(prob, precision="fp64")
    rc, ra = a.solve()
    assert rc == 0
    hs = 0.25
    strong = [W.Strong(s.node, s.comp, s.value * hs, s.set_id) for s in prob.strong]
    b = F.Solver(prob.n, prob.lam, prob.mu, prob.bc, strong, r0_factor=prob.r0_factor, precision="fp64",
                 tol=prob.tol, voxel=hs)
    rc, rb = b.solve()
    assert rc == 0 and rb.iterations == ra.iterations
    assert np.array_equal(b.u.cpu().numpy(), hs * a.u.cpu().numpy())
    _, _, ta = a.reactions()
    _, _, tb = b.reactions()
    assert np.array_equal(tb, hs * hs * ta)
    assert np.array_equal(np.array(rb.mean_stress), np.array(ra.mean_stress))


def test_stiffness_forms():
    """(lam, mu) as FP32 arrays and (E, nu) as FP64 arrays give the solves of the FP64 (lam, mu)
    input: FP32 input rounds the moduli (1e-6 relative), the (E, nu) conversion is done on the
    device (1e-12)."""
    import torch
    F = _lib()
    prob = W.c1_inclusion_patch()
    print("[abi] stiffness forms", flush=True)
    ref = F.Solver.from_problem(prob, precision="fp64", tol=1e-12)
    rc, _ = ref.solve()
    u_ref = ref.u.cpu().numpy()
    g = F.Solver.from_problem(prob, precision="fp64", tol=1e-12)
    F.fftc_set_stiffness(g.h, torch.as_tensor(prob.lam, dtype=torch.float32, device="cuda"),
                         torch.as_tensor(prob.mu, dtype=torch.float32, device="cuda"))
    rc, _ = g.solve()
    assert rc == 0
    assert np.linalg.norm(g.u.cpu().numpy() - u_ref) <= 1e-6 * np.linalg.norm(u_ref)
    E = np.where(prob.lam > 150, 400.0, 200.0)
    nu = np.full(E.shape, 0.3)
    lam, mu = W.lame(E, 0.3)
    assert np.abs(lam - prob.lam).max() < 1e-12 * lam.max()
    F.fftc_set_stiffness_Enu(g.h, torch.as_tensor(E, device="cuda"), torch.as_tensor(nu, device="cuda"))
    rc, _ = g.solve()
    assert rc == 0
    assert np.linalg.norm(g.u.cpu().numpy() - u_ref) <= 1e-12 * np.linalg.norm(u_ref)
    bad = torch.as_tensor(np.full(E.shape, 0.5), device="cuda")
    with pytest.raises(F.FftcError) as e:
        F.fftc_set_stiffness_Enu(g.h, torch.as_tensor(E, device="cuda"), bad)
    assert e.value.code == F.FFTC_E_ARG


def test_constraints_from_device_arrays():
    import torch
    F = _lib()
    prob = W.c1_inclusion_patch()
    print("[abi] device constraint arrays", flush=True)
    a = F.Solver.from_problem(prob, precision="fp64")
    rc, _ = a.solve()
    h = F.fftc_create(prob.n, F.FFTC_FP64)
    F.fftc_set_bc(h, prob.bc)
    import ctypes as C

    def devp(t, ctype):
        return C.cast(C.c_void_p(t.data_ptr()), C.POINTER(ctype))

    for s in prob.strong:
        node = torch.as_tensor(np.asarray(s.node, np.int64), device="cuda")
        comp = torch.as_tensor(np.asarray(s.comp, np.int8), device="cuda")
        val = torch.as_tensor(np.asarray(s.value, np.float64), device="cuda")
        torch.cuda.synchronize()
        rc = F.load().fftc_add_dirichlet(h, len(s.comp), devp(node, C.c_int64), devp(comp, C.c_int8),
                                         devp(val, C.c_double), int(s.set_id))
        assert rc == F.FFTC_OK
    ns, nw = C.c_int64(), C.c_int64()
    F.load().fftc_num_constraints(h, C.byref(ns), C.byref(nw))
    assert ns.value == sum(len(s.comp) for s in prob.strong)
    F.fftc_set_reference_factor(h, prob.r0_factor)
    F.fftc_set_solver(h, tol=prob.tol)
    nb = F.fftc_workspace_bytes(h)
    ws = F._aligned(torch, nb, torch.device("cuda"))
    stream = torch.cuda.current_stream()
    F.fftc_bind_workspace(h, ws, nb, stream.cuda_stream)
    F.fftc_set_stiffness(h, torch.as_tensor(prob.lam, device="cuda"), torch.as_tensor(prob.mu, device="cuda"))
    u = torch.zeros_like(a.u)
    rc, rep = F.fftc_solve(h, u, True)
    assert rc == 0
    assert np.array_equal(u.cpu().numpy(), a.u.cpu().numpy())
    F.fftc_destroy(h)


def test_contact_force_and_area():
    """Force as in the report; area = face area of the nodes of C (half a voxel face along an
    edge of the face), its equivalent radius within a voxel of the Hertz radius sqrt(R d)."""
    F = _lib()
    n = (32, 32, 16); R = 12.0; d = 0.12 * 3
    prob = W.c3_indentation(n=n, R=R)
    print("[abi] contact force and area", flush=True)
    sph = W.Sphere(np.array([16.0, 16.0, 16 + R - d]), R, 5)
    g = F.Solver(n, prob.lam, prob.mu, prob.bc, sphere=sph, r0_factor=5.0, precision="fp64", tol=1e-10)
    rc, rep = g.solve()
    assert rc == 0
    mask, fnc, gap, force, area = F.fftc_get_contact(g.h)
    assert force == rep.force_contact
    m = mask.reshape(n[1] + 1, n[0] + 1).astype(bool)
    assert not m[0].any() and not m[:, 0].any()          # the contact zone stays off the edges
    assert area == float(m.sum())
    assert abs(np.sqrt(area / np.pi) - np.sqrt(R * d)) < 1.0


def test_training_target_kernel():
    import torch
    F = _lib()
    rng = np.random.default_rng(3)
    u = torch.as_tensor(rng.standard_normal(3000), device="cuda")
    u1 = torch.as_tensor(rng.standard_normal(3000), device="cuda")
    t = torch.empty(3000, dtype=torch.float32, device="cuda")
    F.fftc_nn_make_target(u, u1, 0.064, t, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    want = ((u.cpu().numpy() - u1.cpu().numpy()) / 0.064).astype(np.float32)
    assert np.array_equal(t.cpu().numpy(), want) or np.abs(t.cpu().numpy() - want).max() <= 1e-7 * np.abs(want).max()
