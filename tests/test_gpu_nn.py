"""Warm-start network on the GPU against its FP64 oracle (oracle/nn.py).

The GPU runs BF16 operands with FP32 accumulation and stores activations in
BF16, so forward outputs and gradients are compared by relative L2 and
cosine, with bounds derived from BF16's unit roundoff (2^-9): a handful of
roundings per layer over six layers stays below 1e-2 relative.  Binary
channels (prescribed-DOF masks) are compared exactly."""
import numpy as np
import pytest

import workloads as W
from oracle import nn as onn

pytestmark = pytest.mark.gpu


def _bf16_bits(a):
    f = np.ascontiguousarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def _bf16_val(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _torch():
    import torch
    import paper_2607_26082_amd as F
    F.load()
    return torch, F


def _feat_dev(torch, f):
    bits = np.zeros((f.shape[0], 16), np.uint16)
    bits[:, :f.shape[1]] = _bf16_bits(f)
    return torch.as_tensor(bits.view(np.int16), device="cuda"), _bf16_val(bits[:, :f.shape[1]])


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _cos(a, b):
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)))


@pytest.mark.parametrize("case", ["patch64", "patch32", "indent", "periodic"])
def test_features_match_oracle(case):
    torch, F = _torch()
    if case == "patch64":
        prob, prec = W.random_cell(W.BASE_SEED + 21, n=(20, 12, 10)), "fp64"
    elif case == "patch32":
        prob, prec = W.random_cell(W.BASE_SEED + 22, n=(16, 24, 12)), "fp32"
    elif case == "indent":
        prob, prec = W.nn_case(W.NN_TRAIN_SEED + 1, n0=(24, 20, 16)), "fp32"
    else:
        prob, prec = W.random_cell(W.BASE_SEED + 23, n=(12, 10, 8), with_patches=False), "fp64"
        prob.bc[:, 0, :] = W.BC_P
    print(f"[nn features] {case} n={prob.n}", flush=True)
    g = F.Solver.from_problem(prob, precision=prec)
    feat, u1 = g.features()
    got = feat.cpu().numpy().view(np.uint16)
    u1 = u1.cpu().numpy()
    if prec == "fp32":
        # the solver keeps FP32 Lame fields: the oracle sees the same rounded inputs
        import dataclasses
        prob = dataclasses.replace(prob, lam=prob.lam.astype(np.float32).astype(np.float64),
                                   mu=prob.mu.astype(np.float32).astype(np.float64))
    u1_ref = onn.first_iterate(prob).reshape(3, -1)
    # the first iterate: FP64 path to rounding, FP32 form to its arithmetic
    assert np.linalg.norm(u1 - u1_ref) <= (1e-12 if prec == "fp64" else 1e-5) * np.linalg.norm(u1_ref)
    ref = onn.features(prob, u1=u1_ref)
    want = _bf16_bits(ref)
    np.testing.assert_array_equal(got[:, 2:5], want[:, 2:5])
    assert not got[:, 12:].any()
    d = np.abs(got[:, :9].astype(np.int64) - want[:, :9].astype(np.int64))
    assert d.max() <= 1, (case, int(d.max()))
    # first-iterate channels: BF16 of u1 / s_u (the FP32 form differs from FP64 below 1e-5)
    gv, wv = _bf16_val(got[:, 9:12]), ref[:, 9:12]
    assert (np.abs(gv - wv) <= 2.0 ** -8 * np.abs(wv) + 1e-5 * np.abs(wv).max()).all(), case


def _net_case(seed, N, modes=6, blocks=4):
    shape = dict(width=32, modes=modes, blocks=blocks, hidden=64, cin=12, cout=3)
    shapes = [s for _, s in onn.param_layout(**shape)]
    vec = W.nn_init(seed, shapes).astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(seed + 1)
    Nn = int(np.prod(N))
    f = np.concatenate([rng.uniform(0, 1, (Nn, 2)), (rng.random((Nn, 3)) < 0.2).astype(float),
                        rng.standard_normal((Nn, 3)), rng.uniform(-0.2, 0.2, (Nn, 1)),
                        rng.standard_normal((Nn, 3))], 1)
    t = rng.standard_normal((Nn, 3)).astype(np.float32).astype(np.float64)
    return shape, vec, f, t


NETS = [((17, 13, 11), 6, 4), ((9, 8, 7), 2, 1), ((16, 16, 16), 6, 0), ((33, 17, 21), 6, 4)]


@pytest.mark.parametrize("N,modes,blocks", NETS)
def test_forward_matches_oracle(N, modes, blocks):
    torch, F = _torch()
    print(f"[nn forward] N={N} m={modes} B={blocks}", flush=True)
    shape, vec, f, _ = _net_case(11, N, modes, blocks)
    net = F.Net(modes, blocks)
    assert net.P == onn.num_params(**shape)
    net.set_params(vec)
    net.bind(N, training=False)
    fd, fval = _feat_dev(torch, f)
    u0 = torch.zeros((3, int(np.prod(N))), dtype=torch.float64, device="cuda")
    base = torch.randn((3, int(np.prod(N))), dtype=torch.float64, device="cuda")
    y = net.forward(fd, s_u=0.5, base=base, u0=u0)
    torch.cuda.synchronize()
    y = y.cpu().numpy().astype(np.float64)
    yr, _ = onn.forward(onn.unflatten(vec, **shape), fval, N, blocks=blocks, m=modes)
    assert _rel(y, yr) <= 1e-2, _rel(y, yr)
    np.testing.assert_allclose(u0.cpu().numpy(), base.cpu().numpy() + 0.5 * y.T, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("N,modes,blocks", NETS)
def test_gradient_matches_oracle(N, modes, blocks):
    torch, F = _torch()
    print(f"[nn gradient] N={N} m={modes} B={blocks}", flush=True)
    shape, vec, f, t = _net_case(12, N, modes, blocks)
    net = F.Net(modes, blocks)
    net.set_params(vec)
    net.bind(N, training=True)
    fd, fval = _feat_dev(torch, f)
    tt = torch.as_tensor(np.ascontiguousarray(t.T, np.float32), device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    net.train_step(fd, tt, loss)
    g = net.grad().cpu().numpy().astype(np.float64)
    p = onn.unflatten(vec, **shape)
    y, cache = onn.forward(p, fval, N, blocks=blocks, m=modes)
    L, dy = onn.loss(y, t, fval[:, 9:12])
    gr = onn.flatten(onn.backward(p, cache, dy), **shape)
    assert abs(loss.item() - L) <= 1e-2 * L
    assert _cos(g, gr) >= 0.999 and _rel(g, gr) <= 1e-2, (_cos(g, gr), _rel(g, gr))
    # every parameter group gets its own gradient (no group left stale or misplaced)
    o = 0
    for name, s in onn.param_layout(**shape):
        k = int(np.prod(s))
        if np.linalg.norm(gr[o:o + k]) > 1e-6 * np.linalg.norm(gr):
            assert _cos(g[o:o + k], gr[o:o + k]) >= 0.99, name
        o += k


def test_adam_step_matches_oracle():
    torch, F = _torch()
    N = (9, 8, 7)
    shape, vec, f, t = _net_case(13, N, 2, 1)
    net = F.Net(2, 1)
    net.set_params(vec)
    net.bind(N, training=True)
    fd, _ = _feat_dev(torch, f)
    tt = torch.as_tensor(np.ascontiguousarray(t.T, np.float32), device="cuda")
    p0 = net.params().cpu().numpy().astype(np.float64)
    mom = np.zeros_like(p0)
    vel = np.zeros_like(p0)
    for step in (1, 2):
        net.train_step(fd, tt)
        g = net.grad().cpu().numpy().astype(np.float64)
        net.adam(1e-3)
        p1 = net.params().cpu().numpy().astype(np.float64)
        pr, mom, vel = onn.adam(p0, g, mom, vel, step=step, lr=1e-3)
        np.testing.assert_allclose(p1, pr, rtol=1e-5, atol=1e-7)
        p0 = p1


def test_training_reduces_loss():
    torch, F = _torch()
    N = (17, 13, 11)
    prob = W.random_cell(W.BASE_SEED + 31, n=(16, 12, 10))
    g = F.Solver.from_problem(prob, precision="fp32", tol=1e-6, max_iter=4000)
    rc, rep = g.solve()
    assert rc == 0
    su = onn.start_scale(prob.n)
    ustar = g.u.reshape(3, -1).clone()
    feat, u1 = g.features()
    tt = ((ustar - u1) / su).to(torch.float32).contiguous()
    net = F.Net(6, 4)
    net.set_params(W.nn_init(3, [s for _, s in onn.param_layout()]))
    net.bind(N, training=True)
    loss = torch.zeros(200, dtype=torch.float64, device="cuda")
    for i in range(200):
        net.train_step(feat, tt, loss[i:i + 1])
        net.adam(3e-3)
    torch.cuda.synchronize()
    L = loss.cpu().numpy()
    print(f"[nn training] loss {L[0]:.3e} -> {L[-1]:.3e}", flush=True)
    assert np.isfinite(L).all() and L[-10:].mean() < 0.2 * L[:10].mean()


def test_judged_start_uses_good_start_and_falls_back_on_bad():
    torch, F = _torch()
    prob = W.random_cell(W.BASE_SEED + 32, n=(16, 12, 10))
    g = F.Solver.from_problem(prob, precision="fp32", tol=1e-6, max_iter=4000)
    rc, rep = g.solve()
    assert rc == 0
    good = g.u.clone()
    rc2, rep2, used, (r_nn, r_plain) = g.solve_judged(good)
    assert used and r_nn < r_plain and rep2.iterations <= 3
    bad = good + 1e3 * torch.randn_like(good)
    rc3, rep3, used3, (r_bad, r_plain3) = g.solve_judged(bad)
    assert not used3 and r_bad >= r_plain3
    assert rep3.iterations == rep.iterations and rc3 == 0
    np.testing.assert_array_equal(g.u.cpu().numpy(), good.cpu().numpy())


def test_trained_network_judged_start_on_held_out_cases():
    """What the trained network (paper_2607_26082_amd/data, trained by warmstart.py on
    1881 converged 64^3 solves) gains on held-out 64^3 cases: the judged start never
    costs more than the two judge iterations per case over the plain start, and the
    converged answer is the plain one to the solver tolerance (cases that stop at the
    iteration cap must do so from both starts).  The measured gain is
    printed (on this workload it is about 1.0: the network's start is rarely chosen)."""
    torch, F = _torch()
    from paper_2607_26082_amd import warmstart as WS
    net = F.Net(6, 4)
    net.set_params(WS.load_weights())
    specs = [W.nn_case_spec(W.NN_EVAL_SEED + j) for j in range(8)]
    rows = WS.evaluate(net, specs, scale=1)
    s = WS.summary(rows)
    print(f"[nn gain] {s}", flush=True)
    # some held-out cases stop at the iteration cap from either start: same outcome required
    assert all(r["status"][1] == r["status"][0] for r in rows)
    conv = [r for r in rows if r["status"] == [0, 0]]
    assert len(conv) >= len(rows) - 2
    plain = sum(r["iters_plain"] for r in conv)
    judged = sum(r["iters_nn"] for r in conv)
    assert judged <= 1.1 * plain + 2 * len(conv)
    assert max(r["rel_nn_vs_plain"] for r in conv) <= 1e-3
