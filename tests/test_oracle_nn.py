"""Pins of the warm-start network's FP64 reference (oracle/nn.py).

The network is this project's design (the paper only names a better initial
guess as future work, Section 6), so the pins are: scipy's DCT-II/III for the
truncated transforms, discrete orthogonality of the cosine basis, printed
values of the normal CDF, central finite differences for the hand-written
backward pass, the closed form of Adam's first step, and closed forms of the
input channels on simple problems."""
import numpy as np
import pytest
from scipy import fft as sfft

import workloads as W
from oracle import nn
from oracle.plan import Plan


def test_param_count_closed_form():
    w, m, B, H, cin, cout = 32, 6, 4, 64, 12, 3
    expect = w * cin + w + B * (m ** 3 * w * w + w * w + w) + H * w + H + cout * H + cout
    assert nn.num_params() == expect == 891683


def test_analysis_is_truncated_dct2():
    rng = np.random.default_rng(1)
    N, m = (9, 7, 5), 3
    x = rng.standard_normal((N[0] * N[1] * N[2], 2))
    xh = nn.analysis(x, N, m)
    for c in range(2):
        g = x[:, c].reshape(N[2], N[1], N[0])
        d = sfft.dctn(g, type=2, axes=(0, 1, 2))[:m, :m, :m] / (8.0 * x.shape[0])
        np.testing.assert_allclose(xh[:, c], d.ravel(), rtol=0, atol=1e-14)


def test_synthesis_is_dct3_of_halved_modes():
    rng = np.random.default_rng(2)
    N, m = (8, 6, 7), 3
    yh = rng.standard_normal((m ** 3, 2))
    s = nn.synthesis(yh, N, m)
    for c in range(2):
        a = np.zeros((N[2], N[1], N[0]))
        a[:m, :m, :m] = yh[:, c].reshape(m, m, m)
        for ax in range(3):
            sl = [slice(None)] * 3
            sl[ax] = slice(1, None)
            a[tuple(sl)] *= 0.5
        d = sfft.dctn(a, type=3, axes=(0, 1, 2))
        np.testing.assert_allclose(s[:, c], d.ravel(), rtol=0, atol=1e-13)


@pytest.mark.parametrize("k", [(0, 0, 0), (1, 0, 2), (2, 2, 1), (3, 0, 0)])
def test_single_mode_orthogonality(k):
    """phi_k on the grid: analysis returns 2^-(number of nonzero k) at k and 0
    elsewhere; a mode with an index >= m is annihilated."""
    N, m = (10, 8, 6), 3
    fx, fy, fz = nn.cos_basis(N[0], 4), nn.cos_basis(N[1], 4), nn.cos_basis(N[2], 4)
    kx, ky, kz = k
    g = fz[:, kz][:, None, None] * fy[:, ky][None, :, None] * fx[:, kx][None, None, :]
    xh = nn.analysis(g.reshape(-1, 1), N, m)[:, 0]
    expect = np.zeros(m ** 3)
    if max(k) < m:
        expect[(kz * m + ky) * m + kx] = 0.5 ** sum(1 for v in k if v > 0)
    np.testing.assert_allclose(xh, expect, atol=1e-15)


def test_gelu_values():
    # Phi(1) and Phi(-0.5) of the standard normal distribution
    np.testing.assert_allclose(nn.gelu(np.array([1.0, -0.5, 0.0])),
                               [0.8413447460685429, -0.5 * 0.3085375387259869, 0.0], rtol=1e-15, atol=0)
    assert nn.gelu_grad(np.array([0.0]))[0] == 0.5


def _tiny():
    shape = dict(width=4, modes=2, blocks=2, hidden=5, cin=9, cout=3)
    rng = np.random.default_rng(7)
    vec = rng.standard_normal(nn.num_params(**shape)) * 0.5
    N = (5, 4, 3)
    f = rng.standard_normal((N[0] * N[1] * N[2], 9))
    t = rng.standard_normal((f.shape[0], 3))
    return shape, vec, N, f, t


def test_backward_matches_central_differences():
    shape, vec, N, f, t = _tiny()

    def L(v):
        y, _ = nn.forward(nn.unflatten(v, **shape), f, N, blocks=2, m=2)
        return nn.loss(y, t)[0]

    p = nn.unflatten(vec, **shape)
    y, cache = nn.forward(p, f, N, blocks=2, m=2)
    _, dy = nn.loss(y, t)
    g = nn.flatten(nn.backward(p, cache, dy), **shape)
    h = 1e-6
    fd = np.empty_like(vec)
    for i in range(len(vec)):
        e = np.zeros_like(vec)
        e[i] = h
        fd[i] = (L(vec + e) - L(vec - e)) / (2 * h)
    assert np.linalg.norm(g - fd) <= 1e-6 * np.linalg.norm(fd)


def test_loss_zero_at_target_and_gradient_direction():
    t = np.random.default_rng(3).standard_normal((10, 3))
    l0, d0 = nn.loss(t.copy(), t)
    assert l0 == 0.0 and not d0.any()
    l1, d1 = nn.loss(2 * t, t)
    assert abs(l1 - 1.0) < 1e-15
    np.testing.assert_allclose(d1, 2 * t / (t * t).sum(), rtol=1e-15)
    # with b the normaliser is the size of t and b together: here half of it
    l2, _ = nn.loss(2 * t, t, t)
    assert abs(l2 - 0.5) < 1e-15


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    v0 = np.array([1.0, 2.0, 3.0, 4.0])
    v1, m1, s1 = nn.adam(v0, g, np.zeros(4), np.zeros(4), step=1, lr=0.01)
    # bias-corrected moments equal g and g^2 on the first step
    np.testing.assert_allclose(v1, v0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14)
    np.testing.assert_allclose(m1, 0.1 * g)
    np.testing.assert_allclose(s1, 0.001 * g * g)


def test_features_homogeneous_indentation():
    prob = W.c3_indentation(n=(8, 6, 5), R=4.0, d_over_R=0.05)
    f = nn.features(prob).reshape(6, 7, 9, 12)         # [Nz, Ny, Nx, ch]
    np.testing.assert_allclose(f[..., 0], 1.0, rtol=1e-15)
    np.testing.assert_allclose(f[..., 1], 0.3, rtol=1e-14)
    # bottom face: every component fixed; nothing else prescribed
    assert (f[0, :, :, 2:5] == 1).all() and (f[1:, :, :, 2:5] == 0).all()
    assert not f[..., 5:8].any()
    # top node under the sphere centre: gap = (R - d) - R = -d, d = 0.05 R = 0.2, s_u = 0.005
    assert abs(f[5, 3, 4, 8] - np.tanh(-0.2 / 0.04)) < 1e-15
    # off the top face the channel is 0; a top corner sits outside the sphere
    assert not f[:5, :, :, 8].any() and f[5, 0, 0, 8] > 0
    # the first iterate: held at 0 on the fixed bottom, pressed down under the sphere
    u1 = f[..., 9:12] * 0.005
    assert not u1[0].any() and u1[5, 3, 4, 2] < 0


def test_features_patch_cell():
    prob = W.random_cell(W.BASE_SEED + 11, n=(12, 10, 8))
    f = nn.features(prob)
    plan = Plan(prob.n, prob.bc)
    su = nn.start_scale(prob.n)
    Nx, Ny, _ = plan.N
    fixed = plan.amask.reshape(3, -1).T.copy()
    val = np.zeros_like(fixed, dtype=np.float64)
    for s in prob.strong:
        i = s.node[:, 0] + Nx * (s.node[:, 1] + Ny * s.node[:, 2])
        fixed[i, s.comp] = True
        val[i, s.comp] = s.value / su
    np.testing.assert_array_equal(f[:, 2:5], fixed.astype(np.float64))
    np.testing.assert_allclose(f[:, 5:8], val, rtol=1e-15)
    assert f[:, 0].max() <= 1.0 and f[:, 0].min() > 0
    # nodes whose eight voxels are all matrix see the matrix values exactly
    E = prob.mu * (3 * prob.lam + 2 * prob.mu) / (prob.lam + prob.mu)
    assert np.isclose(f[:, 0], E.min() / E.max(), rtol=1e-14).any()
    assert not f[:, 8].any()
    # the first iterate satisfies the prescribed values exactly (proj_U ends the iteration)
    np.testing.assert_allclose(f[:, 9:12][fixed], val[fixed], rtol=1e-13, atol=1e-15)


def test_nn_init_scales():
    shapes = [s for _, s in nn.param_layout()]
    v = W.nn_init(5, shapes)
    p = nn.unflatten(v)
    assert not p["bl"].any() and not p["c3"].any()
    assert abs(p["Ws0"].std() * np.sqrt(32) - 1) < 0.01
    assert abs(p["Wl"].std() * 3 - 1) < 0.2
