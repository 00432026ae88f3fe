"""FP64 reference of the warm-start network, with a hand-written backward pass.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper has no network: it names a better initial guess as future work
(Section 6).  The network here is this project's design, so its plain
definition is the function itself, written out below; its parity pins are
library routines (scipy's DCT-II/III for the truncated transforms), discrete
orthogonality of the cosine basis, values of the normal CDF, and central
finite differences for the backward pass.

Grid: the solver's node grid, N = (Nx, Ny, Nz), flat index x + Nx (y + Ny z);
activations are [Nn, C] (node-major).

Network (defaults width 32, modes m = 6, 4 blocks, head width 64):
  x0 = f Wl^T + bl                                  lift, f = 12 input channels
  x_b = GELU( S_b(x_{b-1}) + x_{b-1} W_b^T + c_b )  b = 1..4
  h  = GELU( x_4 Wp1^T + bp1 )
  y  = h Wp2^T + bp2                                 3 outputs, in units of s_u
Spectral operator S (modes k = (kz, ky, kx), each < m):
  phi_k(i) = cos(pi k (i + 1/2) / N)                 DCT-II basis per axis
  xh[k, c] = (1/Nn) sum_i phi_kz(z) phi_ky(y) phi_kx(x) x[i, c]
  yh[k, o] = sum_c Ws[k, o, c] xh[k, c]
  S(x)[i, o] = sum_k phi_kz(z) phi_ky(y) phi_kx(x) yh[k, o]
GELU(z) = z Phi(z), Phi the standard normal CDF (erf form).
Loss per sample: L = sum (y - t)^2 / (sum t^2 + sum b^2), t = (u* - u1)/s_u
with u1 the solver's first iterate from the plain start and b = u1/s_u (the
misfit of the correction relative to the size of the whole field).
Displacement start: u0 = u1 + s_u y, s_u = 1e-3 min(n).

Input channels (all on nodes):
  0  E / max E, E averaged over the voxels around the node
  1  nu averaged over the voxels around the node
  2-4  per component: 1 where the DOF is prescribed (Dirichlet face or
       strong constraint), else 0
  5-7  per component: prescribed value / s_u (0 where free)
  8  on the contact face of a rigid sphere: tanh(g / (8 s_u)), g = |X - O| - R
     the gap of the undeformed node, so that indentation depths of a few s_u
     map to O(1) values; 0 elsewhere and without a sphere
  9-11 per component: the first iterate u1 / s_u (one iteration of Algorithm 1,
       or Algorithm 2 with a sphere, from the plain start)
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

from .plan import Plan

SQRT2 = np.sqrt(2.0)
INV_SQRT_2PI = 1.0 / np.sqrt(2.0 * np.pi)

DEFAULT_SHAPE = dict(width=32, modes=6, blocks=4, hidden=64, cin=12, cout=3)


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------

def param_layout(width=32, modes=6, blocks=4, hidden=64, cin=12, cout=3):
    """Ordered (name, shape) list; the flat parameter vector concatenates them
    in this order, each row-major."""
    w, M = width, modes ** 3
    out = [("Wl", (w, cin)), ("bl", (w,))]
    for b in range(blocks):
        out += [(f"Ws{b}", (M, w, w)), (f"W{b}", (w, w)), (f"c{b}", (w,))]
    out += [("Wp1", (hidden, w)), ("bp1", (hidden,)), ("Wp2", (cout, hidden)), ("bp2", (cout,))]
    return out


def num_params(**shape):
    return int(sum(np.prod(s) for _, s in param_layout(**shape)))


def unflatten(vec, **shape):
    p, o = {}, 0
    for name, s in param_layout(**shape):
        k = int(np.prod(s))
        p[name] = np.asarray(vec[o:o + k], np.float64).reshape(s)
        o += k
    assert o == len(vec)
    return p


def flatten(p, **shape):
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in param_layout(**shape)])


# ---------------------------------------------------------------------------
# pieces
# ---------------------------------------------------------------------------

def gelu(z):
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


def cos_basis(N, m):
    """phi[i, k] = cos(pi k (i + 1/2) / N), i < N, k < m (DCT-II basis)."""
    i = np.arange(N)[:, None] + 0.5
    k = np.arange(m)[None, :]
    return np.cos(np.pi * k * i / N)


def _bases(N, m):
    Nx, Ny, Nz = N
    return cos_basis(Nx, m), cos_basis(Ny, m), cos_basis(Nz, m)


def analysis(x, N, m):
    """xh[k, c] = (1/Nn) sum_i phi_k(i) x[i, c], k flat = (kz m + ky) m + kx."""
    Nx, Ny, Nz = N
    fx, fy, fz = _bases(N, m)
    C = x.shape[1]
    g = x.reshape(Nz, Ny, Nx, C)
    t = np.einsum("zyxc,xa->zyac", g, fx)
    t = np.einsum("zyac,yb->zbac", t, fy)
    t = np.einsum("zbac,zd->dbac", t, fz)
    return t.reshape(m ** 3, C) / (Nx * Ny * Nz)


def synthesis(yh, N, m):
    """S[i, o] = sum_k phi_k(i) yh[k, o]."""
    Nx, Ny, Nz = N
    fx, fy, fz = _bases(N, m)
    O = yh.shape[1]
    t = yh.reshape(m, m, m, O)                       # (kz, ky, kx, o)
    t = np.einsum("dbac,zd->zbac", t, fz)
    t = np.einsum("zbac,yb->zyac", t, fy)
    t = np.einsum("zyac,xa->zyxc", t, fx)
    return t.reshape(Nx * Ny * Nz, O)


def spectral(x, Ws, N, m):
    xh = analysis(x, N, m)
    yh = np.einsum("koc,kc->ko", Ws, xh)
    return synthesis(yh, N, m), xh


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------

def forward(p, f, N, blocks=None, m=None):
    """Returns y [Nn, cout] and the cache for backward."""
    if m is None:
        m = round(p["Ws0"].shape[0] ** (1 / 3)) if "Ws0" in p else 1
    if blocks is None:
        blocks = sum(1 for k in p if k.startswith("Ws"))
    cache = {"f": f, "x": [], "z": [], "xh": []}
    x = f @ p["Wl"].T + p["bl"]
    cache["x"].append(x)
    for b in range(blocks):
        s, xh = spectral(x, p[f"Ws{b}"], N, m)
        z = s + x @ p[f"W{b}"].T + p[f"c{b}"]
        x = gelu(z)
        cache["xh"].append(xh)
        cache["z"].append(z)
        cache["x"].append(x)
    hp = x @ p["Wp1"].T + p["bp1"]
    h = gelu(hp)
    y = h @ p["Wp2"].T + p["bp2"]
    cache.update(hp=hp, h=h, N=N, m=m, blocks=blocks)
    return y, cache


def loss(y, t, b=None):
    """sum (y - t)^2 / (sum t^2 + sum b^2) and its gradient with respect to y."""
    s = float((t * t).sum()) + (0.0 if b is None else float((b * b).sum()))
    d = y - t
    return float((d * d).sum()) / s, 2.0 * d / s


def backward(p, cache, dy):
    """Gradients of sum(dy * y) with respect to every parameter."""
    N, m, blocks = cache["N"], cache["m"], cache["blocks"]
    Nn = cache["f"].shape[0]
    g = {}
    g["Wp2"] = dy.T @ cache["h"]
    g["bp2"] = dy.sum(0)
    dhp = (dy @ p["Wp2"]) * gelu_grad(cache["hp"])
    g["Wp1"] = dhp.T @ cache["x"][blocks]
    g["bp1"] = dhp.sum(0)
    dx = dhp @ p["Wp1"]
    for b in reversed(range(blocks)):
        dz = dx * gelu_grad(cache["z"][b])
        xin = cache["x"][b]
        g[f"W{b}"] = dz.T @ xin
        g[f"c{b}"] = dz.sum(0)
        # S = synth(Ws . analysis(x)); synth's adjoint is the plain basis sum,
        # analysis's adjoint carries its 1/Nn.
        dyh = analysis(dz, N, m) * Nn
        g[f"Ws{b}"] = np.einsum("ko,kc->koc", dyh, cache["xh"][b])
        dxh = np.einsum("koc,ko->kc", p[f"Ws{b}"], dyh)
        dx = dz @ p[f"W{b}"] + synthesis(dxh, N, m) / Nn
    g["Wl"] = dx.T @ cache["f"]
    g["bl"] = dx.sum(0)
    return g


def adam(vec, grad, mom, vel, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) of the flat parameter vector;
    step counts from 1.  Returns new (vec, mom, vel)."""
    mom = beta1 * mom + (1 - beta1) * grad
    vel = beta2 * vel + (1 - beta2) * grad * grad
    mh = mom / (1 - beta1 ** step)
    vh = vel / (1 - beta2 ** step)
    return vec - lr * mh / (np.sqrt(vh) + eps), mom, vel


# ---------------------------------------------------------------------------
# input channels
# ---------------------------------------------------------------------------

def start_scale(n):
    return 1e-3 * float(min(n))


def first_iterate(prob):
    """u after one iteration from the plain start, [3, Nz, Ny, Nx]."""
    if prob.sphere is None:
        from .solver import Solver
        s = Solver.from_problem(prob)
        return s.solve(tol=0.0, max_iter=1, acv=prob.acv, period=prob.acv_period)["u"]
    from .contact import ContactSolver
    sp = prob.sphere
    cs = ContactSolver(prob.n, prob.lam, prob.mu, prob.bc, face=sp.face, radius=sp.radius,
                       strong=prob.strong, average=prob.average, r0_factor=prob.r0_factor)
    return cs.solve_increment(None, sp.center, tol=0.0, max_iter=1, acv=prob.acv, period=prob.acv_period)["u"]


def features(prob, u1=None):
    """[Nn, 12] input channels of a problem (see the module header); u1 is the first
    iterate (computed when not given)."""
    plan = Plan(prob.n, prob.bc)
    nx, ny, nz = prob.n
    Nx, Ny, Nz = plan.N
    lam, mu = np.asarray(prob.lam, np.float64), np.asarray(prob.mu, np.float64)
    den = lam + mu
    safe = np.where(den > 0, den, 1.0)
    E = np.where(den > 0, mu * (3 * lam + 2 * mu) / safe, 0.0)
    nu = np.where(den > 0, lam / (2 * safe), 0.0)
    Emax = E.max() if E.max() > 0 else 1.0
    Esum = np.zeros((Nz, Ny, Nx))
    nusum = np.zeros((Nz, Ny, Nx))
    cnt = np.zeros((Nz, Ny, Nx))
    # a node touches the voxels at offsets -1 and 0 on each axis (wrapped on periodic axes)
    for dz in (-1, 0):
        for dy in (-1, 0):
            for dx in (-1, 0):
                for z in range(Nz):
                    vz = z + dz
                    if plan.periodic[2]:
                        vz %= nz
                    elif not 0 <= vz < nz:
                        continue
                    ys = np.arange(Ny) + dy
                    xs = np.arange(Nx) + dx
                    if plan.periodic[1]:
                        ys %= ny
                    if plan.periodic[0]:
                        xs %= nx
                    oky = (ys >= 0) & (ys < ny)
                    okx = (xs >= 0) & (xs < nx)
                    for y in np.flatnonzero(oky):
                        row = np.flatnonzero(okx)
                        Esum[z, y, row] += E[vz, ys[y], xs[row]]
                        nusum[z, y, row] += nu[vz, ys[y], xs[row]]
                        cnt[z, y, row] += 1
    f = np.zeros((Nz, Ny, Nx, 12))
    f[..., 0] = Esum / cnt / Emax
    f[..., 1] = nusum / cnt
    su = start_scale(prob.n)
    for c in range(3):
        f[..., 2 + c] = plan.amask[c]
    for s in prob.strong:
        for (i, j, k), c, v in zip(s.node, s.comp, s.value):
            f[k, j, i, 2 + c] = 1.0
            f[k, j, i, 5 + c] = v / su
    if prob.sphere is not None:
        sp = prob.sphere
        a, side = sp.face // 2, sp.face % 2
        idx = 0 if side == 0 else prob.n[a]
        zz, yy, xx = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
        X = np.stack([xx, yy, zz], -1).astype(np.float64)
        g = np.linalg.norm(X - np.asarray(sp.center, np.float64), axis=-1) - sp.radius
        on = [xx, yy, zz][a] == idx
        f[..., 8] = np.where(on, np.tanh(g / (8.0 * su)), 0.0)
    if u1 is None:
        u1 = first_iterate(prob)
    u1 = np.asarray(u1, np.float64).reshape(3, Nz, Ny, Nx)
    for c in range(3):
        f[..., 9 + c] = u1[c] / su
    return f.reshape(-1, 12)
