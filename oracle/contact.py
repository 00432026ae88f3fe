"""Algorithm 2: small-strain frictionless contact with a rigid sphere (active set), and
Algorithm 3: the same with the finite-strain stress (finite_strain=True).

Paper, Section 5.1, eq (24)-(28) and Algorithm 2.  For one load increment:
start from the previous displacement, move the sphere, set the active zone C
to the face nodes whose gap is negative, and iterate the fixed point of
Algorithm 1 with
  proj_U on C: radial projection of the deformed node onto the sphere
  proj_P on C: remove the normal component p.n_c
and a conditional update of C from V_gap (nodes off C with g < 0) and
V_react (nodes on C with f_nc > 0).

Readings:
 * Sign of proj_U (eq 27/28 and the projection step of Algorithm 2 disagree with the definition
   of n_c): M + u <- O' + R (M' - O') / |M' - O'|, the radial projection of
   the deformed point M' = M + u; gap g = |M' - O'| - R; n_c = -(M' - O')/|.|.
 * f_nc = -2^-b p . n_c, from p before the contact projection (the in-cell
   sum, i.e. a layer of null stress outside the face).
 * C is updated only when V_gap and V_react both equal their values at the
   previous iteration, the residual is below the gate (1e-2), and at least one
   of them is non-empty; a change of C restarts Anderson (i = 0).  Strict
   inequalities g < 0 and f_nc > 0.
 * The residual is tested after the contact projection; the loop ends when
   it is below tol and V_gap and V_react are both empty.
 * Finite strain (Section 5.2, eq 29, Algorithm 3): PK1 of the Saint-Venant-Kirchhoff law
   replaces sigma in the residual, in f_nc = -2^-b div(PK1).n_c and in the force
   F = -A0 <PK1_aa> (Section 5.4); contact geometry and projections are unchanged.
Parity against the paper's iteration counts: unpinned.
"""
from __future__ import annotations

import numpy as np

from . import tetra2
from .solver import Anderson, Solver


class ContactSolver(Solver):
    def __init__(self, n, lam, mu, bc, face, radius, strong=(), average=(), r0_factor=5.0,
                 lam0=None, mu0=None, finite_strain=False):
        super().__init__(n, lam, mu, bc, strong, average, r0_factor, lam0, mu0, finite_strain=finite_strain)
        self.radius = float(radius)
        axis, side = divmod(int(face), 2)
        Nx, Ny, Nz = self.plan.N
        kk, jj, ii = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
        coord = [ii, jj, kk][axis]
        on = coord == (0 if side == 0 else self.plan.n[axis])
        self.face_nodes = np.flatnonzero(on.ravel())
        self.X = np.stack([ii.ravel()[self.face_nodes], jj.ravel()[self.face_nodes],
                           kk.ravel()[self.face_nodes]], -1).astype(np.float64)
        self.face_axis = axis
        self.side_sign = 1.0 if side == 1 else -1.0

    def geometry(self, u, center):
        """Deformed positions M', gap g and normal n_c at every face node."""
        uf = u.reshape(3, -1)[:, self.face_nodes].T
        Mp = self.X + uf
        d = Mp - center[None]
        r = np.linalg.norm(d, axis=1)
        g = r - self.radius
        nc = -d / r[:, None]
        return Mp, g, nc

    def proj_U_contact(self, u, center, C):
        Mp, _, nc = self.geometry(u, center)
        target = center[None] - self.radius * nc          # O' + R (M'-O')/|M'-O'|
        uf = u.reshape(3, -1)
        sel = self.face_nodes[C]
        uf[:, sel] = (target[C] - self.X[C]).T
        return u

    def solve_increment(self, u_prev, center, tol=1e-6, max_iter=2000, gate=1e-2,
                        acv="P", period=2, history=False):
        center = np.asarray(center, np.float64)
        u = self.zeros() if u_prev is None else np.array(u_prev, dtype=np.float64, copy=True)
        u[self.plan.amask] = 0.0
        self.cons.proj_U(u)
        _, g, _ = self.geometry(u, center)
        C = g < 0.0                                        # initial active zone
        self.proj_U_contact(u, center, C)
        acc = Anderson(4, period)
        w2b_face = self.plan.w2b.ravel()[self.face_nodes]
        i = 0
        it = 0
        prev = None
        updates = restarts = 0
        hist = []
        converged = False
        while True:
            if acv == "U":
                u = acc.step(i, u)
            p, sig, s2, G = self.stress_residual(u)
            f_s, f_w = self.cons.proj_P(p)
            _, g, nc = self.geometry(u, center)
            pf = p.reshape(3, -1)
            pface = pf[:, self.face_nodes].T                  # [m, 3]
            pn = np.sum(pface * nc, axis=1)
            f_nc = -pn / w2b_face
            pface_proj = pface - (pn * C)[:, None] * nc
            pf[:, self.face_nodes] = pface_proj.T
            res = self.residual(float(np.sum(p * p)), s2)
            hist.append(res)
            if not np.isfinite(res):
                break
            Vgap = (~C) & (g < 0.0)
            Vreact = C & (f_nc > 0.0)
            if res < tol and not Vgap.any() and not Vreact.any():
                converged = True
                break
            if it >= max_iter:
                break
            if (prev is not None and np.array_equal(prev[0], Vgap) and np.array_equal(prev[1], Vreact)
                    and res < gate and (Vgap.any() or Vreact.any())):
                Cold = C
                C = (C | Vgap) & ~Vreact
                updates += 1
                if not np.array_equal(C, Cold):
                    i = 0
                    restarts += 1
            prev = (Vgap, Vreact)
            ptil = p - self.reference_term(G)
            if acv == "P":
                ptil = acc.step(i, ptil)
            u = self.green.apply(ptil)
            u[self.plan.amask] = 0.0
            self.cons.proj_U(u)
            self.proj_U_contact(u, center, C)
            i += 1
            it += 1
        # compressive force along the face normal, from the mean stress (Section 5.4)
        # and from the sum of contact reactions; the two agree at equilibrium
        A0 = float(np.prod([self.plan.n[J] for J in range(3) if J != self.face_axis]))
        ms = tetra2.mean_stress(sig)
        a = self.face_axis
        out = dict(u=u, iterations=it, converged=converged, residual=hist[-1], C=C, f_nc=f_nc,
                   updates=updates, restarts=restarts, gap=g,
                   force_mean_stress=-A0 * ms[a, a],
                   force_contact=-self.side_sign * float(np.sum((f_nc * nc[:, a])[C])),
                   contact_nodes=int(C.sum()), mean_stress=ms)
        if history:
            out["history"] = np.array(hist)
        return out


def hertz_force(E, nu, R, d):
    """Hertz, eq (30): F = 4 E / (3 (1 - nu^2)) sqrt(R d^3)."""
    return 4.0 * E / (3.0 * (1.0 - nu * nu)) * np.sqrt(R * d ** 3)


def hertz_radius(R, d):
    return np.sqrt(R * d)
