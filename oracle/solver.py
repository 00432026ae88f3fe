"""Algorithm 1: displacement-based fixed point with local kinematic constraints.

Paper, Section 4.1.1, eq (9) and Algorithm 1, with the relations on several nodes of
Section 4.2 (averages, eq 10-14; smoothly applied conditions, eq 15-17; see relations.py).
One iteration:

  sigma = C : grad^s_D(u)
  p = div_D(sigma)
  proj_P: strong DOFs p = 0, relation supports per eq 14 / eq 17
  exit if h ||p|| / ||sigma|| < tol                        (eq 5)
  p~ = p - div_D(R0 : grad_D u)
  Anderson on p~ (ACV_P) or on u (ACV_U)
  u = DT^-1( G_hat DT(p~) )                                (eq 3, right)
  proj_U: strong DOFs u = U, relation supports per eq 11 / eq 15

Readings (the paper defers these details to other work):
 * Anderson: type II with mixing 1 over the last four pairs
   (S_k, R_k = g(S_k) - S_k); alpha minimises ||sum alpha_k R_k|| with
   sum alpha_k = 1 from the FP64 Gram matrix, regularised by
   1e-14 tr(G)/4 on the diagonal; accelerated value sum alpha_k (S_k + R_k);
   applied when i >= 4 and i mod period == 0; ring slot i mod 4.
   Parity against the paper's iteration counts: unpinned.
 * Equilibrium norm (eq 5): ||div sigma|| is the Euclidean norm of the
   boundary-weighted p after proj_P; ||sigma||^2 = sum over voxels and both
   IPs of (1/2) sigma:sigma; h = 1.
 * Reactions (Section 4.1.3): the physical nodal force is 2^-b p; the
   reaction of a strong DOF is f = -2^-b p before proj_P, that of a relation the total
   force it applies (relations.py).
 * Relations act on the physical (2^-b weighted) residual.
"""
from __future__ import annotations

import numpy as np

from . import hex1, relations, tetra2
from .green import Green, reference_from_factor
from .plan import Plan


class Anderson:
    """Ring buffers of four (solution, residual) pairs and the accelerated combination."""

    def __init__(self, depth=4, period=2, reg=1e-14):
        self.depth, self.period, self.reg = depth, period, reg
        self.S = [None] * depth
        self.R = [None] * depth
        self.last_alpha = None

    def alpha(self):
        d = self.depth
        G = np.empty((d, d))
        for k in range(d):
            for l in range(d):
                G[k, l] = float(np.dot(self.R[k].ravel(), self.R[l].ravel()))
        G = G + self.reg * np.trace(G) / d * np.eye(d)
        try:
            y = np.linalg.solve(G, np.ones(d))
        except np.linalg.LinAlgError:
            return None
        s = y.sum()
        if not np.isfinite(s) or s == 0.0 or not np.all(np.isfinite(y)):
            return None
        return y / s

    def step(self, i, x):
        """Store the residual, optionally accelerate, store the solution (Algorithm 1, ACV blocks)."""
        d = self.depth
        if i > 0:
            self.R[(i - 1) % d] = x - self.S[(i - 1) % d]
        self.last_alpha = None
        if i >= d and i % self.period == 0:
            a = self.alpha()
            if a is not None:
                self.last_alpha = a
                x = sum(a[k] * (self.S[k] + self.R[k]) for k in range(d))
        self.S[i % d] = x.copy()
        return x


class Constraints:
    """Strong nodal DOFs and relations on several nodes (averages, smooth conditions)."""

    def __init__(self, plan, strong=(), average=(), smooth=()):
        self.plan = plan
        Nx, Ny, Nz = plan.N
        sc, sn, sv, ss = [], [], [], []
        for s in strong:
            node = np.asarray(s.node, np.int64).reshape(-1, 3)
            comp = np.asarray(s.comp, np.int64).ravel()
            val = np.asarray(s.value, np.float64).ravel()
            flat = node[:, 0] + Nx * (node[:, 1] + Ny * node[:, 2])
            keep = ~plan.amask.reshape(3, -1)[comp, flat]
            if np.any(~keep & (val != 0.0)):
                raise ValueError("nonzero value prescribed on an eliminated (A) DOF")
            sc.append(comp[keep]); sn.append(flat[keep]); sv.append(val[keep])
            ss.append(np.full(int(keep.sum()), s.set_id, np.int64))
        self.s_comp = np.concatenate(sc) if sc else np.zeros(0, np.int64)
        self.s_node = np.concatenate(sn) if sn else np.zeros(0, np.int64)
        self.s_val = np.concatenate(sv) if sv else np.zeros(0)
        self.s_set = np.concatenate(ss) if ss else np.zeros(0, np.int64)
        self.rel = relations.relations_from(plan, average, smooth)
        Nn = Nx * Ny * Nz
        relations.check_relations(plan, self.rel, self.s_comp * Nn + self.s_node)
        self.w2b = plan.w2b.ravel()

    def proj_U(self, u):
        uf = u.reshape(3, -1)
        uf[self.s_comp, self.s_node] = self.s_val
        relations.proj_U(u, self.rel)
        return u

    def proj_P(self, p):
        """Projects p in place and returns (strong reactions [m], relation reactions [r])."""
        pf = p.reshape(3, -1)
        f_strong = -pf[self.s_comp, self.s_node] / self.w2b[self.s_node]
        pf[self.s_comp, self.s_node] = 0.0
        f_rel = relations.proj_P(p, self.rel, self.w2b)
        return f_strong, f_rel

    def totals(self, f_strong, f_rel, nsets):
        out = np.zeros((nsets, 3))
        np.add.at(out, (self.s_set, self.s_comp), f_strong)
        for r, rel in enumerate(self.rel):
            out[rel.set_id, rel.comp] += f_rel[r]
        return out


class Solver:
    def __init__(self, n, lam, mu, bc, strong=(), average=(), r0_factor=1.0, lam0=None, mu0=None, smooth=(),
                 finite_strain=False, scheme="tetra2", reference="paux"):
        self.plan = Plan(n, bc)
        self.lam = np.asarray(lam, np.float64)
        self.mu = np.asarray(mu, np.float64)
        if lam0 is None:
            lam0, mu0 = reference_from_factor(self.lam, self.mu, r0_factor)
        self.lam0, self.mu0 = lam0, mu0
        self.scheme, self.reference = scheme, reference
        if reference == "iso":
            self.green = (hex1.IsoGreenPeriodic(self.plan, lam0, mu0) if all(self.plan.periodic)
                          else hex1.IsoGreenDTT(self.plan, lam0, mu0))
            if scheme != "hex1":
                raise ValueError("the isotropic reference medium is built for the HEX1 scheme")
        else:
            self.green = Green(self.plan, lam0, mu0, scheme)
        self.cons = Constraints(self.plan, strong, average, smooth)
        self.finite_strain = bool(finite_strain)
        self.nsets = 1 + max([s.set_id for s in strong] + [a.set_id for a in average] +
                             [m.set_id for m in smooth] + [0])

    @classmethod
    def from_problem(cls, prob):
        return cls(prob.n, prob.lam, prob.mu, prob.bc, prob.strong, prob.average, prob.r0_factor,
                   smooth=prob.smooth, finite_strain=prob.finite_strain, scheme=prob.scheme,
                   reference=prob.reference)

    def zeros(self):
        return np.zeros((3,) + tuple(self.plan.N[J] for J in (2, 1, 0)))

    # -- stages -----------------------------------------------------------
    def stress_residual(self, u):
        """Stress and divergence: boundary-weighted p = 2^b div_D(sigma) (A-DOFs 0), sigma, ||sigma||^2.
        Finite strain (Algorithm 3, lines 10-11): sigma is PK1 of the Saint-Venant-Kirchhoff law."""
        if self.scheme == "hex1":
            G = hex1.gradients(u, self.plan)
        else:
            G = tetra2.tet_gradients(u, self.plan)
        if self.finite_strain:
            sig = tetra2.stress_svk(G, self.lam, self.mu)
        else:
            sig = tetra2.stress(G, self.lam, self.mu)
        if self.scheme == "hex1":
            p = self.plan.w2b[None] * hex1.divergence(sig, self.plan)
            s2 = hex1.stress_norm2(sig)
        else:
            p = self.plan.w2b[None] * tetra2.divergence(sig, self.plan)
            s2 = tetra2.stress_norm2(sig)
        p[self.plan.amask] = 0.0
        return p, sig, s2, G

    def reference_term(self, G):
        """Reference-medium term: 2^b div_D(R0 : grad_D u) (A-DOFs 0)."""
        if self.scheme == "hex1":
            flux = hex1.iso(G, self.lam0, self.mu0) if self.reference == "iso" else tetra2.paux(G, self.lam0, self.mu0)
            q = self.plan.w2b[None] * hex1.divergence(flux, self.plan)
            q[self.plan.amask] = 0.0
            return q
        q = self.plan.w2b[None] * tetra2.divergence(tetra2.paux(G, self.lam0, self.mu0), self.plan)
        q[self.plan.amask] = 0.0
        return q

    def iterate_parts(self, u):
        """K1 semantics for one u: returns dict with p (after proj_P), p_tilde, norms, reactions."""
        p, sig, s2, G = self.stress_residual(u)
        f_s, f_w = self.cons.proj_P(p)
        res_num = float(np.sum(p * p))
        ptil = p - self.reference_term(G)
        return dict(p=p, ptil=ptil, sig=sig, sig2=s2, pnorm2=res_num, f_strong=f_s, f_weak=f_w)

    @staticmethod
    def residual(pnorm2, sig2):
        """Equilibrium measure of eq (5), ||p|| / ||sigma||; undefined (NaN) once either norm
        is no longer finite: the iteration has diverged, whatever the quotient would say."""
        if not (np.isfinite(pnorm2) and np.isfinite(sig2)):
            return np.nan
        if pnorm2 == 0.0:
            return 0.0
        if sig2 == 0.0:
            return np.inf
        return float(np.sqrt(pnorm2) / np.sqrt(sig2))

    # -- Algorithm 1 --------------------------------------------------------
    def solve(self, u0=None, tol=1e-8, max_iter=2000, acv="P", period=2, history=False, snapshots=()):
        """snapshots: iteration counts after which a copy of u is kept (out["snapshots"][k])."""
        u = self.zeros() if u0 is None else np.array(u0, dtype=np.float64, copy=True)
        u[self.plan.amask] = 0.0
        self.cons.proj_U(u)
        acc = Anderson(4, period)
        hist = []
        snap = {}
        it = 0
        converged = False
        parts = None
        while True:
            i = it
            if acv == "U":
                u = acc.step(i, u)
            parts = self.iterate_parts(u)
            res = self.residual(parts["pnorm2"], parts["sig2"])
            hist.append(res)
            if not np.isfinite(res):
                break
            if res < tol:
                converged = True
                break
            if it >= max_iter:
                break
            ptil = parts["ptil"]
            if acv == "P":
                ptil = acc.step(i, ptil)
            u = self.green.apply(ptil)
            u[self.plan.amask] = 0.0
            self.cons.proj_U(u)
            it += 1
            if it in snapshots:
                snap[it] = u.copy()
        tot = self.cons.totals(parts["f_strong"], parts["f_weak"], self.nsets)
        out = dict(u=u, iterations=it, converged=converged, residual=hist[-1], totals=tot,
                   f_strong=parts["f_strong"], f_weak=parts["f_weak"],
                   mean_stress=(hex1 if self.scheme == "hex1" else tetra2).mean_stress(parts["sig"]))
        if history:
            out["history"] = np.array(hist)
        if snapshots:
            out["snapshots"] = snap
        return out
