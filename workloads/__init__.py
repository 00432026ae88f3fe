"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only builds inputs: grid sizes, per-voxel Lame fields, boundary
condition tables, constraint node sets with prescribed values, obstacle
parameters and solver settings.  It performs none of the solver's arithmetic
(no gradients, transforms, Green operator, projections or acceleration), so
both the CPU oracle and the GPU path can consume the same arrays.

Units are voxel units (h = 1).  Node (i, j, k) sits at integer position
(x, y, z) = (i, j, k); voxel (i, j, k) spans [i, i+1] x [j, j+1] x [k, k+1].
Field layout is [z][y][x] (x fastest); vector fields are [3][z][y][x].

Boundary conditions follow the per-face, per-component description of the
paper (Section 3.2.1): bc[comp][axis][face] with face 0 at x_J = 0 and face 1
at x_J = n_J, and the codes below.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
from scipy.spatial import cKDTree

BC_N, BC_D, BC_P = 0, 1, 2
BASE_SEED = 260726082


def lame(E, nu):
    """Isotropic Lame constants (lambda, mu) from Young's modulus and Poisson ratio."""
    E = np.asarray(E, dtype=np.float64)
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


@dataclass
class Strong:
    """Strong nodal constraints: u[comp[k]] at node[k] = value[k] (Section 4.1)."""
    node: np.ndarray          # int64 (i, j, k) triples, shape [m, 3]
    comp: np.ndarray          # int8, shape [m]
    value: np.ndarray         # float64, shape [m]
    set_id: int = 0


@dataclass
class Average:
    """Kinematic relation: mean of u[comp] over a k-node support = value (eq 10: the 8 corners
    of a voxel or the 4 of a face; Section 4.2.3: the 44 nodes of a line of ten voxels)."""
    support: np.ndarray       # int64 node triples, shape [m, k, 3], 2 <= k <= 64
    comp: np.ndarray          # int8, shape [m]
    value: np.ndarray         # float64, shape [m]
    set_id: int = 0


@dataclass
class Smooth:
    """Smoothly applied condition: u[comp] at node = value, reaction spread over the
    neighbouring nodes with the weights of Table 2 (Section 4.2.2, eq 15-17)."""
    node: np.ndarray          # int64 (i, j, k) triples, shape [m, 3]
    comp: np.ndarray          # int8, shape [m]
    value: np.ndarray         # float64, shape [m]
    set_id: int = 0


@dataclass
class Sphere:
    """Rigid spherical obstacle (Section 5): centre, radius, potential-contact face."""
    center: np.ndarray        # float64 [3] (x, y, z)
    radius: float
    face: int                 # axis*2 + side; the contact face of the block


@dataclass
class Problem:
    name: str
    n: tuple                  # voxels (nx, ny, nz)
    lam: np.ndarray           # float64 [nz, ny, nx]
    mu: np.ndarray            # float64 [nz, ny, nx]
    bc: np.ndarray            # int8 [3, 3, 2]
    strong: List[Strong] = field(default_factory=list)
    average: List[Average] = field(default_factory=list)
    smooth: List[Smooth] = field(default_factory=list)
    sphere: Optional[Sphere] = None
    r0_factor: float = 1.0    # reference medium = factor * (max lambda, max mu)
    finite_strain: bool = False   # Saint-Venant-Kirchhoff PK1 instead of linear stress (Section 5.2)
    scheme: str = "tetra2"        # discrete gradient: "tetra2" or "hex1" (Section 3.1.2)
    reference: str = "paux"       # reference medium: "paux" or "iso" (isotropic; periodic cells)
    tol: float = 1e-6
    acv: str = "P"            # "NONE", "U" or "P"
    acv_period: int = 2
    max_iter: int = 2000
    meta: dict = field(default_factory=dict)


def _nodes_box(xs, ys, zs):
    g = np.stack(np.meshgrid(np.asarray(xs), np.asarray(ys), np.asarray(zs), indexing="ij"), -1)
    return g.reshape(-1, 3).astype(np.int64)


def bc_table(default=BC_N):
    return np.full((3, 3, 2), default, dtype=np.int8)


# ---------------------------------------------------------------------------
# Random two-phase microstructures (non-overlapping spheres)
# ---------------------------------------------------------------------------

def random_spheres(rng, n, phi_target, rmin_frac=0.02, rmax_frac=0.10, max_tries=100000, block=512,
                   return_geometry=False):
    """Place non-overlapping spheres uniformly in the cell until the voxelised
    inclusion fraction reaches phi_target.  Returns (mask [nz,ny,nx] bool, phi).

    Candidates (radius, centre) are drawn in blocks and accepted in draw order: a
    candidate is kept if it overlaps no sphere kept before it."""
    nx, ny, nz = n
    L = float(min(n))
    mask = np.zeros((nz, ny, nx), dtype=bool)
    centers = np.zeros((0, 3))
    radii = np.zeros(0)
    total = nx * ny * nz
    count = 0
    tries = 0
    while tries < max_tries and count < phi_target * total:
        m = min(block, max_tries - tries)
        tries += m
        u = rng.random((m, 4))
        r = rmin_frac * L + (rmax_frac - rmin_frac) * L * u[:, 0]
        c = u[:, 1:] * np.array([nx, ny, nz], dtype=np.float64)
        ok = np.ones(m, bool)
        if len(radii):
            # Neighbours within r + max(radii) hold every sphere the candidate can touch.
            pairs = cKDTree(c).sparse_distance_matrix(cKDTree(centers), r.max() + radii.max(),
                                                       output_type="ndarray")
            hit = pairs["v"] < r[pairs["i"]] + radii[pairs["j"]]
            ok[pairs["i"][hit]] = False
        cand = np.flatnonzero(ok)
        cc, rc = c[cand], r[cand]
        clash = (((cc[:, None, :] - cc[None, :, :]) ** 2).sum(-1)
                 < (rc[:, None] + rc[None, :]) ** 2)
        taken = np.zeros(len(cand), bool)
        new_c, new_r = [], []
        for k in range(len(cand)):
            if count >= phi_target * total:
                break
            if np.any(clash[k, :k] & taken[:k]):
                continue
            taken[k] = True
            cq, rq = cc[k], rc[k]
            new_c.append(cq)
            new_r.append(rq)
            lo = np.maximum(np.floor(cq - rq).astype(int), 0)
            hi = np.minimum(np.ceil(cq + rq).astype(int) + 1, [nx, ny, nz])
            xs = np.arange(lo[0], hi[0]) + 0.5
            ys = np.arange(lo[1], hi[1]) + 0.5
            zs = np.arange(lo[2], hi[2]) + 0.5
            d2s = ((zs[:, None, None] - cq[2]) ** 2 + (ys[None, :, None] - cq[1]) ** 2
                   + (xs[None, None, :] - cq[0]) ** 2)
            sub = mask[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
            inside = d2s < rq * rq
            count += int((inside & ~sub).sum())
            sub |= inside
        if new_r:
            centers = np.concatenate([centers, np.array(new_c)])
            radii = np.concatenate([radii, np.array(new_r)])
    if return_geometry:
        return mask, count / total, centers, radii
    return mask, count / total


def voxelize_spheres(centers, radii, n):
    """Voxels whose centre lies inside one of the spheres (same rule as random_spheres)."""
    nx, ny, nz = n
    mask = np.zeros((nz, ny, nx), dtype=bool)
    for cq, rq in zip(centers, radii):
        lo = np.maximum(np.floor(cq - rq).astype(int), 0)
        hi = np.minimum(np.ceil(cq + rq).astype(int) + 1, [nx, ny, nz])
        xs = np.arange(lo[0], hi[0]) + 0.5
        ys = np.arange(lo[1], hi[1]) + 0.5
        zs = np.arange(lo[2], hi[2]) + 0.5
        d2s = ((zs[:, None, None] - cq[2]) ** 2 + (ys[None, :, None] - cq[1]) ** 2
               + (xs[None, None, :] - cq[0]) ** 2)
        mask[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] |= d2s < rq * rq
    return mask


def two_phase_lame(mask, contrast, nu=0.3):
    E = np.where(mask, contrast, 1.0)
    return lame(E, nu)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def c1_inclusion_patch():
    """16^3 block, spherical inclusion, top patch pressed through strong constraints."""
    n = (16, 16, 16)
    nx, ny, nz = n
    zc, yc, xc = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    incl = (xc - 8) ** 2 + (yc - 8) ** 2 + (zc - 8) ** 2 < 16.0
    lam, mu = lame(np.where(incl, 400.0, 200.0), 0.3)
    bc = bc_table(BC_N)
    bc[2, 2, 0] = BC_D                        # u_z = 0 on the bottom face
    patch = _nodes_box(range(4, 13), range(4, 13), [16])
    top = Strong(patch, np.full(len(patch), 2, np.int8), np.full(len(patch), -0.16), set_id=0)
    pins = Strong(np.array([[8, 8, 0], [8, 8, 0], [16, 8, 0], [8, 16, 0]], np.int64),
                  np.array([0, 1, 1, 0], np.int8), np.zeros(4), set_id=1)
    return Problem("C1", n, lam, mu, bc, strong=[top, pins], r0_factor=1.0, tol=1e-8,
                   meta={"inclusion_voxels": int(incl.sum())})


def c2_compact_tension(n=(256, 256, 16), notch_len=64, notch_h=4, radius=8.0, offset=48, disp=None):
    """Plate with a zero-stiffness notch and two pin-loaded cylinders (CT-like)."""
    nx, ny, nz = n
    lam, mu = lame(np.ones((nz, ny, nx)), 0.3)
    y0 = ny // 2 - notch_h // 2
    lam[:, y0:y0 + notch_h, :notch_len] = 0.0
    mu[:, y0:y0 + notch_h, :notch_len] = 0.0
    bc = bc_table(BC_N)
    bc[2, 2, 0] = BC_D
    bc[2, 2, 1] = BC_D
    if disp is None:
        disp = 1e-3 * nx
    xc = notch_len / 2.0
    sets = []
    for sid, (yc, val) in enumerate([(ny // 2 + offset, +disp), (ny // 2 - offset, -disp)]):
        ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="ij")
        sel = (ii - xc) ** 2 + (jj - yc) ** 2 <= radius * radius
        ij = np.stack([ii[sel], jj[sel]], -1)
        nodes = np.concatenate([np.concatenate([ij, np.full((len(ij), 1), k)], 1) for k in range(nz + 1)])
        sets.append(Strong(nodes.astype(np.int64), np.full(len(nodes), 1, np.int8),
                           np.full(len(nodes), val), set_id=sid))
    # reference medium = 2 x max stiffness: on this notched plate the plain map with
    # f = 1 already diverges at 256 x 256 x 16, and with the paper's f = 1/2 the
    # accelerated iteration stalls (oracle and GPU alike) from 128 x 128 x 16 upwards
    return Problem("C2", n, lam, mu, bc, strong=sets, r0_factor=2.0, tol=1e-6)


def c3_indentation(n=(256, 256, 128), R=96.0, d_over_R=0.002, E=1.0, nu=0.3, finite_strain=False):
    """Block fixed at the bottom, traction-free elsewhere, rigid sphere on the top face.
    finite_strain: the Saint-Venant-Kirchhoff form of Algorithm 3 with the reference factor 10
    that Section 5.4 uses for it (5 for small strain)."""
    nx, ny, nz = n
    lam, mu = lame(np.full((nz, ny, nx), E), nu)
    bc = bc_table(BC_N)
    bc[:, 2, 0] = BC_D
    d = d_over_R * R
    sph = Sphere(np.array([nx / 2.0, ny / 2.0, nz + R - d]), R, face=5)
    return Problem("C3", n, lam, mu, bc, sphere=sph, r0_factor=10.0 if finite_strain else 5.0, tol=1e-6,
                   finite_strain=finite_strain, meta={"E": E, "nu": nu, "d": d})


def periodic_centrosymmetric(n=(6, 6, 6), seed=BASE_SEED + 7_000_000, scheme="hex1", reference="iso"):
    """Cell periodic on all axes, stiffness symmetric under the point reflection x -> -x about
    node 0, and voxel-average conditions in reflected pairs with opposite values, so that the
    solution is odd: its mean and its (pi, pi, pi) coefficient vanish, the frequencies where
    the Green operator is set to 0.  Two pairs of voxels, all three components."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)

    def refl(f):
        return f[::-1, ::-1, ::-1]

    lam = rng.uniform(0.5, 2.0, (nz, ny, nx)); lam = 0.5 * (lam + refl(lam))
    mu = rng.uniform(0.4, 1.5, (nz, ny, nx)); mu = 0.5 * (mu + refl(mu))

    def vox(a, b, c):
        return [[(a + i) % nx, (b + j) % ny, (c + k) % nz] for i in (0, 1) for j in (0, 1) for k in (0, 1)]

    pairs = [((1, 1, 1), (0.02, -0.01, 0.015)), ((1, 3, 0), (-0.01, 0.02, 0.01))]
    sup, comp, val = [], [], []
    for (a, b, c), U in pairs:
        r = ((-a - 1) % nx, (-b - 1) % ny, (-c - 1) % nz)
        for cc in range(3):
            sup.append(vox(a, b, c)); comp.append(cc); val.append(U[cc])
            sup.append(vox(*r)); comp.append(cc); val.append(-U[cc])
    avg = [Average(np.array(sup, np.int64), np.array(comp, np.int8), np.array(val))]
    bc = np.full((3, 3, 2), BC_P, np.int8)
    return Problem("periodic-odd", tuple(n), lam, mu, bc, average=avg, tol=1e-8, scheme=scheme,
                   reference=reference)


def random_cell(seed, n=None, edges=(32, 48, 64, 96, 128), with_patches=True):
    """Two-phase cell with random DTT face BCs and local Dirichlet patches."""
    rng = np.random.default_rng(seed)
    if n is None:
        n = tuple(int(rng.choice(edges)) for _ in range(3))
    L = min(n)
    phi = rng.uniform(0.1, 0.4)
    mask, phi_got = random_spheres(rng, n, phi)
    contrast = float(np.exp(rng.uniform(np.log(2.0), np.log(100.0))))
    lam, mu = two_phase_lame(mask, contrast)
    while True:
        bc = (rng.random((3, 3, 2)) < 0.5).astype(np.int8)   # 1 = D, 0 = N
        if all(bc[c].any() for c in range(3)):
            break
    strong = []
    if with_patches:
        npatch = int(rng.integers(1, 5))
        used = []
        for p in range(npatch):
            for _ in range(100):
                s = int(rng.integers(4, 17))
                axis = int(rng.integers(0, 3))
                side = int(rng.integers(0, 2))
                comps = [c for c in range(3) if bc[c, axis, side] == BC_N]
                if not comps:
                    continue
                ta, tb = [a for a in range(3) if a != axis]
                if s + 1 > min(n[ta], n[tb]) - 1:
                    continue
                oa = int(rng.integers(1, n[ta] - s))
                ob = int(rng.integers(1, n[tb] - s))
                box = (axis, side, oa, ob, s)
                clash = any(u[0] == axis and u[1] == side and not (oa + s < u[2] or u[2] + u[4] < oa
                                                                  or ob + s < u[3] or u[3] + u[4] < ob)
                            for u in used)
                if clash:
                    continue
                used.append(box)
                idx = np.zeros((s * s, 3), np.int64)
                aa, bb = np.meshgrid(np.arange(oa, oa + s), np.arange(ob, ob + s), indexing="ij")
                idx[:, ta] = aa.ravel()
                idx[:, tb] = bb.ravel()
                idx[:, axis] = 0 if side == 0 else n[axis]
                for c in comps:
                    val = rng.uniform(-1.0, 1.0) * 1e-3 * L / np.sqrt(3.0)
                    strong.append(Strong(idx.copy(), np.full(len(idx), c, np.int8),
                                         np.full(len(idx), val), set_id=len(strong)))
                break
    return Problem(f"cell{seed}", n, lam, mu, bc, strong=strong, r0_factor=1.0, tol=1e-6,
                   meta={"phi": phi_got, "contrast": contrast})


def c4_batch(count=64, base_seed=BASE_SEED):
    return [random_cell(base_seed + c) for c in range(count)]


def nn_case_spec(seed, kind=None, n0=(64, 64, 64)):
    """Draws of a learned-start case at resolution n0 (geometry, material, loading);
    nn_case_build turns them into a Problem.  Without kind, even seeds give patch
    cases and odd seeds indentation cases."""
    rng = np.random.default_rng(seed)
    if kind is None:
        kind = "patch" if seed % 2 == 0 else "indent"
    phi = rng.uniform(0.1, 0.4)
    _, phi_got, cen, rad = random_spheres(rng, n0, phi, return_geometry=True)
    contrast = float(np.exp(rng.uniform(np.log(2.0), np.log(100.0))))
    spec = {"seed": int(seed), "kind": kind, "n0": tuple(int(v) for v in n0), "phi": phi_got,
            "centers": cen, "radii": rad, "contrast": contrast}
    if kind == "indent":
        spec["d_over_R"] = float(rng.uniform(0.002, 0.03))
        return spec
    while True:
        bc = (rng.random((3, 3, 2)) < 0.5).astype(np.int8)
        if all(bc[c].any() for c in range(3)):
            break
    patches, used = [], []
    for p in range(int(rng.integers(1, 5))):
        for _ in range(100):
            s = int(rng.integers(4, 17))
            axis = int(rng.integers(0, 3))
            side = int(rng.integers(0, 2))
            comps = [c for c in range(3) if bc[c, axis, side] == BC_N]
            if not comps:
                continue
            ta, tb = [a for a in range(3) if a != axis]
            if s + 1 > min(n0[ta], n0[tb]) - 1:
                continue
            oa = int(rng.integers(1, n0[ta] - s))
            ob = int(rng.integers(1, n0[tb] - s))
            if any(u[0] == axis and u[1] == side and not (oa + s < u[2] or u[2] + u[4] < oa
                                                          or ob + s < u[3] or u[3] + u[4] < ob)
                   for u in used):
                continue
            used.append((axis, side, oa, ob, s))
            vals = [(c, float(rng.uniform(-1.0, 1.0))) for c in comps]
            patches.append((axis, side, oa, ob, s, vals))
            break
    spec["bc"] = bc
    spec["patches"] = patches
    return spec


def nn_case_build(spec, scale=1):
    """Problem of a learned-start case voxelised at scale * n0 (geometry scaled with it).

    patch: the drawn DTT face BCs and 1-4 local Dirichlet patches (value
    U[-1, 1] 1e-3 L / sqrt(3) per free component, L = min n0, scaled with the cell);
    indent: bottom face fixed, other faces traction-free, rigid sphere of radius
    0.75 nz pressed into the top face to depth d."""
    k = int(scale)
    n0 = spec["n0"]
    n = tuple(v * k for v in n0)
    mask = voxelize_spheres(spec["centers"] * k, spec["radii"] * k, n)
    lam, mu = two_phase_lame(mask, spec["contrast"])
    meta = {"phi": spec["phi"], "contrast": spec["contrast"], "kind": spec["kind"], "scale": k,
            "seed": spec["seed"]}
    if spec["kind"] == "indent":
        bc = bc_table(BC_N)
        bc[:, 2, 0] = BC_D
        R0 = 0.75 * n0[2]
        d0 = spec["d_over_R"] * R0
        sph = Sphere(np.array([n[0] / 2.0, n[1] / 2.0, n[2] + k * (R0 - d0)]), k * R0, face=5)
        meta["d_over_R"] = spec["d_over_R"]
        return Problem("C5-indent", n, lam, mu, bc, sphere=sph, r0_factor=5.0, tol=1e-6,
                       max_iter=4000, meta=meta)
    L0 = min(n0)
    strong = []
    for axis, side, oa, ob, s, vals in spec["patches"]:
        ta, tb = [a for a in range(3) if a != axis]
        # s nodes span s-1 voxels at n0; the scaled patch spans k (s-1) voxels
        m = k * (s - 1) + 1
        aa, bb = np.meshgrid(np.arange(k * oa, k * oa + m), np.arange(k * ob, k * ob + m), indexing="ij")
        idx = np.zeros((m * m, 3), np.int64)
        idx[:, ta] = aa.ravel()
        idx[:, tb] = bb.ravel()
        idx[:, axis] = 0 if side == 0 else n[axis]
        for c, v in vals:
            val = k * v * 1e-3 * L0 / np.sqrt(3.0)
            strong.append(Strong(idx.copy(), np.full(len(idx), c, np.int8), np.full(len(idx), val),
                                 set_id=len(strong)))
    return Problem("C5-patch", n, lam, mu, spec["bc"].copy(), strong=strong, r0_factor=1.0, tol=1e-6,
                   max_iter=4000, meta=meta)


def nn_case(seed, kind=None, scale=1, n0=(64, 64, 64)):
    """Learned-start case: nn_case_build(nn_case_spec(seed, kind, n0), scale)."""
    return nn_case_build(nn_case_spec(seed, kind, n0), scale)


NN_TRAIN_SEED = BASE_SEED + 1_000_000
NN_EVAL_SEED = BASE_SEED + 2_000_000


def nn_init(seed, shapes):
    """Initial network parameters, flat float64: arrays of rank >= 2 drawn from
    N(0, 1/fan_in) with fan_in the last extent; rank-1 arrays (biases) zero."""
    rng = np.random.default_rng(seed)
    out = []
    for s in shapes:
        s = tuple(s)
        if len(s) >= 2:
            out.append(rng.standard_normal(int(np.prod(s))) / np.sqrt(s[-1]))
        else:
            out.append(np.zeros(int(np.prod(s))))
    return np.concatenate(out)


def m256_metric(n=(256, 256, 256), seed=BASE_SEED + 5_000_000, phi=0.25, contrast=10.0):
    """256^3 two-phase block: bottom fixed, top 16x16 node patch pressed down."""
    rng = np.random.default_rng(seed)
    mask, phi_got = random_spheres(rng, n, phi)
    lam, mu = two_phase_lame(mask, contrast)
    nx, ny, nz = n
    bc = bc_table(BC_N)
    bc[:, 2, 0] = BC_D
    cx, cy = nx // 2, ny // 2
    patch = _nodes_box(range(cx - 8, cx + 8), range(cy - 8, cy + 8), [nz])
    top = Strong(patch, np.full(len(patch), 2, np.int8), np.full(len(patch), -1e-3 * nz))
    return Problem("M256", n, lam, mu, bc, strong=[top], r0_factor=1.0, tol=0.0,
                   meta={"phi": phi_got, "contrast": contrast})


def scaled(problem_fn, n, **kw):
    return problem_fn(n=n, **kw)
