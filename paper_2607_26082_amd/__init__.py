"""Python binding of libfftc (constrained DTT/FFT elasticity solver for MI355X).

The functions below carry the names of the C ABI declared in include/fftc.h and only
marshal arguments (ctypes); every step of the solver runs in the HIP library.  PyTorch
supplies device memory and the stream.  The `Solver` class is a convenience wrapper
that creates a handle from a problem description (see workloads.Problem).

The library must be built (paper_2607_26082_amd/build.py); importing this module on a
machine without it raises ImportError -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FFTC_LIB may name another build of the same sources (the host-sanitized one)
LIB_PATH = os.environ.get("FFTC_LIB") or os.path.join(_HERE, "libfftc.so")

FFTC_OK = 0
FFTC_E_ARG, FFTC_E_BC, FFTC_E_OVERLAP, FFTC_E_WORKSPACE = -1, -2, -3, -4
FFTC_E_NOCONV, FFTC_E_NAN, FFTC_E_UNSUPPORTED, FFTC_E_STATE, FFTC_E_HIP = -5, -6, -7, -8, -9
FFTC_FP64, FFTC_FP32 = 0, 1
FFTC_ACV_NONE, FFTC_ACV_U, FFTC_ACV_P = 0, 1, 2

STAGES = ("residual", "weak+control", "anderson", "dtt_x_fwd", "dtt_y_fwd", "dtt_z_green",
          "dtt_y_inv", "dtt_x_inv", "proj_u")


class fftc_solver_cfg(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("acv", C.c_int32),
                ("depth", C.c_int32), ("period", C.c_int32), ("update_gate", C.c_double),
                ("refine_below", C.c_double), ("anchor_every", C.c_int32), ("reserved", C.c_int32)]


class fftc_report(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("residual", C.c_double),
                ("contact_updates", C.c_int32), ("anderson_restarts", C.c_int32),
                ("contact_nodes", C.c_int32), ("pad", C.c_int32),
                ("force_mean_stress", C.c_double), ("force_contact", C.c_double),
                ("mean_stress", C.c_double * 6)]


_P = C.c_void_p
_SIGS = {
    "fftc_create": (C.c_int, [C.POINTER(_P), C.POINTER(C.c_int32), C.c_double, C.c_int32, C.c_int32]),
    "fftc_destroy": (None, [_P]),
    "fftc_set_bc": (C.c_int, [_P, C.POINTER(C.c_int8)]),
    "fftc_set_reference": (C.c_int, [_P, C.c_int32, C.c_double, C.c_double]),
    "fftc_set_reference_factor": (C.c_int, [_P, C.c_int32, C.c_double]),
    "fftc_add_dirichlet": (C.c_int, [_P, C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_int8),
                                     C.POINTER(C.c_double), C.c_int32]),
    "fftc_add_average": (C.c_int, [_P, C.c_int64, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int8),
                                   C.POINTER(C.c_double), C.c_int32]),
    "fftc_add_smooth": (C.c_int, [_P, C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_int8),
                                  C.POINTER(C.c_double), C.c_int32]),
    "fftc_set_sphere": (C.c_int, [_P, C.POINTER(C.c_double), C.c_double, C.c_int32]),
    "fftc_move_sphere": (C.c_int, [_P, C.POINTER(C.c_double)]),
    "fftc_set_solver": (C.c_int, [_P, C.POINTER(fftc_solver_cfg)]),
    "fftc_set_kinematics": (C.c_int, [_P, C.c_int32]),
    "fftc_stage_residual_form": (C.c_int, [_P, _P, _P, _P, _P, _P, C.c_int32, C.c_int32, _P, _P, _P, _P,
                                           C.POINTER(C.c_double)]),
    "fftc_workspace_bytes": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "fftc_bind_workspace": (C.c_int, [_P, _P, C.c_size_t, _P]),
    "fftc_bind_workspace_static": (C.c_int, [_P, _P]),
    "fftc_set_stiffness": (C.c_int, [_P, _P, _P, C.c_int32]),
    "fftc_set_stiffness_Enu": (C.c_int, [_P, _P, _P, C.c_int32]),
    "fftc_solve": (C.c_int, [_P, _P, C.c_int32, C.POINTER(fftc_report)]),
    "fftc_get_reactions": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), C.c_int32]),
    "fftc_num_constraints": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "fftc_get_contact": (C.c_int, [_P, C.POINTER(C.c_uint8), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "fftc_num_face_nodes": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "fftc_stage_residual": (C.c_int, [_P, _P, _P, _P, C.POINTER(C.c_double)]),
    "fftc_stage_green": (C.c_int, [_P, _P, _P]),
    "fftc_iterate": (C.c_int, [_P, C.c_int32]),
    "fftc_profile_stages": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_double), C.c_int32]),
    "fftc_batch_create": (C.c_int, [C.POINTER(_P), C.c_int32, C.POINTER(_P), _P]),
    "fftc_batch_solve": (C.c_int, [_P, C.POINTER(_P), C.c_int32, C.POINTER(fftc_report)]),
    "fftc_batch_destroy": (None, [_P]),
    "fftc_batch_last_error": (C.c_char_p, [_P]),
    "fftc_nn_create": (C.c_int, [C.POINTER(_P), C.c_int32, C.c_int32]),
    "fftc_nn_destroy": (None, [_P]),
    "fftc_nn_num_params": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "fftc_nn_state_bytes": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "fftc_nn_bind_state": (C.c_int, [_P, _P, C.c_size_t, _P]),
    "fftc_nn_workspace_bytes": (C.c_int, [_P, C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_size_t)]),
    "fftc_nn_bind": (C.c_int, [_P, C.POINTER(C.c_int32), C.c_int32, _P, C.c_size_t, _P]),
    "fftc_nn_set_params": (C.c_int, [_P, _P]),
    "fftc_nn_get_params": (C.c_int, [_P, _P]),
    "fftc_nn_get_grad": (C.c_int, [_P, _P]),
    "fftc_nn_features": (C.c_int, [_P, _P, _P]),
    "fftc_nn_forward": (C.c_int, [_P, _P, _P, C.c_double, _P, _P]),
    "fftc_nn_train_step": (C.c_int, [_P, _P, _P, _P]),
    "fftc_nn_adam_step": (C.c_int, [_P, C.c_float, C.c_float, C.c_float, C.c_float]),
    "fftc_nn_make_target": (C.c_int, [_P, _P, C.c_int64, C.c_double, _P, _P]),
    "fftc_nn_last_error": (C.c_char_p, [_P]),
    "fftc_solve_judged": (C.c_int, [_P, _P, _P, C.POINTER(fftc_report), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_double)]),
    "fftc_status_str": (C.c_char_p, [C.c_int]),
    "fftc_last_error": (C.c_char_p, [_P]),
}

_lib = None


def load():
    """Load libfftc.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libfftc.so not built at {LIB_PATH}; run paper_2607_26082_amd/build.py")
    # torch first: its wheel carries its own HIP runtime, and the library must bind to the
    # runtime torch initialises (loaded the other way round, torch then finds no GPU)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return tuple(_SIGS)


class FftcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _dev(t):
    return C.c_void_p(int(t.data_ptr())) if t is not None else None


# ---------------------------------------------------------------------------
# thin wrappers, named after the C entry points
# ---------------------------------------------------------------------------

FFTC_TETRA2, FFTC_HEX1 = 0, 1
FFTC_F64, FFTC_F32 = 0, 1


def fftc_create(n, precision=FFTC_FP64, h=1.0, scheme=FFTC_TETRA2):
    lib = load()
    hd = C.c_void_p()
    arr = (C.c_int32 * 3)(*[int(v) for v in n])
    rc = lib.fftc_create(C.byref(hd), arr, float(h), int(scheme), int(precision))
    if rc != FFTC_OK:
        raise FftcError(rc, "fftc_create: " + lib.fftc_status_str(rc).decode())
    return hd


def fftc_destroy(h):
    load().fftc_destroy(h)


def _check(h, rc, what, allow=()):
    if rc != FFTC_OK and rc not in allow:
        lib = load()
        raise FftcError(rc, f"{what}: {lib.fftc_status_str(rc).decode()}: {lib.fftc_last_error(h).decode()}")
    return rc


def fftc_set_bc(h, bc):
    a = np.ascontiguousarray(np.asarray(bc, np.int8).reshape(18))
    return _check(h, load().fftc_set_bc(h, _ptr(a, C.c_int8)), "fftc_set_bc")


FFTC_REF_PAUX, FFTC_REF_ISO = 0, 1


def fftc_set_reference(h, lam0, mu0, kind=FFTC_REF_PAUX):
    return _check(h, load().fftc_set_reference(h, int(kind), float(lam0), float(mu0)), "fftc_set_reference")


def fftc_set_reference_factor(h, factor, kind=FFTC_REF_PAUX):
    return _check(h, load().fftc_set_reference_factor(h, int(kind), float(factor)), "fftc_set_reference_factor")



def fftc_add_dirichlet(h, node, comp, value, set_id=0):
    node = np.ascontiguousarray(np.asarray(node, np.int64).reshape(-1, 3))
    comp = np.ascontiguousarray(np.asarray(comp, np.int8).ravel())
    value = np.ascontiguousarray(np.asarray(value, np.float64).ravel())
    return _check(h, load().fftc_add_dirichlet(h, len(comp), _ptr(node, C.c_int64), _ptr(comp, C.c_int8),
                                               _ptr(value, C.c_double), int(set_id)), "fftc_add_dirichlet")


def fftc_add_average(h, support, comp, value, set_id=0):
    comp = np.ascontiguousarray(np.asarray(comp, np.int8).ravel())
    sup = np.ascontiguousarray(np.asarray(support, np.int64).reshape(len(comp), -1, 3))
    value = np.ascontiguousarray(np.asarray(value, np.float64).ravel())
    return _check(h, load().fftc_add_average(h, len(comp), sup.shape[1], _ptr(sup, C.c_int64),
                                             _ptr(comp, C.c_int8), _ptr(value, C.c_double), int(set_id)),
                  "fftc_add_average")


def fftc_add_smooth(h, node, comp, value, set_id=0):
    node = np.ascontiguousarray(np.asarray(node, np.int64).reshape(-1, 3))
    comp = np.ascontiguousarray(np.asarray(comp, np.int8).ravel())
    value = np.ascontiguousarray(np.asarray(value, np.float64).ravel())
    return _check(h, load().fftc_add_smooth(h, len(comp), _ptr(node, C.c_int64), _ptr(comp, C.c_int8),
                                            _ptr(value, C.c_double), int(set_id)), "fftc_add_smooth")


def fftc_set_sphere(h, center, radius, face):
    c = np.ascontiguousarray(np.asarray(center, np.float64))
    return _check(h, load().fftc_set_sphere(h, _ptr(c, C.c_double), float(radius), int(face)), "fftc_set_sphere")


def fftc_move_sphere(h, center):
    c = np.ascontiguousarray(np.asarray(center, np.float64))
    return _check(h, load().fftc_move_sphere(h, _ptr(c, C.c_double)), "fftc_move_sphere")


FFTC_SMALL_STRAIN = 0
FFTC_FINITE_STRAIN = 1


def fftc_set_kinematics(h, kind):
    return _check(h, load().fftc_set_kinematics(h, int(kind)), "fftc_set_kinematics")


def fftc_set_solver(h, tol=1e-6, max_iter=2000, acv=FFTC_ACV_P, depth=4, period=2, update_gate=1e-2,
                    refine_below=None, anchor_every=16):
    """refine_below: FP32 form, residual below which stresses are formed in FP64 (None: 10 tol).
    anchor_every: FP32 form, period of the residual passes from u between incremental ones
    (0: every pass from u)."""
    rb = 10.0 * float(tol) if refine_below is None else float(refine_below)
    cfg = fftc_solver_cfg(float(tol), int(max_iter), int(acv), int(depth), int(period), float(update_gate), rb,
                          int(anchor_every), 0)
    return _check(h, load().fftc_set_solver(h, C.byref(cfg)), "fftc_set_solver")


def fftc_workspace_bytes(h):
    b = C.c_size_t()
    _check(h, load().fftc_workspace_bytes(h, C.byref(b)), "fftc_workspace_bytes")
    return int(b.value)


def fftc_bind_workspace(h, ws, nbytes, stream):
    return _check(h, load().fftc_bind_workspace(h, _dev(ws), int(nbytes), C.c_void_p(stream)),
                  "fftc_bind_workspace")


def fftc_bind_workspace_static(h, stream):
    return _check(h, load().fftc_bind_workspace_static(h, C.c_void_p(stream)), "fftc_bind_workspace_static")


FFTC_STATIC_WORKSPACE_BYTES = 128 << 20


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return FFTC_F64
    if t.dtype == torch.float32:
        return FFTC_F32
    raise TypeError("stiffness arrays must be float64 or float32")


def fftc_set_stiffness(h, lam_dev, mu_dev):
    return _check(h, load().fftc_set_stiffness(h, _dev(lam_dev), _dev(mu_dev), _dtype_code(lam_dev)),
                  "fftc_set_stiffness")


def fftc_set_stiffness_Enu(h, E_dev, nu_dev):
    return _check(h, load().fftc_set_stiffness_Enu(h, _dev(E_dev), _dev(nu_dev), _dtype_code(E_dev)),
                  "fftc_set_stiffness_Enu")


def fftc_solve(h, u_dev, zero_start=True):
    rep = fftc_report()
    rc = load().fftc_solve(h, _dev(u_dev), 1 if zero_start else 0, C.byref(rep))
    _check(h, rc, "fftc_solve", allow=(FFTC_E_NOCONV, FFTC_E_NAN))
    return rc, rep


def fftc_get_reactions(h, nsets):
    lib = load()
    ns, nw = C.c_int64(), C.c_int64()
    lib.fftc_num_constraints(h, C.byref(ns), C.byref(nw))
    per = np.zeros(max(ns.value, 1)); rel = np.zeros(max(nw.value, 1)); tot = np.zeros((max(nsets, 1), 3))
    _check(h, lib.fftc_get_reactions(h, _ptr(per, C.c_double), _ptr(rel, C.c_double), _ptr(tot, C.c_double),
                                     int(nsets)), "fftc_get_reactions")
    return per[:ns.value], rel[:nw.value], tot[:nsets]


def fftc_get_contact(h):
    lib = load()
    m = C.c_int64()
    lib.fftc_num_face_nodes(h, C.byref(m))
    mask = np.zeros(m.value, np.uint8); fnc = np.zeros(m.value); gap = np.zeros(m.value)
    force, area = C.c_double(), C.c_double()
    _check(h, lib.fftc_get_contact(h, _ptr(mask, C.c_uint8), _ptr(fnc, C.c_double), _ptr(gap, C.c_double),
                                   C.byref(force), C.byref(area)), "fftc_get_contact")
    return mask, fnc, gap, force.value, area.value


def fftc_stage_residual(h, u_dev, p_dev=None, ptil_dev=None):
    sums = np.zeros(2)
    _check(h, load().fftc_stage_residual(h, _dev(u_dev), _dev(p_dev), _dev(ptil_dev), _ptr(sums, C.c_double)),
           "fftc_stage_residual")
    return sums


def fftc_stage_residual_form(h, u_dev, delta_dev, e_dev, pprev_dev, rprev_dev, i_local, p_dev=None, r_dev=None,
                             dr_dev=None, dy_dev=None, pass_kind=0):
    sums = np.zeros(2)
    _check(h, load().fftc_stage_residual_form(h, _dev(u_dev), _dev(delta_dev), _dev(e_dev), _dev(pprev_dev),
                                              _dev(rprev_dev), int(i_local), int(pass_kind), _dev(p_dev), _dev(r_dev),
                                              _dev(dr_dev), _dev(dy_dev), _ptr(sums, C.c_double)),
           "fftc_stage_residual_form")
    return sums


def fftc_stage_green(h, ptil_dev, u_dev):
    return _check(h, load().fftc_stage_green(h, _dev(ptil_dev), _dev(u_dev)), "fftc_stage_green")


def fftc_iterate(h, iters):
    return _check(h, load().fftc_iterate(h, int(iters)), "fftc_iterate")


def fftc_profile_stages(h, iters):
    ms = np.zeros(len(STAGES))
    _check(h, load().fftc_profile_stages(h, int(iters), _ptr(ms, C.c_double), len(STAGES)), "fftc_profile_stages")
    return dict(zip(STAGES, ms))


def fftc_batch_create(handles, stream):
    lib = load()
    bh = C.c_void_p()
    arr = (C.c_void_p * len(handles))(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    rc = lib.fftc_batch_create(C.byref(bh), len(handles), arr, C.c_void_p(stream))
    if rc != FFTC_OK:
        raise FftcError(rc, "fftc_batch_create: " + lib.fftc_status_str(rc).decode())
    return bh


def fftc_batch_solve(bh, u_devs, zero_start=True):
    lib = load()
    n = len(u_devs)
    ptrs = (C.c_void_p * n)(*[int(t.data_ptr()) for t in u_devs])
    reps = (fftc_report * n)()
    rc = lib.fftc_batch_solve(bh, ptrs, 1 if zero_start else 0, reps)
    if rc not in (FFTC_OK, FFTC_E_NOCONV, FFTC_E_NAN):
        raise FftcError(rc, "fftc_batch_solve: " + lib.fftc_batch_last_error(bh).decode())
    return rc, list(reps)


def fftc_batch_destroy(bh):
    load().fftc_batch_destroy(bh)


class Batch:
    """Batched solve of several Solver objects (same device)."""

    def __init__(self, solvers):
        self.solvers = list(solvers)
        self.stream = self.solvers[0].stream
        self.bh = fftc_batch_create([s.h for s in self.solvers], self.stream.cuda_stream)

    def solve(self, zero_start=True):
        return fftc_batch_solve(self.bh, [s.u for s in self.solvers], zero_start)

    def __del__(self):
        try:
            if getattr(self, "bh", None) is not None:
                fftc_batch_destroy(self.bh)
                self.bh = None
        except Exception:
            pass


# ---------------------------------------------------------------------------
# learned warm start (include/fftc_nn.h)
# ---------------------------------------------------------------------------

FFTC_NN_CHANNELS = 16


def _nncheck(nn, rc, what):
    if rc != FFTC_OK:
        raise FftcError(rc, f"{what}: " + load().fftc_nn_last_error(nn).decode())


def fftc_nn_create(modes=6, blocks=4):
    h = C.c_void_p()
    rc = load().fftc_nn_create(C.byref(h), int(modes), int(blocks))
    if rc != FFTC_OK:
        raise FftcError(rc, "fftc_nn_create")
    return h


def fftc_nn_destroy(nn):
    load().fftc_nn_destroy(nn)


def fftc_nn_num_params(nn):
    c = C.c_int64()
    _nncheck(nn, load().fftc_nn_num_params(nn, C.byref(c)), "fftc_nn_num_params")
    return c.value


def fftc_nn_state_bytes(nn):
    b = C.c_size_t()
    _nncheck(nn, load().fftc_nn_state_bytes(nn, C.byref(b)), "fftc_nn_state_bytes")
    return b.value


def fftc_nn_bind_state(nn, state_dev, nbytes, stream):
    _nncheck(nn, load().fftc_nn_bind_state(nn, _dev(state_dev), nbytes, C.c_void_p(stream)), "fftc_nn_bind_state")


def fftc_nn_workspace_bytes(nn, N, training):
    b = C.c_size_t()
    Na = (C.c_int32 * 3)(*[int(v) for v in N])
    _nncheck(nn, load().fftc_nn_workspace_bytes(nn, Na, int(training), C.byref(b)), "fftc_nn_workspace_bytes")
    return b.value


def fftc_nn_bind(nn, N, training, ws_dev, nbytes, stream):
    Na = (C.c_int32 * 3)(*[int(v) for v in N])
    _nncheck(nn, load().fftc_nn_bind(nn, Na, int(training), _dev(ws_dev), nbytes, C.c_void_p(stream)),
             "fftc_nn_bind")


def fftc_nn_set_params(nn, params_dev):
    _nncheck(nn, load().fftc_nn_set_params(nn, _dev(params_dev)), "fftc_nn_set_params")


def fftc_nn_get_params(nn, params_dev):
    _nncheck(nn, load().fftc_nn_get_params(nn, _dev(params_dev)), "fftc_nn_get_params")


def fftc_nn_get_grad(nn, grad_dev):
    _nncheck(nn, load().fftc_nn_get_grad(nn, _dev(grad_dev)), "fftc_nn_get_grad")


def fftc_nn_features(h, feat_dev, u1_dev):
    _check(h, load().fftc_nn_features(h, _dev(feat_dev), _dev(u1_dev)), "fftc_nn_features")


def fftc_nn_forward(nn, feat_dev, y_dev=None, s_u=1.0, base_dev=None, u0_dev=None):
    _nncheck(nn, load().fftc_nn_forward(nn, _dev(feat_dev), _dev(y_dev), float(s_u), _dev(base_dev),
                                        _dev(u0_dev)), "fftc_nn_forward")


def fftc_nn_train_step(nn, feat_dev, target_dev, loss_dev=None):
    _nncheck(nn, load().fftc_nn_train_step(nn, _dev(feat_dev), _dev(target_dev), _dev(loss_dev)),
             "fftc_nn_train_step")


def fftc_nn_adam_step(nn, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    _nncheck(nn, load().fftc_nn_adam_step(nn, float(lr), float(beta1), float(beta2), float(eps)),
             "fftc_nn_adam_step")


def fftc_nn_make_target(u_dev, u1_dev, s_u, target_dev, stream):
    rc = load().fftc_nn_make_target(_dev(u_dev), _dev(u1_dev), int(u_dev.numel()), float(s_u), _dev(target_dev),
                                    C.c_void_p(stream))
    if rc != FFTC_OK:
        raise FftcError(rc, "fftc_nn_make_target")


def fftc_solve_judged(h, u0_dev, u_dev):
    rep = fftc_report()
    used = C.c_int32()
    res = (C.c_double * 2)()
    rc = load().fftc_solve_judged(h, _dev(u0_dev), _dev(u_dev), C.byref(rep), C.byref(used), res)
    _check(h, rc, "fftc_solve_judged", allow=(FFTC_E_NOCONV, FFTC_E_NAN))
    return rc, rep, bool(used.value), (res[0], res[1])


class Net:
    """Warm-start network on the current device: handle + torch-owned state buffer."""

    def __init__(self, modes=6, blocks=4, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.h = fftc_nn_create(modes, blocks)
        self.modes, self.blocks = modes, blocks
        self.P = fftc_nn_num_params(self.h)
        nb = fftc_nn_state_bytes(self.h)
        self.stream = torch.cuda.current_stream(self.device)
        self.state = _aligned(torch, nb, self.device)
        fftc_nn_bind_state(self.h, self.state, nb, self.stream.cuda_stream)
        self.grid = None
        self.ws = None

    def bind(self, N, training=False):
        N = tuple(int(v) for v in N)
        if self.grid == (N, bool(training)):
            return
        nb = fftc_nn_workspace_bytes(self.h, N, training)
        self.ws = _aligned(self.torch, nb, self.device)
        fftc_nn_bind(self.h, N, training, self.ws, nb, self.stream.cuda_stream)
        self.grid = (N, bool(training))

    def set_params(self, vec):
        t = self.torch.as_tensor(np.ascontiguousarray(vec, np.float32), device=self.device)
        fftc_nn_set_params(self.h, t)
        self.stream.synchronize()

    def params(self):
        t = self.torch.empty(self.P, dtype=self.torch.float32, device=self.device)
        fftc_nn_get_params(self.h, t)
        return t

    def grad(self):
        t = self.torch.empty(self.P, dtype=self.torch.float32, device=self.device)
        fftc_nn_get_grad(self.h, t)
        return t

    def forward(self, feat, s_u=1.0, base=None, u0=None):
        y = self.torch.empty((feat.shape[0], 3), dtype=self.torch.float32, device=self.device)
        fftc_nn_forward(self.h, feat, y, s_u, base, u0)
        return y

    def train_step(self, feat, target, loss=None):
        fftc_nn_train_step(self.h, feat, target, loss)

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        fftc_nn_adam_step(self.h, lr, beta1, beta2, eps)

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None:
                fftc_nn_destroy(self.h)
                self.h = None
        except Exception:
            pass


def _aligned(torch, nbytes, device):
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + nbytes]


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------

class Solver:
    """One problem on the current CUDA (HIP) device: handle + torch-owned workspace."""

    def __init__(self, n, lam, mu, bc, strong=(), average=(), sphere=None, r0_factor=1.0,
                 precision="fp64", tol=1e-6, max_iter=2000, acv="P", period=2, gate=1e-2, device="cuda",
                 smooth=(), static_workspace=False, finite_strain=False, scheme="tetra2", reference="paux",
                 voxel=1.0, refine_below=None, anchor_every=16):
        import torch
        self.torch = torch
        self.n = tuple(int(v) for v in n)
        self.precision = FFTC_FP64 if precision == "fp64" else FFTC_FP32
        self.h = fftc_create(self.n, self.precision, voxel, FFTC_HEX1 if scheme == "hex1" else FFTC_TETRA2)
        bc = np.asarray(bc, np.int8).reshape(3, 3, 2)
        fftc_set_bc(self.h, bc)
        periodic = [bool((bc[:, J, :] == 2).all()) for J in range(3)]
        self.N = tuple(self.n[J] + (0 if periodic[J] else 1) for J in range(3))
        self.nsets = 1
        for s in strong:
            fftc_add_dirichlet(self.h, s.node, s.comp, s.value, s.set_id)
            self.nsets = max(self.nsets, s.set_id + 1)
        for a in average:
            fftc_add_average(self.h, a.support, a.comp, a.value, a.set_id)
            self.nsets = max(self.nsets, a.set_id + 1)
        for m in smooth:
            fftc_add_smooth(self.h, m.node, m.comp, m.value, m.set_id)
            self.nsets = max(self.nsets, m.set_id + 1)
        if sphere is not None:
            fftc_set_sphere(self.h, sphere.center, sphere.radius, sphere.face)
        fftc_set_reference_factor(self.h, r0_factor, FFTC_REF_ISO if reference == "iso" else FFTC_REF_PAUX)
        if finite_strain:
            fftc_set_kinematics(self.h, FFTC_FINITE_STRAIN)
        fftc_set_solver(self.h, tol=tol, max_iter=max_iter,
                        acv={"NONE": FFTC_ACV_NONE, "U": FFTC_ACV_U, "P": FFTC_ACV_P}[acv],
                        period=period, update_gate=gate, refine_below=refine_below, anchor_every=anchor_every)
        nbytes = fftc_workspace_bytes(self.h)
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        if static_workspace:            # the library's own per-device workspace, no allocation
            self.ws = self.ws_view = None
            fftc_bind_workspace_static(self.h, self.stream.cuda_stream)
        else:
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-self.ws.data_ptr()) % 256
            self.ws_view = self.ws[off:off + nbytes]
            fftc_bind_workspace(self.h, self.ws_view, nbytes, self.stream.cuda_stream)
        lam_t = torch.as_tensor(np.ascontiguousarray(lam, np.float64), device=self.device)
        mu_t = torch.as_tensor(np.ascontiguousarray(mu, np.float64), device=self.device)
        self.stream.synchronize()
        fftc_set_stiffness(self.h, lam_t, mu_t)
        self.u = torch.zeros((3, self.N[2], self.N[1], self.N[0]), dtype=torch.float64, device=self.device)

    @classmethod
    def from_problem(cls, prob, precision="fp64", **kw):
        kw.setdefault("tol", prob.tol)
        kw.setdefault("max_iter", prob.max_iter)
        kw.setdefault("acv", prob.acv)
        kw.setdefault("period", prob.acv_period)
        return cls(prob.n, prob.lam, prob.mu, prob.bc, prob.strong, prob.average, prob.sphere,
                   prob.r0_factor, precision=precision, smooth=prob.smooth, finite_strain=prob.finite_strain,
                   scheme=prob.scheme, reference=prob.reference, **kw)

    def solve(self, zero_start=True):
        rc, rep = fftc_solve(self.h, self.u, zero_start)
        return rc, rep

    def features(self):
        """Network input channels (BF16 bits as int16 [Nn][16]) and the first iterate
        (FP64 [3][Nn]) they carry."""
        Nn = int(np.prod(self.N))
        t = self.torch.empty((Nn, FFTC_NN_CHANNELS), dtype=self.torch.int16, device=self.device)
        u1 = self.torch.empty((3, Nn), dtype=self.torch.float64, device=self.device)
        fftc_nn_features(self.h, t, u1)
        return t, u1

    def solve_judged(self, u0):
        return fftc_solve_judged(self.h, u0, self.u)

    def move_sphere(self, center):
        fftc_move_sphere(self.h, center)

    def reactions(self):
        return fftc_get_reactions(self.h, self.nsets)

    def contact(self):
        """Active set, normal reaction and gap per face node."""
        return fftc_get_contact(self.h)[:3]

    def contact_force_area(self):
        """Contact force along the face normal and contact area of the last solve."""
        return fftc_get_contact(self.h)[3:]

    def stage_residual(self, u):
        t = self.torch
        u_t = t.as_tensor(np.ascontiguousarray(u, np.float64), device=self.device)
        p = t.empty_like(u_t); pt = t.empty_like(u_t)
        sums = fftc_stage_residual(self.h, u_t, p, pt)
        return p.cpu().numpy(), pt.cpu().numpy(), sums

    def stage_residual_form(self, u, delta, e, p_prev, R_prev, i_local, fp64_stress=0, incremental=False):
        """The FP32 iteration's residual pass on given state: (p, R, dR, dY, sums) as numpy.
        fp64_stress: the pass with FP64 stresses; incremental: p = p_prev + the divergence term
        of the stresses of delta (u not read)."""
        t = self.torch
        dev = [t.as_tensor(np.ascontiguousarray(a, np.float64), device=self.device)
               for a in (u, delta, e, p_prev, R_prev)]
        outs = [t.empty_like(dev[0]) for _ in range(4)]
        sums = fftc_stage_residual_form(self.h, *dev, i_local, *outs,
                                        pass_kind=2 if incremental else (1 if fp64_stress else 0))
        return tuple(o.cpu().numpy() for o in outs) + (sums,)

    def stage_green(self, ptil):
        t = self.torch
        p_t = t.as_tensor(np.ascontiguousarray(ptil, np.float64), device=self.device)
        u = t.empty_like(p_t)
        fftc_stage_green(self.h, p_t, u)
        return u.cpu().numpy()

    def iterate(self, iters):
        fftc_iterate(self.h, iters)

    def profile(self, iters):
        return fftc_profile_stages(self.h, iters)

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None:
                fftc_destroy(self.h)
                self.h = None
        except Exception:
            pass
