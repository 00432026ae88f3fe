"""Benchmark: voxel-iterations per second of the constrained DTT/FFT fixed point at 256^3.

One step = one full fixed-point iteration (stress/divergence/projection/reference term,
equilibrium test, Anderson store + Gram + least squares + combination, forward DTTs, Green
solve, inverse DTTs, proj_U) on the 256^3 two-phase block (bottom fixed, 16x16-node patch
pressed on the top face), inputs resident in HBM.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np

METRIC = "voxel-iters/s at 256^3; time to 1e-6 residual, NN warm-start vs plain"
HBM_PEAK_GBS = 8000.0


def stage_bytes(N, nv, s):
    """Algorithmic HBM bytes of each stage per iteration (s = bytes per value).
    Node fields have 3 components; N = nodes, nv = voxels."""
    f = 3 * N * s
    return {
        "residual": 2 * f + 2 * nv * s,        # read u, lam, mu; write p~
        "anderson": 3 * f,                     # read p~, S_prev; write R (Gram reads counted below)
        "dtt_x_fwd": 2 * f, "dtt_y_fwd": 2 * f, "dtt_z_green": 2 * f, "dtt_y_inv": 2 * f, "dtt_x_inv": 2 * f,
    }


def b_alg_per_voxel_iter(N, nv, s, m=4, q=2):
    """Algorithmic bytes of one iteration: 42 nodal values + 2 voxel values (Anderson depth m,
    period q): read u, write p~, forward DT read/write, inverse DT read/write, write S and R,
    and every q-th iteration read m S + m R for the combination and m R for the Gram matrix."""
    vals = 3 + 3 + 6 + 6 + 6 + (2 * m * 3 + m * 3) / q
    return (vals * N * s + 2 * nv * s) / nv


def cpu_baseline(prob):
    """One oracle iteration (FP64 NumPy/SciPy) of the same workload on the host."""
    from oracle.solver import Anderson, Solver as OSolver
    t0 = time.time()
    s = OSolver.from_problem(prob)
    u = s.zeros()
    s.cons.proj_U(u)
    setup = time.time() - t0
    t0 = time.time()
    parts = s.iterate_parts(u)
    acc = Anderson(4, 2)
    x = acc.step(0, parts["ptil"])
    u = s.green.apply(x)
    s.cons.proj_U(u)
    dt = time.time() - t0
    nv = int(np.prod(prob.n))
    return {"value": nv / dt, "unit": "voxel-iters/s", "cores": 1, "kind": "oracle",
            "sample": f"1 iteration of the FP64 NumPy/SciPy oracle on the same 256^3 workload "
                      f"({dt:.1f} s; set-up {setup:.1f} s excluded); NumPy elementwise and scipy.fft "
                      f"(default workers=1) single-threaded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-iters", type=int, default=5)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_2607_26082_amd as F
    import workloads as W

    torch.cuda.set_device(0)
    n = (args.n, args.n, args.n)
    prob = W.m256_metric(n=n)
    nv = int(np.prod(n))
    N = int(np.prod([v + 1 for v in n]))
    print(f"[bench] workload {n} phi={prob.meta['phi']:.3f} precision={args.precision}", file=sys.stderr, flush=True)
    g = F.Solver.from_problem(prob, precision=args.precision, tol=0.0, max_iter=args.warmup)
    rc, rep = g.solve()
    torch.cuda.synchronize()
    print(f"[bench] warmup {rep.iterations} iterations residual {rep.residual:.3e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.iterate(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt / args.steps * 1e3
    value = nv * args.steps / dt
    s = 8 if args.precision == "fp64" else 4
    # per-stage HIP-event timing on the library's stream
    prof = g.profile(args.profile_iters)
    sb = stage_bytes(N, nv, s)
    stages = {}
    for k, t in prof.items():
        stages[k] = {"ms": round(t, 4)}
        if k in sb and t > 0:
            stages[k]["GB/s"] = round(sb[k] / (t * 1e-3) / 1e9, 1)
    dom = max((k for k in sb if prof.get(k, 0) > 0), key=lambda k: prof[k])
    achieved = sb[dom] / (prof[dom] * 1e-3) / 1e9
    balg = b_alg_per_voxel_iter(N, nv, s)
    out = {
        "metric": METRIC, "value": value, "unit": "voxel-iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"two-phase block {n[0]}x{n[1]}x{n[2]} voxels (phi=0.25 spheres, contrast 10), "
                               "bottom face fixed, 16x16-node top patch u_z=-1e-3 L, TETRA2, Paux R0 x1, "
                               "ACV_P depth 4 period 2, no exit test",
                   "voxels": nv, "precision": args.precision},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom},
        "iteration_bytes_alg_GBps": round(balg * value / 1e9, 1),
        "iteration_frac_of_hbm_peak": round(balg * value / 1e9 / HBM_PEAK_GBS, 4),
        "stages": stages,
    }
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle, 1 iteration)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
