"""Benchmark: voxel-iterations per second of the constrained DTT/FFT fixed point at 256^3.

One step = one full fixed-point iteration (stress/divergence/projection/reference term,
equilibrium test, Anderson store + Gram + least squares + combination, forward DTTs, Green
solve, inverse DTTs, proj_U) on the 256^3 two-phase block (bottom fixed, 16x16-node patch
pressed on the top face), inputs resident in HBM.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np

METRIC = "voxel-iters/s at 256^3; time to 1e-6 residual, NN warm-start vs plain"
HBM_PEAK_GBS = 8000.0
BATCH_CELLS_MAX = 4


def stage_bytes(N, nv, precision):
    """Bytes each stage's kernels move per iteration as implemented (N nodes, nv voxels;
    vector node fields have 3 components), averaged over the acceleration period 2: a stage
    that moves some of its bytes only in accelerating iterations is charged half of them.
    FP32 is the residual-form iteration (FP64 displacement); FP64 the literal one.  These are
    implementation bytes, reported as `moved GB/s`; the roofline uses algorithmic bytes."""
    if precision == "fp32":
        f = 3 * N * 4
        # residual pass: incremental (read delta, p_prev, c after accelerating iterations, lam, mu;
        # write p, R, dY), and every 16th iteration from u (also read u in FP64)
        inc, full = f + f + f / 2 + 2 * nv * 4 + 3 * f, 2 * f + f + f + f / 2 + 2 * nv * 4 + 3 * f
        return {
            "residual": (15 * inc + full) / 16,
            "anderson": 4 * f / 2,             # read the ring of four R (accelerating iterations)
            # read p, dY x3 (accelerating); write t, and e (accelerating)
            "dtt_x_fwd": f + 3 * f / 2 + f + f / 2,
            "dtt_y_fwd": 2 * f, "dtt_z_green": 2 * f, "dtt_y_inv": 2 * f,
            "dtt_x_inv": f + 2 * f + 2 * f + f,  # read t, u (FP64); write u (FP64), delta
        }
    f = 3 * N * 8
    return {
        "residual": 2 * f + 2 * nv * 8,        # read u, lam, mu; write p~
        "anderson": 3 * f + 4 * f / 2,         # read p~, S_prev; write R; read 4 R (accelerating)
        "dtt_x_fwd": (8 * f + f) / 2 + 2 * f,  # read 4 S + 4 R (accelerating) or p~; write S, t
        "dtt_y_fwd": 2 * f, "dtt_z_green": 2 * f, "dtt_y_inv": 2 * f, "dtt_x_inv": 2 * f,
    }


def residual_alg_bytes(N, nv, s, precision):
    """Algorithmic bytes of one residual pass (the per-node and per-voxel figures of the
    byte model below, times the nodes and voxels one launch covers): read u~ (3 values; the
    FP32 form's incremental pass reads its increment instead), write p~ (3) and the voxel
    stiffness pair (2 per voxel); the FP32 residual-form pass also writes the Anderson pair
    S_i, R_i (6 values) that it forms in place of a separate store."""
    nodal = 12 if precision == "fp32" else 6
    return s * (nodal * N + 2 * nv)


def b_alg_per_voxel_iter(N, nv, s, m=4, q=2):
    """Algorithmic bytes of one iteration: 42 nodal values + 2 voxel values (Anderson depth m,
    period q): read u, write p~, forward DT read/write, inverse DT read/write, write S and R,
    and every q-th iteration read m S + m R for the combination and m R for the Gram matrix."""
    vals = 3 + 3 + 6 + 6 + 6 + (2 * m * 3 + m * 3) / q
    return (vals * N * s + 2 * nv * s) / nv


def kernel_source_digest():
    h = hashlib.sha256()
    for f in ("fftc_residual.hip", "fftc_common.h", "fftc_internal.h"):
        with open(os.path.join(ROOT, "paper_2607_26082_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(precision, kernel):
    """HBM bytes per launch of the dominant kernel from the committed PMC summary, only if
    the kernel sources are unchanged since the counters were taken (else None)."""
    path = os.path.join(ROOT, "profiles", "residual_dt_m256_fp32_traffic.txt")
    if precision != "fp32" or kernel != "residual" or not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_digest():
        return None
    return float(vals["traffic_bytes_per_launch"])


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, iters=5):
    """The FP64 NumPy/SciPy oracle, as it stands, on the same workload on the host: `iters`
    iterations (stress, divergence, projections, reference term, Anderson, transforms, Green
    solve).  scipy.fft runs with one worker per available core (at most 16, the host share of
    one GPU); NumPy's stencil and elementwise stages run on one thread."""
    import scipy.fft
    from oracle.solver import Anderson, Solver as OSolver
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    t0 = time.time()
    s = OSolver.from_problem(prob)
    u = s.zeros()
    s.cons.proj_U(u)
    setup = time.time() - t0
    with scipy.fft.set_workers(workers):
        t0 = time.time()
        acc = Anderson(4, 2)
        for i in range(iters):
            parts = s.iterate_parts(u)
            x = acc.step(i, parts["ptil"])
            u = s.green.apply(x)
            s.cons.proj_U(u)
        dt = time.time() - t0
    nv = int(np.prod(prob.n))
    N = int(np.prod([v + 1 for v in prob.n]))
    bps = b_alg_per_voxel_iter(N, nv, 8)
    return {"value": nv * iters / dt, "unit": "voxel-iters/s", "cores": workers, "kind": "oracle",
            "GB/s": round(bps * nv * iters / dt / 1e9, 2),
            "cpu_model": _cpu_model(), "host_cpus_visible": os.cpu_count(),
            "threads_per_stage": {"transforms (scipy.fft)": workers, "stencil, projections, Anderson (NumPy)": 1},
            "sample": f"{iters} iterations of the FP64 NumPy/SciPy oracle on the same {prob.n[0]}^3 workload "
                      f"({dt:.1f} s; set-up {setup:.1f} s excluded); GB/s from the byte model with 8-byte values"}


def copy_bandwidth(torch, gib=1, reps=10):
    """A plain device copy of `gib` GiB (read + write), the practical HBM ceiling of a
    streaming kernel on this GPU."""
    n = (gib << 30) // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    a.fill_(1.0)
    c.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        c.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, c
    return {"GB/s": round(2 * (gib << 30) / (ms * 1e-3) / 1e9, 1), "bytes_per_copy": 2 * (gib << 30),
            "ms": round(ms, 4)}


def bench_warmstart(args):
    """Held-out learned-start cases (64^3, or 128^3 with --n 128): per case the plain solve
    and the judged network start (input channels and inference charged), FP32 form to 1e-6."""
    import workloads as W
    from paper_2607_26082_amd import warmstart as WS
    scale = 2 if args.n == 128 else 1          # held-out cells at 64^3, or at 128^3 with --n 128
    specs = WS.make_specs([W.NN_EVAL_SEED + j for j in range(args.cells)], workers=8)
    import torch
    import paper_2607_26082_amd as F
    torch.cuda.set_device(0)
    net = F.Net(6, 4)
    net.set_params(WS.load_weights())
    rows = WS.evaluate(net, specs, scale=scale, ref64=args.ref64)
    s = WS.summary(rows)
    n = 64 * scale
    out = {
        "metric": METRIC, "value": s["time_ratio_total"], "unit": "time-to-1e-6 ratio plain/learned",
        "n_gpus": 1, "steps": len(rows), "warmup": 1, "ms_per_step": 1e3 * s["time_nn_median_s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{len(rows)} held-out learned-start cells at {n}^3 (Dirichlet patches / indentation), "
                               "FP32 form, tol 1e-6, judged start", "precision": "fp32"},
        "summary": s,
    }
    print(json.dumps(out))


def nn_flops_per_node(modes=6, blocks=4, width=32, hidden=64, cin=12, cout=3):
    """Algorithmic FLOPs of one network forward per node: lift, per block the analysis onto
    modes^3 cosine modes and the synthesis back (each 2 M3 width) plus the pointwise map,
    then the two head layers."""
    m3 = modes ** 3
    return (2 * cin * width + blocks * (2 * (2 * m3 * width) + 2 * width * width)
            + 2 * width * hidden + 2 * hidden * cout)


def bench_nn(args):
    """The learned-start network alone on one held-out case at 65^3 nodes (129^3 with
    --n 128): input channels (one plain iteration and the channel build), inference (the
    start u0 = u1 + s_u y) and one training step (forward, backward, Adam)."""
    import torch
    import workloads as W
    import paper_2607_26082_amd as F
    from paper_2607_26082_amd import warmstart as WS
    scale = 2 if args.n == 128 else 1
    torch.cuda.set_device(0)
    prob = W.nn_case(W.NN_EVAL_SEED, None, scale)
    g = F.Solver.from_problem(prob, precision="fp32", tol=1e-6, max_iter=4000)
    net = F.Net(6, 4)
    net.set_params(WS.load_weights())
    Nn = int(np.prod(g.N))
    su = 1e-3 * min(prob.n)
    feat = torch.empty((Nn, F.FFTC_NN_CHANNELS), dtype=torch.int16, device="cuda")
    u1 = torch.empty((3, Nn), dtype=torch.float64, device="cuda")
    u0 = torch.empty_like(u1)

    def timed(fn, reps):
        for _ in range(max(args.warmup, 1)):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    print(f"[bench] network on {g.N} nodes", file=sys.stderr, flush=True)
    t_feat = timed(lambda: F.fftc_nn_features(g.h, feat, u1), args.steps)
    net.bind(g.N, training=False)
    t_fwd = timed(lambda: net.forward(feat, su, u1, u0), args.steps)
    net.bind(g.N, training=True)
    tgt = torch.randn((3, Nn), dtype=torch.float32, device="cuda")
    lr = 1e-12                            # a step that leaves the weights as they are

    def train():
        net.train_step(feat, tgt)
        net.adam(lr)

    t_train = timed(train, args.steps)
    f = nn_flops_per_node()
    tf_fwd = f * Nn / (t_fwd * 1e-3) / 1e12
    tf_train = 3 * f * Nn / (t_train * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": Nn / (t_fwd * 1e-3), "unit": "nodes/s (network inference)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_fwd,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"learned-start network (width 32, 6 modes, 4 blocks) on a held-out case, "
                               f"{'x'.join(str(v) for v in g.N)} nodes", "precision": "bf16 MFMA, fp32 accumulation"},
        "roofline": {"bound": "mfma", "achieved": round(tf_fwd, 1), "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": round(tf_fwd / 2500.0, 4), "traffic": None, "kernel": "network forward (all kernels)",
                     "alg_flops_per_node": f},
        "ms": {"input_channels": round(t_feat, 4), "inference": round(t_fwd, 4), "training_step": round(t_train, 4)},
        "training_tflops": round(tf_train, 1),
    }
    print(json.dumps(out))


def bench_batch(args):
    """64 two-phase cells of uneven size, FP32 form, solved together to 1e-6 as one batch.

    Timed: whole batched solves from a zero start (every cell to its own exit).  The same
    cells are then solved one after another with the single-problem entry point, for the
    batching gain."""
    if args.cells > BATCH_CELLS_MAX:
        print(json.dumps({"error": f"--cells {args.cells}: batches above {BATCH_CELLS_MAX} cells are switched off; "
                                   "the 64-cell batch left the GPU faulted once with a transform variant that has "
                                   "since been removed, and it stays off the GPU until the cause is shown"}))
        sys.exit(3)
    import torch
    import paper_2607_26082_amd as F
    import workloads as W

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    cells = W.c4_batch(args.cells)
    print(f"[bench] generated {len(cells)} cells in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    solvers = [F.Solver.from_problem(p, precision="fp32", tol=1e-6, max_iter=4000) for p in cells]
    batch = F.Batch(solvers)
    for w in range(max(args.warmup, 1)):
        rc, reps = batch.solve()
    torch.cuda.synchronize()
    iters = [r.iterations for r in reps]
    vox = [int(np.prod(p.n)) for p in cells]
    work = float(sum(v * i for v, i in zip(vox, iters)))
    print(f"[bench] warmup batch rc={rc} iterations min/median/max {min(iters)}/{int(np.median(iters))}/{max(iters)}",
          file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        rc, reps = batch.solve()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    bad = [k for k, r in enumerate(reps) if r.status != 0]
    t0 = time.perf_counter()
    for g in solvers:
        g.solve()
    torch.cuda.synchronize()
    dt_solo = time.perf_counter() - t0
    out = {
        "metric": METRIC, "value": work / dt, "unit": "voxel-iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{len(cells)} two-phase cells, edges from {{32,48,64,96,128}} per axis, "
                               "random DTT face BCs and 1-4 Dirichlet patches, FP32 form, tol 1e-6, "
                               "one batched solve per step",
                   "voxels": int(sum(vox)), "precision": "fp32"},
        "time_to_tol_s": round(dt, 4),
        "sequential_solo_s": round(dt_solo, 4),
        "batch_gain": round(dt_solo / dt, 3),
        "iterations": {"min": min(iters), "median": int(np.median(iters)), "max": max(iters),
                       "total_voxel_iters": work},
        "not_converged": bad,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32"])
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (PMC byte-counter calibration)")
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-iters", type=int, default=16,
                    help="iterations of the per-stage HIP-event timing (16: one period of the FP32 form's "
                         "residual passes, fifteen incremental and one from u)")
    ap.add_argument("--workload", default="m256", choices=["m256", "c4", "c5", "nn"],
                    help="m256: 256^3 iteration throughput; c4: 64 uneven cells solved as one batch; "
                         "c5: time to 1e-6 with the learned start vs the plain start on held-out cases; "
                         "nn: the learned-start network alone (inference and a training step)")
    ap.add_argument("--cells", type=int, default=BATCH_CELLS_MAX)
    ap.add_argument("--ref64", type=int, default=16,
                    help="c5: cases also solved by the FP64 path to 1e-10 as the reference solution")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU per process; multi-GPU runs are not supported, --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "c4":
        return bench_batch(args)
    if args.workload == "c5":
        return bench_warmstart(args)
    if args.workload == "nn":
        return bench_nn(args)

    import torch
    import paper_2607_26082_amd as F
    import workloads as W

    torch.cuda.set_device(0)
    n = (args.n, args.n, args.n)
    prob = W.m256_metric(n=n)
    nv = int(np.prod(n))
    N = int(np.prod([v + 1 for v in n]))
    copy = copy_bandwidth(torch)
    print(f"[bench] device copy {copy['GB/s']} GB/s", file=sys.stderr, flush=True)
    out = None
    extra = {}
    for prec in (args.precision, "fp64" if args.precision == "fp32" else None):
        if prec is None:
            break
        main_line = out is None
        print(f"[bench] workload {n} phi={prob.meta['phi']:.3f} precision={prec}", file=sys.stderr, flush=True)
        g = F.Solver.from_problem(prob, precision=prec, tol=0.0, max_iter=args.warmup)
        rc, rep = g.solve()
        torch.cuda.synchronize()
        print(f"[bench] warmup {rep.iterations} iterations residual {rep.residual:.3e}", file=sys.stderr, flush=True)
        steps = args.steps if main_line else max(5, args.steps // 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.iterate(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ms = dt / steps * 1e3
        value = nv * steps / dt
        s = 8 if prec == "fp64" else 4
        # per-stage HIP-event timing on the library's stream
        prof = g.profile(args.profile_iters)
        del g
        torch.cuda.empty_cache()
        sb = stage_bytes(N, nv, prec)
        stages = {}
        for k, t in prof.items():
            stages[k] = {"ms": round(t, 4)}
            if k in sb and t > 0:
                stages[k]["moved GB/s"] = round(sb[k] / (t * 1e-3) / 1e9, 1)
        dom = max((k for k in sb if prof.get(k, 0) > 0), key=lambda k: prof[k])
        alg = residual_alg_bytes(N, nv, s, prec) if dom == "residual" else None
        balg = b_alg_per_voxel_iter(N, nv, s)
        it_gbs = balg * value / 1e9
        iteration = {"bound": "hbm", "achieved": round(it_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(it_gbs / HBM_PEAK_GBS, 4), "frac_of_copy": round(it_gbs / copy["GB/s"], 4),
                     "alg_bytes_per_iteration": round(balg * nv)}
        if not main_line:
            extra["fp64"] = {"value": value, "unit": "voxel-iters/s", "steps": steps, "ms_per_step": ms,
                             "iteration_roofline": iteration, "stages": stages}
            continue
        achieved = alg / (prof[dom] * 1e-3) / 1e9 if alg else None
        out = {
            "metric": METRIC, "value": value, "unit": "voxel-iters/s", "n_gpus": 1, "steps": steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64" if prec == "fp64" else "f32",
            "data": "synthetic",
            "config": {"workload": f"two-phase block {n[0]}x{n[1]}x{n[2]} voxels (phi=0.25 spheres, contrast 10), "
                                   "bottom face fixed, 16x16-node top patch u_z=-1e-3 L, TETRA2, Paux R0 x1, "
                                   "ACV_P depth 4 period 2, no exit test",
                       "voxels": nv, "precision": prec},
            # dominant kernel: its algorithmic bytes per launch over its HIP-event time
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1) if achieved else None, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                         "traffic": measured_traffic(prec, dom),
                         "kernel": dom + (" (k_residual_dt: incremental, from u every 16th iteration)"
                                          if prec == "fp32" and dom == "residual" else ""),
                         "kernel_ms": round(prof[dom], 4),
                         "alg_bytes_per_launch": alg},
            # the whole iteration: algorithmic bytes of one iteration x iterations per second
            "iteration_roofline": iteration,
            "device_copy": copy,
            "stages": stages,
        }
    out.update(extra)
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle, 5 iterations)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
