"""Training and evaluation driver of the learned warm start (include/fftc_nn.h).

Training data are solves of the library itself: learned-start cases
(workloads.nn_case, two-phase cells with Dirichlet patches or a rigid-sphere
indentation) solved in the FP32 form to 1e-6; the target is the converged
field's difference to the first iterate, in units of s_u.  Input channels, the network's
forward and backward passes, Adam and the judged start all run in the
library's kernels; this module only schedules calls and keeps the data on the
device.

    python -m paper_2607_26082_amd.warmstart train --cases 2000 --epochs 6 --out W.npy
    python -m paper_2607_26082_amd.warmstart eval --weights W.npy --cases 200 --scale 2
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "data", "warmstart_m6_b4.npy")
N0 = (64, 64, 64)


def _spec(args):
    import workloads as W
    seed, n0 = args
    return W.nn_case_spec(seed, n0=n0)


def make_specs(seeds, n0=N0, workers=12):
    """Random draws of every case (sphere placement is the costly part).  The worker
    pool is created and joined here, before the caller touches the GPU."""
    jobs = [(int(s), tuple(n0)) for s in seeds]
    if workers <= 1:
        return [_spec(j) for j in jobs]
    with mp.get_context("fork").Pool(workers) as pool:
        out = pool.map(_spec, jobs, chunksize=4)
    return out


def cases(specs, scale=1):
    import workloads as W
    for sp in specs:
        yield W.nn_case_build(sp, scale)


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_dataset(specs, n0=N0, log=_log):
    """Solve every case (FP32 form, tol 1e-6, one at a time) and keep its input
    channels and (converged field - first iterate) / s_u on the device."""
    import torch
    import paper_2607_26082_amd as F
    N = tuple(v + 1 for v in n0)
    Nn = int(np.prod(N))
    su = 1e-3 * min(n0)
    S = len(specs)
    feat = torch.empty((S, Nn, F.FFTC_NN_CHANNELS), dtype=torch.int16, device="cuda")
    tgt = torch.empty((S, 3, Nn), dtype=torch.float32, device="cuda")
    ok = np.zeros(S, bool)
    iters = np.zeros(S, np.int64)
    u1 = torch.empty((3, Nn), dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    for i, prob in enumerate(cases(specs)):
        g = F.Solver.from_problem(prob, precision="fp32", tol=1e-6, max_iter=4000)
        F.fftc_nn_features(g.h, feat[i], u1)
        rc, r = g.solve()
        F.fftc_nn_make_target(g.u.reshape(3, Nn), u1, su, tgt[i], g.stream.cuda_stream)
        ok[i] = r.status == 0
        iters[i] = r.iterations
        del g
        if (i + 1) % 50 == 0 or i + 1 == S:
            torch.cuda.synchronize()
            log(f"[warmstart] data {i + 1}/{S} solved, {time.perf_counter() - t0:.0f} s, "
                f"median iterations {int(np.median(iters[:i + 1]))}, not converged {int((~ok[:i + 1]).sum())}")
    return feat, tgt, ok, iters


def train(net, feat, tgt, ok, epochs, lr, seed=0, warmup=200, log=_log):
    """Adam over the samples in random order, one sample per step, cosine-decayed rate."""
    import torch
    idx = np.flatnonzero(ok)
    rng = np.random.default_rng(seed)
    total = epochs * len(idx)
    losses = torch.zeros(total, dtype=torch.float64, device="cuda")
    step = 0
    t0 = time.perf_counter()
    for e in range(epochs):
        for s in rng.permutation(idx):
            frac = step / max(total - 1, 1)
            rate = lr * min(1.0, (step + 1) / warmup) * 0.5 * (1.0 + math.cos(math.pi * frac))
            net.train_step(feat[s], tgt[s], losses[step:step + 1])
            net.adam(rate)
            step += 1
        torch.cuda.synchronize()
        L = losses[e * len(idx):(e + 1) * len(idx)].cpu().numpy()
        log(f"[warmstart] epoch {e + 1}/{epochs} mean loss {L.mean():.4e} median {np.median(L):.4e}, "
            f"{time.perf_counter() - t0:.0f} s")
    return losses.cpu().numpy()


def evaluate(net, specs, scale=1, ref64=0, log=_log):
    """Per case: plain solve and judged network start (input channels and inference
    charged), both FP32 form to 1e-6, timed with device synchronisation.  For the
    first `ref64` cases also the FP64 solve to 1e-10 as the reference solution."""
    import torch
    import paper_2607_26082_amd as F
    rows = []
    for k, prob in enumerate(cases(specs, scale)):
        g = F.Solver.from_problem(prob, precision="fp32", tol=1e-6, max_iter=4000)
        Nn = int(np.prod(g.N))
        su = 1e-3 * min(prob.n)
        net.bind(g.N, training=False)
        u0 = torch.empty((3, Nn), dtype=torch.float64, device="cuda")
        g.solve()                       # warm the caches of this handle
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc_p, rep_p = g.solve()
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        u_plain = g.u.clone()
        t0 = time.perf_counter()
        feat, u1 = g.features()
        net.forward(feat, s_u=su, base=u1, u0=u0)
        rc_n, rep_n, used, res = g.solve_judged(u0)
        torch.cuda.synchronize()
        t_nn = time.perf_counter() - t0
        u_nn = g.u.clone()
        # the network's start taken unconditionally (no judge), for reference
        g.u.copy_(u0.reshape(g.u.shape))
        rc_f, rep_f = g.solve(zero_start=False)
        g.u.copy_(u_nn)
        row = {"seed": int(prob.meta["seed"]), "kind": prob.meta["kind"], "n": list(prob.n),
               "iters_nn_forced": rep_f.iterations,
               "iters_plain": rep_p.iterations, "iters_nn": rep_n.iterations, "used_nn": bool(used),
               "t_plain_s": t_plain, "t_nn_s": t_nn, "status": [rc_p, rc_n],
               "start_residual": [res[0], res[1]],
               "rel_nn_vs_plain": float(torch.linalg.norm(g.u - u_plain) / torch.linalg.norm(u_plain))}
        if k < ref64:
            g64 = F.Solver.from_problem(prob, precision="fp64", tol=1e-10, max_iter=20000)
            g64.solve()
            nrm = torch.linalg.norm(g64.u)
            row["rel_nn_vs_fp64"] = float(torch.linalg.norm(g.u - g64.u) / nrm)
            row["rel_plain_vs_fp64"] = float(torch.linalg.norm(u_plain - g64.u) / nrm)
            del g64
        rows.append(row)
        if (k + 1) % 10 == 0 or k + 1 == len(specs):
            it = np.array([[r["iters_plain"], r["iters_nn"]] for r in rows], float)
            tt = np.array([[r["t_plain_s"], r["t_nn_s"]] for r in rows])
            log(f"[warmstart] eval {k + 1}/{len(specs)} scale {scale}: median iterations "
                f"{np.median(it[:, 0]):.0f} -> {np.median(it[:, 1]):.0f}, time ratio (geo-mean) "
                f"{np.exp(np.mean(np.log(tt[:, 0] / tt[:, 1]))):.3f}")
        del g
    return rows


def summary(rows):
    it = np.array([[r["iters_plain"], r["iters_nn"]] for r in rows], float)
    tt = np.array([[r["t_plain_s"], r["t_nn_s"]] for r in rows])
    out = {"cases": len(rows),
           "iters_plain_median": float(np.median(it[:, 0])), "iters_nn_median": float(np.median(it[:, 1])),
           "iters_ratio_geomean": float(np.exp(np.mean(np.log(it[:, 0] / np.maximum(it[:, 1], 1))))),
           "time_plain_median_s": float(np.median(tt[:, 0])), "time_nn_median_s": float(np.median(tt[:, 1])),
           "time_ratio_geomean": float(np.exp(np.mean(np.log(tt[:, 0] / tt[:, 1])))),
           "time_ratio_total": float(tt[:, 0].sum() / tt[:, 1].sum()),
           "iters_nn_forced_median": float(np.median([r["iters_nn_forced"] for r in rows])),
           "nn_start_used": int(sum(r["used_nn"] for r in rows)),
           "rel_nn_vs_plain_max": float(np.nanmax([r["rel_nn_vs_plain"] for r in rows]))}
    codes = {0: "ok", -5: "not converged", -6: "non-finite"}
    for j, name in ((0, "status_plain"), (1, "status_nn")):
        cnt = {}
        for r in rows:
            key = codes.get(int(r["status"][j]), str(r["status"][j]))
            cnt[key] = cnt.get(key, 0) + 1
        out[name] = cnt
    # cases whose two final solutions differ by more than the stopping tolerance allows
    out["outliers"] = [{k: r[k] for k in ("seed", "kind", "status", "iters_plain", "iters_nn", "used_nn",
                                          "rel_nn_vs_plain")}
                       for r in rows if not (r["rel_nn_vs_plain"] <= 1e-3)]
    ref = [r for r in rows if "rel_nn_vs_fp64" in r]
    if ref:
        out["fp64_reference_cases"] = len(ref)
        out["rel_nn_vs_fp64_max"] = max(r["rel_nn_vs_fp64"] for r in ref)
        out["rel_plain_vs_fp64_max"] = max(r["rel_plain_vs_fp64"] for r in ref)
        out["rel_plain_vs_fp64_median"] = float(np.median([r["rel_plain_vs_fp64"] for r in ref]))
    kinds = sorted({r["kind"] for r in rows})
    if len(kinds) > 1:
        out["by_kind"] = {}
        for k in kinds:
            rk = [r for r in rows if r["kind"] == k]
            ik = np.array([[r["iters_plain"], r["iters_nn"], r["iters_nn_forced"]] for r in rk], float)
            tk = np.array([[r["t_plain_s"], r["t_nn_s"]] for r in rk])
            out["by_kind"][k] = {"cases": len(rk), "iters_plain_median": float(np.median(ik[:, 0])),
                                 "iters_nn_median": float(np.median(ik[:, 1])),
                                 "iters_nn_forced_median": float(np.median(ik[:, 2])),
                                 "nn_start_used": int(sum(r["used_nn"] for r in rk)),
                                 "time_ratio_total": float(tk[:, 0].sum() / tk[:, 1].sum())}
    return out


def load_weights(path=DEFAULT_WEIGHTS):
    return np.load(path, allow_pickle=False)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["train", "eval"])
    ap.add_argument("--cases", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default=None)
    ap.add_argument("--weights", default=DEFAULT_WEIGHTS)
    ap.add_argument("--scale", type=int, default=1)
    ap.add_argument("--eval-cases", type=int, default=20)
    ap.add_argument("--ref64", type=int, default=0)
    ap.add_argument("--workers", type=int, default=12)
    ap.add_argument("--init-seed", type=int, default=7)
    args = ap.parse_args(argv)
    import workloads as W
    # all random draws first, on the host, before this process touches the GPU
    t0 = time.perf_counter()
    train_specs = []
    if args.mode == "train":
        train_specs = make_specs([W.NN_TRAIN_SEED + j for j in range(args.cases)], workers=args.workers)
    eval_n = args.eval_cases if args.mode == "train" else args.cases
    eval_specs = make_specs([W.NN_EVAL_SEED + j for j in range(eval_n)], workers=args.workers) if eval_n else []
    _log(f"[warmstart] drew {len(train_specs)} training and {len(eval_specs)} evaluation cases "
         f"in {time.perf_counter() - t0:.0f} s")
    import torch
    import paper_2607_26082_amd as F
    F.load()
    torch.cuda.set_device(0)
    net = F.Net(6, 4)
    result = {}
    if args.mode == "train":
        net.set_params(W.nn_init(args.init_seed, _layout(net)))
        t0 = time.perf_counter()
        feat, tgt, ok, iters = make_dataset(train_specs)
        t_data = time.perf_counter() - t0
        net.bind(tuple(v + 1 for v in N0), training=True)
        t0 = time.perf_counter()
        losses = train(net, feat, tgt, ok, args.epochs, args.lr)
        t_train = time.perf_counter() - t0
        vec = net.params().cpu().numpy()
        if args.out:
            os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
            np.save(args.out, vec)
        del feat, tgt
        nok = int(ok.sum())
        result["train"] = {"cases": nok, "epochs": args.epochs, "data_s": t_data, "train_s": t_train,
                           "steps": len(losses), "ms_per_step": 1e3 * t_train / max(len(losses), 1),
                           "loss_first_epoch": float(losses[:nok].mean()),
                           "loss_last_epoch": float(losses[-nok:].mean()),
                           "data_iterations_median": float(np.median(iters[ok]))}
    else:
        net.set_params(load_weights(args.weights))
    if eval_specs:
        rows = evaluate(net, eval_specs, scale=args.scale, ref64=args.ref64)
        result["eval"] = summary(rows)
        result["eval"]["scale"] = args.scale
    print(json.dumps(result))


def _layout(net):
    """Parameter shapes in the order of include/fftc_nn.h."""
    m3, out = net.modes ** 3, [(32, 12), (32,)]
    for _ in range(net.blocks):
        out += [(m3, 32, 32), (32, 32), (32,)]
    return out + [(64, 32), (64,), (3, 64), (3,)]


if __name__ == "__main__":
    main()
