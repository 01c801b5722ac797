"""Train and evaluate the tile/parameter selector on one GPU.

    python -m paper_1504_06474_amd.selector_train --out <out-dir> \
        [--train 2000] [--test 200] [--large-train 160] [--large-test 40] \
        [--reps 5] [--steps 4000]
    python -m paper_1504_06474_amd.selector_train --out <out-dir> --collect A:B
    python -m paper_1504_06474_amd.selector_train --out <out-dir> --fit

The first form does everything in one process.  --collect A:B times
matrices A..B-1 only and saves them as <out-dir>/part_A_B.npz (the timing
can then span several processes); --fit trains and evaluates from every part
file in <out-dir>.

1. Data: matrices 0..train+test-1 of the selector set (2D 5-point and 3D
   27-point stencils, FEM-like bands, web-like lognormal rows, dense rows in a
   sparse matrix; 1e4..2e6 rows) and matrices L..L+large_train+large_test-1
   of its large part (L = csrgen.SELECTOR_LARGE_BASE; 2e6..1.6e7 rows), drawn
   on the GPU, each stored once per value type (FP64, FP32, BF16).  For each sample: the 8 features
   (sss_csr_features; the last is the bytes per stored value) and the median
   time of every (W, S) class of the grid (sss_csr_spmv_autotune, `reps` timed
   runs per trial, plans with bound rows), plus the time of the default
   parameters for that type (also with bound rows)
   (the paper's Table 3 choices for its AMD GPU: W = 8, S = 5 in double
   precision; W = 16, S = 2 in single).
2. Training on the first `train` matrices of each part (`large_train` of the
   large one): features z-scored, soft targets
   q_c ~ exp(-(t_c / t_best - 1) / tau), softmax cross-entropy, full-batch
   Adam -- forward, backward and update all by the library's HIP kernels.
3. Evaluation on the held-out rest of each part against the grid timed in
   the same session: regret = geomean(t(selected) / t(grid best)) - 1, gain =
   geomean(t(default) / t(selected)); reported over all held-out matrices and
   for the large part alone.
Writes selector_params.json (parameters, normalisation, class table) and
selector_report.json (metrics, per-class breakdown) to --out; the dataset goes
to dataset.npz there.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import sss


def log(msg):
    print(msg, flush=True)


def time_plan(plan, args, reps: int, trials: int = 5) -> float:
    """Microseconds per run: two warm-up runs, then `trials` trials of `reps`
    back-to-back runs between two events; the median trial (the autotuner's
    protocol for one class)."""
    plan.execute(*args)
    plan.execute(*args)
    ts = []
    for _ in range(trials):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.execute(*args)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e3 / reps)
    return float(np.median(ts))


# matrices of the selector set's large part that train the shipped network;
# the ones after them are held out
LARGE_TRAIN = 160

VALUE_TYPES = {"f64": (torch.float64, torch.float64), "f32": (torch.float32, torch.float32),
               "bf16": (torch.bfloat16, torch.float32)}  # (val, x and y)


def collect(indices, reps: int, dtypes=("f64", "f32", "bf16")):
    """One sample per (matrix, value type); the default plan is the library's
    per-type default (W = 0, S = 0)."""
    from csrgen.torch_gen import selector_matrix_gpu
    feats, times, t_def, names, kinds, mats, sizes = [], [], [], [], [], [], []
    t0 = t_log = time.time()
    for k, i in enumerate(indices):
        d = selector_matrix_gpu(int(i))
        rp, col = d["row_ptr"], d["col"]
        for kind in dtypes:
            vt, xt = VALUE_TYPES[kind]
            val, x = d["val"].to(vt), d["x"].to(xt)
            y = torch.empty(d["m"], dtype=xt, device="cuda")
            feats.append(sss.features(rp, d["n"], d["nnz"], vt))
            t, _ = sss.autotune(rp, col, val, x, y, d["n"], reps)
            times.append(t)
            plan = sss.Plan(d["m"], d["n"], d["nnz"], dtype=vt, bind_rows=True, row_ptr=rp)
            t_def.append(time_plan(plan, (rp, col, val, x, y), reps))
            plan.close()
            names.append(d["cls"])
            kinds.append(kind)
            mats.append(int(i))
            sizes.append((d["m"], d["nnz"]))
            del val, x, y
        del d, rp, col
        if (k + 1) % 50 == 0 or time.time() - t_log > 30:
            t_log = time.time()
            log(f"[selector] {k + 1}/{len(indices)} matrices timed ({t_log - t0:.0f} s)")
    return (np.array(feats, dtype=np.float32), np.array(times), np.array(t_def), np.array(names),
            np.array(kinds), np.array(mats, dtype=np.int64), np.array(sizes, dtype=np.int64))


def soft_targets(times: np.ndarray, tau: float) -> np.ndarray:
    r = times / times.min(axis=1, keepdims=True) - 1.0
    q = np.exp(-r / tau)
    return q / q.sum(axis=1, keepdims=True)


def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases, packed W1 b1 W2 b2 W3 b3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = [(8, 64), (64,), (64, 64), (64,), (64, 12), (12,)]
    parts = [rng.normal(0, math.sqrt(2.0 / s[0]), size=s) if len(s) == 2 else np.zeros(s) for s in shapes]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def train(X: np.ndarray, Q: np.ndarray, steps: int, lr: float, seed: int):
    N = X.shape[0]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    P = dev(init_params(seed))
    Xd, Qd = dev(X), dev(Q)
    H1 = torch.empty(N, 64, device="cuda")
    H2 = torch.empty(N, 64, device="cuda")
    Z = torch.empty(N, 12, device="cuda")
    g = torch.empty(sss.MLP_PARAMS, device="cuda")
    loss = torch.empty(N, device="cuda")
    work = torch.empty(N * 140, device="cuda")
    m1 = torch.zeros(sss.MLP_PARAMS, device="cuda")
    m2 = torch.zeros(sss.MLP_PARAMS, device="cuda")
    hist = []
    for step in range(1, steps + 1):
        sss.mlp_forward(P, Xd, H1, H2, Z)
        sss.mlp_backward(P, Xd, H1, H2, Z, Qd, g, loss, work)
        lr_t = lr * 0.5 * (1 + math.cos(math.pi * (step - 1) / steps))  # cosine decay
        sss.mlp_adam(P, g, m1, m2, step, lr_t)
        if step % 500 == 0 or step == 1:
            hist.append((step, float(loss.mean())))
    torch.cuda.synchronize()
    return P.cpu().numpy(), hist


def predict(params: np.ndarray, X: np.ndarray) -> np.ndarray:
    N = X.shape[0]
    P = torch.from_numpy(params).cuda()
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    H1 = torch.empty(N, 64, device="cuda")
    H2 = torch.empty(N, 64, device="cuda")
    Z = torch.empty(N, 12, device="cuda")
    sss.mlp_forward(P, Xd, H1, H2, Z)
    torch.cuda.synchronize()
    return Z.cpu().numpy().argmax(axis=1)


def geomean(a) -> float:
    a = np.asarray(a, dtype=np.float64)
    return float(np.exp(np.log(a).mean()))


def evaluate(pred: np.ndarray, times: np.ndarray, t_def: np.ndarray, names: np.ndarray,
             kinds: np.ndarray) -> dict:
    t_sel = times[np.arange(len(pred)), pred]
    t_best = times.min(axis=1)
    out = {"n": int(len(pred)), "regret": geomean(t_sel / t_best) - 1.0,
           "gain_vs_default": geomean(t_def / t_sel), "grid_gain_vs_default": geomean(t_def / t_best),
           "accuracy": float((pred == times.argmin(axis=1)).mean()),
           "worst_ratio": float((t_sel / t_best).max()), "per_class": {}, "per_value_type": {}}
    for key, labels in (("per_class", names), ("per_value_type", kinds)):
        for c in sorted(set(labels.tolist())):
            k = labels == c
            out[key][c] = {"n": int(k.sum()), "regret": geomean(t_sel[k] / t_best[k]) - 1.0,
                           "gain_vs_default": geomean(t_def[k] / t_sel[k]),
                           "worst_ratio": float((t_sel[k] / t_best[k]).max())}
    return out


def sweep(times: np.ndarray, names: np.ndarray, kinds: np.ndarray) -> dict:
    """W and S sweeps (the paper's Section 4.5 studies, per class of matrix):
    for each value type and matrix class, the geometric mean over matrices of
    t(W, S) / t(best) for every class of the grid, in class order."""
    rel = times / times.min(axis=1, keepdims=True)
    out = {}
    for k in sorted(set(kinds.tolist())):
        out[k] = {}
        for c in sorted(set(names.tolist())):
            sel = (kinds == k) & (names == c)
            out[k][c] = [round(float(np.exp(np.log(rel[sel, j]).mean())), 3) for j in range(rel.shape[1])]
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--test", type=int, default=200)
    ap.add_argument("--large-train", type=int, default=LARGE_TRAIN)
    ap.add_argument("--large-test", type=int, default=40)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--tau", type=float, default=0.03)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--dtypes", default="f64,f32,bf16", help="value types to time each matrix in")
    ap.add_argument("--out", required=True)
    ap.add_argument("--collect", default="", help="A:B -- time matrices A..B-1 only, save part_A_B.npz")
    ap.add_argument("--fit", action="store_true", help="train and evaluate from the part files in --out")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    sss.lib()
    import csrgen
    base = csrgen.SELECTOR_LARGE_BASE
    if args.train + args.test > base:
        raise SystemExit(f"--train + --test must stay below {base}, where the large part begins")
    indices = list(range(args.train + args.test)) + list(range(base, base + args.large_train + args.large_test))
    n_all = len(indices)
    dtypes = tuple(args.dtypes.split(","))
    keys = ("feats", "times", "t_default", "names", "kinds", "mats", "sizes")
    if args.collect:
        a, b = (int(v) for v in args.collect.split(":"))
        log(f"[selector] timing matrices {a}..{b - 1} x {dtypes}, {sss.N_CLASSES} classes, {args.reps} runs per trial")
        arrays = collect(range(a, b), args.reps, dtypes)
        np.savez(os.path.join(args.out, f"part_{a}_{b}.npz"), **dict(zip(keys, arrays)))
        log(f"[selector] saved part_{a}_{b}.npz")
        return
    if args.fit:
        import glob
        parts = [np.load(f) for f in sorted(glob.glob(os.path.join(args.out, "part_*.npz")))]
        feats, times, t_def, names, kinds, mats, sizes = (np.concatenate([p[k] for p in parts]) for k in keys)
        have = set(mats.tolist())
        if not set(indices) <= have:
            raise SystemExit(f"the part files cover {len(have & set(indices))} of the {n_all} matrices asked for")
        keep = np.isin(mats, indices)
        feats, times, t_def, names, kinds, mats, sizes = (a[keep] for a in (feats, times, t_def, names, kinds,
                                                                              mats, sizes))
    else:
        log(f"[selector] timing {n_all} matrices x {dtypes}, {sss.N_CLASSES} classes, {args.reps} runs per trial")
        feats, times, t_def, names, kinds, mats, sizes = collect(indices, args.reps, dtypes)
    np.savez(os.path.join(args.out, "dataset.npz"), feats=feats, times=times, t_default=t_def, names=names,
             kinds=kinds, mats=mats, sizes=sizes)
    large = mats >= base
    tr = np.where(large, mats < base + args.large_train, mats < args.train)
    te = ~tr
    Xtr, Xte = feats[tr], feats[te]
    mean = Xtr.mean(axis=0)
    std = Xtr.std(axis=0)
    std[std == 0] = 1.0
    Q = soft_targets(times[tr], args.tau)
    params, hist = train((Xtr - mean) / std, Q, args.steps, args.lr, args.seed)
    log(f"[selector] loss {hist}")
    res_tr = evaluate(predict(params, (Xtr - mean) / std), times[tr], t_def[tr], names[tr], kinds[tr])
    pred_te = predict(params, (Xte - mean) / std)
    res_te = evaluate(pred_te, times[te], t_def[te], names[te], kinds[te])
    lte = large[te]
    res_large = evaluate(pred_te[lte], times[te][lte], t_def[te][lte], names[te][lte], kinds[te][lte]) \
        if lte.any() else None
    classes = [list(sss.class_params(c)) for c in range(sss.N_CLASSES)]
    json.dump({"params": [float(v) for v in params], "feature_mean": [float(v) for v in mean],
               "feature_std": [float(v) for v in std], "classes_WS": classes,
               "features": ["log2(m+1)", "log2(n+1)", "log2(nnz+1)", "log2(1+mean)", "log2(1+var)",
                            "log2(1+max)", "empty_frac", "bytes_per_value"],
               "trained_on": f"selector matrices 0..{args.train - 1} and {base}..{base + args.large_train - 1} "
                             f"(seed base 10000) as {'/'.join(dtypes)}, T=64 B=2",
               "command": "python -m paper_1504_06474_amd.selector_train " + " ".join(sys.argv[1:])},
              open(os.path.join(args.out, "selector_params.json"), "w"))
    report = {"train": res_tr, "test": res_te, "test_large": res_large, "loss_history": hist, "args": vars(args),
              "sweep_geomean_t_over_best": sweep(times, names, kinds),
              "class_best_counts": {k: np.bincount(times[kinds == k].argmin(axis=1), minlength=12).tolist()
                                    for k in dtypes}}
    json.dump(report, open(os.path.join(args.out, "selector_report.json"), "w"), indent=1)
    log(f"[selector] test regret {res_te['regret']:.4f} gain {res_te['gain_vs_default']:.3f} "
        f"(grid gain {res_te['grid_gain_vs_default']:.3f}) accuracy {res_te['accuracy']:.3f}")
    for k, v in res_te["per_value_type"].items():
        log(f"[selector]   {k}: regret {v['regret']:.4f} gain {v['gain_vs_default']:.3f} worst {v['worst_ratio']:.3f}")
    if res_large:
        log(f"[selector] large part ({res_large['n']} held-out samples): regret {res_large['regret']:.4f} "
            f"gain {res_large['gain_vs_default']:.3f} (grid gain {res_large['grid_gain_vs_default']:.3f}) "
            f"worst {res_large['worst_ratio']:.3f}")


if __name__ == "__main__":
    main()
