#!/usr/bin/env python3
"""Benchmark of the speculative segmented sum CSR SpMV on one MI355X.

Workload: the 1M-row power-law matrix (m = n = 1e6, Zipf-Mandelbrot exponent 2
row lengths on [1, 2e5], mean ~20, 3% empty rows, ~19M nonzeros), double
precision, synthetic and seeded.  A step is one y = A x through both stages
(speculative execution + device fixup).  Inputs are resident in HBM before the
timed region; three copies of the matrix and vectors rotate so that one step
does not find the previous step's data in the 256 MB last-level cache.

Prints one JSON line: GFLOP/s (2 nnz / t, the paper's throughput metric),
the stage-1 kernel against the HBM roofline, and the CPU oracle beside it.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
  python bench.py --mode copy     # plain device copy of known size (counter calibration)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

PEAK_HBM_GBPS = 8000.0  # MI355X HBM3E, datasheet
METRIC = "CSR SpMV % of HBM roofline + GFLOP/s; learned/batched/FP32 vs plain FP64"


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def alg_bytes(m: int, n: int, nnz: int, val_size: int, vec_size: int) -> int:
    """Each matrix entry once, row_ptr once, x once, y once (int32 indices)."""
    return nnz * (val_size + 4) + (m + 1) * 4 + n * vec_size + m * vec_size


def paper_bytes(m: int, nnz: int, val_size: int) -> int:
    """The paper's bandwidth formula (Section 4.3): x counted once per nonzero."""
    return (m + 1 + nnz) * 4 + (2 * nnz + m) * val_size


def measured_traffic(W: int, S: int, B: int, bind_rows: bool):
    """HBM-side bytes per stage-1 launch from the committed counter records
    (one per launch shape), or None when the device code (the kernel source
    file up to its host side) differs from the one the counters were taken
    on, or no record has this launch shape."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        doc = json.load(open(os.path.join(here, "profiles", "traffic.json")))
        src = open(os.path.join(here, "paper_1504_06474_amd", "csrc", "sss_spmv.hip"), "rb").read()
    except (OSError, ValueError):
        return None
    src = src[:src.index(b"struct sss_plan_s {")]  # the device code: every kernel precedes the host side
    if hashlib.sha256(src).hexdigest()[:16] != doc.get("source_sha256_16"):
        return None
    for rec in doc.get("sss_stage1", []):
        if (W, S, B) == (rec["W"], rec["S"], rec["B"]) and bool(rec["bind_rows"]) == bool(bind_rows):
            return int(rec["fetch_kib_raw"] * doc["fetch_factor"] * 1024 + rec["write_kib_raw"] * doc["write_factor"] * 1024)
    return None


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _time_reps(fn, seconds: float):
    """Repetitions of fn() and the seconds they took, at least one, about `seconds`."""
    reps, t0 = 0, time.perf_counter()
    while True:
        fn()
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            return reps, el


def _finite(v):
    """The JSON line holds no NaN or infinity: such a figure (a block that was
    skipped, an empty sample) becomes null."""
    if isinstance(v, dict):
        return {k: _finite(u) for k, u in v.items()}
    if isinstance(v, (list, tuple)):
        return [_finite(u) for u in v]
    if isinstance(v, float) and not np.isfinite(v):
        return None
    return v


def row_sums(row_ptr, col, val, x):
    """Reference for the error figures this script reports: y_i = sum of
    val*x[col] over row i, and (|A||x|)_i, both summed in long double (64-bit
    mantissa) and rounded to double.  Each product carries a relative error
    below 2^-64 and the sums of up to 2*10^5 terms stay within ~1e-14 of
    (|A||x|)_i of the exact values: far inside the 1e-12 checks.  Plain
    numpy, independent of the library."""
    if np.finfo(np.longdouble).nmant < 63:
        raise RuntimeError("long double is not the 64-bit-mantissa extended type on this host")
    rp = np.asarray(row_ptr, dtype=np.int64)
    m = rp.shape[0] - 1
    p = np.asarray(val, dtype=np.longdouble) * np.asarray(x, dtype=np.longdouble)[np.asarray(col)]
    y = np.zeros(m, dtype=np.longdouble)
    sc = np.zeros(m, dtype=np.longdouble)
    rows = np.flatnonzero(rp[1:] > rp[:-1])  # a non-empty row's entries run to the next non-empty row's start
    if rows.size:
        y[rows] = np.add.reduceat(p, rp[rows])
        sc[rows] = np.add.reduceat(np.abs(p), rp[rows])
    return y.astype(np.float64), sc.astype(np.float64)


def cpu_baseline(A, x, seconds: float) -> dict:
    """The oracle on the host cores (the reported CPU baseline), then the paper's
    CPU comparators on the same matrix (Section 4.3): the oracle's Dot2 row
    loop on one thread, the plain OpenMP row-block loop, and the plain
    single-thread loop.  Each comparator gets a fifth of `seconds`."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    oracle.spmv(A.row_ptr, A.col, A.val, x, threads)  # warm caches / page in
    reps, el = _time_reps(lambda: oracle.spmv(A.row_ptr, A.col, A.val, x, threads), seconds)
    gflops = 2.0 * A.nnz * reps / el / 1e9
    nbytes = A.nnz * 12 + (A.m + 1) * 4 + A.n * 8 + A.m * 8
    comparators = {}
    for name, t, fn in (
            ("dot2_1_thread", 1, lambda: oracle.spmv(A.row_ptr, A.col, A.val, x, 1)),
            ("rowblock_openmp", threads, lambda: oracle.spmv_rowblock(A.row_ptr, A.col, A.val, x, threads)),
            ("naive_1_thread", 1, lambda: oracle.spmv_naive(A.row_ptr, A.col, A.val, x))):
        r, e = _time_reps(fn, seconds / 5)
        comparators[name] = {"GFLOPs": round(2.0 * A.nnz * r / e / 1e9, 3), "GBps": round(nbytes * r / e / 1e9, 2),
                             "threads": t, "reps": r}
    return {"value": round(gflops, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"the full benchmark matrix ({A.nnz} nnz), {reps} repetitions of the Dot2 FP64 "
                      f"row loop with OpenMP over rows, {el:.1f} s",
            "cpu_model": _cpu_model(), "comparators": comparators}


class PlanSet:
    """The plans for a set of rotated copies: with bound rows one plan per
    copy (a bound plan serves only the row_ptr array it was made for), else
    one plan shared by all.  Calls go to the plan of the copy's row_ptr."""

    def __init__(self, sss, copies, m, n, nnz, bind_rows: bool, **kw):
        if bind_rows:
            self.plans = {c[0].data_ptr(): sss.Plan(m, n, nnz, bind_rows=True, row_ptr=c[0], **kw) for c in copies}
        else:
            shared = sss.Plan(m, n, nnz, row_ptr=copies[0][0], **kw)
            self.plans = {c[0].data_ptr(): shared for c in copies}
        self.first = next(iter(self.plans.values()))

    def for_rp(self, rp):
        return self.plans[rp.data_ptr()]

    def execute(self, rp, col, v, xx, y):
        return self.for_rp(rp).execute(rp, col, v, xx, y)

    def stage1(self, rp, col, v, xx, y):
        self.for_rp(rp).stage1(rp, col, v, xx, y)

    def stage2(self, rp, y):
        self.for_rp(rp).stage2(rp, y)

    def floor_probe(self, col, v, xx, out, gather):
        return self.first.floor_probe(col, v, xx, out, gather)  # the probe reads no row structure

    def info(self):
        return self.first.info()

    def close(self):
        for p in {id(p): p for p in self.plans.values()}.values():
            p.close()


def time_steps(torch, plan, copies, steps: int, warmup: int) -> float:
    """Average ms per y = A x over `steps` launches, rotating the copies."""
    for k in range(warmup):
        rp, col, v, xx, y = copies[k % len(copies)]
        plan.execute(rp, col, v, xx, y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for k in range(steps):
        rp, col, v, xx, y = copies[k % len(copies)]
        plan.execute(rp, col, v, xx, y)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def error_stats(y, ref, scale) -> dict:
    """Per-row error scaled by (|A||x|)_i, and plain relative error over rows
    that do not cancel (|y_i| >= 1e-3 (|A||x|)_i)."""
    y = np.asarray(y, dtype=np.float64)
    nz = scale > 0
    e = np.abs(y - ref)[nz] / scale[nz]
    keep = nz & (np.abs(ref) >= 1e-3 * scale)
    rel = np.abs(y - ref)[keep] / np.abs(ref)[keep]
    return {"max_scaled": float(e.max()) if e.size else 0.0, "median_scaled": float(np.median(e)) if e.size else 0.0,
            "max_rel": float(rel.max()) if rel.size else 0.0, "median_rel": float(np.median(rel)) if rel.size else 0.0}


def graph_time_us(torch, fn, copies) -> float:
    """Device time per call of fn(copy): a run of calls captured once into a
    graph (enough for ~2 ms of work) and replayed for ~0.3 s, so that the
    host's per-call launch cost does not hide small kernels."""
    fn(copies[0])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    fn(copies[1 % len(copies)])
    e1.record()
    torch.cuda.synchronize()
    approx = max(e0.elapsed_time(e1), 1e-3)  # ms
    reps = int(max(1, min(64, 2.0 / approx)))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn(copies[0])
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for k in range(reps):
            fn(copies[k % len(copies)])
    g.replay()
    torch.cuda.synchronize()
    trials = int(max(3, min(200, 300.0 / (approx * reps))))
    e0.record()
    for _ in range(trials):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) / (trials * reps) * 1e3
    del g
    return us


def rowwise_comparison(torch, sss, copies, n: int, sss_call) -> dict:
    """The row-wise comparators (CSR-scalar = 1 lane per row ... CSR-vector =
    64 lanes) against the speculative plan's call sss_call(copy), all timed
    the same way (graph_time_us) on the same rotated copies."""
    t_sss = graph_time_us(torch, sss_call, copies)
    times = {}
    for lanes in (1, 2, 4, 8, 16, 32, 64):
        times[lanes] = graph_time_us(torch, lambda c, L=lanes: sss.csr_rowwise(c[0], c[1], c[2], c[3], c[4], n, L),
                                     copies)
    best = min(times, key=times.get)
    return {"sss_us": round(t_sss, 2), "rowwise_us": {str(k): round(v, 2) for k, v in times.items()},
            "speedup_vs_csr_scalar": round(times[1] / t_sss, 2), "speedup_vs_csr_vector": round(times[64] / t_sss, 2),
            "best_rowwise_lanes": best, "speedup_vs_best_rowwise": round(times[best] / t_sss, 2),
            "timing": "graph replay"}


def precision_block(torch, sss, steps: int, warmup: int) -> dict:
    """The 4M-row Zipf-1.8 matrix stored FP64 / FP32 / BF16: time per y = A x
    and the error against the exact product of the FP64 values (row_sums), for
    uniform and lognormal values."""
    import csrgen
    log("[bench] precision: generating the 4M-row Zipf 1.8 matrix (seed 5)")
    A, x = csrgen.config5()
    out = {"workload": "zipf18_4M", "m": A.m, "nnz": A.nnz}
    sizes = {"f64": (8, 8), "f32": (4, 4), "bf16": (2, 4)}
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}
    for values in ("uniform", "lognormal"):
        Av = A if values == "uniform" else csrgen.with_values(A, "lognormal", 55)
        ref64, sc64 = row_sums(Av.row_ptr, Av.col, Av.val, x)
        for kind in ("f64", "f32", "bf16"):
            vs, xs, ve, xe = csrgen.quantize(Av, x, kind)
            rp = torch.from_numpy(Av.row_ptr).cuda()
            col = torch.from_numpy(Av.col).cuda()
            if kind == "bf16":
                v = torch.from_numpy(vs.view(np.int16)).cuda().view(torch.bfloat16)
            else:
                v = torch.from_numpy(np.ascontiguousarray(vs)).cuda()
            xx = torch.from_numpy(np.ascontiguousarray(xs)).cuda()
            ydt = torch.float64 if kind == "f64" else torch.float32
            copies = [(rp, col, v, xx, torch.empty(A.m, dtype=ydt, device="cuda"))]
            if values == "uniform":
                for _ in range(2):
                    copies.append((rp.clone(), col.clone(), v.clone(), xx.clone(),
                                   torch.empty(A.m, dtype=ydt, device="cuda")))
            plan = PlanSet(sss, copies, A.m, A.n, A.nnz, True, dtype=tdt[kind])
            info = plan.info()
            rec = out.setdefault(kind, {"W": info["W"], "S": info["S"]})
            if values == "uniform":
                ms = time_steps(torch, plan, copies, steps, warmup)
                vb, xb = sizes[kind]
                rec.update({"us": round(ms * 1e3, 2), "GFLOPs": round(2 * A.nnz / (ms * 1e-3) / 1e9, 2),
                            "alg_GBps": round(alg_bytes(A.m, A.n, A.nnz, vb, xb) / (ms * 1e-3) / 1e9, 1)})
                # memory floors of this plan's access pattern (see the headline)
                fo = torch.empty(info["n_bunches"] * 64, dtype=ydt, device="cuda")
                fl = {}
                for name, gather in (("stream_us", False), ("stream_gather_us", True)):
                    for k in range(warmup):
                        c = copies[k % len(copies)]
                        plan.floor_probe(c[1], c[2], c[3], fo, gather)
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    torch.cuda.synchronize()
                    e0.record()
                    for k in range(steps):
                        c = copies[k % len(copies)]
                        plan.floor_probe(c[1], c[2], c[3], fo, gather)
                    e1.record()
                    torch.cuda.synchronize()
                    fl[name] = round(e0.elapsed_time(e1) / steps * 1e3, 2)
                rec["floors"] = fl
                del fo
                # stage 1 alone, and the design-independent ceiling of this matrix's reads
                rec["stage1_us"] = round(events_us(torch, lambda c: plan.stage1(*c), copies, steps, warmup), 2)
                rec["gather_ceiling"] = gather_ceiling(torch, sss, copies, alg_bytes(A.m, A.n, A.nnz, vb, xb),
                                                       max(5, steps // 2), 2)
                rec["stage1_frac_of_probe_ceiling"] = round(rec["gather_ceiling"]["best_us"] / rec["stage1_us"], 3)
                rec["stage1_frac_of_probe_ceiling_with_rows"] = round(
                    rec["gather_ceiling"]["with_rows"]["best_us"] / rec["stage1_us"], 3)
                for c in copies:  # every copy's y back to a full product
                    plan.execute(*c)
                if kind == "f64":
                    rec["vs_rowwise"] = rowwise_comparison(torch, sss, copies, A.n, lambda c: plan.execute(*c))
                    log(f"[bench] precision f64 row-wise comparators: {rec['vs_rowwise']}")
                # the learned selector's plan for the same matrix and value type
                if sss.load_selector():
                    sel = PlanSet(sss, copies, A.m, A.n, A.nnz, True, dtype=tdt[kind], mode=sss.MODE_SELECTOR)
                    ms_sel = time_steps(torch, sel, copies, steps, warmup)
                    rec["selected"] = {"W": sel.info()["W"], "S": sel.info()["S"], "us": round(ms_sel * 1e3, 2)}
                    sel.close()
                    # the timed output must stay the default plan's
                    plan.execute(*copies[0])
                y = copies[0][4]
            else:
                y = copies[0][4]
                plan.execute(*copies[0])
            del copies
            torch.cuda.synchronize()
            yh = y.double().cpu().numpy()
            rec.setdefault("err_vs_f64", {})[values] = error_stats(yh, ref64, sc64)
            if kind != "f64":
                refq, scq = row_sums(Av.row_ptr, Av.col, ve, xe)
                st = error_stats(yh, refq, scq)
                # in units of u = 2^-24: products rounded once and y rounded once give at most 2
                st["max_scaled_in_u"] = round(st["max_scaled"] / 2.0 ** -24, 4)
                rec.setdefault("err_arith_only", {})[values] = st
            del rp, col, v, xx, y
            plan.close()
            log(f"[bench] precision {values} {kind}: {rec.get('us')} us")
    for kind in ("f32", "bf16"):
        out[kind]["speedup_vs_f64"] = round(out["f64"]["us"] / out[kind]["us"], 3)
    for kind in ("f64", "f32", "bf16"):
        if "selected" in out[kind]:
            out[kind]["selected"]["speedup_vs_f64_default"] = round(out["f64"]["us"] / out[kind]["selected"]["us"], 3)
    return out


def reduced_on_benchmark_matrix(torch, sss, A, x, ms_f64: float, steps: int, warmup: int) -> dict:
    """The benchmark matrix stored FP32 and BF16 (x and y FP32), each type's
    default plan with rows bound, three rotated copies: time per y = A x, the
    speedup over the FP64 step, and the error against the exact product of
    the FP64 values."""
    import csrgen
    ref, sc = row_sums(A.row_ptr, A.col, A.val, x)
    out = {}
    for kind, vdt in (("f32", torch.float32), ("bf16", torch.bfloat16)):
        vs, xs, _, _ = csrgen.quantize(A, x, kind)
        rp = torch.from_numpy(A.row_ptr).cuda()
        col = torch.from_numpy(A.col).cuda()
        v = (torch.from_numpy(vs.view(np.int16)).cuda().view(torch.bfloat16) if kind == "bf16"
             else torch.from_numpy(np.ascontiguousarray(vs)).cuda())
        xx = torch.from_numpy(np.ascontiguousarray(xs)).cuda()
        copies = [(rp, col, v, xx, torch.empty(A.m, dtype=torch.float32, device="cuda"))]
        for _ in range(2):
            copies.append((rp.clone(), col.clone(), v.clone(), xx.clone(),
                           torch.empty(A.m, dtype=torch.float32, device="cuda")))
        plan = PlanSet(sss, copies, A.m, A.n, A.nnz, True, dtype=vdt)
        ms = time_steps(torch, plan, copies, steps, warmup)
        info = plan.info()
        vb = 4 if kind == "f32" else 2
        out[kind] = {"W": info["W"], "S": info["S"], "us": round(ms * 1e3, 2),
                     "GFLOPs": round(2 * A.nnz / (ms * 1e-3) / 1e9, 2),
                     "alg_GBps": round(alg_bytes(A.m, A.n, A.nnz, vb, 4) / (ms * 1e-3) / 1e9, 1),
                     "speedup_vs_f64": round(ms_f64 / ms, 3),
                     "err_vs_f64": error_stats(copies[0][4].double().cpu().numpy(), ref, sc)}
        plan.close()
        del copies, rp, col, v, xx
        log(f"[bench] benchmark matrix {kind}: {out[kind]['us']} us")
    return out


def events_us(torch, fn, copies, steps: int, warmup: int) -> float:
    """Average microseconds of fn(copy) over `steps` launches rotating the
    copies, between two events on the current stream."""
    for k in range(warmup):
        fn(copies[k % len(copies)])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for k in range(steps):
        fn(copies[k % len(copies)])
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps * 1e3


# the probe configurations timed by gather_ceiling: (mode, in flight, waves
# per SIMD); mode 0 plain loads over the whole grid as one front, 4 the same
# with one contiguous chunk per wavefront, 2 direct-to-LDS gathers
PROBE_CONFIGS = [(0, 1, 4), (0, 4, 4), (0, 16, 4), (0, 16, 8), (0, 2, 2), (4, 4, 4), (4, 16, 2), (4, 8, 1),
                 (2, 1, 4), (2, 8, 1)]


def gather_ceiling(torch, sss, copies, alg: int, steps: int, warmup: int) -> dict:
    """The device's rate for the reads of a CSR SpMV on this matrix with
    none of the method's choices (sss_gather_probe with val streamed: col and
    val coalesced, x gathered), over a set of issue modes, depths and
    occupancies; the best reading is the design-independent ceiling.  Each
    configuration is also timed with the row part (sss_gather_probe_rows:
    row_ptr read, y written), which moves every algorithmic byte; that
    ceiling matters where rows are short.  The copies' y are overwritten."""
    xdt = copies[0][3].dtype
    with_val = copies[0][2].dtype == xdt  # the probe streams val only when it shares x's type
    out_buf = torch.empty(1 << 20, dtype=xdt, device="cuda")
    res, res_rows = {}, {}
    for mode, U, wps in PROBE_CONFIGS:
        try:
            sss.gather_probe(copies[0][1], copies[0][3], out_buf, copies[0][2] if with_val else None, mode, U, wps)
        except sss.SSSError:
            continue
        name = f"{sss.GATHER_MODES[mode & 3]}{'_chunked' if mode & 4 else ''}_u{U}_w{wps}"
        us = events_us(torch, lambda c: sss.gather_probe(c[1], c[3], out_buf, c[2] if with_val else None, mode, U, wps),
                       copies, steps, warmup)
        res[name] = round(us, 2)
        for after in (0, 8):  # rows spread over the gathers, or after them
            us = events_us(torch, lambda c: sss.gather_probe(c[1], c[3], out_buf, c[2] if with_val else None,
                                                             mode | after, U, wps, row_ptr=c[0], y=c[4]),
                           copies, steps, warmup)
            res_rows[name + ("_rows_after" if after else "_rows_spread")] = round(us, 2)
    del out_buf
    best = min(res, key=res.get)
    best_r = min(res_rows, key=res_rows.get)
    return {"probe_us": res, "val_streamed": with_val, "best": best, "best_us": res[best],
            "best_alg_GBps": round(alg / (res[best] * 1e-6) / 1e9, 1),
            "best_frac_of_peak": round(alg / (res[best] * 1e-6) / 1e9 / PEAK_HBM_GBPS, 4),
            "with_rows": {"probe_us": res_rows, "best": best_r, "best_us": res_rows[best_r],
                          "best_alg_GBps": round(alg / (res_rows[best_r] * 1e-6) / 1e9, 1),
                          "best_frac_of_peak": round(alg / (res_rows[best_r] * 1e-6) / 1e9 / PEAK_HBM_GBPS, 4)}}


def stencil_block(torch, sss, steps: int, warmup: int) -> dict:
    """Where gathers are cheap: the 27-point stencil on a 160^3 grid (4.1M
    rows, 109M nnz, 1.39 GB in FP64: far past the 256 MB last-level cache, so
    one copy streams from HBM every call).  The selector's plan and the
    default plan, stage 1 against the floor of its own access pattern, the
    design-independent probe, and the fraction of the HBM peak."""
    from csrgen.torch_gen import _stencil
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    d = _stencil(160, 3, gen, "cuda")
    m, nnz = d["m"], d["nnz"]
    c = (d["row_ptr"], d["col"], d["val"], d["x"], torch.empty(m, dtype=torch.float64, device="cuda"))
    copies = [c]
    alg = alg_bytes(m, m, nnz, 8, 8)
    out = {"workload": "stencil3d_160_f64", "m": m, "nnz": nnz, "alg_bytes": alg}
    # the exact product on sampled rows, to check each plan's timed output
    rows = np.random.default_rng(7).choice(m, size=2000, replace=False)
    rp = d["row_ptr"].cpu().numpy().astype(np.int64)
    colh, valh, xh = d["col"].cpu().numpy(), d["val"].cpu().numpy(), d["x"].cpu().numpy()
    idx = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in rows])
    sub = np.zeros(rows.size + 1, dtype=np.int64)
    np.cumsum(rp[rows + 1] - rp[rows], out=sub[1:])
    ref, sc = row_sums(sub, colh[idx], valh[idx], xh)
    ok = True
    named = [("default", {})]
    if sss.load_selector():
        named.insert(0, ("selected", {"mode": sss.MODE_SELECTOR}))
    sets = {name: PlanSet(sss, copies, m, m, nnz, True, dtype=torch.float64, **kw) for name, kw in named}
    # both plans warmed up, then timed in alternating rounds (median per plan):
    # the first calls on a freshly written matrix run slower whichever plan
    # makes them, so timing one plan after the other favours the second
    for ps in sets.values():
        for _ in range(warmup):
            ps.execute(*c)
    # every figure of every plan in short runs, round after round (stage 1
    # alone, back to back for long, runs at a lower clock than the same calls
    # with stage 2 between them)
    n_run = max(5, steps // 10)
    fos = {name: torch.empty(ps.info()["n_bunches"] * 64, dtype=torch.float64, device="cuda")
           for name, ps in sets.items()}
    figs = ("execute", "stage1", "stage2", "floor_stream", "floor_stream_gather")
    rounds = {name: {f: [] for f in figs} for name in sets}
    for _ in range(5):
        for name, ps in sets.items():
            fo, r = fos[name], rounds[name]
            r["execute"].append(events_us(torch, lambda cc: ps.execute(*cc), copies, n_run, 2))
            r["stage1"].append(events_us(torch, lambda cc: ps.stage1(*cc), copies, n_run, 2))
            r["stage2"].append(events_us(torch, lambda cc: ps.stage2(cc[0], cc[4]), copies, n_run, 2))
            r["floor_stream"].append(events_us(torch, lambda cc: ps.floor_probe(cc[1], cc[2], cc[3], fo, False),
                                               copies, n_run, 2))
            r["floor_stream_gather"].append(events_us(
                torch, lambda cc: ps.floor_probe(cc[1], cc[2], cc[3], fo, True), copies, n_run, 2))
    del fos
    for name, ps in sets.items():
        info = ps.info()
        ex, s1, s2, fs, fg = (float(np.median(rounds[name][f])) for f in figs)
        ps.execute(*c)
        torch.cuda.synchronize()
        got = c[4].cpu().numpy()[rows]
        ok = ok and bool(np.all(np.abs(got - ref) <= 1e-12 * sc))
        out[name] = {"W": info["W"], "S": info["S"], "execute_us": round(ex, 2), "stage1_us": round(s1, 2),
                     "stage2_us": round(s2, 2), "floor_stream_us": round(fs, 2), "floor_stream_gather_us": round(fg, 2),
                     "stage1_frac_of_floor": round(fg / s1, 3),
                     "execute_alg_GBps": round(alg / (ex * 1e-6) / 1e9, 1),
                     "execute_frac_of_peak": round(alg / (ex * 1e-6) / 1e9 / PEAK_HBM_GBPS, 4),
                     "stage1_frac_of_peak": round(alg / (s1 * 1e-6) / 1e9 / PEAK_HBM_GBPS, 4)}
    for ps in sets.values():
        ps.close()
    out["gather_ceiling"] = gather_ceiling(torch, sss, copies, alg, steps, warmup)
    out["sampled_rows_within_1e-12"] = ok
    log(f"[bench] stencil: {out}")
    del d, c, copies
    torch.cuda.empty_cache()
    return out


def classes_block(torch, sss, steps: int, warmup: int) -> dict:
    """Bandwidth utilisation per matrix class (the paper's Section 4.4
    bandwidth figure, and its Section 4.5 parameter sweeps): one large matrix
    of every selector class, FP64, enough rotated copies to pass 1 GB, the
    selector's plan: time, algorithmic GB/s and fraction of the 8 TB/s peak,
    stage 1 against the floor of its access pattern and against the
    design-independent probe; and every (W, S) class timed on it."""
    from csrgen.torch_gen import _stencil, _fem_band, _weblike, _dense_rows
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    rng = np.random.default_rng(11)
    mats = {
        "stencil2d": lambda: _stencil(1414, 2, gen, "cuda"),
        "stencil3d": lambda: _stencil(125, 3, gen, "cuda"),
        "fem_band": lambda: _fem_band(2_000_000, gen, "cuda"),
        "weblike": lambda: _weblike(2_000_000, gen, "cuda"),
        "dense_rows": lambda: _dense_rows(1_000_000, gen, "cuda", 8, rng.integers(10_000, 1_000_000, size=8)),
    }
    out = {}
    for cls, make in mats.items():
        d = make()
        m, n, nnz = d["m"], d["n"], d["nnz"]
        alg = alg_bytes(m, n, nnz, 8, 8)
        k = max(1, int(np.ceil((1 << 30) / alg)))
        copies = [(d["row_ptr"], d["col"], d["val"], d["x"], torch.empty(m, dtype=torch.float64, device="cuda"))]
        for _ in range(k - 1):
            copies.append(tuple(t.clone() for t in copies[0][:4]) + (torch.empty(m, dtype=torch.float64, device="cuda"),))
        ps = PlanSet(sss, copies, m, n, nnz, True, dtype=torch.float64, mode=sss.MODE_SELECTOR)
        info = ps.info()
        ex = events_us(torch, lambda cc: ps.execute(*cc), copies, steps, warmup)
        s1 = events_us(torch, lambda cc: ps.stage1(*cc), copies, steps, warmup)
        fo = torch.empty(info["n_bunches"] * 64, dtype=torch.float64, device="cuda")
        fg = events_us(torch, lambda cc: ps.floor_probe(cc[1], cc[2], cc[3], fo, True), copies, steps, warmup)
        del fo
        ceil = gather_ceiling(torch, sss, copies, alg, max(5, steps // 2), 2)
        grid, best = sss.autotune(*copies[0], n=n, reps=5)
        out[cls] = {"m": m, "nnz": nnz, "alg_bytes": alg, "copies_rotated": k, "W": info["W"], "S": info["S"],
                    "execute_us": round(ex, 2), "stage1_us": round(s1, 2),
                    "alg_GBps": round(alg / (ex * 1e-6) / 1e9, 1),
                    "frac_of_peak": round(alg / (ex * 1e-6) / 1e9 / PEAK_HBM_GBPS, 4),
                    "stage1_frac_of_own_floor": round(fg / s1, 3),
                    "stage1_frac_of_probe_ceiling": round(ceil["best_us"] / s1, 3),
                    "probe_ceiling_frac_of_peak": ceil["best_frac_of_peak"],
                    "stage1_frac_of_probe_ceiling_with_rows": round(ceil["with_rows"]["best_us"] / s1, 3),
                    "probe_ceiling_with_rows_frac_of_peak": ceil["with_rows"]["best_frac_of_peak"],
                    "grid_us_by_class": {f"W{sss.class_params(c)[0]}S{sss.class_params(c)[1]}": round(float(t), 2)
                                         for c, t in enumerate(grid)},
                    "grid_best": "W{}S{}".format(*sss.class_params(best))}
        log(f"[bench] class {cls}: {out[cls]}")
        ps.close()
        del copies, d
        torch.cuda.empty_cache()
    return out


def host_stage2_block(torch, sss, plan, copies, A, x, reps: int = 20) -> dict:
    """The paper's split on this discrete GPU: stage 1 on the device, y and
    the plan's small arrays to host memory, stage 2 on one host core, y back;
    against the device stage 2 (the product path).  Wall-clock per call."""
    y_pin = torch.empty(A.m, dtype=torch.float64, pin_memory=True)
    parts = np.zeros((reps, 3))
    for k in range(reps + 2):
        rp, col, v, xx, y = copies[k % len(copies)]
        p = plan.for_rp(rp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p.stage1(rp, col, v, xx, y)
        y_pin.copy_(y, non_blocking=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        p.stage2_host(A.row_ptr, y_pin)
        t2 = time.perf_counter()
        y.copy_(y_pin, non_blocking=True)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        if k >= 2:
            parts[k - 2] = (t1 - t0, t2 - t1, t3 - t2)
    rows = np.random.default_rng(1).choice(A.m, size=500, replace=False)
    ref, scale = row_sums(A.row_ptr, A.col, A.val, x)
    ref, scale = ref[rows], scale[rows]
    got = copies[(reps + 1) % len(copies)][4].cpu().numpy()[rows]
    mean = [float(v) for v in parts.mean(axis=0) * 1e6]
    return {"stage1_and_copy_to_host_us": round(mean[0], 1), "host_stage2_us": round(mean[1], 1),
            "copy_back_us": round(mean[2], 1), "total_us": round(sum(mean), 1),
            "sampled_rows_within_1e-12": bool(np.all(np.abs(got - ref) <= 1e-12 * scale))}


def _cg_torch_ops(torch, plan, rp, col, v, b, iters: int):
    """The same CG iteration with PyTorch's dot and elementwise kernels for
    the vector steps and the plan's product: the comparison for the
    library's own vector kernels."""
    x = torch.zeros_like(b)
    Ap = torch.empty_like(b)
    r = b.clone()
    p = r.clone()
    rr = torch.dot(r, r)
    for _ in range(iters):
        plan.execute(rp, col, v, p, Ap)
        alpha = rr / torch.dot(p, Ap)
        x.add_(p * alpha)
        r.sub_(Ap * alpha)
        rr_new = torch.dot(r, r)
        p.mul_(rr_new / rr).add_(r)
        rr = rr_new
    return x


def cg_block(torch, sss, iters: int = 300) -> dict:
    """Iterative-solver use: CG on the 5-point Laplacian of a 1024 x 1024
    grid, one bound plan with the selector's (W, S) reused for every
    product; the plan's one-off analysis time (features, the network, the
    first-row search), the time per iteration (the library's loop, and one
    iteration replayed from a graph), the product's share, and the same
    iteration with PyTorch's vector kernels."""
    import csrgen
    from paper_1504_06474_amd.cg import cg
    A = csrgen.laplacian2d_csr(1024)
    rp, col, v = (torch.from_numpy(a).cuda() for a in (A.row_ptr, A.col, A.val))
    x_true = torch.from_numpy(np.random.default_rng(3).uniform(-1, 1, A.n)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = sss.Plan(A.m, A.n, A.nnz, mode=sss.MODE_SELECTOR, bind_rows=True, row_ptr=rp)  # learned (W, S)
    t_plan_ms = (time.perf_counter() - t0) * 1e3
    info = plan.info()
    b = torch.empty_like(x_true)
    plan.execute(rp, col, v, x_true, b)
    cg(plan, rp, col, v, b, max_iter=10)  # warm
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    x, it, hist = cg(plan, rp, col, v, b, rtol=0.0, max_iter=iters, check_every=50)
    e1.record()
    torch.cuda.synchronize()
    it_us = e0.elapsed_time(e1) / it * 1e3
    # one library iteration replayed from a graph (the state keeps iterating)
    cx, cr, cp, cq = (torch.zeros_like(b) for _ in range(4))
    work = torch.empty(sss.cg_workspace_size() // 8, dtype=torch.float64, device="cuda")
    sss.cg_start(plan, rp, col, v, b, cx, cr, cp, cq, work)
    it_graph_us = graph_time_us(torch, lambda c: sss.cg_iterate(plan, rp, col, v, cx, cr, cp, cq, work, 1), [None])
    _cg_torch_ops(torch, plan, rp, col, v, b, 10)  # warm
    torch.cuda.synchronize()
    e0.record()
    _cg_torch_ops(torch, plan, rp, col, v, b, iters)
    e1.record()
    torch.cuda.synchronize()
    torch_it_us = e0.elapsed_time(e1) / iters * 1e3
    del cx, cr, cp, cq, work
    y = torch.empty_like(b)
    spmv_us = graph_time_us(torch, lambda c: plan.execute(*c), [(rp, col, v, x_true, y)])
    s1_us = graph_time_us(torch, lambda c: plan.stage1(*c), [(rp, col, v, x_true, y)])
    fo = torch.empty(plan.info()["n_bunches"] * 64, dtype=torch.float64, device="cuda")
    fl_us = graph_time_us(torch, lambda c: plan.floor_probe(c[1], c[2], c[3], fo, True), [(rp, col, v, x_true, y)])
    # the design-independent probe moving every algorithmic byte (col, val, x,
    # row_ptr, y), best over the probe configurations
    pout = torch.empty(1 << 20, dtype=torch.float64, device="cuda")
    probe_us = {}
    for mode, U, wps in PROBE_CONFIGS:
        try:
            sss.gather_probe(col, x_true, pout, v, mode, U, wps, row_ptr=rp, y=y)
        except sss.SSSError:
            continue
        for after in (0, 8):
            name = f"{sss.GATHER_MODES[mode & 3]}{'_chunked' if mode & 4 else ''}_u{U}_w{wps}"
            probe_us[name + ("_rows_after" if after else "_rows_spread")] = graph_time_us(
                torch, lambda c: sss.gather_probe(c[1], c[3], pout, c[2], mode | after, U, wps, row_ptr=c[0],
                                                  y=c[4]), [(rp, col, v, x_true, y)])
    del pout
    best_probe = min(probe_us, key=probe_us.get)
    byts = alg_bytes(A.m, A.n, A.nnz, 8, 8)
    out = {"workload": "laplacian2d_1024", "m": A.m, "nnz": A.nnz, "W": info["W"], "S": info["S"],
           "plan_ms": round(t_plan_ms, 3),
           "iterations": it, "us_per_iteration": round(it_us, 2),
           "us_per_iteration_graph": round(it_graph_us, 2),
           "us_per_iteration_torch_vector_ops": round(torch_it_us, 2),
           "vector_kernels_us": round(it_graph_us - spmv_us, 2), "spmv_us": round(spmv_us, 2),
           "spmv_alg_GBps": round(byts / (spmv_us * 1e-6) / 1e9, 1), "stage1_us": round(s1_us, 2),
           "stream_gather_floor_us": round(fl_us, 2),
           "probe_with_rows_best": best_probe, "probe_with_rows_us": round(probe_us[best_probe], 2),
           "stage1_frac_of_probe_with_rows": round(probe_us[best_probe] / s1_us, 3),
           "spmv_share": round(spmv_us / it_us, 3), "rel_residual": hist[-1][1],
           "rel_error": float(torch.linalg.vector_norm(x - x_true) / torch.linalg.vector_norm(x_true))}
    plan.close()
    log(f"[bench] cg: {out}")
    return out


def batched_block(torch, sss, steps: int, warmup: int) -> dict:
    """512 uneven power-law matrices: one batched plan (one persistent launch
    per stage, eager and as a replayed HIP graph) against 512 separate plans
    launched one after another (eager and captured in a graph)."""
    import csrgen
    log("[bench] batched: generating 512 matrices (seeds 20000..20511)")
    mats = csrgen.batched_set(512)
    out = {"workload": "batch512_zipf2", "count": len(mats), "sum_m": int(sum(A.m for A, _ in mats)),
           "sum_nnz": int(sum(A.nnz for A, _ in mats))}
    refs, scales = zip(*[row_sums(A.row_ptr, A.col, A.val, x) for A, x in mats])

    def timed(fn, k):
        for _ in range(warmup):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    for kind, tdt in (("f64", torch.float64), ("f32", torch.float32)):
        dev = []
        for A, x in mats:
            dev.append((torch.from_numpy(A.row_ptr).cuda(), torch.from_numpy(A.col).cuda(),
                        torch.from_numpy(A.val).cuda().to(tdt), torch.from_numpy(x).cuda().to(tdt),
                        torch.empty(A.m, dtype=tdt, device="cuda"), A.n))
        bp = sss.BatchPlan(dev, dtype=tdt)
        info = bp.info()
        ms_batch = timed(bp.execute, steps)
        ms_graph = timed(bp.graph_launch, steps)
        # memory floors of the batched stage 1's access pattern (same launch,
        # the probe's loads in place of the method's work)
        fo = torch.empty(info["n_bunches"] * 64, dtype=tdt, device="cuda")
        bfl = {}
        for name, gather in (("stream_us", False), ("stream_gather_us", True)):
            bfl[name] = round(timed(lambda: bp.floor_probe(fo, gather), steps) * 1e3, 1)
        del fo
        # the same plan with a persistent stage 1 (batch_persistent)
        bp_p = sss.BatchPlan(dev, dtype=tdt, persistent=True)
        ms_persistent = timed(bp_p.execute, steps)
        bp_p.close()
        bp.execute()  # the checked output below is the default plan's
        # correctness of the batched result (every matrix, every row)
        worst = 0.0
        for (A, x), d, ref, sc in zip(mats, dev, refs, scales):
            err = np.abs(d[4].double().cpu().numpy() - ref)
            nz = sc > 0
            if nz.any():
                worst = max(worst, float((err[nz] / sc[nz]).max()))
        plans = [sss.Plan(A.m, A.n, A.nnz, dtype=tdt, bind_rows=True, row_ptr=d[0]) for (A, _), d in zip(mats, dev)]

        def separate():
            for pl, d in zip(plans, dev):
                pl.execute(d[0], d[1], d[2], d[3], d[4])

        ms_sep = timed(separate, max(3, steps // 4))
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            separate()
        torch.cuda.current_stream().wait_stream(side)
        with torch.cuda.graph(g):
            separate()
        ms_sep_graph = timed(g.replay, max(3, steps // 4))
        # the batch autotuner's tile schedule (every class timed on this batch)
        bp_grid, grid_us, grid_best = sss.BatchPlan.grid(dev, dtype=tdt, reps=3)
        ginfo = bp_grid.info()
        ms_grid = timed(bp_grid.execute, steps)
        ms_grid_graph = timed(bp_grid.graph_launch, steps)
        worst_grid = 0.0
        for (A, x), d, ref, sc in zip(mats, dev, refs, scales):
            err = np.abs(d[4].double().cpu().numpy() - ref)
            nz = sc > 0
            if nz.any():
                worst_grid = max(worst_grid, float((err[nz] / sc[nz]).max()))
        bp_grid.close()
        # the learned selector's per-matrix schedule (W by its votes, each
        # matrix its own S)
        sel_rec = None
        if sss.load_selector():
            bp_sel = sss.BatchPlan(dev, dtype=tdt, mode=sss.MODE_SELECTOR)
            sW, sS = bp_sel.schedule()
            ms_sel = timed(bp_sel.execute, steps)
            ms_sel_graph = timed(bp_sel.graph_launch, steps)
            worst_sel = 0.0
            for (A, x), d, ref, sc in zip(mats, dev, refs, scales):
                err = np.abs(d[4].double().cpu().numpy() - ref)
                nz = sc > 0
                if nz.any():
                    worst_sel = max(worst_sel, float((err[nz] / sc[nz]).max()))
            bp_sel.close()
            sel_rec = {"W": sW, "S_counts": {str(k): int(sum(1 for v in sS if v == k)) for k in (1, 2, 4, 8)},
                       "batched_us": round(ms_sel * 1e3, 1), "batched_graph_us": round(ms_sel_graph * 1e3, 1),
                       "speedup_vs_separate": round(ms_sep / ms_sel, 2),
                       "vs_autotuned_grid": round(ms_grid / ms_sel, 3), "max_err_scaled_vs_f64": worst_sel}
        vb = 8 if kind == "f64" else 4
        byts = sum(alg_bytes(A.m, A.n, A.nnz, vb, vb) for A, _ in mats)
        out[kind] = {"W": info["W"], "S": info["S"], "n_bunches": info["n_bunches"],
                     "batched_us": round(ms_batch * 1e3, 1), "batched_graph_us": round(ms_graph * 1e3, 1),
                     "persistent_stage1_us": round(ms_persistent * 1e3, 1),
                     "floors": bfl,
                     "separate_us": round(ms_sep * 1e3, 1), "separate_graph_us": round(ms_sep_graph * 1e3, 1),
                     "speedup_vs_separate": round(ms_sep / ms_batch, 2),
                     "speedup_vs_separate_graph": round(ms_sep_graph / ms_batch, 2),
                     "batched_GFLOPs": round(2 * out["sum_nnz"] / (ms_batch * 1e-3) / 1e9, 1),
                     "batched_alg_GBps": round(byts / (ms_batch * 1e-3) / 1e9, 1),
                     "max_err_scaled_vs_f64": worst,
                     "autotuned": {"W": ginfo["W"], "S": ginfo["S"], "grid_class_us": [round(float(t), 1) for t in grid_us],
                                   "batched_us": round(ms_grid * 1e3, 1),
                                   "batched_graph_us": round(ms_grid_graph * 1e3, 1),
                                   "speedup_vs_separate": round(ms_sep / ms_grid, 2),
                                   "speedup_vs_separate_graph": round(ms_sep_graph / ms_grid, 2),
                                   "max_err_scaled_vs_f64": worst_grid},
                     "selector_scheduled": sel_rec}
        log(f"[bench] batched {kind}: {out[kind]}")
        del g, plans, bp, dev
        torch.cuda.synchronize()
    return out


def selector_block(torch, sss, n_matrices: int, bench_matrix, n_large: int = 10) -> dict:
    """The trained selector on held-out selector matrices (indices 2000..,
    not trained on) and on held-out matrices of the set's large part (2e6 to
    1.6e7 rows, indices 2360..), each stored as FP64, FP32 and BF16: regret
    against the grid timed here, gain over the default parameters of that
    value type; and its pick for the benchmark matrix."""
    from csrgen.torch_gen import selector_matrix_gpu
    if not sss.load_selector():
        return {"error": "no trained selector parameters"}

    from paper_1504_06474_amd.selector_train import VALUE_TYPES, time_plan as t_plan

    gm = lambda a: float(np.exp(np.mean(np.log(a))))

    def evaluate(indices, by_class):
        acc = {k: {"ratios": [], "gains": [], "hits": 0, "misses": []} for k in VALUE_TYPES}
        for i in indices:
            d = selector_matrix_gpu(i)
            for kind, (vt, xt) in VALUE_TYPES.items():
                a = acc[kind]
                args = (d["row_ptr"], d["col"], d["val"].to(vt), d["x"].to(xt),
                        torch.empty(d["m"], dtype=xt, device="cuda"))
                grid, best = sss.autotune(*args, n=d["n"], reps=5)
                cls = sss.selector_predict(sss.features(d["row_ptr"], d["n"], d["nnz"], vt))
                W, S = sss.class_params(cls)
                p_def = sss.Plan(d["m"], d["n"], d["nnz"], dtype=vt, bind_rows=True, row_ptr=d["row_ptr"])
                p_sel = sss.Plan(d["m"], d["n"], d["nnz"], dtype=vt, W=W, S=S, bind_rows=True,
                                 row_ptr=d["row_ptr"])
                t_def, t_sel = t_plan(p_def, args, 5), t_plan(p_sel, args, 5)
                if by_class is not None and kind == "f64" and i < 2005:  # one matrix of each selector class
                    by_class[d["cls"]] = dict(rowwise_comparison(torch, sss, [args], d["n"],
                                                                 lambda c: p_sel.execute(*c)),
                                              matrix=d["name"], m=d["m"], nnz=d["nnz"], sss_plan=[W, S])
                p_def.close()
                p_sel.close()
                a["ratios"].append(grid[cls] / grid.min())
                a["gains"].append(t_def / t_sel)
                a["hits"] += int(cls == best)
                if a["ratios"][-1] > 1.1:
                    a["misses"].append({"i": i, "name": d["name"], "picked": [W, S],
                                        "best": list(sss.class_params(best)),
                                        "picked_us": round(float(grid[cls]), 1),
                                        "best_us": round(float(grid.min()), 1)})
                del args
            del d
        res = {}
        for kind, a in acc.items():
            res[kind] = {"regret_vs_grid": round(gm(a["ratios"]) - 1, 4), "gain_vs_default": round(gm(a["gains"]), 3),
                         "top1": round(a["hits"] / len(indices), 3), "worst_ratio": round(float(max(a["ratios"])), 3),
                         "picks_over_10pct": a["misses"]}
        res["regret_vs_grid"] = round(gm([r for a in acc.values() for r in a["ratios"]]) - 1, 4)
        res["gain_vs_default"] = round(gm([g for a in acc.values() for g in a["gains"]]), 3)
        return res

    by_class = {}
    out = {"held_out_matrices": n_matrices, "vs_rowwise_by_class": by_class}
    out.update(evaluate(range(2000, 2000 + n_matrices), by_class))
    if n_large:
        import csrgen
        from paper_1504_06474_amd.selector_train import LARGE_TRAIN
        first = csrgen.SELECTOR_LARGE_BASE + LARGE_TRAIN  # the large part's held-out matrices
        out["large"] = dict(held_out_matrices=n_large, rows="2e6..1.6e7",
                            **evaluate(range(first, first + n_large), None))
    rp, col, v, xx, y, A = bench_matrix
    grid, best = sss.autotune(rp, col, v, xx, y, n=A.n, reps=5)
    cls = sss.selector_predict(sss.features(rp, A.n, A.nnz))
    p_def = sss.Plan(A.m, A.n, A.nnz, bind_rows=True, row_ptr=rp)
    t_def = t_plan(p_def, (rp, col, v, xx, y), 5)
    p_def.close()
    out["benchmark_matrix"] = {"selected": list(sss.class_params(cls)), "selected_us": round(float(grid[cls]), 2),
                               "grid_best": list(sss.class_params(best)), "grid_best_us": round(float(grid.min()), 2),
                               "default_W8S5_us": round(float(t_def), 2)}
    log(f"[bench] selector: {out}")
    return out


def device_copy_ms(torch, steps: int, nbytes: int = 1 << 30) -> float:
    """Average ms of a plain device-to-device copy of nbytes (torch's copy_)."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps


def run_copy_calibration(steps: int):
    import torch
    nbytes = 1 << 30
    ms = device_copy_ms(torch, steps, nbytes)
    print(json.dumps({"mode": "copy", "bytes_read": nbytes, "bytes_written": nbytes, "ms": ms,
                      "GBps": 2 * nbytes / (ms * 1e-3) / 1e9}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--copies", type=int, default=3)
    ap.add_argument("--W", type=int, default=0)
    ap.add_argument("--S", type=int, default=0)
    ap.add_argument("--B", type=int, default=0)
    ap.add_argument("--skip-extras", action="store_true",
                    help="time only the headline plan (no floor probes, no second plan variant): for profiling runs")
    ap.add_argument("--extras", choices=["all", "ceiling", "none"], default="all",
                    help="headline blocks beside the timed steps: all; only the floors and the gather ceiling "
                         "(for counter runs); none (= --skip-extras)")
    ap.add_argument("--no-bind-rows", action="store_true",
                    help="search each thread-bunch's first row in every call instead of once at plan time")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", choices=["spmv", "copy"], default="spmv")
    ap.add_argument("--skip-precision", action="store_true", help="skip the FP32/BF16 comparison")
    ap.add_argument("--skip-batched", action="store_true", help="skip the 512-matrix batched comparison")
    ap.add_argument("--skip-selector", action="store_true", help="skip the tile-selector evaluation")
    ap.add_argument("--skip-cg", action="store_true", help="skip the conjugate-gradient workload")
    ap.add_argument("--skip-stencil", action="store_true", help="skip the 1.39 GB stencil block")
    ap.add_argument("--skip-classes", action="store_true", help="skip the per-class bandwidth block")
    ap.add_argument("--plan", choices=["grid", "selector", "default"], default="grid",
                    help="the headline plan's (W, S): the library's grid autotuner (GRID plans), the learned "
                         "selector (SELECTOR plans) or the per-type default; --W/--S fix them instead")
    args = ap.parse_args()
    if args.skip_extras:
        args.extras = "none"
    args.skip_extras = args.extras == "none"
    comparators = args.extras == "all"

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the multi-GPU path is not built (see the design notes on "
              "sharding); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.mode == "copy":
        run_copy_calibration(args.steps)
        return

    import csrgen
    from paper_1504_06474_amd import sss

    log("[bench] generating the 1M-row power-law matrix (seed 1)")
    A, x = csrgen.config2()
    m, n, nnz = A.m, A.n, A.nnz
    log(f"[bench] m={m} nnz={nnz} max_row={int(np.diff(A.row_ptr).max())}")

    dev = "cuda"
    copies = []
    for _ in range(max(1, args.copies)):
        copies.append((torch.from_numpy(A.row_ptr).to(dev), torch.from_numpy(A.col).to(dev),
                       torch.from_numpy(A.val).to(dev), torch.from_numpy(x).to(dev),
                       torch.empty(m, dtype=torch.float64, device=dev)))
    # plan / analyse (outside the timed region): the parameters from the
    # learned selector (SELECTOR mode: features on the device, the network),
    # or the default, or the fixed --W/--S; with bind_rows the tile boundary
    # search runs once here instead of in every call
    bind = not args.no_bind_rows
    plan_name = "fixed" if (args.W or args.S) else args.plan
    if plan_name == "selector" and not sss.load_selector():
        plan_name = "default"
    plan_kw = {"W": args.W, "S": args.S}
    if plan_name == "selector":
        plan_kw = {"mode": sss.MODE_SELECTOR}
    elif plan_name == "grid":
        # the autotuner's timing of every class on this matrix (what a GRID
        # plan does), then one bound plan of that class per rotated copy
        _, best = sss.autotune(*copies[0], n=n, reps=5)
        W_g, S_g = sss.class_params(best)
        plan_kw = {"W": W_g, "S": S_g}
    plan = PlanSet(sss, copies, m, n, nnz, bind, dtype=torch.float64, B=args.B, **plan_kw)
    info = plan.info()
    log(f"[bench] plan ({plan_name}) {info}")
    torch.cuda.synchronize()

    def step(k):
        rp, col, v, xx, y = copies[k % len(copies)]
        plan.execute(rp, col, v, xx, y)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} done")

    # headline: K whole steps, rotating copies
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for k in range(args.steps):
        step(k)
    ev1.record()
    torch.cuda.synchronize()
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    gflops = 2.0 * nnz / (ms_step * 1e-3) / 1e9
    log(f"[bench] timed {args.steps} steps: {ms_step * 1e3:.2f} us/step, {gflops:.1f} GFLOP/s")

    # per-stage durations: events around each stage on the launch stream
    ea = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    eb = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ec = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    for k in range(args.steps):
        rp, col, v, xx, y = copies[k % len(copies)]
        ea[k].record()
        plan.stage1(rp, col, v, xx, y)
        eb[k].record()
        plan.stage2(rp, y)
        ec[k].record()
    torch.cuda.synchronize()
    s1 = np.array([ea[k].elapsed_time(eb[k]) for k in range(args.steps)])
    s2 = np.array([eb[k].elapsed_time(ec[k]) for k in range(args.steps)])
    s1_each_ms = float(s1.mean())
    s2_ms = float(s2.mean())
    # the roofline's kernel duration: stage 1 alone, K launches back to back
    # between two events on the launch stream (an event pair around every
    # launch adds a few microseconds per launch to what the kernel takes)
    s1_ms = events_us(torch, lambda c: plan.stage1(*c), copies, args.steps, args.warmup) * 1e-3
    for c in copies:  # every copy's y back to a full product
        plan.execute(*c)
    log(f"[bench] stage1 {s1_ms * 1e3:.2f} us back to back ({s1_each_ms * 1e3:.2f} us with events around each), "
        f"stage2 {s2_ms * 1e3:.2f} us")

    # the distribution of whole steps: events around every step (the headline
    # above is the bracketed K-step time)
    torch.cuda.synchronize()
    for k in range(args.steps):
        ea[k].record()
        step(k)
        eb[k].record()
    torch.cuda.synchronize()
    st = np.array([ea[k].elapsed_time(eb[k]) for k in range(args.steps)]) * 1e3
    per_step = {"mean": round(float(st.mean()), 2), "median": round(float(np.median(st)), 2),
                "p10": round(float(np.percentile(st, 10)), 2), "p90": round(float(np.percentile(st, 90)), 2)}

    # memory floors of stage 1's access pattern with the same tiling and the
    # same rotated copies: col/val streamed alone, and streamed with x gathered
    floor_out = torch.empty(info["n_bunches"] * 64, dtype=torch.float64, device="cuda")
    floors = {"stream_us": float("nan"), "stream_gather_us": float("nan")}
    for name, gather in (() if args.skip_extras else (("stream_us", False), ("stream_gather_us", True))):
        for k in range(args.warmup):
            rp, col, v, xx, y = copies[k % len(copies)]
            plan.floor_probe(col, v, xx, floor_out, gather)
        torch.cuda.synchronize()
        for k in range(args.steps):
            rp, col, v, xx, y = copies[k % len(copies)]
            ea[k].record()
            plan.floor_probe(col, v, xx, floor_out, gather)
            eb[k].record()
        torch.cuda.synchronize()
        floors[name] = float(np.mean([ea[k].elapsed_time(eb[k]) for k in range(args.steps)])) * 1e3
    del floor_out
    log(f"[bench] floors {floors}")

    # a plain device copy on the same device: the practical streaming rate
    copy_GBps = None
    if comparators:
        copy_GBps = round(2 * (1 << 30) / (device_copy_ms(torch, 10) * 1e-3) / 1e9, 1)
        log(f"[bench] device copy {copy_GBps} GB/s (read + write)")

    # the other plan variant (first rows searched in every call, or bound)
    ms_other = s1_other = float("nan")
    if comparators:
        other = PlanSet(sss, copies, m, n, nnz, not bind, dtype=torch.float64, W=info["W"], S=info["S"], B=args.B)
        ms_other = time_steps(torch, other, copies, args.steps, args.warmup)
        torch.cuda.synchronize()
        for k in range(args.steps):
            rp, col, v, xx, y = copies[k % len(copies)]
            ea[k].record()
            other.stage1(rp, col, v, xx, y)
            eb[k].record()
            other.stage2(rp, y)
        torch.cuda.synchronize()
        s1_other = float(np.mean([ea[k].elapsed_time(eb[k]) for k in range(args.steps)]))
        other.close()
        log(f"[bench] {'searching' if bind else 'bound-rows'} plan: {ms_other * 1e3:.2f} us/step, "
            f"stage1 {s1_other * 1e3:.2f} us")

    # the per-type default plan (the paper's Table 3 values for its AMD GPU)
    # beside the headline plan, and the device's gather ceiling on this matrix
    default_rec = ceiling = None
    if comparators:
        dp = PlanSet(sss, copies, m, n, nnz, bind, dtype=torch.float64, B=args.B)
        dinfo = dp.info()
        default_rec = {"W": dinfo["W"], "S": dinfo["S"],
                       "us_per_step": round(events_us(torch, lambda c: dp.execute(*c), copies, args.steps,
                                                      args.warmup), 2),
                       "stage1_us": round(events_us(torch, lambda c: dp.stage1(*c), copies, args.steps,
                                                    args.warmup), 2)}
        for c in copies:  # restore every copy's y to a full product of the headline plan
            plan.execute(*c)
        dp.close()
        log(f"[bench] default plan: {default_rec}")
    if not args.skip_extras:
        ceiling = gather_ceiling(torch, sss, copies, alg_bytes(m, n, nnz, 8, 8), args.steps, args.warmup)
        ceiling["stage1_frac_of_ceiling"] = round(ceiling["best_us"] / (s1_ms * 1e3), 3)
        ceiling["stage1_frac_of_ceiling_with_rows"] = round(ceiling["with_rows"]["best_us"] / (s1_ms * 1e3), 3)
        log(f"[bench] gather ceiling: {ceiling}")

    # the paper's comparison (Section 4.3) on this matrix: row-wise kernels
    comp_c2 = None
    if comparators:
        comp_c2 = rowwise_comparison(torch, sss, copies, n, lambda c: plan.execute(*c))
        log(f"[bench] row-wise comparators: {comp_c2}")

    # the paper's heterogeneous split (stage 2 on a host core) on this part
    host_s2 = None
    if comparators:
        host_s2 = host_stage2_block(torch, sss, plan, copies, A, x)
        host_s2["device_execute_us"] = round(ms_step * 1e3, 2)
        log(f"[bench] stage 2 on the host: {host_s2}")

    # the same matrix stored FP32 and BF16
    reduced = None
    if comparators:
        reduced = reduced_on_benchmark_matrix(torch, sss, A, x, ms_step, args.steps, args.warmup)

    # warm cache: the same copy every step
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        step(0)
    ev1.record()
    torch.cuda.synchronize()
    ms_warm = ev0.elapsed_time(ev1) / args.steps

    # correctness of the benchmarked launch configuration: every row, within
    # 1e-12 of (|A||x|)_i; the plain relative error over rows that do not
    # cancel (|y_i| >= 1e-3 (|A||x|)_i)
    y0 = copies[0][4].cpu().numpy()
    ref, scale = row_sums(A.row_ptr, A.col, A.val, x)
    err = np.abs(y0 - ref)
    err_ok = bool(np.all(err <= 1e-12 * scale))
    max_scaled = float(np.max(err / np.where(scale > 0, scale, 1.0)))
    big = (scale > 0) & (np.abs(ref) >= 1e-3 * scale)
    max_rel = float(np.max(err[big] / np.abs(ref[big]))) if big.any() else 0.0
    del ref, scale, err, big

    B = alg_bytes(m, n, nnz, 8, 8)
    achieved = B / (s1_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "powerlaw_1M_zipf2_f64", "m": m, "n": n, "nnz": nnz, "plan": plan_name,
                   "W": info["W"], "S": info["S"], "B": info["B"], "T": 64, "bind_rows": bind,
                   "copies_rotated": len(copies)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBPS, 4),
                     "traffic": measured_traffic(info["W"], info["S"], info["B"], bind),
                     "kernel": "sss_stage1<f64,W>", "alg_bytes_per_launch": B,
                     "avg_launch_us": round(s1_ms * 1e3, 2)},
        "extras": {
            "step_GBps": round(B / (ms_step * 1e-3) / 1e9, 1),
            "step_frac_of_peak": round(B / (ms_step * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4),
            "stage1_us": round(s1_ms * 1e3, 2),
            "stage1_us_events_each": round(s1_each_ms * 1e3, 2),
            "stage2_us": round(s2_ms * 1e3, 2),
            ("searching_plan" if bind else "bound_rows_plan"): None if not comparators else {
                "us_per_step": round(ms_other * 1e3, 2), "stage1_us": round(s1_other * 1e3, 2)},
            "per_step_us": per_step,
            "device_copy_GBps": copy_GBps,
            "warm_cache_us_per_step": round(ms_warm * 1e3, 2),
            "warm_cache_GFLOPs": round(2.0 * nnz / (ms_warm * 1e-3) / 1e9, 2),
            "paper_formula_GBps": round(paper_bytes(m, nnz, 8) / (ms_step * 1e-3) / 1e9, 1),
            "default_plan": default_rec,
            "gather_ceiling": ceiling,
            "floors": None if args.skip_extras else {"stream_us": round(floors["stream_us"], 2),
                       "stream_GBps": round(12.0 * nnz / (floors["stream_us"] * 1e-6) / 1e9, 1),
                       "stream_gather_us": round(floors["stream_gather_us"], 2),
                       "stage1_frac_of_stream_gather_floor": round(floors["stream_gather_us"] / (s1_ms * 1e3), 3)},
            "vs_rowwise": comp_c2,
            "stage2_on_host": host_s2,
            "reduced_precision": reduced,
            "all_rows_within_1e-12": err_ok,
            "max_err_over_abs_Ax": max_scaled,
            "max_rel_err": max_rel,
        },
    }
    if not args.skip_selector:
        out["extras"]["selector"] = selector_block(torch, sss, 40, copies[0] + (A,))
    del copies
    if not args.skip_precision:
        out["extras"]["precision"] = precision_block(torch, sss, min(args.steps, 50), min(args.warmup, 5))
    if not args.skip_batched:
        out["extras"]["batched"] = batched_block(torch, sss, min(args.steps, 20), 2)
    if not args.skip_cg:
        out["extras"]["cg"] = cg_block(torch, sss)
    if not args.skip_stencil:
        out["extras"]["stencil"] = stencil_block(torch, sss, min(args.steps, 50), min(args.warmup, 5))
    if not args.skip_classes:
        out["extras"]["classes"] = classes_block(torch, sss, min(args.steps, 30), min(args.warmup, 3))
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(A, x, args.cpu_seconds)
    print(json.dumps(_finite(out), allow_nan=False), flush=True)


if __name__ == "__main__":
    main()
