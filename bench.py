#!/usr/bin/env python3
"""Throughput of the linearized-implicit thermochemistry update on one
MI355X.

Workload: the 128^3 = 2,097,152-cell grid population (independent cells,
log-uniform densities 1..1e8 cm^-3, temperatures 10..1e4 K, photon
densities over six decades, Z in {0.01, 0.1, 1} per cell, dt = 10 kyr),
inputs resident in HBM before the timed region.  One step = one call of
sfc_chem_step over all cells (every subcycle of every cell), preceded by a
device-to-device restore of the initial state so that each step does the
same work.

Metric: cell-updates/s (one cell advanced over the whole dt, all subcycles
included) of the binary64 path at dust factor 1 (C_d = 1e4 erg/g/K).
Also reported: the dust-capacity sweep (factors 10, 100, 1000), the mixed
binary32/binary64 path, and the CPU reference timed on a sample of the same
cells.

    python bench.py [--steps K] [--warmup W] [--no-sweep] [--no-mixed] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic operations per subcycle of the LI update (add/sub, mul, div,
# sqrt with a multiply-add counted as 2, plus 44 transcendental calls counted
# as 1 each), from the counting build of the CPU reference on a seeded
# sample of this workload: python -m oracle.count_ops
FLOP_PER_SUBCYCLE = 1539.0
PEAK_FP64_VALU = 78.6e12      # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
BYTES_PER_CELL = 132          # 8 float64 reads, 7 float64 writes, 3 int32 writes
STATE_KEYS = ("y_h2", "y_e", "eint", "tdust")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stats(a):
    a = np.asarray(a, np.float64)
    return dict(mean=float(a.mean()), p50=float(np.median(a)), p99=float(np.percentile(a, 99)),
                max=float(a.max()))


def relerr(a, b, floor=1e-20):
    e = np.abs(a - b) / np.maximum(np.abs(b), floor)
    return dict(max=float(np.nanmax(e)), p99=float(np.nanpercentile(e, 99)),
                median=float(np.nanmedian(e)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-cells", type=int, default=8192)
    ap.add_argument("--cells", type=int, default=None, help="fewer cells (testing only)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run three device-to-device copies of MIB MiB (a kernel of "
                         "known traffic, to scale the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; the update has no cross-GPU "
              "step (cells are independent), so --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copied {args.calibrate_copy} MiB three times "
            f"(each: {n * 8} bytes read, {n * 8} bytes written)")
        return

    import paper_2604_21438_amd as sfc
    from paper_2604_21438_amd import workloads as W

    cells, dt = W.grid128(n=args.cells)
    n = cells["nh"].shape[0]
    log(f"[bench] workload grid128: {n} cells, dt = {dt:.4e} s")
    pristine = sfc.to_device(cells, outputs=False)
    work = sfc.to_device(cells)
    stream = torch.cuda.current_stream()

    def restore():
        for k in STATE_KEYS:
            work[k].copy_(pristine[k])

    def run(ctx, prec, steps, warmup, label):
        for i in range(warmup):
            restore()
            ctx.step(work, dt, prec)
            torch.cuda.synchronize()
            log(f"[bench] {label}: warmup {i + 1}/{warmup} done")
        evs = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            restore()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ctx.step(work, dt, prec)
            e1.record(stream)
            evs.append((e0, e1))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kern = [a.elapsed_time(b) * 1e-3 for a, b in evs]
        out = {k: v.cpu().numpy() for k, v in work.items()}
        log(f"[bench] {label}: {steps} steps in {t1 - t0:.3f} s, kernel {np.mean(kern):.3f} s/launch")
        return (t1 - t0) / steps, float(np.mean(kern)), out

    def describe(out):
        ns = out["nsub"].astype(np.int64)
        fl = out["flags"].view(np.uint32)
        return dict(nsub=stats(ns), tight_fraction=float(((fl & sfc.F_TIGHT) != 0).mean()),
                    niter_mean_tight=float(out["niter"][(fl & sfc.F_TIGHT) != 0].mean())
                    if np.any(fl & sfc.F_TIGHT) else 0.0,
                    cap_fraction=float(((fl & sfc.F_CAP) != 0).mean()),
                    subcycles=int(ns.sum()))

    # ---- headline: binary64 at dust factor 1 ----
    ctx = sfc.Context(dust_factor=1.0)
    step_s, kern_s, out64 = run(ctx, sfc.FP64, args.steps, args.warmup, "fp64 factor 1")
    ctx.close()
    d64 = describe(out64)
    flops = FLOP_PER_SUBCYCLE * d64["subcycles"]
    achieved = flops / kern_s
    result = {
        "metric": "chem cell-updates/s",
        "value": n / step_s,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "grid128: 128^3 = 2,097,152 independent cells, log n_H ~ U[0,8], "
                        "log T ~ U[1,4], T_d = T, Z in {0.01,0.1,1}, dt = 10 kyr, "
                        "dust factor 1 (C_d = 1e4 erg/g/K), IR fixed",
            "cells": n, "dt_s": dt, "dust_factor": 1.0, "precision": "fp64",
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_FP64_VALU / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_VALU,
            "traffic": None,
            "kernel": "li_step_kernel<double>",
            "flop_per_subcycle": FLOP_PER_SUBCYCLE,
            "subcycles_per_launch": d64["subcycles"],
            "kernel_s_per_launch": kern_s,
            "hbm_gbs_algorithmic": n * BYTES_PER_CELL / kern_s / 1e9,
        },
        "stats_fp64": d64,
    }

    # ---- dust-capacity sweep ----
    if not args.no_sweep:
        sweep = {"1": dict(value=n / step_s, **{k: d64[k] for k in ("nsub", "tight_fraction",
                                                                     "niter_mean_tight")})}
        for f in (10.0, 100.0, 1000.0):
            c = sfc.Context(dust_factor=f)
            s, ks, o = run(c, sfc.FP64, 1, 0, f"fp64 factor {f:g}")
            c.close()
            dd = describe(o)
            acc = {k: relerr(o[k], out64[k]) for k in ("y_h2", "y_e", "y_h", "y_hp", "tgas",
                                                        "tdust")}
            sweep[f"{f:g}"] = dict(value=n / s, nsub=dd["nsub"],
                                   tight_fraction=dd["tight_fraction"],
                                   niter_mean_tight=dd["niter_mean_tight"],
                                   vs_factor1=acc)
        result["dust_factor_sweep"] = sweep

    # ---- mixed binary32 / binary64 ----
    outmx = None
    if not args.no_mixed:
        c = sfc.Context(dust_factor=1.0)
        s, ks, outmx = run(c, sfc.MIXED, args.steps, args.warmup, "mixed factor 1")
        c.close()
        result["mixed"] = dict(value=n / s, ms_per_step=s * 1e3, kernel_s_per_launch=ks,
                               speedup_vs_fp64=step_s / s,
                               vs_fp64={k: relerr(outmx[k], out64[k])
                                        for k in ("y_h2", "y_e", "y_h", "y_hp", "y_hm", "tgas",
                                                  "tdust")},
                               stats=describe(outmx))

    # ---- CPU reference on a sample of the same cells ----
    if not args.no_cpu:
        import oracle
        m = min(args.cpu_cells, n)
        sub, idx = W.subsample(cells, m, seed=99)
        threads = max(1, min(16, os.cpu_count() or 1))
        log(f"[bench] cpu reference: {m} cells on {threads} threads")
        t0 = time.perf_counter()
        ref = oracle.li_step(sub, dt, nthreads=threads)
        el = time.perf_counter() - t0
        log(f"[bench] cpu reference done in {el:.1f} s")
        result["cpu_baseline"] = {"value": m / el, "unit": "cell-updates/s", "cores": threads,
                                  "kind": "oracle",
                                  "sample": f"{m} seeded cells of the same 128^3 population, "
                                            f"dt = 10 kyr, dust factor 1, binary64"}
        par = {"fp64": {k: relerr(out64[k][idx], ref[k]) for k in
                        ("y_h2", "y_e", "y_h", "y_hp", "y_hm", "tgas", "tdust")}}
        par["fp64_nsub_mismatch"] = int((out64["nsub"][idx] != ref["nsub"]).sum())
        if outmx is not None:
            par["mixed"] = {k: relerr(outmx[k][idx], ref[k]) for k in
                            ("y_h2", "y_e", "y_h", "y_hp", "y_hm", "tgas", "tdust")}
        result["parity_on_cpu_sample"] = par

    print(json.dumps(result))


if __name__ == "__main__":
    main()
