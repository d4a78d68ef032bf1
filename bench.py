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
# as 1 each, and the tight dust solve's Newton iterations), from the counting
# build of the CPU reference on a seeded sample of this workload with E_IR
# evolved: python -m oracle.count_ops; with the IR field held (FIXED):
# python -m oracle.count_ops --fixed-ir
FLOP_PER_SUBCYCLE = 1705.0
FLOP_PER_SUBCYCLE_FIXED_IR = 1552.0
PEAK_FP64_VALU = 78.6e12      # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
BYTES_PER_CELL = 148          # 9 float64 reads, 8 float64 writes, 3 int32 writes (E_IR evolved)
# HBM bytes of one binary64 step on the 128^3 workload (the two launches of
# the LI kernel under progress dispatch, first pass and resumed pass), from
# rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each scaled
# by what the same counter reads for a 256 MiB device-to-device copy
# (bench.py --calibrate-copy 256).  Valid only for the plain-step sources
# whose combined SHA-1 is given (sfk.h, sfk_lane.h, sfk_li.hip,
# sfk_exp_table.h, in that order): with any other source the figure is
# reported as null.
TRAFFIC = {"kernel_sha1": "bf797566d6fa5ad099df9ed33212b57751a3201c",
           "fetch_bytes": 3.2300e+09, "write_bytes": 9.9822e+08}
KERNEL_SRCS = [os.path.join(ROOT, "paper_2604_21438_amd", "csrc", f)
               for f in ("sfk.h", "sfk_lane.h", "sfk_li.hip", "sfk_exp_table.h")]


def kernel_sha1():
    import hashlib
    h = hashlib.sha1()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(n):
    """The counted bytes, for the full 128^3 step of the sources they were
    taken on; None for anything else."""
    if n != 128 ** 3 or TRAFFIC["kernel_sha1"] is None or TRAFFIC["kernel_sha1"] != kernel_sha1():
        return None
    return TRAFFIC["fetch_bytes"] + TRAFFIC["write_bytes"]
STATE_KEYS = ("y_h2", "y_e", "eint", "tdust", "eir")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stats(a):
    a = np.asarray(a, np.float64)
    return dict(mean=float(a.mean()), p50=float(np.median(a)), p99=float(np.percentile(a, 99)),
                max=float(a.max()))


def relerr(a, b, floor=1e-20):
    e = np.abs(a - b) / np.maximum(np.abs(b), floor)
    return dict(max=float(np.nanmax(e)), p99=float(np.nanpercentile(e, 99)),
                median=float(np.nanmedian(e)), frac_above_1e9=float(np.mean(e > 1e-9)))


def worst_rel(out, ref, idx, floor=1e-20):
    """Largest relative error of each sampled cell over the outputs (y_H by
    the binary64 bar: within 4 ulp of 1 absolute counts as exact)."""
    w = np.zeros(len(idx))
    for k in ("y_h2", "y_e", "y_h", "y_hp", "y_hm", "tgas", "tdust"):
        d = np.abs(out[k][idx] - ref[k])
        e = d / np.maximum(np.abs(ref[k]), floor)
        if k == "y_h":
            e = np.where(d <= 4 * np.finfo(float).eps, 0.0, e)
        w = np.maximum(w, np.nan_to_num(e, nan=np.inf))
    return w


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def pct(a, q):
    return float(np.percentile(np.asarray(a, np.float64), q))


def served_leg(args, sfc, W, torch):
    """Requests of 8^3 blocks (count log-uniform in [1, max_blocks]) cut out
    of the log-normal / point-source population, levels 0..5 with
    dt = 10 kyr / 2^L, dust factor 100.  Legs: the plain path called
    request by request (binary64, then mixed), the served form with every
    request queued at once (its capacity), and the served form fed by a
    Poisson process at a fraction of that capacity (latency = done - arrival)."""
    reqs, _ = W.amr_requests(args.served_requests, max_blocks=args.served_max_blocks,
                             side=args.served_side)
    sizes = np.array([r["cells"]["nh"].shape[0] for r in reqs])
    total = int(sizes.sum())
    log(f"[bench] served workload: {len(reqs)} requests, {total} cells, "
        f"blocks/request mean {sizes.mean() / 512:.1f} max {sizes.max() // 512}")
    bufs = [sfc.to_device(r["cells"]) for r in reqs]
    prist = [{k: b[k].clone() for k in STATE_KEYS} for b in bufs]

    def restore():
        for b, p in zip(bufs, prist):
            for k in STATE_KEYS:
                b[k].copy_(p[k])
        torch.cuda.synchronize()

    factor = 100.0
    out = dict(workload=f"{len(reqs)} requests of 8^3 blocks, blocks/request log-uniform in "
                        f"[1,{args.served_max_blocks}], levels 0..5 (dt = 10 kyr / 2^L), "
                        f"cells from the {args.served_side}^3 log-normal + 8 point-source "
                        f"population, dust factor 100",
               requests=len(reqs), cells=total)
    ctx = sfc.Context(dust_factor=factor, served_budget_bytes=args.served_budget_mib << 20)

    m = min(args.served_plain_requests, len(reqs))
    plain_cells = int(sizes[:m].sum())

    def plain(prec, label):
        # the plain path, one sfc_chem_step per request in arrival order, on
        # the first m requests (each call waits for its slowest cell)
        restore()
        t0 = time.perf_counter()
        for b, r in zip(bufs[:m], reqs[:m]):
            ctx.step(b, r["dt"], prec)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        log(f"[bench] served/{label}: {m} requests, {plain_cells} cells in {el:.3f} s")
        return el

    def served(prec, arrivals, label):
        restore()
        tickets = []
        t0 = sfc.now()
        for i, (b, r) in enumerate(zip(bufs, reqs)):
            if arrivals is not None:
                while sfc.now() - t0 < arrivals[i]:
                    time.sleep(50e-6)
            tickets.append(ctx.submit(b, r["dt"], prec, level=r["level"], tag=i, sync=False))
        ctx.drain()
        res = [ctx.poll(t) for t in tickets]
        t_first = min(x["t_submit"] for x in res)
        t_last = max(x["t_done"] for x in res)
        lat = np.array([x["t_done"] - x["t_submit"] for x in res])
        qd = np.array([x["t_admit"] - x["t_submit"] for x in res])
        log(f"[bench] served/{label}: makespan {t_last - t_first:.3f} s, latency p50 "
            f"{np.median(lat) * 1e3:.1f} ms p99 {pct(lat, 99) * 1e3:.1f} ms")
        return dict(value=total / (t_last - t_first), makespan_s=t_last - t_first,
                    latency_ms=dict(p50=pct(lat, 50) * 1e3, p99=pct(lat, 99) * 1e3,
                                    max=float(lat.max()) * 1e3),
                    admission_wait_ms=dict(p50=pct(qd, 50) * 1e3, p99=pct(qd, 99) * 1e3))

    def snapshot():
        torch.cuda.synchronize()
        return {k: torch.cat([b[k] for b in bufs]).cpu().numpy()
                for k in ("y_h2", "y_e", "y_h", "y_hp", "y_hm", "tgas", "tdust", "nsub")}

    # the plain path on the same cells at its best: every request of one
    # AMR level (one dt) concatenated into one array, one sfc_chem_step per
    # level, levels one after the other
    by_level = {}
    for b, r in zip(bufs, reqs):
        by_level.setdefault(r["level"], []).append((b, r["dt"]))
    batched = {L: ({k: torch.cat([b[k] for b, _ in lst]) for k in bufs[0]}, lst[0][1])
               for L, lst in sorted(by_level.items())}
    bprist = {L: {k: c[k].clone() for k in STATE_KEYS} for L, (c, _) in batched.items()}

    def plain_batched(prec, label):
        for L, (c, _) in batched.items():
            for k in STATE_KEYS:
                c[k].copy_(bprist[L][k])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for L, (c, dt_l) in batched.items():
            ctx.step(c, dt_l, prec)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ns = int(torch.cat([c["nsub"] for c, _ in batched.values()]).to(torch.int64).sum())
        log(f"[bench] served/{label}: {len(batched)} launches, {total} cells in {el:.3f} s")
        return dict(value=total / el, seconds=el, launches=len(batched),
                    roofline_frac=FLOP_PER_SUBCYCLE * ns / el / PEAK_FP64_VALU)

    el = plain(sfc.FP64, "plain fp64")
    out["plain_fp64"] = dict(value=plain_cells / el, seconds=el, requests=m, cells=plain_cells)
    el = plain(sfc.MIXED, "plain mixed")
    out["plain_mixed"] = dict(value=plain_cells / el, seconds=el, requests=m, cells=plain_cells)
    out["plain_fp64_by_level"] = plain_batched(sfc.FP64, "plain fp64, one launch per level")
    out["plain_mixed_by_level"] = plain_batched(sfc.MIXED, "plain mixed, one launch per level")
    # binary64 reference for the accuracy of the served mixed results
    sref = served(sfc.FP64, None, "served_fp64 reference")
    ref = snapshot()
    for prec, name in ((sfc.MIXED, "served_mixed"), (sfc.FP64, "served_fp64")):
        cap = sref if prec == sfc.FP64 else served(prec, None, f"{name} all queued")
        got = snapshot()
        if prec == sfc.MIXED:
            mixed_ref = got
        # algorithmic binary64-equivalent FLOP of the drained work over the
        # makespan, against the binary64 VALU peak
        cap["roofline_frac"] = (FLOP_PER_SUBCYCLE * float(got["nsub"].astype(np.int64).sum()) /
                                cap["makespan_s"] / PEAK_FP64_VALU)
        leg = dict(all_queued=cap)
        if prec == sfc.MIXED:
            leg["vs_fp64"] = {k: relerr(got[k], ref[k]) for k in got if k != "nsub"}
        rate = args.served_load * cap["value"] / sizes.mean()
        arr = W.poisson_arrivals(len(reqs), rate)
        leg["poisson"] = dict(load=args.served_load, rate_req_per_s=rate,
                              **served(prec, arr, f"{name} poisson load {args.served_load}"))
        out[name] = leg
    out["served_mixed_vs_plain_fp64_throughput"] = (out["served_mixed"]["all_queued"]["value"] /
                                                    out["plain_fp64"]["value"])
    out["served_mixed_vs_plain_fp64_by_level"] = (out["served_mixed"]["all_queued"]["value"] /
                                                  out["plain_fp64_by_level"]["value"])
    out["served_fp64_vs_plain_fp64_by_level"] = (out["served_fp64"]["all_queued"]["value"] /
                                                 out["plain_fp64_by_level"]["value"])
    ctx.close()
    # admission under a budget far below the workload's arena need: requests
    # wait for slots and memory while earlier ones drain
    if args.served_tight_budget_mib > 0:
        ctx = sfc.Context(dust_factor=factor,
                          served_budget_bytes=args.served_tight_budget_mib << 20)
        tight = served(sfc.MIXED, None,
                       f"served_mixed all queued, budget {args.served_tight_budget_mib} MiB")
        got = snapshot()
        tight["budget_mib"] = args.served_tight_budget_mib
        tight["arena_need_mib"] = total * 108 / 2 ** 20
        tight["bitwise_equal_to_8gib_budget"] = bool(all(
            np.array_equal(got[k].view(np.int64), mixed_ref[k].view(np.int64))
            for k in got if k != "nsub") and np.array_equal(got["nsub"], mixed_ref["nsub"]))
        out["served_mixed_tight_budget"] = tight
        ctx.close()
    return out


def hii_leg(args, sfc, W, torch):
    """LI (dust factors 1 to 1e4, C_d = 1e4 to 1e8) and the NR comparator on
    a static H II region stand-in (n_H = 100 cm^-3 around a 40 M_sun star,
    front at the Stromgren radius), dt = 100 yr: once as drawn (gas off its
    thermal and ionisation balance), once after 200 kyr of the chemistry
    alone at realistic C_d (gas near balance, as inside an H II region long
    after the front has passed).  The ageing is preparation, not timed."""
    cells, dt = W.hii_region(args.hii_cells)
    n = cells["nh"].shape[0]
    t = sfc.to_device(cells)
    fresh = {k: t[k].clone() for k in STATE_KEYS}
    ctx = sfc.Context(dust_factor=1.0)
    for _ in range(20):
        ctx.step(t, 10.0 * W.KYR, sfc.FP64)
    torch.cuda.synchronize()
    ctx.close()
    aged = {k: t[k].clone() for k in STATE_KEYS}
    out = dict(cells=n, dt_s=dt, workload="n_H = 100, S_EUV = 1.36e49 /s, R_st = 2.67 pc, 6 pc box, Z = 1")

    def timed(state, run):
        for k in STATE_KEYS:
            t[k].copy_(state[k])
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        run()
        e1.record()
        torch.cuda.synchronize()
        s = e0.elapsed_time(e1) * 1e-3
        ns = t["nsub"].cpu().numpy()
        fl = t["flags"].cpu().numpy().view(np.uint32)
        return dict(seconds=s, value=n / s, nsub_mean=float(ns.mean()), nsub_max=int(ns.max()),
                    tight_fraction=float(((fl & sfc.F_TIGHT) != 0).mean()),
                    niter_mean=float(t["niter"].cpu().numpy().mean()))

    for name, state in (("fresh", fresh), ("aged_200kyr", aged)):
        leg = {}
        for f in (1.0, 10.0, 100.0, 1000.0, 10000.0):
            c = sfc.Context(dust_factor=f)
            c.step(t, dt, sfc.FP64)  # allocation and warm-up
            leg[f"li_factor{f:g}"] = timed(state, lambda: c.step(t, dt, sfc.FP64))
            c.close()
        c = sfc.Context(dust_factor=1.0)
        c.step_nr(t, dt)
        leg["nr_factor1"] = timed(state, lambda: c.step_nr(t, dt))
        c.close()
        for k, v in leg.items():
            log(f"[bench] hii {name} {k}: {v['seconds'] * 1e3:.2f} ms, nsub {v['nsub_mean']:.2f}, "
                f"tight {v['tight_fraction']:.3f}, niter {v['niter_mean']:.2f}")
        out[name] = leg
    return out


def nr_leg(args, sfc, cells, dt, torch):
    """The paper's comparison: LI (dust factor 1 and 1000) against the fully
    implicit NR solver (realistic C_d) on the first nr_cells cells of the
    headline population, one binary64 launch each."""
    m = min(args.nr_cells, cells["nh"].shape[0])
    sub = {k: np.ascontiguousarray(v[:m]) for k, v in cells.items()}
    out = dict(cells=m, dt_s=dt)
    for name, factor, nr in (("li_factor1", 1.0, False), ("li_factor1000", 1000.0, False),
                             ("nr_factor1", 1.0, True)):
        ctx = sfc.Context(dust_factor=factor)
        t = sfc.to_device(sub)
        stream = torch.cuda.current_stream()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if nr:
            ctx.step_nr(t, dt)
        else:
            ctx.step(t, dt, sfc.FP64)
        e1.record(stream)
        torch.cuda.synchronize()
        s = e0.elapsed_time(e1) * 1e-3
        ctx.close()
        ns = t["nsub"].cpu().numpy().astype(np.int64)
        it = t["niter"].cpu().numpy().astype(np.int64)
        fl = t["flags"].cpu().numpy().view(np.uint32)
        out[name] = dict(value=m / s, seconds=s, nsub_mean=float(ns.mean()), nsub_max=int(ns.max()),
                         niter_mean=float(it.mean()),
                         nrfail_fraction=float(((fl & sfc.F_NRFAIL) != 0).mean()))
        log(f"[bench] {name}: {m} cells in {s:.3f} s")
    out["li_factor1_over_nr"] = out["li_factor1"]["value"] / out["nr_factor1"]["value"]
    out["li_factor1000_over_nr"] = out["li_factor1000"]["value"] / out["nr_factor1"]["value"]
    return out


def collapse_leg(sfc):
    """Free-fall collapse 1e2 -> 1e11 cm^-3 for Z = 1, 1e-2, 1e-4 (three
    cells per call, one call per 0.1 t_ff): LI at dust factors 1 and 1000
    and the NR comparator; wall time per track and how far the factor-1000
    and NR tracks stray from the factor-1 LI track."""
    from paper_2604_21438_amd import collapse as CO
    out = {}
    tracks = {}
    for name, factor, method in (("li_factor1", 1.0, "li"), ("li_factor1000", 1000.0, "li"),
                                 ("nr_factor1", 1.0, "nr")):
        ctx = sfc.Context(dust_factor=factor, params=sfc.default_params(ir_mode=sfc.IR_FIXED))
        t0 = time.perf_counter()
        tr = CO.run(CO.gpu_step(ctx, method), CO.initial_parcels())
        el = time.perf_counter() - t0
        ctx.close()
        tracks[name] = tr
        out[name] = dict(seconds=el, steps=int(tr["nh"].shape[0]), nsub_total=int(tr["nsub"].sum()))
        log(f"[bench] collapse {name}: {el:.2f} s")
    base = tracks["li_factor1"]
    for name in ("li_factor1000", "nr_factor1"):
        out[name]["max_rel_vs_li_factor1"] = {
            k: float((np.abs(tracks[name][k] - base[k]) / np.abs(base[k])).max())
            for k in ("tgas", "tdust", "y_h2")}
    return out


def gmc_leg(args, sfc, W, torch):
    """One coarse step of a GMC-like AMR hierarchy (levels 0..5, level L
    advanced 2^L times with dt = 10 kyr / 2^L, Z = 0.1, 64 point sources).
    Plain path: one call per level substep in Berger-Colella order.  Served
    form: every level submits its next substep as soon as its previous one
    is done (the same device buffers carry the state), so the levels overlap
    on the device; latency per request = done - submit."""
    levels = W.gmc_levels(target_cells=args.gmc_cells, progress=lambda m: log(f"[bench] {m}"))
    nl = len(levels)
    sizes = [lv["cells"]["nh"].shape[0] for lv in levels]
    updates = sum(m * 2 ** L for L, m in enumerate(sizes))
    log(f"[bench] gmc hierarchy: cells per level {sizes}, {updates} cell-updates per coarse step")
    bufs = [sfc.to_device(lv["cells"]) for lv in levels]
    prist = [{k: b[k].clone() for k in STATE_KEYS} for b in bufs]

    def restore():
        for b, p in zip(bufs, prist):
            for k in STATE_KEYS:
                b[k].copy_(p[k])
        torch.cuda.synchronize()

    def bc_order(L=0):
        o = [L]
        if L + 1 < nl:
            o += bc_order(L + 1) + bc_order(L + 1)
        return o

    order = bc_order()
    out = dict(cells_per_level=sizes, cell_updates_per_coarse_step=updates)
    factors = (1.0, 1000.0) if args.gmc_both_factors else (1.0,)
    if args.gmc_factor is not None:
        factors = (args.gmc_factor,)
    precs = ((sfc.FP64, "fp64"),) if args.gmc_no_mixed else ((sfc.FP64, "fp64"), (sfc.MIXED, "mixed"))
    for factor in factors:
        ctx = sfc.Context(dust_factor=factor, z_default=0.1,
                          served_budget_bytes=args.served_budget_mib << 20)
        legs = {}
        for prec, pname in precs:
            if prec == sfc.FP64 and not args.gmc_skip_plain:
                restore()
                t0 = time.perf_counter()
                for i, L in enumerate(order):
                    ctx.step(bufs[L], levels[L]["dt"], prec)
                    if args.gmc_cells >= 8_000_000:  # long legs report each level step
                        torch.cuda.synchronize()
                        log(f"[bench] gmc plain {pname}: step {i + 1}/{len(order)} (level {L}) "
                            f"done at {time.perf_counter() - t0:.1f} s")
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                legs[f"plain_{pname}"] = dict(value=updates / el, seconds=el)
                log(f"[bench] gmc factor {factor:g} {pname}: plain {el:.2f} s")
            if args.gmc_served in ("both", "copy"):
                legs.update(gmc_served_copy(ctx, bufs, levels, prec, pname, factor, restore,
                                            updates, verbose=args.gmc_cells >= 8_000_000))
            if args.gmc_served in ("both", "resident"):
                legs.update(gmc_served_resident(ctx, bufs, levels, prec, pname, factor, restore,
                                                updates, torch))
        ctx.close()
        out[f"dust_factor_{factor:g}"] = legs
    return out


def gmc_served_copy(ctx, bufs, levels, prec, pname, factor, restore, updates, verbose=False):
    """Served GMC step, every request copied in and out of the arena."""
    nl = len(levels)
    legs = {}
    restore()
    remaining = [2 ** L for L in range(nl)]
    inflight = [None] * nl
    lat = []
    t0 = time.perf_counter()
    while any(remaining) or any(t is not None for t in inflight):
        for L in range(nl):
            if inflight[L] is not None:
                r = ctx.poll(inflight[L])
                if r is not None:
                    lat.append(r["t_done"] - r["t_submit"])
                    inflight[L] = None
                    if verbose:
                        log(f"[bench] gmc served {pname}: level {L} substep done at "
                            f"{time.perf_counter() - t0:.1f} s")
            if inflight[L] is None and remaining[L] > 0:
                inflight[L] = ctx.submit(bufs[L], levels[L]["dt"], prec, level=L,
                                         sync=False)
                remaining[L] -= 1
        time.sleep(100e-6)
    el = time.perf_counter() - t0
    legs[f"served_{pname}"] = dict(value=updates / el, seconds=el,
                                   latency_ms=dict(p50=pct(lat, 50) * 1e3,
                                                   p99=pct(lat, 99) * 1e3,
                                                   max=float(np.max(lat)) * 1e3))
    log(f"[bench] gmc factor {factor:g} {pname}: served {el:.2f} s")
    return legs


def gmc_served_resident(ctx, bufs, levels, prec, pname, factor, restore, updates, torch):
    """The same with each level's state resident under a block key: the
    first substep uploads, the others continue in the arena (no copy-in, no
    copy-out); the results are fetched at the end."""
    nl = len(levels)
    legs = {}
    restore()
    remaining = [2 ** L for L in range(nl)]
    inflight = [None] * nl
    last = [None] * nl
    lat = []
    t0 = time.perf_counter()
    while any(remaining) or any(t is not None for t in inflight):
        for L in range(nl):
            if inflight[L] is not None:
                r = ctx.poll(inflight[L])
                if r is not None:
                    lat.append(r["t_done"] - r["t_submit"])
                    inflight[L] = None
            if inflight[L] is None and remaining[L] > 0:
                first = remaining[L] == 2 ** L
                inflight[L] = ctx.submit(bufs[L] if first else None, levels[L]["dt"],
                                         prec, level=L, sync=False,
                                         block_key=1 + L, resume=not first)
                last[L] = inflight[L]
                remaining[L] -= 1
        time.sleep(100e-6)
    for L in range(nl):
        ctx.fetch(last[L], bufs[L])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    for L in range(nl):
        ctx.release(1 + L)
    legs[f"served_{pname}_resident"] = dict(
        value=updates / el, seconds=el,
        latency_ms=dict(p50=pct(lat, 50) * 1e3, p99=pct(lat, 99) * 1e3,
                        max=float(np.max(lat)) * 1e3))
    log(f"[bench] gmc factor {factor:g} {pname}: served, resident blocks {el:.2f} s")
    return legs


def grid256_leg(args, sfc, W, torch):
    """The 256^3 population (log-normal n_H with an n^-1.5 tail, 8 point
    sources, Z = 1, dust factor 100, dt = 10 kyr): one binary64 and one mixed
    step over all cells, timed with events after a warm-up step, and the
    error of both against the CPU reference on a seeded sample of cells."""
    import oracle
    cells, dt = W.grid256(side=args.grid256_side)
    n = cells["nh"].shape[0]
    log(f"[bench] grid256: {n} cells")
    prist = sfc.to_device(cells, outputs=False)
    work = sfc.to_device(cells)
    out = dict(workload=f"{args.grid256_side}^3 log-normal density (mu = ln 100, sigma = 2) with "
                        "an n^-1.5 tail above 1e4, 8 point sources, Z = 1, dust factor 100, "
                        "dt = 10 kyr", cells=n, dt_s=dt)
    res = {}
    # progress dispatch (the default) and density dispatch, whose results are
    # bitwise the same: this population has few long cells (see DESIGN)
    for prec, name, disp in ((sfc.FP64, "fp64", None), (sfc.MIXED, "mixed", None),
                             (sfc.FP64, "fp64_density", sfc.DISPATCH_DENSITY),
                             (sfc.MIXED, "mixed_density", sfc.DISPATCH_DENSITY)):
        ctx = sfc.Context(dust_factor=100.0, params=sfc.default_params(dispatch=disp)
                          if disp is not None else None)
        times = []
        for rep in range(2):
            for k in STATE_KEYS:
                work[k].copy_(prist[k])
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            ctx.step(work, dt, prec)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) * 1e-3)
        ctx.close()
        o = {k: v.cpu().numpy() for k, v in work.items()}
        ns = o["nsub"].astype(np.int64)
        s = times[-1]
        out[name] = dict(value=n / s, seconds=s, nsub=stats(ns),
                         roofline_frac=FLOP_PER_SUBCYCLE * float(ns.sum()) / s / PEAK_FP64_VALU)
        if disp is None:
            res[name] = o
        else:
            base = res[name.split("_")[0]]
            out[name]["bitwise_same_as_progress"] = bool(all(
                np.array_equal(o[k].view(np.int64) if o[k].dtype == np.float64 else o[k],
                               base[k].view(np.int64) if base[k].dtype == np.float64 else base[k])
                for k in o))
        log(f"[bench] grid256 {name}: {s:.3f} s, {n / s:.3e} cell-updates/s")
    out["mixed_speedup_vs_fp64"] = out["fp64"]["seconds"] / out["mixed"]["seconds"]
    if not args.no_cpu:
        m = min(args.grid256_sample, n)
        sub, idx = W.subsample(cells, m, seed=77)
        threads = max(1, min(16, os.cpu_count() or 1))
        p = oracle.default_params(dust_cap=1e6)
        t0 = time.perf_counter()
        ref = oracle.li_step(sub, dt, params=p, nthreads=threads)
        log(f"[bench] grid256 reference on {m} cells: {time.perf_counter() - t0:.1f} s")
        for name in ("fp64", "mixed"):
            errs = {k: relerr(res[name][k][idx], ref[k]) for k in
                    ("y_h2", "y_e", "y_h", "y_hp", "y_hm", "tgas", "tdust")}
            w = np.zeros(m)
            for k in ("y_h2", "y_e", "y_h", "y_hp", "y_hm", "tgas", "tdust"):
                e = np.abs(res[name][k][idx] - ref[k]) / np.maximum(np.abs(ref[k]), 1e-20)
                w = np.maximum(w, np.nan_to_num(e, nan=np.inf))
            out[f"{name}_vs_reference"] = dict(
                sample=m, per_output=errs, cells_beyond_1e9=int((w > 1e-9).sum()),
                cells_beyond_1e4=int((w > 1e-4).sum()),
                nsub_mismatch=int((res[name]["nsub"][idx] != ref["nsub"]).sum()))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-collapse", action="store_true")
    ap.add_argument("--gmc-cells", type=int, default=1_000_000,
                    help="cells of the GMC-like hierarchy for the served leg (0 skips it)")
    ap.add_argument("--gmc-skip-plain", action="store_true",
                    help="GMC leg: served runs only (no plain per-level baseline)")
    ap.add_argument("--gmc-both-factors", action="store_true",
                    help="run the GMC leg at dust factor 1000 too")
    ap.add_argument("--gmc-factor", type=float, default=None,
                    help="run the GMC leg at this dust factor only")
    ap.add_argument("--gmc-served", choices=("both", "copy", "resident", "none"), default="both",
                    help="GMC leg: which served runs (copy in/out per request, resident "
                         "block keys, both, or none)")
    ap.add_argument("--gmc-no-mixed", action="store_true",
                    help="GMC leg: binary64 only")
    ap.add_argument("--hii-cells", type=int, default=262144,
                    help="cells of the H II region stand-in leg (0 skips it)")
    ap.add_argument("--nr-cells", type=int, default=262144,
                    help="cells of the LI-vs-NR comparison (0 skips it)")
    ap.add_argument("--served-requests", type=int, default=120)
    ap.add_argument("--served-plain-requests", type=int, default=40)
    ap.add_argument("--served-max-blocks", type=int, default=256)
    ap.add_argument("--served-side", type=int, default=128)
    ap.add_argument("--served-budget-mib", type=int, default=8192)
    ap.add_argument("--served-load", type=float, default=0.8)
    ap.add_argument("--served-tight-budget-mib", type=int, default=64,
                    help="second served budget that forces queueing (0 skips it)")
    ap.add_argument("--cpu-cells", type=int, default=32768)
    ap.add_argument("--grid256-side", type=int, default=256,
                    help="side of the log-normal / point-source grid leg (0 skips it)")
    ap.add_argument("--grid256-sample", type=int, default=65536,
                    help="cells of that leg checked against the CPU reference")
    ap.add_argument("--cells", type=int, default=None, help="fewer cells (testing only)")
    ap.add_argument("--ir", choices=("evolve", "fixed"), default="evolve",
                    help="IR mode of the headline step (fixed: the IR field held at the CMB's)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run three device-to-device copies of MIB MiB (a kernel of "
                         "known traffic, to scale the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the thermochemistry update runs on one GPU only; cells are "
              "independent and the update has no cross-GPU step, so --gpus must be 1",
              file=sys.stderr)
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
        log(f"[bench] {label}: {steps} steps in {t1 - t0:.3f} s, kernel {np.mean(kern):.3f} s/step")
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
    evolve = args.ir == "evolve"
    flop_sub = FLOP_PER_SUBCYCLE if evolve else FLOP_PER_SUBCYCLE_FIXED_IR
    ctx = sfc.Context(dust_factor=1.0,
                      params=sfc.default_params(ir_mode=sfc.IR_EVOLVE if evolve else sfc.IR_FIXED))
    step_s, kern_s, out64 = run(ctx, sfc.FP64, args.steps, args.warmup, "fp64 factor 1")
    ctx.close()
    d64 = describe(out64)
    flops = flop_sub * d64["subcycles"]
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
                        "dust factor 1 (C_d = 1e4 erg/g/K), " +
                        ("E_IR evolved (T_IR log-uniform in [T_CMB, T_d])" if evolve
                         else "IR field held at the CMB's (FIXED)"),
            "cells": n, "dt_s": dt, "dust_factor": 1.0, "precision": "fp64",
            "dispatch": "progress", "phase_nsub": int(sfc.default_params().phase_nsub),
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_FP64_VALU / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_VALU,
            "traffic": measured_traffic(n) if evolve else None,
            "traffic_unit": "bytes per step (both launches)",
            "algorithmic_bytes": n * (BYTES_PER_CELL if evolve else BYTES_PER_CELL - 16),
            "kernel": "li_step_kernel<double>",
            "launches_per_step": 2,
            "flop_per_subcycle": flop_sub,
            "subcycles_per_step": d64["subcycles"],
            "kernel_s_per_step": kern_s,
            "hbm_gbs_algorithmic": n * (BYTES_PER_CELL if evolve else BYTES_PER_CELL - 16) / kern_s / 1e9,
        },
        "stats_fp64": d64,
    }

    # ---- the same step with the IR field held at the CMB's (FIXED IR) ----
    if not args.no_sweep:
        c = sfc.Context(dust_factor=1.0, params=sfc.default_params(ir_mode=sfc.IR_FIXED))
        s, ks, o = run(c, sfc.FP64, 1, 0, "fp64 factor 1 fixed IR")
        c.close()
        dd = describe(o)
        result["fixed_ir"] = dict(value=n / s, kernel_s=ks, nsub=dd["nsub"],
                                  tight_fraction=dd["tight_fraction"],
                                  flop_per_subcycle=FLOP_PER_SUBCYCLE_FIXED_IR,
                                  roofline_frac=FLOP_PER_SUBCYCLE_FIXED_IR * dd["subcycles"] / ks /
                                  PEAK_FP64_VALU)

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
        result["mixed"] = dict(value=n / s, ms_per_step=s * 1e3, kernel_s_per_step=ks,
                               speedup_vs_fp64=step_s / s,
                               vs_fp64={k: relerr(outmx[k], out64[k])
                                        for k in ("y_h2", "y_e", "y_h", "y_hp", "y_hm", "tgas",
                                                  "tdust")},
                               stats=describe(outmx))

    # ---- LI against the Newton-Raphson comparator on the same cells ----
    if args.nr_cells > 0:
        result["li_vs_nr"] = nr_leg(args, sfc, cells, dt, torch)

    # ---- one-zone free-fall collapse (hydro-free analogue) ----
    if args.hii_cells > 0:
        result["hii_stand_in"] = hii_leg(args, sfc, W, torch)

    if not args.no_collapse:
        result["collapse"] = collapse_leg(sfc)

    # ---- 256^3 log-normal population, binary64 and mixed ----
    if args.grid256_side > 0:
        result["grid256"] = grid256_leg(args, sfc, W, torch)

    # ---- served form: AMR-shaped requests with Poisson arrivals ----
    if not args.no_served:
        result["served"] = served_leg(args, sfc, W, torch)

    # ---- served form: one coarse step of a GMC-like AMR hierarchy ----
    if args.gmc_cells > 0:
        result["served_gmc"] = gmc_leg(args, sfc, W, torch)

    # ---- CPU reference on a sample of the same cells ----
    if not args.no_cpu:
        import oracle
        m = min(args.cpu_cells, n)
        sub, idx = W.subsample(cells, m, seed=99)
        # the host's share of one GPU on the benchmark machines is 16 cores
        threads = max(1, min(16, os.cpu_count() or 1))
        log(f"[bench] cpu reference: {m} cells on {threads} threads")
        t0 = time.perf_counter()
        ref = oracle.li_step(sub, dt, nthreads=threads)
        el = time.perf_counter() - t0
        log(f"[bench] cpu reference done in {el:.1f} s")
        result["cpu_baseline"] = {"value": m / el, "unit": "cell-updates/s", "cores": threads,
                                  "kind": "oracle", "cpu_model": cpu_model(),
                                  "sample": f"{m} seeded cells of the same 128^3 population, "
                                            f"dt = 10 kyr, dust factor 1, binary64"}
        # one core over the whole 4096-cell population (dt = 1 kyr)
        small, dt1 = W.small_cells()
        t0 = time.perf_counter()
        oracle.li_step(small, dt1, nthreads=1)
        el1 = time.perf_counter() - t0
        result["cpu_single_core_4096_cells"] = {
            "value": small["nh"].shape[0] / el1, "unit": "cell-updates/s", "cores": 1,
            "seconds": el1, "workload": "16^3 = 4096 independent cells, dt = 1 kyr, dust factor 1"}
        log(f"[bench] cpu reference, one core, 4096 cells: {el1:.1f} s")
        par = {"fp64": {k: relerr(out64[k][idx], ref[k]) for k in
                        ("y_h2", "y_e", "y_h", "y_hp", "y_hm", "tgas", "tdust")}}
        par["fp64_nsub_mismatch"] = int((out64["nsub"][idx] != ref["nsub"]).sum())
        w64 = worst_rel(out64, ref, idx)
        par["fp64_cells_beyond_1e9"] = int((w64 > 1e-9).sum())
        if outmx is not None:
            par["mixed"] = {k: relerr(outmx[k][idx], ref[k]) for k in
                            ("y_h2", "y_e", "y_h", "y_hp", "y_hm", "tgas", "tdust")}
            par["mixed_cells_beyond_1e4"] = int((worst_rel(outmx, ref, idx) > 1e-4).sum())
        par["cells"] = m
        result["parity_on_cpu_sample"] = par

    print(json.dumps(result))


if __name__ == "__main__":
    main()
