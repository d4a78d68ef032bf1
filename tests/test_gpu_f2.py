"""The pieces beside the solver on the GPU, against the CPU reference: H2
self-shielding (shield_mode 1), photoelectric heating with grain charging
and recombination cooling (pe_mode 1), and the absorption of EUV/FUV
photons over the step (photon_absorb 1), each on the binary64 bar of the
plain step; the mixed path with all of them on stays finite and conserves
H nuclei and charge."""
import numpy as np
import pytest

import oracle
from parity_util import (EXEMPT_SPREAD, FP64_TOL, SPREAD_FACTOR, check_fp64_bar, host_threads,
                         oracle_net_params, rel)
from paper_2604_21438_amd import workloads as W

pytestmark = pytest.mark.gpu


def _run(cells, dt, prec, net, par, factor=1.0, photons=False, label=""):
    import torch
    import paper_2604_21438_amd as sfc
    print(f"[gpu f2] {label}: n={cells['nh'].shape[0]} prec={prec}", flush=True)
    ctx = sfc.Context(network=net, dust_factor=factor, params=par)
    try:
        t = sfc.to_device(cells, photons=photons)
        ctx.step(t, dt, prec)
        torch.cuda.synchronize()
        out = {k: v.cpu().numpy() for k, v in t.items()}
    finally:
        ctx.close()
    out["flags"] = out["flags"].view(np.uint32)
    return out


def _population(n, seed):
    """4096-cell population cells with FUV fields raised so that both
    stand-ins matter (G0 ~ 0.3 - 3e3)."""
    cells, dt = W.small_cells()
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(cells["nh"].shape[0], n, replace=False))
    sub = {k: np.ascontiguousarray(v[idx]) for k, v in cells.items()}
    sub["n_fuv"] = 3.7e-3 * 10.0 ** rng.uniform(-0.5, 3.5, n)
    return sub, dt


@pytest.mark.parametrize("modes", [dict(shield_mode=1), dict(pe_mode=1),
                                   dict(shield_mode=1, pe_mode=1)])
def test_fp64_with_shielding_and_photoelectric(modes):
    import paper_2604_21438_amd as sfc
    cells, dt = _population(1024, 3)
    net = sfc.default_network(**modes)
    par = sfc.default_params()
    gpu = _run(cells, dt, sfc.FP64, net, par, label=str(modes))
    onet, opar = oracle_net_params(net, par, 1.0)
    ref = oracle.li_step(cells, dt, onet, opar, host_threads())
    spread = oracle.rounding_spread(cells, dt, ref, onet, opar, host_threads())
    check_fp64_bar(gpu, ref, spread, f"f2 {modes}", cells)


def test_fp64_photon_absorption():
    """Photon densities after the step on the binary64 bar, the condition
    number of N exp(-tau) being tau: a cell is held to max(1, tau) times
    the bar of its other outputs; invalid cells keep their photons."""
    import paper_2604_21438_amd as sfc
    cells, dt = _population(1024, 5)
    cells["nh"][7] = -1.0
    net = sfc.default_network(shield_mode=1, pe_mode=1)
    par = sfc.default_params(photon_absorb=1)
    gpu = _run(cells, dt, sfc.FP64, net, par, photons=True, label="photon absorption")
    onet, opar = oracle_net_params(net, par, 1.0)
    ref = oracle.li_step(cells, dt, onet, opar, host_threads())
    spread = oracle.rounding_spread(cells, dt, ref, onet, opar, host_threads())
    check_fp64_bar(gpu, ref, spread, "photon absorption", cells)
    assert gpu["n_euv_out"][7] == cells["n_euv"][7] and gpu["n_fuv_out"][7] == cells["n_fuv"][7]
    for k, src in (("n_euv_out", "n_euv"), ("n_fuv_out", "n_fuv")):
        r = ref[k]
        tau = np.log(np.maximum(cells[src], 1e-300) / np.maximum(r, 1e-300))
        tau = np.where(r > 0, tau, 0.0)
        both_zero = (gpu[k] == 0) & (r == 0)
        e = np.where(both_zero, 0.0, rel(gpu[k], r, floor=1e-300))
        tol = np.maximum(FP64_TOL, np.where(spread <= EXEMPT_SPREAD, FP64_TOL,
                                            SPREAD_FACTOR * spread)) * np.maximum(1.0, tau)
        bad = np.nonzero(e > tol)[0]
        print(f"[gpu f2] {k}: max err {e.max():.2e}, max tau {tau.max():.1f}, "
              f"absorbed to zero: {int(both_zero.sum())}", flush=True)
        assert bad.size == 0, (k, bad[:5], e[bad[:5]], tol[bad[:5]])
        assert np.all(gpu[k] >= 0) and np.all(gpu[k] <= cells[src])


def test_nr_with_shielding_and_photoelectric():
    """The NR comparator shares the source assembly: same substeps and
    outer iterations as the reference NR, 1e-9 where determined."""
    import torch
    import paper_2604_21438_amd as sfc
    cells, dt = _population(256, 7)
    net = sfc.default_network(shield_mode=1, pe_mode=1)
    par = sfc.default_params()
    ctx = sfc.Context(network=net, params=par)
    try:
        t = sfc.to_device(cells)
        ctx.step_nr(t, dt)
        torch.cuda.synchronize()
        gpu = {k: v.cpu().numpy() for k, v in t.items()}
    finally:
        ctx.close()
    onet, opar = oracle_net_params(net, par, 1.0)
    ref = oracle.nr_step(cells, dt, onet, opar, host_threads())
    spread = oracle.rounding_spread(cells, dt, ref, onet, opar, host_threads(), method="nr")
    same = (gpu["nsub"] == ref["nsub"]) & (gpu["niter"] == ref["niter"])
    w = np.zeros(len(same))
    for k in ("y_h2", "y_e", "y_h", "y_hp", "y_hm", "tgas", "tdust"):
        w = np.maximum(w, rel(gpu[k], ref[k]))
    det = same & (spread <= EXEMPT_SPREAD)
    print(f"[gpu f2] NR: same path {int(same.sum())}/{len(same)}, determined {int(det.sum())}, "
          f"max err there {w[det].max() if det.any() else 0:.2e}", flush=True)
    assert det.any() and w[det].max() <= FP64_TOL
    tol = np.where(same, np.maximum(FP64_TOL, SPREAD_FACTOR * spread), 1e-3)
    assert np.all(w <= tol), np.nonzero(w > tol)[0][:5]


def test_mixed_with_every_piece_on():
    import paper_2604_21438_amd as sfc
    cells, dt = _population(2048, 9)
    net = sfc.default_network(shield_mode=1, pe_mode=1)
    par = sfc.default_params(photon_absorb=1)
    gpu = _run(cells, dt, sfc.MIXED, net, par, photons=True, label="mixed, all pieces")
    for k in ("y_h2", "y_e", "y_h", "y_hp", "y_hm", "tgas", "tdust", "eint", "n_euv_out",
              "n_fuv_out"):
        assert np.all(np.isfinite(gpu[k])), k
    s = gpu["y_h"] + 2 * gpu["y_h2"] + gpu["y_hp"] + gpu["y_hm"]
    assert np.all(np.abs(s - 1) <= 8 * np.finfo(float).eps)
    onet, opar = oracle_net_params(net, par, 1.0)
    ref = oracle.li_step(cells, dt, onet, opar, host_threads())
    w = np.zeros(cells["nh"].shape[0])
    for k in ("y_h2", "y_e", "tgas", "tdust"):
        w = np.maximum(w, rel(gpu[k], ref[k]))
    print(f"[gpu f2] mixed: median {np.median(w):.2e} p99 {np.percentile(w, 99):.2e} "
          f"max {w.max():.2e}", flush=True)
    assert np.median(w) <= 1e-6


def test_served_photon_absorption_matches_plain():
    """The served form applies the same absorption at the store: for each
    request the photon densities after the step (and every other output)
    are bitwise the plain step's, in both precisions, and a second context
    without photon_absorb leaves the output buffers untouched."""
    import torch
    import paper_2604_21438_amd as sfc
    net = sfc.default_network(shield_mode=1, pe_mode=1)
    par = sfc.default_params(photon_absorb=1)
    reqs = []
    for j, (n, dt) in enumerate(((700, 3.15576e11), (333, 3.15576e11 / 4), (1024, 3.15576e10))):
        cells, _ = _population(n, 20 + j)
        cells["nh"][j] = -1.0  # an invalid cell keeps its photons
        reqs.append((cells, dt))
    keys = ("y_h2", "y_e", "eint", "tdust", "eir", "y_h", "y_hp", "y_hm", "tgas", "nsub",
            "niter", "flags", "n_euv_out", "n_fuv_out")
    ctx = sfc.Context(network=net, params=par, served_budget_bytes=32 << 20)
    try:
        for prec in (sfc.FP64, sfc.MIXED):
            print(f"[gpu f2] served photon absorption prec={prec}: {len(reqs)} requests", flush=True)
            bufs = [sfc.to_device(c, photons=True) for c, _ in reqs]
            torch.cuda.synchronize()
            tickets = [ctx.submit(b, dt, prec, level=i, tag=i)
                       for i, (b, (_, dt)) in enumerate(zip(bufs, reqs))]
            ctx.drain()
            for tk in tickets:
                assert ctx.poll(tk)["status"] == 0
            for i, (b, (c, dt)) in enumerate(zip(bufs, reqs)):
                t = sfc.to_device(c, photons=True)
                ctx.step(t, dt, prec)
                torch.cuda.synchronize()
                for k in keys:
                    x, y = b[k].cpu().numpy(), t[k].cpu().numpy()
                    same = x.view(np.int64) == y.view(np.int64) if x.dtype.kind == "f" else x == y
                    assert same.all(), (prec, i, k, int((~same).sum()))
                out = b["n_euv_out"].cpu().numpy()
                assert out[i] == c["n_euv"][i] and np.all(out <= c["n_euv"])
                assert np.any(out < c["n_euv"])
    finally:
        ctx.close()
    # without photon_absorb the served form does not touch the photon outputs
    ctx = sfc.Context(network=net, params=sfc.default_params(), served_budget_bytes=32 << 20)
    try:
        c, dt = reqs[0]
        b = sfc.to_device(c, photons=True)
        b["n_euv_out"].fill_(-7.0)
        torch.cuda.synchronize()
        tk = ctx.submit(b, dt, sfc.FP64, level=0, tag=0)
        ctx.drain()
        assert ctx.poll(tk)["status"] == 0
        assert np.all(b["n_euv_out"].cpu().numpy() == -7.0)
    finally:
        ctx.close()
