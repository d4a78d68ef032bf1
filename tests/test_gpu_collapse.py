"""One-zone free-fall collapse driven by the library (LI plain path and NR
comparator) against the same driver on the CPU reference: the whole track
(208 steps, 1e2 -> 1e11 cm^-3, three metallicities) agrees step by step."""
import numpy as np
import pytest

import oracle
from parity_util import oracle_net_params
from paper_2604_21438_amd import collapse as CO

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("method,factor", [("li", 1.0), ("li", 1000.0), ("nr", 1.0)])
def test_collapse_track_matches_reference(method, factor):
    import paper_2604_21438_amd as sfc
    print(f"[gpu collapse] {method} factor {factor}", flush=True)
    par = sfc.default_params(ir_mode=sfc.IR_FIXED)  # optically thin parcel
    ctx = sfc.Context(dust_factor=factor, params=par)
    try:
        gpu = CO.run(CO.gpu_step(ctx, method), CO.initial_parcels())
    finally:
        ctx.close()
    onet, opar = oracle_net_params(sfc.default_network(), par, factor)
    f = oracle.nr_step if method == "nr" else oracle.li_step
    ref = CO.run(lambda c, dt: f(c, dt, onet, opar, 4), CO.initial_parcels())
    assert gpu["nh"].shape == ref["nh"].shape
    worst = 0.0
    for k in ("tgas", "tdust", "y_h2", "y_e"):
        r = np.abs(gpu[k] - ref[k]) / np.maximum(np.abs(ref[k]), 1e-20)
        worst = max(worst, float(r.max()))
    print(f"[collapse] {method} factor {factor}: {gpu['nh'].shape[0]} steps, max rel diff {worst:.2e}, "
          f"nsub gpu {int(gpu['nsub'].sum())} ref {int(ref['nsub'].sum())}", flush=True)
    assert worst <= 1e-6
