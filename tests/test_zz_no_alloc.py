"""sfc_chem_step_noalloc (the plain step with its dispatch buffers in the
library's static device array) through the C ABI, against sfc_chem_step on
the same inputs: bitwise equal on two calls in a row, the second with fewer
cells (the array keeps the first call's contents), in both precisions, and
sizes beyond the array rejected."""
import ctypes as C

import numpy as np
import pytest

from paper_2604_21438_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("y_h2", "y_e", "eint", "tdust", "y_h", "y_hp", "y_hm", "tgas", "nsub", "niter", "flags")


def _same(a, b, label):
    for k in KEYS:
        x, y = a[k].cpu().numpy(), b[k].cpu().numpy()
        same = (x.view(np.int64) == y.view(np.int64)) if x.dtype.kind == "f" else (x == y)
        assert same.all(), (label, k, int((~same).sum()))


def test_noalloc_matches_step_twice_second_smaller():
    import torch
    import paper_2604_21438_amd as sfc
    cells, dt = W.grid128(n=300_000)
    small = {k: np.ascontiguousarray(v[:70_001]) for k, v in cells.items()}
    for prec in (sfc.FP64, sfc.MIXED):
        ctx = sfc.Context(dust_factor=1.0)
        try:
            for label, c in (("300000 cells", cells), ("70001 cells", small)):
                print(f"[noalloc] precision {prec}, {label}", flush=True)
                a = sfc.to_device(c)
                b = sfc.to_device(c)
                torch.cuda.synchronize()
                ctx.step(a, dt, prec)
                ctx.step_noalloc(b, dt, prec)
                torch.cuda.synchronize()
                assert torch.all(b["nsub"] > 0)
                _same(a, b, f"precision {prec}, {label}")
        finally:
            ctx.close()


def test_noalloc_rejects_more_cells_than_the_array_holds():
    import paper_2604_21438_amd as sfc
    ctx = sfc.Context()
    try:
        c = sfc.SfcCells()
        c.n = sfc.NOALLOC_MAX_CELLS + 1
        rc = sfc.lib().sfc_chem_step_noalloc(ctx._h, C.byref(c), 1e10, sfc.FP64, None)
        assert rc == sfc.E_INVAL
        assert b"at most" in sfc.lib().sfc_last_error(ctx._h)
    finally:
        ctx.close()
