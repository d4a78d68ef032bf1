"""The kernels' hand-written binary64 math against references of 60
significant digits: e^x, ln x, 1/x and sqrt x each within one unit in the
last place (ulp of the correctly rounded result) over their working
ranges, with exact special values (e^0 = 1, ln 1 = 0, 1/1 = 1, sqrt 1 = 1,
sqrt of an exact square).  The functions are those that the LI, NR and
served kernels inline; tests/math_probe.hip runs them over an array."""
import ctypes as C
import math
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
PROBE = os.path.join(HERE, "libmathprobe.so")


def _probe(fn, x):
    import torch
    import paper_2604_21438_amd  # noqa: F401  (torch's HIP runtime first)
    assert os.path.exists(PROBE), "tests/libmathprobe.so missing: run the package build"
    lib = C.CDLL(PROBE)
    lib.sfk_math_probe.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_void_p]
    lib.sfk_math_probe.restype = C.c_int
    xd = torch.tensor(np.asarray(x, np.float64), device="cuda")
    out = torch.empty_like(xd)
    s = torch.cuda.current_stream()
    rc = lib.sfk_math_probe(xd.data_ptr(), out.data_ptr(), xd.numel(), fn, C.c_void_p(s.cuda_stream))
    assert rc == 0, rc
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _ulp_errors(got, x, exact):
    getcontext().prec = 60
    errs = np.empty(len(x))
    for i, (g, v) in enumerate(zip(got, x)):
        e = exact(Decimal(float(v)))
        errs[i] = float(abs(Decimal(float(g)) - e) / Decimal(math.ulp(float(e))))
    return errs


def _check(name, fn, x, exact, bound=1.0):
    print(f"[gpu math] {name}: {len(x)} arguments", flush=True)
    got = _probe(fn, x)
    errs = _ulp_errors(got, x, exact)
    print(f"[gpu math] {name}: max {errs.max():.3f} ulp, mean {errs.mean():.3f}", flush=True)
    assert np.all(np.isfinite(got))
    assert errs.max() <= bound, (name, x[np.argmax(errs)], errs.max())


def test_exp_within_one_ulp():
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.uniform(-700.0, 700.0, 6000), rng.uniform(-1.0, 1.0, 3000),
                        rng.uniform(-1e-3, 1e-3, 1000),
                        # near the table nodes (j ln2 / 512) and the reduction's halfway points
                        np.arange(-2000, 2000) * (math.log(2) / 1024.0)])
    _check("exp", 0, x, lambda d: d.exp())
    assert _probe(0, [0.0])[0] == 1.0
    big = _probe(0, [-800.0, 800.0])
    assert big[0] == 0.0 and np.isinf(big[1])


def test_log_within_one_ulp():
    rng = np.random.default_rng(12)
    x = np.concatenate([10.0 ** rng.uniform(-300, 300, 6000), rng.uniform(0.5, 2.0, 3000),
                        1.0 + rng.uniform(-1e-6, 1e-6, 1000)])
    x = x[x != 1.0]
    _check("log", 1, x, lambda d: d.ln())
    assert _probe(1, [1.0])[0] == 0.0


def test_reciprocal_and_root_within_one_ulp():
    rng = np.random.default_rng(13)
    x = 10.0 ** rng.uniform(-300, 300, 8000)
    _check("rcp", 2, x, lambda d: 1 / d)
    _check("sqrt", 3, x, lambda d: d.sqrt())
    sq = np.array([1.0, 4.0, 9.0, 2.25, 1e10, 6.25e-4])
    assert np.array_equal(_probe(3, sq), np.sqrt(sq))
    assert _probe(2, [1.0])[0] == 1.0
