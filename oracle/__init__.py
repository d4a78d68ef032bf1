"""CPU reference ("oracle") for the linearized-implicit thermochemistry of
SFUMATO# (arXiv 2604.21438) -- Python access through ctypes.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP implementation in ``paper_2604_21438_amd``.

The arithmetic lives in ``orc_chem.cpp`` (plain serial C++, binary64,
-ffp-contract=off).  ``build()`` compiles eight libraries next to this
file: ``liborc.so`` (the reference), ``liborc_count.so`` (counting build,
algorithmic operation count per cell-update), ``liborc_fma.so`` and
``liborc_dn.so`` (other valid roundings: contracted multiply-adds and
transcendentals nudged up / uncontracted and nudged down),
``liborc_rcp.so`` / ``liborc_rcpdn.so`` (every quotient formed as a
product with a reciprocal moved one ulp up, contracted / down,
uncontracted), ``liborc_all.so`` (all of these classes at once) and
``liborc_c32.so`` (exponentials and powers rounded to binary32) and
``liborc_j32.so`` (the Jacobian of the chemistry + energy solve rounded to
binary32).  The alternative builds only measure each cell's conditioning:
to binary64 rounding, and to coefficients and partials of binary32
accuracy.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liborc.so")
LIB_COUNT = os.path.join(HERE, "liborc_count.so")
# the same source with multiply-add contraction and every transcendental
# result moved by one ulp: a second, equally valid rounding of the same
# algorithm, used to measure how far rounding alone moves each cell
LIB_FMA = os.path.join(HERE, "liborc_fma.so")
# and a third: no contraction, transcendentals nudged down, powers formed
# as exp(y log x)
LIB_DN = os.path.join(HERE, "liborc_dn.so")
# and two more in the rounding class of division through a refined
# hardware reciprocal: a / b = a * rcp(b), the reciprocal one ulp up with
# contraction, or one ulp down without
LIB_RCP = os.path.join(HERE, "liborc_rcp.so")
LIB_RCPDN = os.path.join(HERE, "liborc_rcpdn.so")
# every class at once: contraction, transcendentals and reciprocals one ulp up
LIB_ALL = os.path.join(HERE, "liborc_all.so")
# exponentials and powers rounded to binary32, everything else binary64:
# the error floor of binary32 rate coefficients (mixed-precision bar)
LIB_C32 = os.path.join(HERE, "liborc_c32.so")
# the partial derivatives of the chemistry + energy system (its Jacobian)
# rounded to binary32 before the solve, everything else binary64: the
# rounding of the mixed path's binary32 partials (mixed-precision bar)
LIB_J32 = os.path.join(HERE, "liborc_j32.so")
# the subcycle's Lie split in the other order (Appendix C step first, then
# chemistry + energy at the updated state): a study of the split order, not
# another rounding
LIB_DF = os.path.join(HERE, "liborc_df.so")
SRC = os.path.join(HERE, "orc_chem.cpp")

NREAC, NPROC, NLINE = 12, 14, 5
IR_FIXED, IR_EVOLVE = 0, 1
THERMAL_EVOLVE, THERMAL_ISOTHERMAL = 0, 1
DUST_EVOLVE, DUST_FROZEN = 0, 1
F_CAP, F_TIGHT, F_NOCONV, F_INVALID, F_FLOOR, F_NRFAIL = 1, 2, 4, 8, 16, 32

CFLAGS = ["-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
          "-shared", "-Wall", "-pthread"]


def build(force: bool = True) -> None:
    """Compile the plain, counting and contracted oracle libraries (g++)."""
    variants = ((LIB, []), (LIB_COUNT, ["-DORC_COUNT"]),
                (LIB_FMA, ["-mfma", "-ffp-contract=fast", "-DORC_NUDGE"]),
                (LIB_DN, ["-DORC_NUDGE", "-DORC_NUDGE_DOWN"]),
                (LIB_RCP, ["-DORC_RCP", "-mfma", "-ffp-contract=fast"]),
                (LIB_RCPDN, ["-DORC_RCP", "-DORC_NUDGE_DOWN"]),
                (LIB_ALL, ["-DORC_RCP", "-DORC_NUDGE", "-mfma", "-ffp-contract=fast"]),
                (LIB_C32, ["-DORC_COEF32"]), (LIB_J32, ["-DORC_JAC32"]),
                (LIB_DF, ["-DORC_DUST_FIRST"]))
    for out, extra in variants:
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
            continue
        tmp = out + ".tmp"
        subprocess.check_call(["g++", *CFLAGS, *extra, "-o", tmp, SRC])
        os.replace(tmp, out)


class Network(C.Structure):
    _fields_ = [
        ("reac_mult", C.c_double * NREAC),
        ("proc_mult", C.c_double * NPROC),
        ("sigma_euv", C.c_double), ("k10_per_g0", C.c_double),
        ("g0_photon_density", C.c_double), ("zeta_cr", C.c_double),
        ("k4_pre", C.c_double), ("k4_theta", C.c_double),
        ("heat_euv_ev", C.c_double), ("heat_h2diss_ev", C.c_double),
        ("pe_coef", C.c_double), ("pe_eps", C.c_double),
        ("kappa_max", C.c_double), ("kappa_tnorm", C.c_double),
        ("kappa_uv", C.c_double), ("e_fuv_ev", C.c_double), ("e_euv_ev", C.c_double),
        ("x_c", C.c_double), ("x_o", C.c_double), ("f_oiii", C.c_double),
        ("line_tul", C.c_double * NLINE), ("line_a", C.c_double * NLINE),
        ("line_g", C.c_double * NLINE), ("line_qn", C.c_double * NLINE),
        ("line_qe100", C.c_double * NLINE),
        ("shield_len", C.c_double), ("shield_b5", C.c_double),
        ("pe_mode", C.c_int32), ("shield_mode", C.c_int32),
    ]


class Params(C.Structure):
    _fields_ = [
        ("f_chem", C.c_double), ("y_abs", C.c_double), ("newton_rtol", C.c_double),
        ("c_red", C.c_double), ("t_cmb", C.c_double), ("y_he", C.c_double),
        ("gamma_ad", C.c_double), ("dust_cap", C.c_double), ("z_default", C.c_double),
        ("n_cyc", C.c_int32), ("n_sub_max", C.c_int32), ("newton_max", C.c_int32),
        ("ir_mode", C.c_int32), ("thermal_mode", C.c_int32), ("dust_mode", C.c_int32),
        ("photon_absorb", C.c_int32), ("reserved", C.c_int32),
    ]


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_up = C.POINTER(C.c_uint32)


class Cells(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("y_h2", _dp), ("y_e", _dp), ("eint", _dp), ("tdust", _dp), ("eir", _dp),
        ("y_h", _dp), ("y_hp", _dp), ("y_hm", _dp), ("tgas", _dp),
        ("nh", _dp), ("n_euv", _dp), ("n_fuv", _dp), ("zmet", _dp),
        ("nsub", _ip), ("niter", _ip), ("flags", _up),
        ("n_euv_out", _dp), ("n_fuv_out", _dp),
    ]


_libs: dict = {}


def _lib(counting: bool = False, variant: str = "plain"):
    """The plain build, or a named rounding variant ("fma", "dn", "rcp",
    "rcpdn", "all", "c32", "j32"), or any other
    build of the same source given by its path (the pins' mutation test
    builds copies with planted mistakes)."""
    if variant.endswith(".so"):
        path = variant
    else:
        path = LIB_COUNT if counting else {"fma": LIB_FMA, "dn": LIB_DN, "rcp": LIB_RCP,
                                       "rcpdn": LIB_RCPDN, "all": LIB_ALL,
                                       "c32": LIB_C32, "j32": LIB_J32, "df": LIB_DF}.get(variant, LIB)
    if path not in _libs:
        if variant.endswith(".so"):
            if not os.path.exists(path):
                raise FileNotFoundError(path)
        elif not os.path.exists(path):
            build(force=False)
        lib = C.CDLL(path)
        P = C.POINTER
        lib.orc_network_default.argtypes = [P(Network)]
        lib.orc_params_default.argtypes = [P(Params)]
        for name in ("orc_li_step", "orc_nr_step"):
            f = getattr(lib, name)
            f.argtypes = [P(Network), P(Params), P(Cells), C.c_double, C.c_int]
            f.restype = C.c_int
        lib.orc_rk_reference.argtypes = [P(Network), P(Params), P(Cells), C.c_double, C.c_double]
        lib.orc_rk_reference.restype = C.c_int
        lib.orc_rate_coeffs.argtypes = [P(Network), P(Params)] + [C.c_double] * 6 + [_dp, _dp]
        lib.orc_chem_sources.argtypes = [P(Network), P(Params)] + [C.c_double] * 8 + [_dp, _dp, _dp]
        lib.orc_dust_system.argtypes = [P(Network), P(Params)] + [C.c_double] * 9 + [_dp, _dp, _dp]
        lib.orc_count_li_cell.argtypes = [P(Network), P(Params), P(Cells), C.c_int64, C.c_double, _dp]
        lib.orc_count_li_cell.restype = C.c_int
        _libs[path] = lib
    return _libs[path]


def default_network(**overrides) -> Network:
    net = Network()
    _lib().orc_network_default(C.byref(net))
    for k, v in overrides.items():
        _assign(net, k, v)
    return net


def default_params(**overrides) -> Params:
    p = Params()
    _lib().orc_params_default(C.byref(p))
    for k, v in overrides.items():
        _assign(p, k, v)
    return p


def _assign(obj, k, v):
    cur = getattr(obj, k)
    if isinstance(cur, C.Array):
        for i, x in enumerate(v):
            cur[i] = x
    else:
        setattr(obj, k, v)


STATE = ("y_h2", "y_e", "eint", "tdust", "eir")
INPUTS = ("nh", "n_euv", "n_fuv", "zmet")
OUT_F = ("y_h", "y_hp", "y_hm", "tgas")
PHOTON_OUT = ("n_euv_out", "n_fuv_out")


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


def _cells(arrs: dict, n: int):
    """Build the ctypes SoA view; returns (Cells, keepalive)."""
    keep = {}
    c = Cells()
    c.n = n
    for k in STATE + INPUTS + OUT_F + PHOTON_OUT:
        a = arrs.get(k)
        if a is not None:
            assert a.dtype == np.float64 and a.flags.c_contiguous and a.shape == (n,), k
        keep[k] = a
        setattr(c, k, _ptr(a, C.c_double))
    for k, ct in (("nsub", C.c_int32), ("niter", C.c_int32), ("flags", C.c_uint32)):
        a = arrs.get(k)
        keep[k] = a
        setattr(c, k, _ptr(a, ct))
    return c, keep


def _prepare(cells: dict, ir_mode: int, photon_absorb: int = 0):
    """Copy the inputs, allocate outputs; returns the dict the oracle writes."""
    n = int(np.asarray(cells["nh"]).shape[0])
    out = {}
    for k in STATE + INPUTS:
        if k in cells and cells[k] is not None:
            out[k] = np.ascontiguousarray(cells[k], dtype=np.float64).copy()
    if ir_mode != IR_EVOLVE:
        out.pop("eir", None)
    for k in OUT_F:
        out[k] = np.empty(n, np.float64)
    out["nsub"] = np.zeros(n, np.int32)
    out["niter"] = np.zeros(n, np.int32)
    out["flags"] = np.zeros(n, np.uint32)
    if photon_absorb:
        for k in PHOTON_OUT:
            out[k] = np.empty(n, np.float64)
    return out, n


def li_step(cells: dict, dt: float, net: Network | None = None, params: Params | None = None,
            nthreads: int = 1, variant: str = "plain") -> dict:
    """LI update of every cell over dt [s]; returns a new dict of arrays.
    variant names another rounding of the same arithmetic ("fma", "dn",
    "rcp", "rcpdn", "all", "c32", "j32"; see build)."""
    net = net or default_network()
    params = params or default_params()
    out, n = _prepare(cells, params.ir_mode, params.photon_absorb)
    c, keep = _cells(out, n)
    rc = _lib(variant=variant).orc_li_step(C.byref(net), C.byref(params), C.byref(c), float(dt),
                                            int(nthreads))
    if rc != 0:
        raise ValueError("orc_li_step rejected its arguments")
    return out


def nr_step(cells: dict, dt: float, net: Network | None = None, params: Params | None = None,
            nthreads: int = 1, variant: str = "plain") -> dict:
    """Newton-Raphson comparator over dt [s]; same variants as li_step."""
    net = net or default_network()
    params = params or default_params()
    out, n = _prepare(cells, params.ir_mode, params.photon_absorb)
    c, keep = _cells(out, n)
    rc = _lib(variant=variant).orc_nr_step(C.byref(net), C.byref(params), C.byref(c), float(dt),
                                            int(nthreads))
    if rc != 0:
        raise ValueError("orc_nr_step rejected its arguments")
    return out


def rk_reference(cells: dict, dt: float, net: Network | None = None,
                 params: Params | None = None, step_frac: float = 1e-3) -> dict:
    net = net or default_network()
    params = params or default_params()
    out, n = _prepare(cells, params.ir_mode, params.photon_absorb)
    c, keep = _cells(out, n)
    rc = _lib().orc_rk_reference(C.byref(net), C.byref(params), C.byref(c), float(dt),
                                 float(step_frac))
    if rc != 0:
        raise ValueError("orc_rk_reference rejected its arguments")
    return out


def rate_coeffs(T, tdust, nh=1.0, fd=1.0, n_euv=0.0, n_fuv=0.0, net=None, params=None):
    """(k[12], dk/dT[12]) at one temperature."""
    net = net or default_network()
    params = params or default_params()
    k = np.zeros(NREAC)
    dk = np.zeros(NREAC)
    _lib().orc_rate_coeffs(C.byref(net), C.byref(params), T, tdust, nh, fd, n_euv, n_fuv,
                           _ptr(k, C.c_double), _ptr(dk, C.c_double))
    return k, dk


def chem_sources(y_h2, y_e, T, tdust, nh, fd=1.0, n_euv=0.0, n_fuv=0.0, net=None, params=None):
    """((R_H2, R_e, Q), jac[3x3] w.r.t. (y_H2, y_e, T), terms[14])."""
    net = net or default_network()
    params = params or default_params()
    out = np.zeros(3)
    jac = np.zeros(9)
    terms = np.zeros(NPROC)
    _lib().orc_chem_sources(C.byref(net), C.byref(params), y_h2, y_e, T, tdust, nh, fd, n_euv,
                            n_fuv, _ptr(out, C.c_double), _ptr(jac, C.c_double),
                            _ptr(terms, C.c_double))
    return out, jac.reshape(3, 3), terms


def dust_system(tg, tdust, eir, nh, fd, ntot, n_euv, n_fuv, h, net=None, params=None):
    """Appendix C matrix (3x3 over dT_d, dE_IR, dT_g), rhs, (S_d, S_IR, S_g, alpha_g)."""
    net = net or default_network()
    params = params or default_params()
    A = np.zeros(9)
    rhs = np.zeros(3)
    src = np.zeros(4)
    _lib().orc_dust_system(C.byref(net), C.byref(params), tg, tdust, eir, nh, fd, ntot, n_euv,
                           n_fuv, h, _ptr(A, C.c_double), _ptr(rhs, C.c_double),
                           _ptr(src, C.c_double))
    return A.reshape(3, 3), rhs, src


def count_li(cells: dict, dt: float, idx, net=None, params=None) -> np.ndarray:
    """Operation counts (add, mul, div, sqrt, transcendental, cmp) of the LI
    update for each cell index in idx, from the counting build."""
    net = net or default_network()
    params = params or default_params()
    lib = _lib(counting=True)
    out, n = _prepare(cells, params.ir_mode, params.photon_absorb)
    c, keep = _cells(out, n)
    res = np.zeros((len(idx), 6))
    buf = np.zeros(6)
    for j, i in enumerate(idx):
        # the counting build writes its results into the arrays of `out`;
        # each cell is counted from its original input state
        rc = lib.orc_count_li_cell(C.byref(net), C.byref(params), C.byref(c), int(i), float(dt),
                                   _ptr(buf, C.c_double))
        if rc != 0:
            raise RuntimeError("counting build not available")
        res[j] = buf
    return res


OUT_KEYS = ("y_h2", "y_e", "y_h", "y_hp", "y_hm", "tgas", "tdust")


def _rel(a, b, floor=1e-20):
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


def rounding_spread(cells: dict, dt: float, ref: dict, net=None, params=None,
                    nthreads: int = 1, method: str = "li") -> np.ndarray:
    """Per cell, the largest relative change of any output between the
    reference result `ref` and seven (nine with E_IR evolved) other valid roundings of the same
    computation: the contracted build with transcendentals nudged up; the
    uncontracted build with them nudged down and powers formed as
    exp(y log x); quotients formed through a reciprocal moved one ulp up
    (contracted) or down (uncontracted); all of the first kinds at once
    (contracted, transcendentals and reciprocals one ulp up); and the input
    internal energy moved by one unit in the last place either way, and so
    the IR energy density when it evolves (the two energies of the state
    that enter temperatures through a root or a ratio).  A cell whose spread
    exceeds a tolerance is not determined to that tolerance by binary64
    arithmetic.  Cells that the reference marks invalid (NaN outputs) have
    spread 0 here; comparisons treat them separately."""
    params = params or default_params()
    step = li_step if method == "li" else nr_step
    alt = [step(cells, dt, net, params, nthreads, variant=v)
           for v in ("fma", "dn", "rcp", "rcpdn", "all")]
    energies = ["eint"] + (["eir"] if params.ir_mode == IR_EVOLVE and "eir" in cells else [])
    for key in energies:
        for direction in (np.inf, -np.inf):
            nudged = dict(cells)
            nudged[key] = np.nextafter(np.asarray(cells[key], np.float64), direction)
            alt.append(step(nudged, dt, net, params, nthreads))
    spread = np.zeros(ref["nsub"].shape[0])
    invalid = (np.asarray(ref["flags"]) & F_INVALID) != 0
    for o in alt:
        for k in OUT_KEYS:
            spread = np.maximum(spread, np.where(invalid, 0.0, _rel(o[k], ref[k])))
    return spread


def step_sensitivity(cells: dict, dt: float, ref: dict, net=None, params=None,
                     nthreads: int = 1, eps: float = 1e-6) -> np.ndarray:
    """Per cell, the largest relative output change when every subcycle is
    made larger by the factor (1 + eps) (f_chem scaled): how strongly the
    result depends on the step-size sequence."""
    params = params or default_params()
    p2 = Params.from_buffer_copy(params)
    p2.f_chem = params.f_chem * (1.0 + eps)
    o = li_step(cells, dt, net, p2, nthreads)
    s = np.zeros(ref["nsub"].shape[0])
    invalid = (np.asarray(ref["flags"]) & F_INVALID) != 0
    for k in OUT_KEYS:
        s = np.maximum(s, np.where(invalid, 0.0, _rel(o[k], ref[k])))
    return s


def coefficient_sensitivity(cells: dict, dt: float, ref: dict, net=None, params=None,
                            nthreads: int = 1) -> np.ndarray:
    """Per cell, the largest relative output change when every exponential
    and power of the reference (its rate, cooling and opacity coefficients)
    is rounded to binary32: how far coefficients of binary32 accuracy alone
    move the result.  Invalid cells get 0."""
    params = params or default_params()
    o = li_step(cells, dt, net, params, nthreads, variant="c32")
    s = np.zeros(ref["nsub"].shape[0])
    invalid = (np.asarray(ref["flags"]) & F_INVALID) != 0
    for k in OUT_KEYS:
        s = np.maximum(s, np.where(invalid, 0.0, _rel(o[k], ref[k])))
    return s


def jacobian_sensitivity(cells: dict, dt: float, ref: dict, net=None, params=None,
                         nthreads: int = 1) -> np.ndarray:
    """Per cell, the largest relative output change when the Jacobian of
    every chemistry + energy solve is rounded to binary32 (the sources and
    the solve stay binary64): how far partials of binary32 accuracy alone
    move the result, which a near-singular I - h J amplifies.  Invalid
    cells get 0."""
    params = params or default_params()
    o = li_step(cells, dt, net, params, nthreads, variant="j32")
    s = np.zeros(ref["nsub"].shape[0])
    invalid = (np.asarray(ref["flags"]) & F_INVALID) != 0
    for k in OUT_KEYS:
        s = np.maximum(s, np.where(invalid, 0.0, _rel(o[k], ref[k])))
    return s
