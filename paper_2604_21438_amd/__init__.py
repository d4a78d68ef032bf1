"""MI355X (gfx950) linearized-implicit thermochemistry of SFUMATO#
(arXiv 2604.21438): Python binding of libsfchem.so.

The binding only marshals arguments: every step of the update runs in the
HIP kernels of the library, PyTorch provides device memory and streams.
Names follow the C ABI in include/sfchem.h.  There is no CPU fallback: if
the library is not built, loading it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsfchem.so")

FP64, MIXED = 0, 1
DISPATCH_INDEX, DISPATCH_DENSITY, DISPATCH_PROGRESS = 0, 1, 2
IR_FIXED, IR_EVOLVE = 0, 1
THERMAL_EVOLVE, THERMAL_ISOTHERMAL = 0, 1
DUST_EVOLVE, DUST_FROZEN = 0, 1
F_CAP, F_TIGHT, F_NOCONV, F_INVALID, F_FLOOR, F_NRFAIL = 1, 2, 4, 8, 16, 32
OK, E_INVAL, E_NOMEM, E_BUDGET, E_DEVICE, E_PENDING, E_VERSION, E_STATE = 0, -1, -2, -3, -4, -5, -6, -7
ABI_VERSION = 4
NOALLOC_MAX_CELLS = 2097152
REQ_RESUME, REQ_WRITEBACK = 1, 2
NREAC, NPROC, NLINE = 12, 14, 5

_d = C.c_double


class SfcNetwork(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("size", C.c_uint32),
        ("reac_mult", _d * NREAC), ("proc_mult", _d * NPROC),
        ("sigma_euv", _d), ("k10_per_g0", _d), ("g0_photon_density", _d), ("zeta_cr", _d),
        ("k4_pre", _d), ("k4_theta", _d), ("heat_euv_ev", _d), ("heat_h2diss_ev", _d),
        ("pe_coef", _d), ("pe_eps", _d), ("kappa_max", _d), ("kappa_tnorm", _d),
        ("kappa_uv", _d), ("e_fuv_ev", _d), ("e_euv_ev", _d),
        ("x_c", _d), ("x_o", _d), ("f_oiii", _d),
        ("line_tul", _d * NLINE), ("line_a", _d * NLINE), ("line_g", _d * NLINE),
        ("line_qn", _d * NLINE), ("line_qe100", _d * NLINE),
        ("shield_len", _d), ("shield_b5", _d), ("pe_mode", C.c_int32),
        ("shield_mode", C.c_int32),
    ]


class SfcParams(C.Structure):
    _fields_ = [
        ("f_chem", _d), ("y_abs", _d), ("newton_rtol", _d), ("c_red", _d), ("t_cmb", _d),
        ("y_he", _d), ("gamma_ad", _d),
        ("n_cyc", C.c_int32), ("n_sub_max", C.c_int32), ("newton_max", C.c_int32),
        ("ir_mode", C.c_int32), ("thermal_mode", C.c_int32), ("dust_mode", C.c_int32),
        ("dispatch", C.c_int32), ("phase_nsub", C.c_int32),
        ("photon_absorb", C.c_int32), ("reserved", C.c_int32),
    ]


_vp = C.c_void_p


class SfcCells(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, _vp) for k in (
        "y_h2", "y_e", "eint", "tdust", "eir", "y_h", "y_hp", "y_hm", "tgas",
        "nh", "n_euv", "n_fuv", "zmet", "nsub", "niter", "flags", "n_euv_out", "n_fuv_out")]


class SfcRequest(C.Structure):
    _fields_ = [("cells", SfcCells), ("dt_seconds", _d), ("level", C.c_int32),
                ("precision", C.c_int32), ("tag", C.c_uint64), ("block_key", C.c_uint64),
                ("flags", C.c_uint32), ("reserved", C.c_uint32), ("hip_stream", C.c_void_p)]


class SfcResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("level", C.c_int32), ("tag", C.c_uint64),
                ("cells", C.c_int64), ("t_submit", _d), ("t_admit", _d), ("t_done", _d)]


EXPORTS = ("sfc_network_default", "sfc_params_default", "sfc_chem_init", "sfc_chem_step",
           "sfc_chem_step_nr", "sfc_chem_step_noalloc", "sfc_chem_submit", "sfc_chem_poll",
           "sfc_chem_fetch",
           "sfc_chem_release", "sfc_chem_drain", "sfc_chem_destroy", "sfc_strerror",
           "sfc_last_error", "sfc_now")

_LIB = None


def lib():
    """Load libsfchem.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first "
                               "(python -m paper_2604_21438_amd.build)")
        # PyTorch ships its own HIP runtime; importing it first makes the
        # library's libamdhip64 dependency resolve to that same runtime, so
        # the process holds one HIP runtime and torch's streams and device
        # pointers are valid for the library's launches.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.sfc_network_default.argtypes = [P(SfcNetwork)]
        L.sfc_params_default.argtypes = [P(SfcParams)]
        L.sfc_chem_init.argtypes = [P(SfcNetwork), _d, _d, P(SfcParams), C.c_int, C.c_uint64,
                                    P(C.c_void_p)]
        L.sfc_chem_step.argtypes = [C.c_void_p, P(SfcCells), _d, C.c_int, C.c_void_p]
        L.sfc_chem_step_nr.argtypes = [C.c_void_p, P(SfcCells), _d, C.c_void_p]
        L.sfc_chem_step_noalloc.argtypes = [C.c_void_p, P(SfcCells), _d, C.c_int, C.c_void_p]
        L.sfc_chem_submit.argtypes = [C.c_void_p, P(SfcRequest), P(C.c_uint64)]
        L.sfc_chem_poll.argtypes = [C.c_void_p, C.c_uint64, P(SfcResult)]
        L.sfc_chem_fetch.argtypes = [C.c_void_p, C.c_uint64, P(SfcCells), C.c_void_p]
        L.sfc_chem_release.argtypes = [C.c_void_p, C.c_uint64]
        L.sfc_chem_drain.argtypes = [C.c_void_p]
        L.sfc_chem_destroy.argtypes = [C.c_void_p]
        L.sfc_strerror.argtypes = [C.c_int]
        L.sfc_strerror.restype = C.c_char_p
        L.sfc_last_error.argtypes = [C.c_void_p]
        L.sfc_last_error.restype = C.c_char_p
        L.sfc_now.restype = _d
        for name in ("sfc_chem_init", "sfc_chem_step", "sfc_chem_step_nr", "sfc_chem_step_noalloc",
                     "sfc_chem_submit",
                     "sfc_chem_poll", "sfc_chem_fetch", "sfc_chem_release", "sfc_chem_drain",
                     "sfc_chem_destroy"):
            getattr(L, name).restype = C.c_int
        _LIB = L
    return _LIB


def default_network(**overrides) -> SfcNetwork:
    net = SfcNetwork()
    lib().sfc_network_default(C.byref(net))
    _apply(net, overrides)
    return net


def default_params(**overrides) -> SfcParams:
    p = SfcParams()
    lib().sfc_params_default(C.byref(p))
    _apply(p, overrides)
    return p


def _apply(obj, overrides):
    for k, v in overrides.items():
        cur = getattr(obj, k)
        if isinstance(cur, C.Array):
            for i, x in enumerate(v):
                cur[i] = x
        else:
            setattr(obj, k, v)


class SfcError(RuntimeError):
    pass


STATE = ("y_h2", "y_e", "eint", "tdust", "eir")
INPUTS = ("nh", "n_euv", "n_fuv", "zmet")
OUT_F = ("y_h", "y_hp", "y_hm", "tgas")
PHOTON_OUT = ("n_euv_out", "n_fuv_out")
OUT_I = ("nsub", "niter", "flags")


def to_device(cells: dict, device="cuda", outputs=True, photons=False) -> dict:
    """Copy a dict of host arrays (numpy or torch) to contiguous device
    tensors and allocate the optional outputs (with photons, also the photon
    densities after absorption)."""
    import torch
    out = {}
    n = None
    for k, v in cells.items():
        if v is None:
            continue
        t = torch.as_tensor(np.ascontiguousarray(v) if isinstance(v, np.ndarray) else v)
        t = t.to(device=device, dtype=torch.float64).contiguous()
        out[k] = t
        n = t.shape[0]
    if outputs and n is not None:
        for k in OUT_F:
            out[k] = torch.empty(n, dtype=torch.float64, device=device)
        out["nsub"] = torch.zeros(n, dtype=torch.int32, device=device)
        out["niter"] = torch.zeros(n, dtype=torch.int32, device=device)
        out["flags"] = torch.zeros(n, dtype=torch.int32, device=device)
        if photons:
            for k in PHOTON_OUT:
                out[k] = torch.empty(n, dtype=torch.float64, device=device)
    return out


def make_cells(t: dict) -> SfcCells:
    """SfcCells view of a dict of device tensors (missing keys -> NULL)."""
    import torch
    n = None
    for k in STATE + INPUTS + OUT_F + OUT_I:
        if k in t and t[k] is not None:
            n = t[k].shape[0]
            break
    if n is None:
        raise ValueError("no cell arrays")
    c = SfcCells()
    c.n = n
    for k in STATE + INPUTS + OUT_F + PHOTON_OUT:
        v = t.get(k)
        if v is not None:
            if v.dtype != torch.float64 or not v.is_cuda or not v.is_contiguous() or v.shape != (n,):
                raise ValueError(f"{k}: need a contiguous float64 device tensor of length {n}")
            setattr(c, k, v.data_ptr())
    for k in OUT_I:
        v = t.get(k)
        if v is not None:
            if v.dtype != torch.int32 or not v.is_cuda or not v.is_contiguous() or v.shape != (n,):
                raise ValueError(f"{k}: need a contiguous int32 device tensor of length {n}")
            setattr(c, k, v.data_ptr())
    return c


class Context:
    """sfc_chem_init / sfc_chem_step / sfc_chem_submit / sfc_chem_poll."""

    def __init__(self, network: SfcNetwork | None = None, z_default: float = 1.0,
                 dust_factor: float = 1.0, params: SfcParams | None = None, device: int = 0,
                 served_budget_bytes: int = 0):
        L = lib()
        # let PyTorch bring up its HIP context first: it owns the device
        # memory and streams this context works on
        import torch
        torch.cuda.init()
        torch.cuda.set_device(int(device))
        h = C.c_void_p()
        rc = L.sfc_chem_init(C.byref(network) if network is not None else None, float(z_default),
                             float(dust_factor), C.byref(params) if params is not None else None,
                             int(device), int(served_budget_bytes), C.byref(h))
        if rc != OK:
            raise SfcError(f"sfc_chem_init: {L.sfc_strerror(rc).decode()} ({rc})")
        self._h = h
        self.device = device
        self._keep = {}

    def _check(self, rc, what):
        if rc != OK:
            L = lib()
            raise SfcError(f"{what}: {L.sfc_strerror(rc).decode()} ({rc}): "
                           f"{L.sfc_last_error(self._h).decode()}")

    def step(self, cells: dict, dt: float, precision: int = FP64, stream=None) -> None:
        """Advance the cells (dict of device tensors, updated in place)."""
        import torch
        c = make_cells(cells)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        sp = C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        self._check(lib().sfc_chem_step(self._h, C.byref(c), float(dt), int(precision), sp),
                    "sfc_chem_step")

    def step_noalloc(self, cells: dict, dt: float, precision: int = FP64, stream=None) -> None:
        """sfc_chem_step through the entry point that allocates nothing (at
        most NOALLOC_MAX_CELLS cells; calls on one GPU must not overlap)."""
        c = make_cells(cells)
        self._check(lib().sfc_chem_step_noalloc(self._h, C.byref(c), float(dt), int(precision),
                                                self._stream(stream)), "sfc_chem_step_noalloc")

    def step_nr(self, cells: dict, dt: float, stream=None) -> None:
        """Advance the cells with the Newton-Raphson comparator (binary64)."""
        import torch
        c = make_cells(cells)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        sp = C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        self._check(lib().sfc_chem_step_nr(self._h, C.byref(c), float(dt), sp), "sfc_chem_step_nr")

    def _stream(self, stream):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))

    def submit(self, cells, dt: float, precision: int = MIXED, level: int = 0, tag: int = 0,
               sync: bool = True, block_key: int = 0, resume: bool = False,
               writeback: bool = False, stream=None) -> int:
        """Queue a request; without a block key the tensors are updated in
        place once poll() reports it done.  The library reads the inputs on
        its own stream: by default torch's current stream is synchronised
        first; with sync=False the library instead waits (on the device) for
        the work queued on `stream` (default: torch's current stream).
        `level` is the AMR level: waves holding cells of finer levels issue
        first, and with SFC_SERVE_LEVEL_CLAIMS=1 (read when the context is
        created) finer levels are also handed out first.  With a block key
        the block's state stays resident between requests: `resume`
        continues from it (cells may be None), results are read with
        fetch(), and `writeback` also copies them into `cells`."""
        import torch
        r = SfcRequest()
        if cells is not None:
            r.cells = make_cells(cells)
        if sync:
            torch.cuda.current_stream(self.device).synchronize()
            r.hip_stream = None
        else:
            r.hip_stream = self._stream(stream)
        r.dt_seconds = float(dt)
        r.level = int(level)
        r.precision = int(precision)
        r.tag = int(tag)
        r.block_key = int(block_key)
        r.flags = (REQ_RESUME if resume else 0) | (REQ_WRITEBACK if writeback else 0)
        t = C.c_uint64()
        self._check(lib().sfc_chem_submit(self._h, C.byref(r), C.byref(t)), "sfc_chem_submit")
        if cells is not None:
            self._keep[t.value] = cells  # buffers must outlive the request
        return t.value

    def poll(self, ticket: int):
        """None while pending, else a dict with the request's timing."""
        res = SfcResult()
        rc = lib().sfc_chem_poll(self._h, int(ticket), C.byref(res))
        if rc == E_PENDING:
            return None
        self._check(rc, "sfc_chem_poll")
        self._keep.pop(int(ticket), None)
        return dict(status=res.status, level=res.level, tag=res.tag, cells=res.cells,
                    t_submit=res.t_submit, t_admit=res.t_admit, t_done=res.t_done)

    def fetch(self, ticket: int, cells: dict, stream=None) -> bool:
        """Copy the results of a completed keyed request into `cells`
        (device tensors; missing keys are skipped), queued on `stream`
        (default: torch's current stream).  False while it is pending."""
        c = make_cells(cells)
        rc = lib().sfc_chem_fetch(self._h, int(ticket), C.byref(c), self._stream(stream))
        if rc == E_PENDING:
            return False
        self._check(rc, "sfc_chem_fetch")
        return True

    def release(self, block_key: int) -> None:
        """Give a block key's arena range back."""
        self._check(lib().sfc_chem_release(self._h, int(block_key)), "sfc_chem_release")

    def drain(self) -> None:
        self._check(lib().sfc_chem_drain(self._h), "sfc_chem_drain")

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().sfc_chem_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def now() -> float:
    return float(lib().sfc_now())
