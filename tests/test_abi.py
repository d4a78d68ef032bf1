"""The C-ABI library loads on a machine without a GPU and exports every
symbol include/sfchem.h declares; host-side argument checks that need no
device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sfchem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sfc_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("sfc_chem_init", "sfc_chem_step", "sfc_chem_submit", "sfc_chem_poll",
              "sfc_chem_destroy"):
        assert n in names


def test_library_exports_declared_symbols():
    import paper_2604_21438_amd as sfc
    L = sfc.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(_declared()) == set(sfc.EXPORTS)


def test_defaults_and_structs_match_header():
    import paper_2604_21438_amd as sfc
    net = sfc.default_network()
    assert net.abi_version == sfc.ABI_VERSION
    assert net.size == C.sizeof(sfc.SfcNetwork)
    p = sfc.default_params()
    assert p.f_chem == 0.03 and p.n_cyc == 300 and p.n_sub_max == 100000


def test_strerror_and_init_errors_without_device():
    import paper_2604_21438_amd as sfc
    L = sfc.lib()
    assert L.sfc_strerror(sfc.E_BUDGET).decode().startswith("request exceeds")
    h = C.c_void_p()
    # bad dust factor is rejected before any device call
    assert L.sfc_chem_init(None, 1.0, -1.0, None, 0, 0, C.byref(h)) == sfc.E_INVAL
    net = sfc.default_network()
    net.abi_version = 99
    assert L.sfc_chem_init(C.byref(net), 1.0, 1.0, None, 0, 0, C.byref(h)) == sfc.E_VERSION
    assert L.sfc_chem_destroy(None) == sfc.OK
    assert L.sfc_chem_step(None, None, 1.0, 0, None) == sfc.E_INVAL


def test_dispatch_default_and_validation():
    import paper_2604_21438_amd as sfc
    L = sfc.lib()
    p = sfc.default_params()
    assert p.dispatch == sfc.DISPATCH_PROGRESS
    assert p.phase_nsub == 4096
    h = C.c_void_p()
    p.phase_nsub = 0
    assert L.sfc_chem_init(None, 1.0, 1.0, C.byref(p), 0, 0, C.byref(h)) == sfc.E_INVAL
    p.phase_nsub = 4096
    p.dispatch = 7
    assert L.sfc_chem_init(None, 1.0, 1.0, C.byref(p), 0, 0, C.byref(h)) == sfc.E_INVAL


def test_hii_region_inputs_are_valid():
    """The H II stand-in draws feasible states: positive densities and
    temperatures, H-nuclei conservation room for the drawn H2, ionised gas
    inside the Stromgren radius and neutral gas outside."""
    import numpy as np
    from paper_2604_21438_amd import workloads as W
    c, dt = W.hii_region(4096)
    assert dt == 100.0 * W.YR
    for k in W.FIELDS:
        assert np.all(np.isfinite(c[k])), k
    assert np.all(c["nh"] > 0) and np.all(c["eint"] > 0) and np.all(c["tdust"] > 0)
    assert np.all(c["n_euv"] >= 0) and np.all(c["n_fuv"] > 0)
    assert np.all(2 * c["y_h2"] + c["y_e"] <= 1.0)
    ionised = c["y_e"] > 0.5
    assert 0.2 < ionised.mean() < 0.6          # sphere of 2.67 pc in a 6 pc box: ~0.37
    assert np.all(c["n_euv"][~ionised] < c["n_euv"][ionised].min())


def test_struct_layouts_match_header(tmp_path):
    """sizeof and field offsets of every ABI struct, from the header through
    a C compiler, equal the binding's ctypes layouts."""
    import paper_2604_21438_amd as sfc
    structs = {"sfc_request": sfc.SfcRequest, "sfc_result": sfc.SfcResult,
               "sfc_cells": sfc.SfcCells, "sfc_network": sfc.SfcNetwork,
               "sfc_params": sfc.SfcParams}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "sfchem.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = str(tmp_path / "layout")
    import subprocess
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src),
                           "-o", exe])
    out = dict(line.rsplit(" ", 1) for line in subprocess.check_output([exe], text=True).splitlines())
    for cname, py in structs.items():
        assert int(out[f"{cname} size"]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(out[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def test_served_calls_reject_bad_arguments_without_device():
    import paper_2604_21438_amd as sfc
    L = sfc.lib()
    t = C.c_uint64()
    assert L.sfc_chem_submit(None, None, C.byref(t)) == sfc.E_INVAL
    assert L.sfc_chem_fetch(None, 1, None, None) == sfc.E_INVAL
    assert L.sfc_chem_release(None, 1) == sfc.E_INVAL
