"""The oracle's pins catch plausible mistakes.

Each mutant is a copy of oracle/orc_chem.cpp with one planted mistake (a
textual substitution), built with the oracle's own flags into a temporary
directory.  A pin set is only worth something if every such mistake makes
at least one of its pins fail; the plain build passes them all
(tests/test_oracle_pins.py).  All of this runs on the CPU.
"""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

import oracle
import tight_pins

# tight gas-dust step: Phi, its derivative, the frozen coefficients and the
# back-substitution of T_g and E_IR (Appendix C equations under backward
# Euler, Sec. 2 "Time stepping")
TIGHT_MUTANTS = {
    "phi_coupling_sign": ("real coup = t.ggd * t.dg * (x - t.tg0);",
                          "real coup = t.ggd * t.dg * (t.tg0 - x);"),
    "phi_emission_power": ("real emis = k * ac * x3 * x;",
                           "real emis = k * ac * x3;"),
    "phi_uv_dropped": ("phi = t.p->dust_cap * (x - t.td0) - t.h * (ab + t.c->e_uv - emis - coup);",
                       "phi = t.p->dust_cap * (x - t.td0) - t.h * (ab - emis - coup);"),
    "dphi_emission_dropped": ("dphi = t.p->dust_cap - t.h * (dab - demis - t.ggd * t.dg);",
                              "dphi = t.p->dust_cap - t.h * (dab - t.ggd * t.dg);"),
    "dphi_coupling_sign": ("dphi = t.p->dust_cap - t.h * (dab - demis - t.ggd * t.dg);",
                           "dphi = t.p->dust_cap - t.h * (dab - demis + t.ggd * t.dg);"),
    "ir_absorption_explicit": ("real E = (t.e0 + t.P * emis) / t.qd;", "real E = t.e0;"),
    "dg_complement": ("t.dg = t.alpha / (t.alpha + t.w);", "t.dg = t.w / (t.alpha + t.w);"),
    "coupling_without_fd": ("t.w = h * c.fd * t.ggd;", "t.w = h * t.ggd;"),
    "ir_coupling_without_fd": ("t.P = h * c.rho * c.fd;", "t.P = h * c.rho;"),
    "qd_without_reduced_c": ("t.qd = 1.0 + t.P * ctil * t.kir;", "t.qd = 1.0 + t.P * t.kir;"),
    "tg_backsub_swapped": ("real tg = (t.alpha * t.tg0 + t.w * x) / (t.alpha + t.w);",
                           "real tg = (t.w * t.tg0 + t.alpha * x) / (t.alpha + t.w);"),
    "eir_backsub_no_qd": ("s.Eir = (t.e0 + t.P * k * ac * x * x * x * x) / t.qd;",
                          "s.Eir = t.e0 + t.P * k * ac * x * x * x * x;"),
    "gas_energy_update_sign": ("s.E = s.E + cv * (tg - Tg0);\n  return it;",
                               "s.E = s.E - cv * (tg - Tg0);\n  return it;"),
    "gamma_d_sign": ("real gd = 1.0 - 0.8 * rexp(-T_LOW / Tg0);",
                     "real gd = 1.0 + 0.8 * rexp(-T_LOW / Tg0);"),
}


def _checks():
    """(name, callable(variant)) of every tight-step pin."""
    return [
        ("convergence_fixed", lambda v: tight_pins.check_convergence(oracle.IR_FIXED, v)),
        ("convergence_evolve", lambda v: tight_pins.check_convergence(oracle.IR_EVOLVE, v)),
        ("energy_identity", tight_pins.check_energy_identity),
        ("newton", tight_pins.check_newton),
        ("steady_state", tight_pins.check_steady_state),
    ]


@pytest.fixture(scope="module")
def mutant_libs(tmp_path_factory):
    with open(oracle.SRC) as f:
        src = f.read()
    d = tmp_path_factory.mktemp("mutants")
    jobs = []
    for name, (old, new) in TIGHT_MUTANTS.items():
        assert src.count(old) == 1, (name, src.count(old))
        cpp = d / f"{name}.cpp"
        cpp.write_text(src.replace(old, new))
        # the copies include the oracle's headers from its own directory
        jobs.append((name, ["g++", *oracle.CFLAGS, "-I" + oracle.HERE, "-o",
                            str(d / f"lib_{name}.so"), str(cpp)]))
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        rcs = list(ex.map(lambda j: subprocess.run(j[1], capture_output=True).returncode, jobs))
    assert all(rc == 0 for rc in rcs), dict(zip([j[0] for j in jobs], rcs))
    return {name: str(d / f"lib_{name}.so") for name in TIGHT_MUTANTS}


def test_plain_build_passes_tight_pins():
    for _, check in _checks():
        check("plain")


@pytest.mark.parametrize("name", sorted(TIGHT_MUTANTS))
def test_tight_pins_catch_mutant(mutant_libs, name):
    caught = []
    for cname, check in _checks():
        try:
            check(mutant_libs[name])
        except AssertionError:
            caught.append(cname)
    assert caught, f"no tight-step pin fails for the planted mistake {name}"
