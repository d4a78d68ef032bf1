"""Pins of the oracle's tightly coupled gas-dust step (Sec. 2, "Time
stepping": dust iterations only where gas and grains are tightly coupled;
Appendix C: the dust temperature, IR energy and gas temperature equations).

In the oracle the tight step is backward Euler over the subcycle with the
gas-grain coefficient and kappa(T_IR) frozen: T_g and E_IR follow from
T_d, and one scalar equation Phi(T_d) = 0 is solved by safeguarded Newton.
None of these checks reads that construction back; each one holds for the
exact mathematics and fails for a plausible mistake in Phi, in its
derivative, or in the back-substitution of T_g and E_IR:

  check_convergence     every subcycle forced tight (N_cyc = 0): LI
                        converges at first order to a fine RK4 integration
                        of the ODE (whose right-hand side is the Appendix C
                        source terms, written separately from Phi) in T_g,
                        T_d, E_IR and y_H2: the error falls in proportion to
                        the mean subcycle length as f_chem falls 0.03 ->
                        0.01 -> 1/300.  (In strongly coupled cells the step
                        is set by the split's own residual and shrinks only
                        as f_chem^1/2, so the error's ratio per f_chem step
                        is ~sqrt 3 there, ~3 elsewhere.)
  check_energy_identity one tight step over the whole interval with the
                        chemistry and heating/cooling switched off, EVOLVE
                        IR: the energy given to gas, dust and IR field
                        equals the UV energy the grains absorbed,
                        rho alpha_g dT_g + rho f_d C_d dT_d + dE_IR
                        = dt rho f_d E_UV (gas-grain exchange and IR
                        emission/absorption only move energy around), for
                        weakly and for strongly gas-grain coupled cells.
  check_newton          single tight steps of strongly coupled cells at
                        the realistic C_d = 1e4 over 1e5-1e9 s: the Newton
                        iteration, started on the convex side, ends without
                        NOCONV within 20 iterations (quadratic once close;
                        the quartic emission term makes the first steps
                        contract by about 3/4).
  check_steady_state    one tight step of 1e24 s, FIXED IR: backward Euler
                        of infinite length lands on the ODE's steady state,
                        T_g = T_d and S_d = 0 (grain radiative equilibrium).

Each takes `variant`, the oracle build to check (the plain build by
default); tests/test_oracle_mutants.py runs them on builds with planted
mistakes.
"""
import numpy as np

import oracle
from conftest import cell_dict

YR = 3.15576e7
A_RAD = 7.5657e-15
C_LIGHT = 2.99792458e10
M_H = 1.67262192e-24
EV = 1.602176634e-12
Y_HE = 0.1


def _coupled_cells(evolve_ir):
    """Five cells whose dust is far from balance (T_d changes by factors
    0.5-3 over the interval, E_IR by 2 in the n_H = 1e5 cell), three weakly
    and two strongly gas-grain coupled, Z != 1 in four of them so that
    every f_d factor matters."""
    c = cell_dict([1e2, 1e3, 1e5, 3e6, 1e7], [100.0, 60.0, 50.0, 100.0, 200.0],
                  [30.0, 8.0, 30.0, 15.0, 20.0], [0.1, 0.3, 0.4, 0.3, 0.3],
                  [1e-3, 1e-4, 1e-5, 1e-6, 1e-6], n_euv=[0.0] * 5,
                  n_fuv=[1e-2, 3e-3, 1e-1, 1e-2, 1e-2], z=[1.0, 0.5, 0.3, 0.5, 0.5])
    if evolve_ir:
        # T_IR = 10, 25, 5, 10, 10 K: E_IR = a T^4 / (c~/c)
        c["eir"] = np.array([A_RAD * T ** 4 / 1e-4 for T in (10.0, 25.0, 5.0, 10.0, 10.0)])
    return c


def _dense_cells():
    """Strongly gas-grain coupled cells (n_H 1e6-1e8) with dust far from
    the gas temperature."""
    c = cell_dict([1e6, 1e7, 1e8, 1e8], [200.0, 100.0, 300.0, 30.0], [20.0, 15.0, 20.0, 60.0],
                  [0.3] * 4, [1e-6] * 4, n_euv=[0.0, 0.0, 1e-2, 0.0],
                  n_fuv=[1e-2, 1e-1, 1.0, 1e-3], z=[0.5, 1.0, 0.3, 1.0])
    c["eir"] = np.array([A_RAD * T ** 4 / 1e-4 for T in (10.0, 25.0, 5.0, 10.0)])
    return c


def _no_chemistry():
    """Network with every reaction and heating/cooling process off except
    the gas-grain exchange (process 14)."""
    return oracle.default_network(reac_mult=[0.0] * oracle.NREAC,
                                  proc_mult=[0.0] * 13 + [1.0])


def check_convergence(ir_mode, variant="plain"):
    """First-order convergence of the forced-tight LI update to RK4: with
    C_d = 1e10 erg/g/K the dust relaxes in ~1e2-1e3 yr, shorter than the
    1 kyr interval, so every tight subcycle's implicit solve decides T_d."""
    evolve = ir_mode == oracle.IR_EVOLVE
    cells = _coupled_cells(evolve)
    dt = 1.0e3 * YR

    def par(f):
        return oracle.default_params(ir_mode=ir_mode, dust_cap=1e10, f_chem=f, n_cyc=0)

    ref = oracle.rk_reference(cells, dt, params=par(0.03), step_frac=1e-3)
    keys = ("y_h2", "tgas", "tdust") + (("eir",) if evolve else ())
    errs = {k: [] for k in keys}
    nsub = []
    for f in (0.03, 0.01, 1.0 / 300):
        o = oracle.li_step(cells, dt, params=par(f), variant=variant)
        assert np.all(o["flags"] & oracle.F_TIGHT), o["flags"]
        assert not np.any(o["flags"] & oracle.F_NOCONV), o["flags"]
        # safeguarded Newton from the convex side: ~3 iterations per subcycle
        assert np.all(o["niter"] <= 6 * o["nsub"]), (o["niter"], o["nsub"])
        nsub.append(o["nsub"].astype(float))
        for k in keys:
            errs[k].append(np.abs(o[k] / ref[k] - 1.0))
    nsub = np.array(nsub)
    step_ratio = nsub[1:] / nsub[:-1]          # mean subcycle length, before / after
    assert np.all(step_ratio > 1.5), nsub
    for k in keys:
        e = np.array(errs[k])
        assert e[-1].max() < 2.5e-2, (k, e[-1])
        # cells whose error is far above rounding (E_IR hardly moves in the
        # thinnest cells)
        live = e[-1] > 1e-9
        assert live.sum() >= 3, (k, e[-1])
        ratio = (e[:-1] / np.where(e[1:] > 0, e[1:], np.inf)) / step_ratio
        assert np.all((ratio[:, live] > 0.7) & (ratio[:, live] < 1.4)), (k, ratio)


def check_energy_identity(variant="plain"):
    """dE_th + rho f_d C_d dT_d + dE_IR = dt rho f_d E_UV after one tight
    step, to rounding.  E_UV (UV energy absorbed per gram of gas) is
    c kappa_UV (N_FUV e_FUV + N_EUV e_EUV) with the network's stand-in
    constants; rho = (1 + 4 y_He) m_H n_H."""
    weak = _coupled_cells(True)
    weak["n_euv"] = np.array([1e-3, 0.0, 3e-2, 0.0, 1e-3])
    net = _no_chemistry()
    for cells, cd, dt in ((weak, 1e9, 3.0e2 * YR), (_dense_cells(), 1e4, 1e7)):
        par = oracle.default_params(ir_mode=oracle.IR_EVOLVE, dust_cap=cd, n_cyc=0,
                                    f_chem=1e30)
        o = oracle.li_step(cells, dt, net=net, params=par, variant=variant)
        assert np.all(o["nsub"] == 1) and np.all(o["flags"] & oracle.F_TIGHT), (o["nsub"],
                                                                               o["flags"])
        # the composition does not change, so dE_th = c_v dT_g exactly
        np.testing.assert_array_equal(o["y_h2"], cells["y_h2"])
        np.testing.assert_array_equal(o["y_e"], cells["y_e"])
        rho = (1.0 + 4.0 * Y_HE) * M_H * cells["nh"]
        fd = cells["zmet"]
        e_uv = C_LIGHT * net.kappa_uv * (cells["n_fuv"] * net.e_fuv_ev +
                                         cells["n_euv"] * net.e_euv_ev) * EV
        d_gas = o["eint"] - cells["eint"]
        d_dust = rho * fd * cd * (o["tdust"] - cells["tdust"])
        d_ir = o["eir"] - cells["eir"]
        src = dt * rho * fd * e_uv
        # rounding bound: the changes are differences of the stored energies
        # (E_IR is up to ~1e6 times its change here), and T_d is solved to
        # ~1e-12
        tol = 1e-12 * (np.abs(cells["eir"]) + np.abs(cells["eint"]) +
                       rho * fd * cd * cells["tdust"] + np.abs(src))
        # every term moves by far more than that: the identity is not trivial
        for d in (d_gas, d_dust, d_ir, src):
            assert np.all(np.abs(d) > 100.0 * tol), (d, tol)
        resid = np.abs(d_gas + d_dust + d_ir - src)
        assert np.all(resid < tol), (cd, resid, tol)


def check_newton(variant="plain"):
    """Single tight steps of strongly coupled cells at C_d = 1e4 (h times
    the gas-grain term of Phi' is comparable to C_d + h times the emission
    term): no NOCONV, at most 20 Newton iterations."""
    cells = _dense_cells()
    net = _no_chemistry()
    for ir in (oracle.IR_FIXED, oracle.IR_EVOLVE):
        par = oracle.default_params(ir_mode=ir, dust_cap=1e4, n_cyc=0, f_chem=1e30)
        for dt in (1e5, 1e6, 1e7, 1e8, 1e9):
            o = oracle.li_step(cells, dt, net=net, params=par, variant=variant)
            assert np.all(o["nsub"] == 1) and np.all(o["flags"] & oracle.F_TIGHT)
            assert not np.any(o["flags"] & oracle.F_NOCONV), (ir, dt, o["flags"])
            assert np.all(o["niter"] <= 20), (ir, dt, o["niter"])


def check_steady_state(variant="plain"):
    """One tight step of 1e24 s (chemistry and heating/cooling off, FIXED
    IR): the grains end in radiative equilibrium with the UV and the CMB,
    S_d = 0, and the gas at the grain temperature, T_g = T_d."""
    cells = _coupled_cells(False)
    net = _no_chemistry()
    par = oracle.default_params(ir_mode=oracle.IR_FIXED, dust_cap=1e4, n_cyc=0, f_chem=1e30)
    o = oracle.li_step(cells, 1e24, net=net, params=par, variant=variant)
    assert np.all(o["nsub"] == 1) and np.all(o["flags"] & oracle.F_TIGHT)
    np.testing.assert_allclose(o["tgas"], o["tdust"], rtol=1e-9)
    e_uv = C_LIGHT * net.kappa_uv * (cells["n_fuv"] * net.e_fuv_ev +
                                     cells["n_euv"] * net.e_euv_ev) * EV
    for i in range(cells["nh"].shape[0]):
        ntot = 1.0 - o["y_h2"][i] + o["y_e"][i] + Y_HE
        _, _, src = oracle.dust_system(o["tgas"][i], o["tdust"][i], 0.0, cells["nh"][i],
                                       cells["zmet"][i], ntot, cells["n_euv"][i],
                                       cells["n_fuv"][i], 1.0, net=net, params=par)
        # S_d = kappa(T_CMB) a c T_CMB^4 + E_UV - kappa(T_d) a c T_d^4 - (gas-grain)
        assert abs(src[0]) < 1e-9 * e_uv[i], (i, src[0], e_uv[i])
        assert o["tdust"][i] > 3.0
