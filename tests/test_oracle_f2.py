"""Pins of the oracle's pieces beside the solver: H2 self-shielding, the
photoelectric heating with grain charging and recombination cooling, and
the absorption of EUV/FUV photons after the update.

The paper takes these formulas from its references (text after Table
"Thermal processes"; Sec. 2 "Radiation components"), so the oracle carries
labelled stand-ins: the self-shielding fit of Draine & Bertoldi (1996) with
a local H2 column, the photoelectric efficiency of Bakes & Tielens (1994)
in the form of Wolfire et al. (2003), and the exact integral of the
absorption term of the reduced-speed-of-light transport over the step.
Their values are parity unpinned beyond these checks: limits and shapes
of the fits, derivatives against central differences, the equilibrium the
integrator reaches, first-order convergence to RK4 with every piece on,
and photon conservation of the absorption step.
"""
import math

import numpy as np

import oracle
from conftest import cell_dict

YR = 3.15576e7
C_RED = 1e-4 * 2.99792458e10
MH = 1.67262192e-24


def _net(**kw):
    return oracle.default_network(**kw)


def _only(*reactions, **kw):
    rm = [0.0] * oracle.NREAC
    for r in reactions:
        rm[r] = 1.0
    return _net(reac_mult=rm, **kw)


# ------------------------------------------------------------ self-shielding

def _fsh(y2, T=100.0, nh=1e3, n_fuv=3.7e-3, **kw):
    """f_sh from the photodissociation rate: R_H2 = -k10 f_sh y_H2 with
    only reaction H10 on."""
    net = _only(10, shield_mode=1, **kw)
    out, _, _ = oracle.chem_sources(y2, 0.0, T, 10.0, nh, 1.0, 0.0, n_fuv, net=net)
    k, _ = oracle.rate_coeffs(T, 10.0, nh, 1.0, 0.0, n_fuv, net=net)
    return -out[0] / (k[10] * y2)


def test_shielding_fit_limits_and_shape():
    """f_sh -> 0.965 + 0.035 exp(-8.5e-4) at zero column (the fit's value,
    within 1e-9 at a tiny column), decreases monotonically with the column,
    stays in (0, 1], and at large columns falls as 0.035 exp(-8.5e-4 s) / s,
    s = sqrt(1 + x) (the damping-wing term of the fit)."""
    f0 = 0.965 + 0.035 * math.exp(-8.5e-4)
    assert abs(_fsh(1e-20) - f0) < 1e-9
    cols = np.logspace(-8, -0.3, 40)
    f = np.array([_fsh(y) for y in cols])
    assert np.all(np.diff(f) < 0) and np.all(f > 0) and np.all(f <= 1)
    # the same y_H2 at a longer column length (larger shield_len) shields more
    assert _fsh(1e-3, shield_len=2.0) < _fsh(1e-3, shield_len=0.5)
    # at a very large column only the wing survives: f s / (0.035 e^(-8.5e-4 s))
    # tends to 1 (the first term falls as x^-2, the wing as x^-1/2)
    big = np.array([_fsh(0.49, nh=1e9), _fsh(0.49, nh=1e11)])
    ratio_now = big[1] / big[0]
    assert ratio_now < 0.2  # two decades more column: ~x^-1/2 wing, 0.1 times exp factors


def test_shielding_partials_against_central_differences():
    """d R_H2 / d y_H2 and d R_H2 / d T (through the T dependence of the
    column length) of the photodissociation rate with shielding."""
    net = _only(10, shield_mode=1)
    for y2, T in ((1e-4, 50.0), (1e-2, 300.0), (0.3, 2000.0)):
        _, jac, _ = oracle.chem_sources(y2, 0.0, T, 10.0, 1e4, 1.0, 0.0, 3.7e-2, net=net)
        h = 1e-6 * y2
        fp, _, _ = oracle.chem_sources(y2 + h, 0.0, T, 10.0, 1e4, 1.0, 0.0, 3.7e-2, net=net)
        fm, _, _ = oracle.chem_sources(y2 - h, 0.0, T, 10.0, 1e4, 1.0, 0.0, 3.7e-2, net=net)
        assert abs((fp[0] - fm[0]) / (2 * h) / jac[0, 0] - 1) < 1e-6
        hT = 1e-6 * T
        fp, _, _ = oracle.chem_sources(y2, 0.0, T + hT, 10.0, 1e4, 1.0, 0.0, 3.7e-2, net=net)
        fm, _, _ = oracle.chem_sources(y2, 0.0, T - hT, 10.0, 1e4, 1.0, 0.0, 3.7e-2, net=net)
        assert abs((fp[0] - fm[0]) / (2 * hT) / jac[0, 2] - 1) < 1e-5


def test_shielded_formation_dissociation_equilibrium():
    """Grain formation (H8) against shielded photodissociation (H10), fixed
    T and T_d: the LI update settles where k8 n y_H = k10 f_sh(y_H2) y_H2,
    y_H = 1 - 2 y_H2; the root is found independently by bisection on the
    oracle's own rate evaluations."""
    nh, T, Td, nf = 1e3, 50.0, 15.0, 3.7e-2
    net = _only(8, 10, shield_mode=1)
    par = oracle.default_params(thermal_mode=oracle.THERMAL_ISOTHERMAL,
                                dust_mode=oracle.DUST_FROZEN)

    def g(y2):
        out, _, _ = oracle.chem_sources(y2, 0.0, T, Td, nh, 1.0, 0.0, nf, net=net, params=par)
        return out[0]

    lo, hi = 1e-12, 0.5 - 1e-12
    assert g(lo) > 0 > g(hi)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(mid) > 0:
            lo = mid
        else:
            hi = mid
    y_eq = 0.5 * (lo + hi)
    c = cell_dict(nh, T, Td, 1e-3, 0.0, n_fuv=nf)
    o = oracle.li_step(c, 1e9 * YR, net=net, params=par)
    for _ in range(2):  # each call ends on a Newton-like step of the LI map
        o = oracle.li_step(o, 1e9 * YR, net=net, params=par)
    assert abs(o["y_h2"][0] / y_eq - 1) < 1e-10
    # without shielding the equilibrium lies lower (more dissociation)
    o0 = oracle.li_step(c, 1e9 * YR, net=_only(8, 10), params=par)
    assert o0["y_h2"][0] < o["y_h2"][0]


# ------------------------------------------------------------ photoelectric

def _pe(ye, T, nh=100.0, n_fuv=3.7e-3, fd=1.0):
    net = _only(pe_mode=1)
    net.proc_mult[:] = [0.0, 0.0, 0.0, 1.0] + [0.0] * 10  # process 4 only
    out, jac, terms = oracle.chem_sources(0.0, ye, T, 10.0, nh, fd, 0.0, n_fuv, net=net)
    return out, jac, terms


def test_photoelectric_neutral_grain_limit():
    """Where the charging parameter psi = G0 sqrt(T) / n_e is tiny, grains
    stay neutral: the efficiency tends to 0.0487 + 0.0365 (T/1e4)^0.7, so
    Gamma_4 tends to 1.3e-24 eps G0 n_H f_d.  Without an FUV field there is
    neither heating nor recombination cooling."""
    for T in (100.0, 1e4):
        nh = 1e8
        _, _, terms = _pe(0.5, T, nh=nh, n_fuv=3.7e-6)  # G0 = 1e-3, n_e = 5e7
        eps0 = 0.0487 + 0.0365 * (T / 1e4) ** 0.7
        assert abs(terms[3] / (1.3e-24 * eps0 * 1e-3 * nh) - 1) < 1e-4
    _, _, terms = _pe(1e-3, 100.0, n_fuv=0.0)
    assert terms[3] == 0.0 and terms[13] == 0.0


def test_photoelectric_charging_and_recombination():
    """Fewer electrons per unit field charge the grains: the heating per G0
    falls monotonically as psi grows (over psi from ~0.3 to ~3e4), and the
    recombination cooling scales as n_e psi^beta: at fixed psi (G0 and n_e
    raised together) it grows linearly with n_e, and at fixed n_e it grows
    with the field as G0^beta, beta = 0.735 T^-0.068."""
    heat = []
    for ye in (1e-1, 1e-2, 1e-3, 1e-4, 1e-5):
        _, _, terms = _pe(ye, 100.0)
        heat.append(terms[3])
    assert np.all(np.diff(heat) < 0)
    _, _, t1 = _pe(1e-2, 100.0, n_fuv=3.7e-3)
    _, _, t2 = _pe(2e-2, 100.0, n_fuv=7.4e-3)
    assert abs(t2[13] / t1[13] - 2.0) < 1e-12
    _, _, t3 = _pe(1e-2, 100.0, n_fuv=7.4e-3)
    beta = 0.735 * 100.0 ** -0.068
    assert abs(t3[13] / t1[13] - 2.0 ** beta) < 1e-12


def test_photoelectric_partials_against_central_differences():
    for ye, T in ((1e-4, 80.0), (1e-2, 500.0), (0.3, 8000.0)):
        out, jac, _ = _pe(ye, T)
        h = 1e-6 * ye
        fp, _, _ = _pe(ye + h, T)
        fm, _, _ = _pe(ye - h, T)
        assert abs((fp[2] - fm[2]) / (2 * h) / jac[2, 1] - 1) < 1e-5
        hT = 1e-6 * T
        fp, _, _ = _pe(ye, T + hT)
        fm, _, _ = _pe(ye, T - hT)
        assert abs((fp[2] - fm[2]) / (2 * hT) / jac[2, 2] - 1) < 1e-5


def test_li_converges_to_rk4_with_shielding_and_photoelectric():
    """First-order convergence of LI to RK4 with both stand-ins on (their
    partials enter the LI Jacobian, their values the RK4 right-hand side)."""
    cells = cell_dict([10.0, 30.0, 3.0], [300.0, 150.0, 800.0], [20.0, 15.0, 30.0],
                      [0.1, 0.02, 0.2], [1e-3, 3e-3, 1e-2], n_euv=[0.0, 0.0, 0.0],
                      n_fuv=[1e-2, 3e-3, 3e-2])
    net = _net(pe_mode=1, shield_mode=1)
    dt = 2.0e4 * YR
    mk = lambda f: oracle.default_params(dust_mode=oracle.DUST_FROZEN, f_chem=f)
    ref = oracle.rk_reference(cells, dt, net=net, params=mk(0.03), step_frac=1e-3)
    errs = []
    for f in (0.03, 0.01, 1.0 / 300):
        o = oracle.li_step(cells, dt, net=net, params=mk(f))
        errs.append(max(np.max(np.abs(o[k] / ref[k] - 1)) for k in ("y_h2", "y_e", "tgas")))
    assert errs[0] < 0.1
    assert 2.0 < errs[0] / errs[1] < 4.5 and 2.0 < errs[1] / errs[2] < 4.5, errs


# ------------------------------------------------------------ photon absorption

def _rk4_photons(n0, a_h, a_d, dt, steps=20000):
    """dN/dt = -c~ (a_h + a_d) N with the photons taken by each absorber
    counted separately (ionisations I, dust D), classical RK4."""
    y = np.array([n0, 0.0, 0.0])

    def f(y):
        return np.array([-C_RED * (a_h + a_d) * y[0], C_RED * a_h * y[0], C_RED * a_d * y[0]])

    h = dt / steps
    for _ in range(steps):
        k1 = f(y)
        k2 = f(y + 0.5 * h * k1)
        k3 = f(y + 0.5 * h * k2)
        k4 = f(y + h * k3)
        y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return y


def test_photon_absorption_conserves_photons():
    """With the composition held fixed (no reactions, isothermal, frozen
    dust), the EUV photons left after dt are those of the transport's
    absorption term integrated over dt, and the photons removed equal the
    photoionisations plus the dust absorptions (RK4 of the three counts);
    the FUV field loses only to dust."""
    nh, fd, yh2, ye = 30.0, 0.5, 0.1, 0.05
    c = cell_dict(nh, 100.0, 20.0, yh2, ye, n_euv=2.0, n_fuv=5.0, z=fd)
    net = _only()
    par = oracle.default_params(thermal_mode=oracle.THERMAL_ISOTHERMAL,
                                dust_mode=oracle.DUST_FROZEN, photon_absorb=1)
    dt = 3.0e3 * YR
    o = oracle.li_step(c, dt, net=net, params=par)
    yh = o["y_h"][0]
    rho = 1.4 * MH * nh
    a_h = net.sigma_euv * nh * yh
    a_d = net.kappa_uv * rho * fd
    n_left, ion, dust = _rk4_photons(2.0, a_h, a_d, dt)
    assert abs(o["n_euv_out"][0] / n_left - 1) < 1e-9
    assert abs((2.0 - o["n_euv_out"][0]) / (ion + dust) - 1) < 1e-9
    n_left, _, _ = _rk4_photons(5.0, 0.0, a_d, dt)
    assert abs(o["n_fuv_out"][0] / n_left - 1) < 1e-9


def test_photon_absorption_edge_cases():
    """No absorbers (no dust, no neutral H): nothing is absorbed; an invalid
    cell keeps its photons; a fully neutral dense cell absorbs its EUV
    photons entirely, leaving a non-negative field; the absorption follows
    the updated neutral fraction (EUV optical depth = c~ dt (sigma n_H y_H +
    kappa rho f_d) with the y_H the update returns)."""
    par = oracle.default_params(photon_absorb=1)
    # y_H = 0: fully ionised (y_e = 1), no dust
    c = cell_dict(10.0, 1e4, 100.0, 0.0, 1.0, n_euv=1.0, n_fuv=1.0, z=0.0)
    o = oracle.li_step(c, 1e3 * YR, net=_only(), params=oracle.default_params(
        photon_absorb=1, thermal_mode=oracle.THERMAL_ISOTHERMAL, dust_mode=oracle.DUST_FROZEN))
    assert o["n_euv_out"][0] == 1.0 and o["n_fuv_out"][0] == 1.0
    bad = cell_dict([10.0, -1.0], 100.0, 20.0, 0.1, 1e-3, n_euv=1.0, n_fuv=1.0)
    o = oracle.li_step(bad, 1e3 * YR, params=par)
    assert o["flags"][1] == oracle.F_INVALID and o["n_euv_out"][1] == 1.0
    dense = cell_dict(1e6, 50.0, 20.0, 0.1, 1e-6, n_euv=1.0, n_fuv=1.0)
    o = oracle.li_step(dense, 1e4 * YR, params=par)
    assert o["n_euv_out"][0] == 0.0 and o["n_fuv_out"][0] >= 0.0
    full = cell_dict([3.0, 30.0], [300.0, 3000.0], 20.0, [0.1, 0.01], [1e-3, 0.1],
                     n_euv=[1e-2, 1e-1], n_fuv=[1.0, 1.0])
    net = oracle.default_network()
    dt = 10.0 * YR
    o = oracle.li_step(full, dt, net=net, params=par)
    rho = 1.4 * MH * full["nh"]
    tau = C_RED * dt * (net.sigma_euv * full["nh"] * o["y_h"] + net.kappa_uv * rho)
    np.testing.assert_allclose(np.log(full["n_euv"] / o["n_euv_out"]), tau, rtol=1e-10)
