"""One-zone free-fall collapse: a hydro-free workload for the update.

A parcel of gas contracts on its own free-fall time
t_ff = sqrt(3 pi / (32 G rho)), rho = (1 + 4 y_He) m_H n_H, so that over a
step dt its density grows by exp(dt / t_ff) and its internal energy by the
adiabatic factor exp(gamma dt / t_ff) (compressional heating); the
thermochemistry then advances it over the same dt.  Several parcels (one
per metallicity) run side by side as one batch of cells.  This stands in
for the collapse histories the paper follows with hydrodynamics and
gravity (its Bonnor-Ebert tests), which are out of scope here: the tracks
T_g(n), T_d(n), y_H2(n) show how the pseudo dust heat capacity and the
LI scheme behave along a collapse, qualitatively.

The parcels carry no IR field: the one-zone model has no transport to
carry the grains' emission away, so it is run with FIXED IR (the IR field
held at the CMB's, an optically thin parcel); an E_IR evolved inside the
parcel alone would keep all the energy the grains radiate.

The compression is plain binary64 numpy arithmetic on the host, identical
whichever implementation advances the chemistry: `step(cells, dt)` is any
callable that returns the advanced cell dict (the library's plain path, its
NR comparator, or the CPU reference in the tests).
"""
from __future__ import annotations

import math

import numpy as np

from .workloads import GAMMA, KB, Y_HE, internal_energy

G_NEWTON = 6.6743e-8
M_H = 1.67262192e-24


def free_fall_time(nh: float) -> float:
    rho = (1.0 + 4.0 * Y_HE) * M_H * nh
    return math.sqrt(3.0 * math.pi / (32.0 * G_NEWTON * rho))


def initial_parcels(zmets=(1.0, 1e-2, 1e-4), n0=1.0e2, t0=100.0, td0=10.0, y_h2=1.0e-6,
                    y_e=1.0e-4):
    """One parcel per metallicity, no external radiation."""
    m = len(zmets)
    nh = np.full(m, n0)
    yh2 = np.full(m, y_h2)
    ye = np.full(m, y_e)
    return dict(nh=nh, n_euv=np.zeros(m), n_fuv=np.zeros(m), zmet=np.asarray(zmets, np.float64),
                y_h2=yh2, y_e=ye, eint=internal_energy(nh, yh2, ye, np.full(m, t0)),
                tdust=np.full(m, td0))


def gas_temperature(c: dict) -> np.ndarray:
    ntot = 1.0 - c["y_h2"] + c["y_e"] + Y_HE
    return c["eint"] * (GAMMA - 1.0) / (KB * c["nh"] * ntot)


def run(step, cells: dict, n_end: float = 1.0e11, dt_frac: float = 0.1, max_steps: int = 100000):
    """Collapse from the parcels' density to n_end.  Returns the track as
    arrays of shape (steps, parcels): nh, tgas, tdust, y_h2, y_e, nsub."""
    c = {k: np.array(v, dtype=np.float64) for k, v in cells.items()}
    rec = {k: [] for k in ("nh", "tgas", "tdust", "y_h2", "y_e", "nsub")}
    for _ in range(max_steps):
        n = float(c["nh"][0])
        if n >= n_end:
            break
        dt = dt_frac * free_fall_time(n)
        grow = math.exp(dt / free_fall_time(n))
        c["nh"] = c["nh"] * grow
        c["eint"] = c["eint"] * grow ** GAMMA
        out = step(c, dt)
        for k in ("y_h2", "y_e", "eint", "tdust"):
            c[k] = np.array(out[k], dtype=np.float64)
        rec["nh"].append(c["nh"].copy())
        rec["tgas"].append(gas_temperature(c))
        rec["tdust"].append(c["tdust"].copy())
        rec["y_h2"].append(c["y_h2"].copy())
        rec["y_e"].append(c["y_e"].copy())
        rec["nsub"].append(np.asarray(out["nsub"]).copy())
    return {k: np.array(v) for k, v in rec.items()}


def gpu_step(ctx, method: str = "li", precision: int = 0):
    """A step callable advancing host cells with the library (plain path or
    NR comparator) on the current device."""
    import torch

    from . import to_device

    def step(c, dt):
        t = to_device(c)
        if method == "nr":
            ctx.step_nr(t, dt)
        else:
            ctx.step(t, dt, precision)
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in t.items()}

    return step
