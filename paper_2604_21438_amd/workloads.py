"""Seeded synthetic cell populations for the thermochemistry update.

This module only draws inputs.  It contains none of the update's arithmetic
and is shared by the HIP path's tests and benchmark and by the CPU
reference's tests, which must see the same bits.  The paper's own snapshots
(Bonnor-Ebert collapse, H II region, giant molecular cloud) are not
available, so these distributions stand in for them.

Every population is a dict of contiguous float64 numpy arrays (SoA):

  nh     H-nuclei number density [cm^-3]
  n_euv  EUV photon number density [cm^-3]
  n_fuv  FUV photon number density [cm^-3]
  zmet   metallicity in solar units (dust-to-gas ratio scales with it)
  y_h2   H2 abundance per H nucleus
  y_e    electron abundance per H nucleus
  eint   gas internal energy density [erg cm^-3]
  tdust  dust temperature [K]
  eir    IR radiation energy density [erg cm^-3] (read when E_IR evolves)

The IR field is drawn as a radiation temperature log-uniform between
T_CMB = 2.73 K and the cell's dust temperature (a field diluted below the
dust's own emission), E_IR = (c / c~) a T_IR^4 with c~/c = 1e-4, the
default reduced speed of light.

The internal energy is built from a drawn gas temperature with the ideal-gas
relation E = k_B n_H (1 - y_H2 + y_e + y_He) T / (gamma - 1), y_He = 0.1,
gamma = 5/3, so that both implementations read identical bits.

Seeds: numpy PCG64 with SeedSequence(21438 + 100 * i) for population i,
one spawned child stream per drawn field (fixed order).
"""
from __future__ import annotations

import numpy as np

KB = 1.380649e-16
A_RAD = 7.5657e-15        # radiation constant [erg cm^-3 K^-4]
C_RED = 1.0e-4            # reduced speed of light / c (default)
T_CMB = 2.73
Y_HE = 0.1
GAMMA = 5.0 / 3.0
YR = 3.15576e7            # Julian year [s]
KYR = 1.0e3 * YR

FIELDS = ("nh", "n_euv", "n_fuv", "zmet", "y_h2", "y_e", "eint", "tdust", "eir")


def _streams(cfg_index: int, nstreams: int, seed_offset: int = 0):
    ss = np.random.SeedSequence(21438 + 100 * cfg_index + seed_offset)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(nstreams)]


def internal_energy(nh, y_h2, y_e, tgas):
    """Ideal-gas internal energy density from a temperature (input construction)."""
    return KB * nh * (1.0 - y_h2 + y_e + Y_HE) * tgas / (GAMMA - 1.0)


def _abundances(g_h2, g_hp, n):
    y_hp = 10.0 ** g_hp.uniform(-8.0, -1.0, n)
    y_hm = np.full(n, 1.0e-12)
    y_e = y_hp - y_hm                        # charge neutral
    y_h2 = 10.0 ** g_h2.uniform(-6.0, -0.3, n)
    # the upper end of the H2 draw can exceed what H-nuclei conservation
    # allows; clamp it just inside the feasible range
    y_h2 = np.minimum(y_h2, 0.5 * (1.0 - y_hp - y_hm) * (1.0 - 1.0e-9))
    return y_h2, y_e


def uniform_population(n: int, cfg_index: int = 0, z_choices=None, seed_offset: int = 0):
    """Independent cells: log10 n_H ~ U[0,8], log10 T ~ U[1,4], T_d = T,
    log10 y_H2 ~ U[-6,-0.3], log10 y_H+ ~ U[-8,-1], y_H- = 1e-12, y_e from
    charge neutrality, log10 N_EUV, log10 N_FUV ~ U[-5,1] independently,
    Z = 1 or drawn uniformly from z_choices, E_IR as in the module notes."""
    g = _streams(cfg_index, 8, seed_offset)
    nh = 10.0 ** g[0].uniform(0.0, 8.0, n)
    tg = 10.0 ** g[1].uniform(1.0, 4.0, n)
    y_h2, y_e = _abundances(g[2], g[3], n)
    n_euv = 10.0 ** g[4].uniform(-5.0, 1.0, n)
    n_fuv = 10.0 ** g[5].uniform(-5.0, 1.0, n)
    if z_choices is None:
        zmet = np.ones(n)
    else:
        zmet = np.asarray(z_choices, np.float64)[g[6].integers(0, len(z_choices), n)]
    return _pack(nh, n_euv, n_fuv, zmet, y_h2, y_e, tg, tg.copy(), g[7].uniform(0.0, 1.0, n))


def ir_energy(tdust, u):
    """E_IR for a radiation temperature T_CMB (td / T_CMB)^u, u in [0, 1]."""
    tir = T_CMB * (np.maximum(tdust, T_CMB) / T_CMB) ** u
    return A_RAD * tir ** 4 / C_RED


def _pack(nh, n_euv, n_fuv, zmet, y_h2, y_e, tg, td, u_ir):
    out = dict(nh=nh, n_euv=n_euv, n_fuv=n_fuv, zmet=zmet, y_h2=y_h2, y_e=y_e,
               eint=internal_energy(nh, y_h2, y_e, tg), tdust=td, eir=ir_energy(td, u_ir))
    return {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in out.items()}


# ---- the named workloads ------------------------------------------------

def small_cells():
    """16^3 = 4096 independent cells, Z = 1, dt = 1 kyr (dust factor 1)."""
    return uniform_population(4096, cfg_index=0), 1.0 * KYR


def grid128(n: int | None = None):
    """128^3 = 2,097,152 cells, Z in {0.01, 0.1, 1} per cell, dt = 10 kyr.
    n < 128^3 returns the first n cells of the same draw."""
    full = 128 ** 3
    cells = uniform_population(full, cfg_index=1, z_choices=(0.01, 0.1, 1.0))
    if n is not None and n < full:
        cells = {k: np.ascontiguousarray(v[:n]) for k, v in cells.items()}
    return cells, 10.0 * KYR


PC = 3.0857e18            # parsec [cm]
C_LIGHT = 2.99792458e10   # [cm/s]


def hii_region(n: int = 262_144, dt_yr: float = 100.0):
    """Static stand-in for the paper's H II region test (its hydrodynamic
    run is out of scope): a uniform n_H = 100 cm^-3 medium around a 40 M_sun
    star emitting S_EUV = 1.36e49 ionising photons/s, the state of the gas
    near the time when the ionisation front has reached the Stromgren
    radius R_st = 2.67 pc.  Cells sit at uniform positions in a 6 pc box
    centred on the star (r >= 0.05 pc).
      - inside the front (width 0.05 pc): ionised, T = 8000 K, T_d = 60 K;
      - outside: neutral (y_H+ = 1e-4), T = 100 K, T_d = 20 K, turning
        molecular over 0.3 pc beyond the front (y_H2 -> 0.5);
      - N_EUV = S_EUV / (4 pi r^2 c), cut off past the front; N_FUV half of
        the unattenuated value everywhere (dust attenuation neglected);
      - n_H and T carry 5 % log-normal scatter; Z = 1.
    dt = 100 yr stands for the step of a reduced-speed-of-light (1e-4 c)
    radiation solver on a ~0.01 pc cell, which the paper does not state."""
    g = _streams(5, 4)  # g[3]: E_IR
    x = g[0].uniform(-3.0, 3.0, (n, 3))
    r = np.maximum(np.sqrt(np.sum(x * x, axis=1)), 0.05)
    r_st, w = 2.67, 0.05
    front = 1.0 / (1.0 + np.exp(np.clip((r - r_st) / w, -60.0, 60.0)))
    nh = 100.0 * np.exp(0.05 * g[1].standard_normal(n))
    tg = (8000.0 * front + 100.0 * (1.0 - front)) * np.exp(0.05 * g[2].standard_normal(n))
    td = 60.0 * front + 20.0 * (1.0 - front)
    y_hp = front * (1.0 - 1.0e-4) + (1.0 - front) * 1.0e-4
    y_hm = np.full(n, 1.0e-12)
    y_e = y_hp - y_hm
    y_h2 = (1.0 - front) * 0.5 * (1.0 - np.exp(-np.maximum(r - r_st, 0.0) / 0.3))
    y_h2 = np.maximum(np.minimum(y_h2, 0.5 * (1.0 - y_hp - y_hm) * (1.0 - 1.0e-9)), 1.0e-10)
    flux = 1.36e49 / (4.0 * np.pi * (r * PC) ** 2 * C_LIGHT)
    n_euv = flux * front
    n_fuv = 0.5 * flux
    return _pack(nh, n_euv, n_fuv, np.ones(n), y_h2, y_e, tg, td, g[3].uniform(0.0, 1.0, n)), \
        dt_yr * YR


def subsample(cells: dict, m: int, seed: int = 7):
    """Seeded subset of m cells (sorted indices) and the indices."""
    n = cells["nh"].shape[0]
    if m >= n:
        return cells, np.arange(n)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    idx = np.sort(rng.choice(n, size=m, replace=False))
    return {k: np.ascontiguousarray(v[idx]) for k, v in cells.items()}, idx


def _density_tail(g_u, g_n, n, mu=np.log(100.0), sigma=2.0, n_break=1.0e4, n_max=1.0e11,
                  slope=1.5):
    """n_H with a log-normal body below n_break and a continuous power-law
    tail p(n) ~ n^-slope on [n_break, n_max] (pdf in n, joined continuously
    at n_break), drawn by inverse CDF."""
    from math import erf, sqrt, log, exp, pi
    lb = log(n_break)
    z = (lb - mu) / sigma
    mass_body = 0.5 * (1.0 + erf(z / sqrt(2.0)))
    # pdf in n of the log-normal at the break
    pdf_b = exp(-0.5 * z * z) / (n_break * sigma * sqrt(2.0 * pi))
    # tail pdf A n^-slope continuous at the break
    A = pdf_b * n_break ** slope
    mass_tail = A * (n_break ** (1.0 - slope) - n_max ** (1.0 - slope)) / (slope - 1.0)
    total = mass_body + mass_tail
    u = g_u.uniform(0.0, 1.0, n) * total
    out = np.empty(n)
    body = u < mass_body
    # body: invert the normal CDF by drawing a truncated normal in ln n
    nb = int(body.sum())
    ln = np.empty(nb)
    filled = 0
    while filled < nb:
        x = g_n.normal(mu, sigma, 2 * (nb - filled) + 16)
        x = x[x < lb]
        k = min(nb - filled, x.size)
        ln[filled:filled + k] = x[:k]
        filled += k
    out[body] = np.exp(ln)
    ut = (u[~body] - mass_body) / A  # = int_{n_b}^{n} x^-s dx
    base = n_break ** (1.0 - slope) - (slope - 1.0) * ut
    out[~body] = base ** (1.0 / (1.0 - slope))
    return out, mass_tail / total


def point_source_field(pos, src_pos, amp, h):
    """sum_s amp_s (h / max(|x - x_s|, h))^2 (photon density, 1/r^2)."""
    out = np.zeros(pos.shape[0])
    for s in range(src_pos.shape[0]):
        d = np.sqrt(((pos - src_pos[s]) ** 2).sum(axis=1))
        out += amp[s] * (h / np.maximum(d, h)) ** 2
    return out


def grid256(n: int | None = None, side: int = 256):
    """256^3 cells on the unit cube: n_H log-normal (mu = ln 100, sigma = 2)
    with an n^-1.5 tail above 1e4 to 1e11 cm^-3, log10 T ~ U[1,4], T_d = T,
    abundances as the uniform population, 8 point sources at uniform
    positions giving N_EUV = sum A_s (h/r)^2, A_s ~ logU[1,100] cm^-3 and
    N_FUV = sum r_s A_s (h/r)^2, r_s ~ logU[1,10]; Z = 1; dt = 10 kyr.
    n < side^3 returns the first n cells (x-fastest ordering)."""
    full = side ** 3
    m = full if n is None else min(n, full)
    g = _streams(2, 10)
    nh, _ = _density_tail(g[0], g[1], full)
    tg = 10.0 ** g[2].uniform(1.0, 4.0, full)
    y_h2, y_e = _abundances(g[3], g[4], full)
    src = g[5].uniform(0.0, 1.0, (8, 3))
    amp = 10.0 ** g[6].uniform(0.0, 2.0, 8)
    ratio = 10.0 ** g[7].uniform(0.0, 1.0, 8)
    h = 1.0 / side
    i = np.arange(m)
    pos = np.stack([(i % side + 0.5) * h, ((i // side) % side + 0.5) * h,
                    (i // (side * side) + 0.5) * h], axis=1)
    n_euv = point_source_field(pos, src, amp, h)
    n_fuv = point_source_field(pos, src, amp * ratio, h)
    u_ir = g[8].uniform(0.0, 1.0, full)
    sl = slice(0, m)
    return _pack(nh[sl], n_euv, n_fuv, np.ones(m), y_h2[sl], y_e[sl], tg[sl], tg[sl].copy(),
                 u_ir[sl]), 10.0 * KYR


BLOCK = 8  # AMR block edge (8^3 = 512 cells)


def amr_requests(n_req: int, max_blocks: int = 4096, side: int = 256, n_levels: int = 6,
                 seed_offset: int = 0):
    """Served workload: n_req requests, each a set of 8^3-cell blocks cut
    at seeded block-aligned offsets out of the grid256 fields (on a side^3
    grid), with the block count floor(exp(U[0, ln(max_blocks + 1)])) in
    [1, max_blocks], AMR level L ~ U{0..n_levels-1} and dt = 10 kyr / 2^L.

    Returns (requests, field) where each request is a dict with 'cells'
    (SoA dict, blocks concatenated, x-fastest inside a block), 'dt',
    'level' and 'blocks' (block indices into the field)."""
    field, dt0 = grid256(side=side)
    g = _streams(3, 3, seed_offset)
    nbmax = int(max_blocks)
    nblk = np.floor(np.exp(g[0].uniform(0.0, np.log(nbmax + 1.0), n_req))).astype(np.int64)
    nblk = np.clip(nblk, 1, nbmax)
    level = g[1].integers(0, n_levels, n_req)
    nb = side // BLOCK
    # cell offsets of one block relative to its first cell
    i = np.arange(BLOCK ** 3)
    local = (i % BLOCK) + side * ((i // BLOCK) % BLOCK) + side * side * (i // (BLOCK * BLOCK))
    reqs = []
    for j in range(n_req):
        b = g[2].integers(0, nb ** 3, int(nblk[j]))
        bx, by, bz = b % nb, (b // nb) % nb, b // (nb * nb)
        first = BLOCK * (bx + side * by + side * side * bz)
        idx = (first[:, None] + local[None, :]).reshape(-1)
        cells = {k: np.ascontiguousarray(v[idx]) for k, v in field.items()}
        reqs.append(dict(cells=cells, dt=dt0 / 2.0 ** int(level[j]), level=int(level[j]),
                         blocks=b))
    return reqs, field


def poisson_arrivals(n: int, rate: float, seed: int = 3):
    """Arrival times [s] of a Poisson process of the given rate, from 0."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(21438 + seed)))
    gaps = rng.exponential(1.0 / rate, n)
    return np.concatenate([[0.0], np.cumsum(gaps[1:])])


def _gaussian_field(g, side: int, slope: float = 11.0 / 3.0):
    """Unit-variance Gaussian random field on a periodic side^3 grid with
    power spectrum P(k) ~ |k|^-slope (random phases), via FFT."""
    k = np.fft.fftfreq(side) * side
    kx, ky, kz = np.meshgrid(k, k, np.fft.rfftfreq(side) * side, indexing="ij")
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    amp = np.zeros_like(kk)
    amp[kk > 0] = kk[kk > 0] ** (-slope / 2.0)
    spec = amp * (g.normal(size=kk.shape) + 1j * g.normal(size=kk.shape))
    f = np.fft.irfftn(spec, s=(side, side, side), axes=(0, 1, 2))
    return (f - f.mean()) / f.std()


def gmc_levels(target_cells: int = 4_000_000, base_side: int = 64, n_levels: int = 6,
               sigma: float = 2.5, n_sources: int = 64, zmet: float = 0.1, seed_offset: int = 0,
               progress=None):
    """A GMC-like AMR hierarchy of 8^3-cell blocks for the served form.

    Level 0 covers the unit cube with base_side^3 cells; ln n_H = ln 100 +
    sigma g on the level-0 grid (g a Gaussian random field, P(k) ~ k^-11/3).
    A block of level L is refined into 8 blocks of level L + 1 (twice the
    resolution) where its densest cell exceeds n0 4^L; child cells take
    their parent cell's density times exp(0.5 G), G a fresh unit normal per
    cell.  n0 is bisected so that the hierarchy holds target_cells +- 2 %
    (levels 1..n_levels-1 non-empty when possible).  T, abundances as the
    uniform population; 64 point sources at uniform positions give N_EUV =
    sum A_s (h/max(r, h))^2 and N_FUV = r_s times that (h the level-0 cell,
    A_s ~ logU[1, 100] cm^-3, r_s ~ logU[1, 10]); Z = zmet.

    Returns a list of levels, each a dict with 'cells' (SoA, blocks
    concatenated), 'dt' = 10 kyr / 2^L, 'blocks' and 'level'.  progress,
    if given, is called with a line of text after each trial threshold."""
    g = _streams(4, 8, seed_offset)
    base = np.exp(np.log(100.0) + sigma * _gaussian_field(g[0], base_side))
    nb0 = base_side // BLOCK
    # level-0 blocks: (corner index in level-L cell units, densities 8x8x8)
    def blocks_of(field, side):
        nb = side // BLOCK
        f = field.reshape(nb, BLOCK, nb, BLOCK, nb, BLOCK).transpose(0, 2, 4, 1, 3, 5)
        corners = np.stack(np.meshgrid(np.arange(nb), np.arange(nb), np.arange(nb),
                                       indexing="ij"), -1).reshape(-1, 3) * BLOCK
        return corners, f.reshape(-1, BLOCK, BLOCK, BLOCK)

    cap = 4 * target_cells

    def build(n0, count_only=False):
        """The hierarchy for threshold n0, or None once it exceeds cap cells
        (count_only: its cell count, without drawing the finest level)."""
        levels = []
        corners, dens = blocks_of(base, base_side)
        total = 0
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(21438 + 400 + seed_offset)))
        for L in range(n_levels):
            levels.append((corners, dens))
            total += dens.size
            if L == n_levels - 1:
                break
            refine = dens.reshape(dens.shape[0], -1).max(axis=1) > n0 * 4.0 ** L
            if not refine.any():
                break
            if total + 8 * int(refine.sum()) * BLOCK ** 3 > cap:
                return None
            if count_only and L == n_levels - 2:
                return total + 8 * int(refine.sum()) * BLOCK ** 3
            pc, pd = corners[refine], dens[refine]
            # each parent block -> 8 children at twice the resolution
            up = pd.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)  # (m, 16, 16, 16)
            up = up * np.exp(0.5 * rng.normal(size=up.shape))
            ch_c, ch_d = [], []
            for ox in (0, 1):
                for oy in (0, 1):
                    for oz in (0, 1):
                        ch_c.append(2 * pc + BLOCK * np.array([ox, oy, oz]))
                        ch_d.append(up[:, ox * BLOCK:(ox + 1) * BLOCK, oy * BLOCK:(oy + 1) * BLOCK,
                                       oz * BLOCK:(oz + 1) * BLOCK])
            corners, dens = np.concatenate(ch_c), np.concatenate(ch_d)
        return levels

    def count(n0):
        c = build(n0, count_only=True)
        return c if isinstance(c, (int, np.integer)) or c is None else sum(d.size for _, d in c)

    # bisection on n0 over counts, then one full build at the chosen threshold
    lo, hi = 1.0, 1.0e12
    chosen = None
    for _ in range(80):
        mid = np.sqrt(lo * hi)
        c = count(mid)
        total = cap + 1 if c is None else c
        if progress:
            progress(f"gmc threshold n0 = {mid:.4g}: {'over the cap' if c is None else int(c)} cells")
        if c is not None:
            chosen = mid
        if abs(total - target_cells) <= 0.02 * target_cells:
            break
        if total > target_cells:
            lo = mid
        else:
            hi = mid
    levels = build(chosen if chosen is not None else hi)
    src = g[1].uniform(0.0, 1.0, (n_sources, 3))
    amp = 10.0 ** g[2].uniform(0.0, 2.0, n_sources)
    ratio = 10.0 ** g[3].uniform(0.0, 1.0, n_sources)
    h0 = 1.0 / base_side
    out = []
    for L, (corners, dens) in enumerate(levels):
        m = dens.shape[0] * BLOCK ** 3
        hL = h0 / 2.0 ** L
        i = np.arange(BLOCK ** 3)
        local = np.stack([i // (BLOCK * BLOCK), (i // BLOCK) % BLOCK, i % BLOCK], 1)
        pos = ((corners[:, None, :] + local[None, :, :]).reshape(-1, 3) + 0.5) * hL
        nh = dens.reshape(-1)
        tg = 10.0 ** g[4].uniform(1.0, 4.0, m)
        y_h2, y_e = _abundances(g[5], g[6], m)
        n_euv = point_source_field(pos, src, amp, h0)
        n_fuv = point_source_field(pos, src, amp * ratio, h0)
        cells = _pack(nh, n_euv, n_fuv, np.full(m, zmet), y_h2, y_e, tg, tg.copy(),
                      g[7].uniform(0.0, 1.0, m))
        out.append(dict(cells=cells, dt=10.0 * KYR / 2.0 ** L, blocks=dens.shape[0], level=L))
    return out
