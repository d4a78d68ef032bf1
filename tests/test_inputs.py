"""Host-side checks (no GPU): the seeded input recipes of each workload
match the distributions they are meant to stand in for, they are
reproducible, and bench.py refuses more than one GPU before touching one."""
import os
import subprocess
import sys

import numpy as np

from paper_2604_21438_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KYR = 3.15576e10
STATE = ("nh", "n_euv", "n_fuv", "zmet", "y_h2", "y_e", "eint", "tdust")


def _neutrality_and_bounds(c):
    y_h2, y_e = c["y_h2"], c["y_e"]
    assert np.all(y_h2 > 0) and np.all(y_h2 <= 0.5)
    assert np.all(y_e > 0) and np.all(y_e < 1)
    # H nuclei: y_H = 1 - 2 y_H2 - y_H+ - y_H- stays non-negative
    assert np.all(1.0 - 2.0 * y_h2 - y_e >= -1e-12)
    assert np.all(c["eint"] > 0) and np.all(np.isfinite(c["eint"]))


def test_small_population_recipe():
    """4096 cells: log n_H ~ U[0,8], log T ~ U[1,4], T_d = T, dt = 1 kyr."""
    c, dt = W.small_cells()
    assert c["nh"].shape == (4096,)
    assert dt == 1.0 * KYR
    ln = np.log10(c["nh"])
    assert ln.min() >= 0 and ln.max() <= 8 and ln.min() < 0.1 and ln.max() > 7.9
    assert np.all(c["tdust"] >= 10) and np.all(c["tdust"] <= 1e4)
    for k in ("n_euv", "n_fuv"):
        lk = np.log10(c[k])
        assert lk.min() >= -5 and lk.max() <= 1 and lk.max() - lk.min() > 5.5  # six decades
    _neutrality_and_bounds(c)


def test_grid128_recipe_and_prefix():
    """128^3 cells, Z drawn from {0.01, 0.1, 1} per cell, dt = 10 kyr; a
    shorter request is the prefix of the same draw."""
    c, dt = W.grid128(65536)
    assert dt == 10.0 * KYR
    assert set(np.unique(c["zmet"])) == {0.01, 0.1, 1.0}
    frac = np.array([(c["zmet"] == z).mean() for z in (0.01, 0.1, 1.0)])
    assert np.all(np.abs(frac - 1 / 3) < 0.02)
    _neutrality_and_bounds(c)
    c2, _ = W.grid128(4096)
    for k in STATE:
        assert np.array_equal(c2[k], c[k][:4096])


def test_grid256_density_tail():
    """Log-normal n_H (median ~100 cm^-3, sigma 2 in ln) with an n^-1.5
    tail above 1e4 cm^-3; photon densities fall off from point sources."""
    c, dt = W.grid256(262144)
    assert dt == 10.0 * KYR
    ln = np.log(c["nh"])
    assert abs(np.median(ln) - np.log(100.0)) < 0.1
    body = ln[c["nh"] < 1e3]
    assert 1.5 < np.std(body) < 2.5
    tail = np.sort(c["nh"][c["nh"] > 1e4])
    assert tail.size > 100
    # survival function of a power-law density p(n) ~ n^-1.5 falls as n^-0.5
    s = 1.0 - np.arange(tail.size) / tail.size
    slope = np.polyfit(np.log(tail[: tail.size * 9 // 10]), np.log(s[: tail.size * 9 // 10]), 1)[0]
    assert -0.7 < slope < -0.3, slope
    assert np.all(c["zmet"] == 1.0)
    _neutrality_and_bounds(c)


def test_amr_requests_recipe():
    """Requests of whole 8^3 blocks, level L in 0..5 with dt = 10 kyr / 2^L,
    block counts within [1, max_blocks]; reproducible for a seed."""
    reqs, _ = W.amr_requests(64, max_blocks=64, side=64)
    levels = set()
    for r in reqs:
        n = r["cells"]["nh"].shape[0]
        assert n % 512 == 0 and 512 <= n <= 64 * 512
        assert r["dt"] == 10.0 * KYR / 2 ** r["level"]
        levels.add(r["level"])
    assert levels == set(range(6))
    again, _ = W.amr_requests(64, max_blocks=64, side=64)
    assert all(np.array_equal(a["cells"]["nh"], b["cells"]["nh"]) for a, b in zip(reqs, again))


def test_gmc_levels_recipe():
    """Nested 8^3 blocks, level L advanced with dt = 10 kyr / 2^L, Z = 0.1,
    finer levels denser than coarser ones on average."""
    lv = W.gmc_levels(target_cells=40000, base_side=16)
    assert len(lv) >= 3
    for L, l in enumerate(lv):
        assert l["cells"]["nh"].shape[0] % 512 == 0
        assert l["dt"] == 10.0 * KYR / 2 ** L
        assert np.all(l["cells"]["zmet"] == 0.1)
    med = [np.median(l["cells"]["nh"]) for l in lv]
    assert med[-1] > med[0]


def test_poisson_arrivals():
    t = W.poisson_arrivals(20000, rate=50.0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps >= 0)
    assert abs(gaps.mean() - 1 / 50.0) < 0.05 / 50.0 * 10
    # exponential gaps: coefficient of variation 1
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_ir_field_recipe():
    """Every population carries E_IR for a radiation temperature
    log-uniform between T_CMB and the dust temperature (E_IR = (c/c~) a
    T_IR^4)."""
    for cells in (W.small_cells()[0], W.grid128(n=50_000)[0], W.hii_region(20_000)[0],
                  W.grid256(n=30_000, side=64)[0]):
        tir = (cells["eir"] * W.C_RED / W.A_RAD) ** 0.25
        td = np.maximum(cells["tdust"], W.T_CMB)
        assert np.all(tir >= W.T_CMB * (1 - 1e-12)) and np.all(tir <= td * (1 + 1e-12))
        u = np.log(tir / W.T_CMB) / np.log(td / W.T_CMB)
        assert abs(np.mean(u) - 0.5) < 0.02 and abs(np.mean(u < 0.25) - 0.25) < 0.02


def test_bench_traffic_only_for_the_counted_step():
    """The HBM bytes bench.py reports were counted on the full 128^3 step of
    the plain-step sources whose hash they carry: any other cell count, or
    a changed source, reports null instead of a stale figure."""
    sys.path.insert(0, ROOT)
    import bench
    full = 128 ** 3
    ok = bench.kernel_sha1() == bench.TRAFFIC["kernel_sha1"]
    got = bench.measured_traffic(full)
    assert (got == bench.TRAFFIC["fetch_bytes"] + bench.TRAFFIC["write_bytes"]) if ok else got is None
    assert bench.measured_traffic(65536) is None
    assert bench.measured_traffic(full - 1) is None
