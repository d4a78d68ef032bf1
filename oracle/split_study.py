"""Split-order study: the subcycle's Lie split in both orders on a seeded
sample of the 128^3 grid population (dt = 10 kyr, dust factor 1).

The method's split (chemistry + energy, renormalisation, then the Appendix C
dust/IR/gas-grain step) is a reading; the paper does not state the order.
This runs the same sample through the oracle built both ways (the other
order is the measurement build ORC_DUST_FIRST, which takes the chemistry's
coefficients again after the dust step) and prints the subcycle statistics,
the fraction of cells at the subcycle cap, and how far the results of the
two orders lie apart.

    python -m oracle.split_study [n_cells]

TEST / MEASUREMENT INFRASTRUCTURE: calls only this package.
"""
import sys

import numpy as np


def main(n=2048, threads=8):
    import oracle
    from paper_2604_21438_amd import workloads as W
    cells, dt = W.grid128(n=200_000)
    sub, _ = W.subsample(cells, n, seed=31)
    p = oracle.default_params(dust_cap=1e4)
    out = {}
    for variant, name in (("plain", "chemistry first"), ("df", "dust first")):
        o = oracle.li_step(sub, dt, params=p, nthreads=threads, variant=variant)
        ns = o["nsub"].astype(np.float64)
        capped = (o["flags"] & oracle.F_CAP) != 0
        out[variant] = o
        print(f"{name}: {n} cells, nsub mean {ns.mean():.0f} p50 {np.median(ns):.0f} "
              f"p99 {np.percentile(ns, 99):.0f}; at the cap {capped.mean():.4f} "
              f"(carrying {ns[capped].sum() / ns.sum():.3f} of the subcycles)")
    a, b = out["plain"], out["df"]
    for k in ("tgas", "tdust", "y_h2", "y_e"):
        r = np.abs(a[k] - b[k]) / np.maximum(np.abs(a[k]), 1e-300)
        print(f"  {k}: relative difference between the orders median {np.median(r):.2e} "
              f"p90 {np.percentile(r, 90):.2e} p99 {np.percentile(r, 99):.2e}")
    both = ((a["flags"] & oracle.F_CAP) != 0) & ((b["flags"] & oracle.F_CAP) != 0)
    print(f"  cells at the cap in both orders: {int(both.sum())}")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 2048)
