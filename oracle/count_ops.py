"""Algorithmic operation count per subcycle of the LI update.

Runs the counting build of the CPU reference on a seeded sample of the
128^3 grid population (dt = 10 kyr) and prints the ratio of total counted
operations to total subcycles: add/sub, mul, div, sqrt (FMA-free code, so
a multiply-add counts 2) and transcendental calls (exp, log, log1p, pow),
plus the same per Newton iteration of the tight dust solve.

    python -m oracle.count_ops [n_cells] [--fixed-ir]

E_IR is evolved unless --fixed-ir (the IR field held at the CMB's).

TEST / MEASUREMENT INFRASTRUCTURE: calls only this package.
"""
import sys

import numpy as np


def main(n=120, factors=(1.0, 1000.0), fixed_ir=False):
    import oracle
    from paper_2604_21438_amd import workloads as W
    cells, dt = W.grid128(n=100000)
    sub, _ = W.subsample(cells, n, seed=21)
    for f in factors:
        p = oracle.default_params(dust_cap=1e4 * f)
        if fixed_ir:
            p.ir_mode = 0
        o = oracle.li_step(sub, dt, params=p)
        cnt = oracle.count_li(sub, dt, range(n), params=p)
        tot = cnt.sum(axis=0)
        nsub = o["nsub"].sum()
        per = tot / nsub
        print(f"dust factor {f:g}, {'FIXED' if fixed_ir else 'evolved'} E_IR: {n} cells, {nsub} subcycles, "
              f"{o['niter'].sum()} tight Newton iterations")
        print("  per subcycle: add %.1f mul %.1f div %.1f sqrt %.1f transcendental %.1f" %
              tuple(per[:5]))
        print("  algorithmic FLOP per subcycle (basic + transcendental as 1): %.0f" %
              per[:5].sum())


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if not a.startswith("--")]
    main(int(args[0]) if args else 120, fixed_ir="--fixed-ir" in sys.argv[1:])
