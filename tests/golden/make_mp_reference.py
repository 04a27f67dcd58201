"""Write mp256_ising_small.txt: the 256-bit TT cross (oracle/ttcross_mp.py) on small D_d cases.

D_d in the paper form (Sec. 5.1, eq. d) at n = 3..6 Gauss-Legendre nodes per
mode, rank cap 64, tol 1e-21, seed d, and the brute-force tensor-product
sum over the same nodes (T2), both at 256 bits.  The double-double GPU path is
compared with them (tests/test_gpu_dd.py): with the cross's value at 1e-20 where
both runs end on the same ranks, and with T2 where rounding-level ties took
them to different ranks.  Only oracle/ is called.  Pins of the 256-bit
oracle: tests/test_oracle_mp.py.

Usage: python tests/golden/make_mp_reference.py  (about two minutes on one core)
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import mpmath as mp  # noqa: E402

from oracle import ttcross_mp  # noqa: E402

CASES = [(4, 3), (4, 4), (4, 5), (4, 6), (5, 3), (5, 4), (5, 5), (5, 6), (6, 3), (6, 4), (6, 5),
         (7, 3), (7, 4), (8, 3), (8, 4)]
RANK, TOL = 64, 1e-21


def main():
    lines = ["# D_d, paper form (Sec. 5.1, eq. d), n Gauss-Legendre nodes per mode: the oracle's TT cross",
             f"# in 256-bit arithmetic (oracle/ttcross_mp.py), rank cap {RANK}, tol {TOL:g}, seed d.",
             "# Written by tests/golden/make_mp_reference.py.",
             "# With it, the brute-force tensor-product sum over the same nodes at 256 bits (T2).",
             "# d  n  value(60 digits)  sweeps  stop_reason  ranks(comma-separated)  T2(60 digits)"]
    for d, n in CASES:
        tt = ttcross_mp.solve("ising_d", d, n, RANK, TOL, seed=d)
        t2 = ttcross_mp.tensor_quadrature_mp("ising_d", d, n)
        lines.append(f"{d} {n} {mp.nstr(tt.history[-1], 60, min_fixed=1, max_fixed=0)} {tt.sweeps} "
                     f"{tt.stop_reason} {','.join(str(r) for r in tt.ranks())} "
                     f"{mp.nstr(t2, 60, min_fixed=1, max_fixed=0)}")
        print(lines[-1], flush=True)
    with open(os.path.join(HERE, "mp256_ising_small.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
