"""Write ising_d_n64_reference.txt: D_5..D_10 from the oracle's TT cross (test infrastructure).

The paper form of D_d (Sec. 5.1, eq. d) on 64 Gauss-Legendre nodes per mode,
rank cap 48, stopping tolerance 1e-13, seed d: the oracle's own run (plain
float64, nothing incremental; oracle/ttcross.py), well below the 1e-10 the
benchmark checks its results against.  Only oracle/ is called.  The stored
values are pinned in tests/test_oracle_reference_values.py (the paper's printed
D_8, brute-force quadrature of D_5).

Usage: python tests/golden/make_ising_reference.py  (about two minutes on one core)
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ttcross  # noqa: E402

N, RANK, TOL = 64, 48, 1e-13


def main():
    lines = ["# D_d, paper form (Sec. 5.1, eq. d), 64 Gauss-Legendre nodes per mode: the oracle's",
             f"# TT cross (oracle/ttcross.py) with rank cap {RANK}, tol {TOL:g}, seed d.",
             "# Written by tests/golden/make_ising_reference.py.",
             "# d  value  sweeps  max_rank"]
    for d in range(5, 11):
        tt = ttcross.solve("ising_d", d, N, RANK, TOL, seed=d)
        assert tt.stop_reason == "converged", (d, tt.stop_reason)
        lines.append(f"{d} {tt.history[-1]!r} {tt.sweeps} {max(tt.ranks())}")
        print(lines[-1], flush=True)
    with open(os.path.join(HERE, "ising_d_n64_reference.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
