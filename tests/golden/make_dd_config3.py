"""Write dd_d8_n128_r64.txt: the double-double oracle's run of D_8 at the full precision-workload size.

D_8 in the paper form (Sec. 5.1, eq. d), 128 Gauss-Legendre nodes per mode,
rank cap 64, tol 1e-21, seed 8, every value in double-double
(oracle/ttcross_dd.py, plain: every sweep rebuilds the cores and crosses from
the definition of B).  Stored: the pivot log (per sweep and bond: row, col,
accepted, rook iterations, the error's leading and low doubles, B's leading
double, whether the last column step was at the final column) and the
integral after the start and after every sweep (leading and low doubles).
The double-double GPU path runs the same job with its rank-64 sweep kernels
and is compared record by record (tests/test_gpu_dd.py).  Only oracle/ is
called.

Usage: python tests/golden/make_dd_config3.py  (some ten minutes on four cores)
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.ttcross_dd import TTCrossDD  # noqa: E402

D, N, RANK, TOL, SEED = 8, 128, 64, 1e-21, 8


def main():
    tt = TTCrossDD("ising_d", D, N, RANK, TOL, SEED)
    while tt.stop_reason is None:
        tt.sweep()
        print(f"sweep {tt.sweeps} ranks {tt.ranks()} value {tt.history[-1]!r} {tt.history_lo[-1]!r}", flush=True)
    out = [f"# D_{D}, paper form (Sec. 5.1, eq. d), {N} Gauss-Legendre nodes, rank cap {RANK}, tol {TOL:g},",
           f"# seed {SEED}: the double-double oracle (oracle/ttcross_dd.py).  Written by",
           "# tests/golden/make_dd_config3.py.",
           f"stop {tt.stop_reason} sweeps {tt.sweeps} evals {tt.evals} ranks {','.join(map(str, tt.ranks()))}",
           "# hist k value_hi value_lo"]
    for k, (h, lo) in enumerate(zip(tt.history, tt.history_lo)):
        out.append(f"hist {k} {h!r} {lo!r}")
    out.append("# piv sweep bond row col accepted iters err_hi err_lo value_hi col_fresh")
    for s, recs in enumerate(tt.pivot_log):
        for r in recs:
            out.append(f"piv {s} {r.bond} {r.row} {r.col} {int(r.accepted)} {r.iters} {r.err!r} {r.err_lo!r} "
                       f"{r.value!r} {int(r.col_fresh)}")
    with open(os.path.join(HERE, "dd_d8_n128_r64.txt"), "w") as fh:
        fh.write("\n".join(out) + "\n")


if __name__ == "__main__":
    main()
