"""CPU oracle for tensor-train (TT) cross integration — TEST INFRASTRUCTURE ONLY.

This package is the slow, plain, obviously-correct reference that the GPU
library is checked against.  It is written from the paper (Dolgov &
Savostyanov, "Parallel cross interpolation for high-precision calculation of
high-dimensional integrals", arXiv:1903.11554) in float64 numpy, with a
double-double counterpart for the high-precision runs, and mpmath used only
where a pin needs more digits.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything from here.  The product library
(``paper_1903_11554_amd``) never imports, links or calls it, and the oracle
never imports the product library: the two share no code.

Modules
-------
rng          SplitMix64 counter-based generator (Steele, Lea & Flood 2014).
gauss        Gauss--Legendre rule on [0,1] (Sec. 4.1, "Tensor product quadratures").
integrands   Ising integrands C_d, D_d, E_d (eqs. c/d/e, Sec. 5.1), the
             u-form of the same integrals, and synthetic product test functions.
quadrature   Brute-force tensor-product quadrature (eq. quad_product).
ttcross      Alg. 2 (matrix cross step: random + rook pivoting) run on every
             superblock at once with the previous sweep's index sets (Alg. 6),
             and the TT quadrature as a product of 2d-1 matrices (Sec. 4.1),
             with the folded weights and the chain scaled by exact powers
             of two so that a thousand modes stay in the double range.
ddarith      Double-double arithmetic on numpy arrays from the error-free
             transformations (Knuth two-sum, Dekker/Veltkamp two-product).
ttcross_dd   The same TT cross with every value in double-double (the
             quadruple/multiple-precision runs of Sec. 5.2), paper form only.
montecarlo   Monte Carlo and randomly shifted lattice rules with the
             empirical error estimate (Sec. 4.2).

Parity status of every function is listed in the module headers.  Functions
pinned by closed forms, the paper's printed values or exact-recovery theorems
are marked "pinned"; none is "parity unpinned" except where a header says so.
"""
