"""Bounds of the LDS and private-array indices of the sweep kernel's core update and quadrature.

A host model of the index arithmetic of update_core, refresh_core and the
quadrature's factor staging in paper_1903_11554_amd/csrc/tt_kernels.hpp: every
index expression is restated with the kernel's loop bounds and checked against
the size of the array it addresses, for every rank bucket, every old and new
rank the kernel admits, and the extreme mode counts.  The staging rule that an
earlier double-double version used (the first factor of a stage admitted
whatever its size) is checked too: it overruns the stage with a rank-64
double-double factor, the cause of a GPU memory fault met while the
double-double path was written; the rule in the kernel does not.
"""
import itertools

import pytest

MAX_RANK, MAX_MODES, WAVE, BLOCK = 64, 1024, 64, 512
STAGE_BYTES = 49152


def chain_block(t_bytes, rmax):
    return 4 if t_bytes != 8 else (16 if rmax in (16, 32) else 8)


def stage_elems(t_bytes):
    """IntSmem::kStage: 48 KiB of T, but never less than one factor of the largest rank."""
    return max(STAGE_BYTES // t_bytes, MAX_RANK * (MAX_RANK + 1))


def pad(r, cb):
    return (r + cb - 1) // cb * cb + 1


@pytest.mark.parametrize("t_bytes", [8, 16])
@pytest.mark.parametrize("rmax", [8, 16, 32, 64])
def test_quadrature_stage_holds_every_factor(t_bytes, rmax):
    cb = chain_block(t_bytes, rmax)
    assert WAVE % cb == 0
    kstage = stage_elems(t_bytes)
    for rl, rr in itertools.product(range(1, rmax + 1), repeat=2):
        assert pad(rl, cb) * rr <= kstage            # one factor always fits a stage
        # chain: v[a0 + u] for a0 < rl in steps of cb, u < cb, within v's 64 entries
        assert (rl + cb - 1) // cb * cb <= WAVE
        # a lane above the rank reads the last column: offset + (rr - 1) pad + a0 + u inside the factor
        assert (rr - 1) * pad(rl, cb) + (rl + cb - 1) // cb * cb <= pad(rl, cb) * rr


def stage_plan(ranks, kstage, cb, admit_first_whatever_size):
    """Factors c0..c1-1 staged together (the binary search of the kernel, or the earlier rule)."""
    m = len(ranks) + 1
    sizes = [pad(ranks[c - 1], cb) * (ranks[c] if c <= m - 2 else 1) for c in range(1, m)]
    plans, c0 = [], 1
    while c0 < m:
        total, c1 = 0, c0
        while c1 < m:
            s = sizes[c1 - 1]
            if total + s > kstage and (c1 > c0 or not admit_first_whatever_size):
                break
            total += s
            c1 += 1
        plans.append((c0, c1, total))
        c0 = c1
    return plans


def test_earlier_double_double_staging_overran_and_the_kernel_rule_does_not():
    ranks = [64] * 8                                 # D_10 at the rank cap 64, double-double
    cb = chain_block(16, 64)
    # the earlier rule: a 6144-double stage, the first factor admitted whatever its size
    old = stage_plan(ranks, 6144 // 2, cb, admit_first_whatever_size=True)
    assert any(total > 6144 // 2 for _, _, total in old)
    new = stage_plan(ranks, stage_elems(16), cb, admit_first_whatever_size=False)
    assert all(total <= stage_elems(16) for _, _, total in new) and new[-1][1] == len(ranks) + 1


@pytest.mark.parametrize("maxm", [0, 4, 8, 10, 12, 16, 24, 32])
@pytest.mark.parametrize("rmax", [8, 16, 32, 64])
def test_update_core_indices(maxm, rmax):
    """LDS of update_core (UpdateSmem) and the register rows of the incremental updates."""
    ld, la = maxm + 1, rmax + 1
    lx_size = MAX_RANK * ld
    a_size = rmax * la
    ms = [m for m in (2, 3, maxm) if maxm == 0 or m <= maxm] if maxm else [2, 40, MAX_MODES]
    for m in ms:
        for c in sorted({0, 1, m // 2, m - 2, m - 1}):
            if not 0 <= c < m:
                continue
            for r_new in range(1, rmax + 1):
                r_old = r_new - 1
                if maxm:   # staged coordinates: left rows k < c, right rows c+1 <= k < m
                    if c > 0:
                        assert (r_new - 1) * ld + (c - 1) < lx_size
                    if c + 1 < m:
                        assert (r_new - 1) * ld + (m - 1) < lx_size
                else:      # streaming C_d: summaries written at rR_old + idx (+ 64, + 128), idx < 1
                    assert 2 * MAX_RANK + r_old + 0 < 3 * MAX_RANK
                # stored LU, zero-padded to rmax; rowidx, u, cp indexed below the old rank
                assert (rmax - 1) * la + rmax - 1 < a_size
                assert r_old < rmax
                # refresh_core: rowidx[r0] = prow only when a pivot was accepted (r0 = r - 1)
                assert r_new - 1 < rmax
                # elimination: A[i * LA + j] for i, j < r; the solves' blocks of four below r
                assert (r_new - 1) * la + (r_new - 1) < a_size
                for q0 in range(0, r_new, 4):
                    for t in range(4):
                        if q0 + t < r_new:
                            assert (q0 + t) * la + q0 + t < a_size
    assert BLOCK // WAVE == 8                        # rv[tid / 64] for 512 threads


def test_register_rows_are_indexed_by_constants():
    """x[RMAX], acc[4]: every access sits in a loop over the compile-time bound (checked in the source)."""
    import os
    import re
    src = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "paper_1903_11554_amd", "csrc", "tt_kernels.hpp")).read()
    body = src[src.index("void refresh_core"):src.index("// ------------------------------------------------------------ k_integral")]
    # every x[...] and acc[...] subscript is a loop variable of a loop bounded by RMAX or kB
    for name, bound in (("x", "RMAX"), ("acc", "kB")):
        for sub in set(re.findall(rf"\b{name}\[([a-z0-9_+ ]+)\]", body)):
            var = sub.strip()
            assert var in ("q", "pp", "a", "bb", "k", "t", "u"), (name, sub)
            assert re.search(rf"for \(int {var} = [^;]+; {var} (<|>=) [^;]*;", body), (name, var)
