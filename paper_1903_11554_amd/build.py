"""Build the gfx950 HIP library in-tree (hipcc, no JIT cache).

The library is the host translation units ``csrc/ttcross.hip`` (job API) and
``csrc/tt_server.hip`` (serving loop) plus one kernel
translation unit per integrand class (``csrc/tt_inst.hip`` compiled with
-DTT_FAM=0..3, and once more with -DTT_INST_DD=1 for the double-double kernels of
the paper-form class), compiled in parallel for gfx950 only, with floating-point
contraction off (every FMA is written in the source) and packed-FP32
instructions disabled, then linked into ``libttcross.so``.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libttcross.so")
OBJDIR = os.path.join(HERE, "_build")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unused-value", "-Wno-pass-failed",
]

UNITS = [("ttcross.hip", [], "ttcross.o"), ("tt_server.hip", [], "tt_server.o")] + [
    ("tt_inst.hip", [f"-DTT_FAM={f}"], f"tt_inst_{f}.o") for f in range(4)] + [
    ("tt_inst.hip", ["-DTT_FAM=0", "-DTT_INST_DD=1"], "tt_inst_dd.o"),
    ("tt_inst.hip", ["-DTT_FAM=0", "-DTT_INST_QD=1"], "tt_inst_qd.o")]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with status {res.returncode}: {' '.join(cmd)}")


def build(verbose=False):
    """Compile libttcross.so next to this file; raises on failure."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = []
    for src, defs, obj in UNITS:
        jobs.append([hipcc, *FLAGS, *defs, "-c", "-o", os.path.join(OBJDIR, obj), os.path.join(CSRC, src)])
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(lambda c: _run(c, verbose), jobs))
    tmp = LIB + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
          *[os.path.join(OBJDIR, o) for _, _, o in UNITS]], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
