"""MI355X-native tensor-train cross integration (Dolgov & Savostyanov, arXiv:1903.11554).

Python binding over the C ABI of ``include/ttcross.h`` (``libttcross.so``,
hand-written gfx950 HIP kernels).  The binding only marshals arguments; every
step of the method runs in the library's kernels.  Importing this package does
not need a GPU; creating a context does, and fails loudly without one or
without the built library.
"""
from .ttcross import (Context, Job, Problem, Server, TTError, FAMILY_IDS, STOP_REASONS,  # noqa: F401
                      library_path, load_library)

__all__ = ["Context", "Job", "Problem", "Server", "TTError", "FAMILY_IDS", "STOP_REASONS",
           "library_path", "load_library"]
