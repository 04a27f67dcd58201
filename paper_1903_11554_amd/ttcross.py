"""ctypes binding of libttcross.so (include/ttcross.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  There is no CPU fallback: without the built library or a GPU the
calls raise.  PyTorch is used only to hand device buffers (and optionally its
current stream) to the library.
"""
import ctypes
import os

import numpy as np

from .workloads import Problem

HERE = os.path.dirname(os.path.abspath(__file__))

FAMILY_IDS = {
    "ising_c": 1, "ising_d": 2, "ising_e": 3,
    "ising_c_u": 11, "ising_d_u": 12,
    "prod_exp": 21, "sum2_exp_cos": 22,
}
STOP_REASONS = {0: "running", 1: "converged", 2: "rank_cap", 3: "max_sweeps", 4: "error"}
PRECISION_IDS = {"fp64": 0, "dd": 1, "qd": 2}

TT_OK, TT_CONVERGED, TT_NOT_CONVERGED, TT_PENDING = 0, 1, 2, 3
TT_EINVAL, TT_ENOMEM, TT_EDEVICE, TT_ENUMERIC = -1, -2, -3, -4


class TTError(RuntimeError):
    """A negative tt_status.  `infos` holds the per-integral infos when the call filled them
    (TT_ENUMERIC from tt_cross_sweep / tt_cross_run: an integral stopped on a numeric error)."""

    def __init__(self, status, what, infos=None):
        self.status = status
        self.infos = infos
        super().__init__(f"{what}: {_status_name(status)} ({status})")


class _Problem(ctypes.Structure):
    _fields_ = [("integrand", ctypes.c_int32), ("d", ctypes.c_int32),
                ("n_nodes", ctypes.c_int32), ("rank_cap", ctypes.c_int32),
                ("tol", ctypes.c_double), ("precision", ctypes.c_int32),
                ("max_sweeps", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("params", ctypes.POINTER(ctypes.c_double)),
                ("stop_rule", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _TuneResult(ctypes.Structure):
    _fields_ = [("mode_bucket", ctypes.c_int32), ("rank_policy", ctypes.c_int32),
                ("rule_mode_bucket", ctypes.c_int32), ("candidates", ctypes.c_int32),
                ("matching", ctypes.c_int32), ("search_group", ctypes.c_int32),
                ("rule_ms", ctypes.c_double), ("tuned_ms", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("max_rank", ctypes.c_int32),
                ("reason", ctypes.c_int32), ("err_flags", ctypes.c_int32),
                ("evals", ctypes.c_int64), ("value", ctypes.c_double),
                ("rel_change", ctypes.c_double), ("value_lo", ctypes.c_double),
                ("value_mant", ctypes.c_double), ("value_exp2", ctypes.c_int32),
                ("recomputes", ctypes.c_int32), ("value_scale", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("running", ctypes.c_int64),
                ("max_running", ctypes.c_int64), ("sweep_launches", ctypes.c_int64),
                ("admissions", ctypes.c_int64), ("busy_s", ctypes.c_double)]


class _Pivot(ctypes.Structure):
    _fields_ = [("row", ctypes.c_int32), ("col", ctypes.c_int32),
                ("accepted", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("err", ctypes.c_double), ("value", ctypes.c_double),
                ("col_fresh", ctypes.c_int32), ("reserved", ctypes.c_int32)]


EXPORTS = [
    "tt_ctx_create", "tt_ctx_destroy", "tt_ctx_synchronize", "tt_job_footprint",
    "tt_cross_init", "tt_cross_sweep", "tt_cross_run", "tt_cross_integrate",
    "tt_job_pivot_log", "tt_job_history", "tt_job_index_sets", "tt_job_nodes",
    "tt_cross_free", "tt_eval_points", "tt_eval_fibers", "tt_status_string",
    "tt_ctx_profile", "tt_ctx_set_search_group", "tt_ctx_kernel_time", "tt_job_phase_times",
    "tt_server_create", "tt_server_submit", "tt_server_poll", "tt_server_wait",
    "tt_server_get_stats", "tt_server_destroy", "tt_cross_enqueue", "tt_mc_integrate",
    "tt_mc_integrate_noalloc", "tt_job_core", "tt_batch_run", "tt_autotune", "tt_cross_refresh",
    "tt_job_history_parts", "tt_job_nodes_parts",
]

STOP_RULE_IDS = {"rel2": 0, "strict": 1}   # tt_stop_rule
KERNEL_KINDS = {"sweep": 0, "update": 1, "integral": 2, "start": 3, "gl": 4,
                "eval_points": 5, "eval_fibers": 6, "mc": 7, "refresh": 8}
MC_RANDOM, MC_LATTICE = 0, 1

_lib = None


def library_path():
    return os.environ.get("TTCROSS_LIB", os.path.join(HERE, "libttcross.so"))


def load_library():
    """Load libttcross.so and declare the C signatures (no GPU needed to load)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"libttcross.so not built at {path}: run `python -m paper_1903_11554_amd.build`")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "tt_ctx_create": (i32, [ctypes.c_int, vp, P(vp)]),
        "tt_ctx_destroy": (None, [vp]),
        "tt_ctx_synchronize": (i32, [vp]),
        "tt_job_footprint": (ctypes.c_size_t, [P(_Problem)]),
        "tt_cross_init": (i32, [vp, P(_Problem), i32, P(vp)]),
        "tt_cross_sweep": (i32, [vp, i32, P(_Info)]),
        "tt_cross_run": (i32, [vp, P(_Info)]),
        "tt_cross_integrate": (i32, [vp, P(dbl), P(_Info)]),
        "tt_job_pivot_log": (i32, [vp, i32, P(_Pivot), i64, P(i64)]),
        "tt_job_history": (i32, [vp, i32, P(dbl), P(dbl), P(i32), i64, P(i64)]),
        "tt_job_index_sets": (i32, [vp, i32, P(i32), P(i32), i64, P(i64)]),
        "tt_job_nodes": (i32, [vp, i32, P(dbl), P(dbl), P(dbl), P(dbl)]),
        "tt_cross_free": (None, [vp]),
        "tt_eval_points": (i32, [vp, P(_Problem), vp, i64, vp]),
        "tt_eval_fibers": (i32, [vp, P(_Problem), i32, vp, i32, vp, i32, vp]),
        "tt_status_string": (ctypes.c_char_p, [i32]),
        "tt_ctx_profile": (i32, [vp, i32]),
        "tt_ctx_set_search_group": (i32, [vp, i32]),
        "tt_ctx_kernel_time": (i32, [vp, i32, P(i64), P(dbl)]),
        "tt_job_phase_times": (i32, [vp, i32, P(i64), i64, P(i64), P(dbl)]),
        "tt_server_create": (i32, [vp, ctypes.c_size_t, i32, P(vp)]),
        "tt_server_submit": (i32, [vp, P(_Problem), P(ctypes.c_uint64)]),
        "tt_server_poll": (i32, [vp, ctypes.c_uint64, P(_Info), P(dbl)]),
        "tt_server_wait": (i32, [vp, ctypes.c_uint64, P(_Info), P(dbl)]),
        "tt_server_get_stats": (i32, [vp, P(_ServerStats)]),
        "tt_server_destroy": (None, [vp]),
        "tt_cross_enqueue": (i32, [vp, i32]),
        "tt_mc_integrate": (i32, [vp, P(_Problem), i32, i64, i32, P(i64), P(dbl), P(dbl), P(dbl)]),
        "tt_mc_integrate_noalloc": (i32, [vp, P(_Problem), i32, i64, i32, P(i64), vp]),
        "tt_job_core": (i32, [vp, i32, i32, P(dbl), P(dbl), i64, P(i32), P(i32)]),
        "tt_batch_run": (i32, [vp, P(_Problem), i32, P(_Info)]),
        "tt_autotune": (i32, [vp, P(_Problem), i32, i32, P(_TuneResult)]),
        "tt_cross_refresh": (i32, [vp, P(_Info)]),
        "tt_job_history_parts": (i32, [vp, i32, i32, P(ctypes.c_double), P(i32), i64, P(i64)]),
        "tt_job_nodes_parts": (i32, [vp, i32, i32, P(ctypes.c_double), P(ctypes.c_double)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _status_name(status):
    try:
        return load_library().tt_status_string(status).decode()
    except Exception:  # noqa: BLE001 - only used to format an error message
        return str(status)


def _check(status, what):
    if status < 0:
        raise TTError(status, what)
    return status


def _c_problem(p: Problem, keep):
    params = None
    if p.params is not None:
        arr = np.ascontiguousarray(np.concatenate([np.asarray(p.params["a"], np.float64)[:p.d],
                                                   np.asarray(p.params["b"], np.float64)[:p.d]]))
        keep.append(arr)
        params = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return _Problem(FAMILY_IDS[p.family], p.d, p.n, p.rank_cap, float(p.tol), PRECISION_IDS[p.precision],
                    int(p.max_sweeps), int(p.seed) & ((1 << 64) - 1), params, STOP_RULE_IDS[p.stop], 0)


def footprint(p: Problem):
    keep = []
    return int(load_library().tt_job_footprint(ctypes.byref(_c_problem(p, keep))))


class Context:
    """A device + stream.  stream: a torch.cuda.Stream (its handle is passed) or None."""

    def __init__(self, device=0, stream=None):
        lib = load_library()
        self._lib = lib
        handle = ctypes.c_void_p()
        sptr = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
        _check(lib.tt_ctx_create(device, sptr, ctypes.byref(handle)), "tt_ctx_create")
        self.handle = handle

    def close(self):
        if self.handle:
            self._lib.tt_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def synchronize(self):
        _check(self._lib.tt_ctx_synchronize(self.handle), "tt_ctx_synchronize")

    def profile(self, enable=True):
        """Switch per-kernel event timing on/off (clears the totals)."""
        _check(self._lib.tt_ctx_profile(self.handle, 1 if enable else 0), "tt_ctx_profile")

    def set_search_group(self, group):
        """Workgroups per superblock search for later double jobs (0: the rule; results are identical)."""
        _check(self._lib.tt_ctx_set_search_group(self.handle, int(group)), "tt_ctx_set_search_group")

    def kernel_time(self, kind):
        """(launches, total_ms) of a kernel kind since profiling was switched on."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(self._lib.tt_ctx_kernel_time(self.handle, KERNEL_KINDS[kind], ctypes.byref(n),
                                            ctypes.byref(ms)), "tt_ctx_kernel_time")
        return n.value, ms.value

    def job(self, problems):
        return Job(self, problems)

    def mc_integrate(self, p: Problem, n_points, n_sets, kind=MC_RANDOM, gen=None):
        """Monte Carlo / shifted lattice estimators: (estimates, mean, relative error)."""
        keep = []
        est = (ctypes.c_double * n_sets)()
        mean, err = ctypes.c_double(), ctypes.c_double()
        g = None
        if gen is not None:
            g = (ctypes.c_int64 * len(gen))(*[int(v) for v in gen])
        _check(self._lib.tt_mc_integrate(self.handle, ctypes.byref(_c_problem(p, keep)), kind, n_points,
                                         n_sets, g, est, ctypes.byref(mean), ctypes.byref(err)),
               "tt_mc_integrate")
        return list(est), mean.value, err.value

    def mc_integrate_noalloc(self, p: Problem, n_points, n_sets, out_dev, kind=MC_RANDOM, gen=None):
        """The estimators of mc_integrate with no allocation: estimates, mean and relative error
        are written to the device array out_dev (n_sets + 2 doubles) on the context stream."""
        keep = []
        g = None
        if gen is not None:
            g = (ctypes.c_int64 * len(gen))(*[int(v) for v in gen])
        _check(self._lib.tt_mc_integrate_noalloc(self.handle, ctypes.byref(_c_problem(p, keep)), kind,
                                                 n_points, n_sets, g, ctypes.c_void_p(out_dev)),
               "tt_mc_integrate_noalloc")

    def batch_run(self, problems):
        """tt_batch_run: solve the problems together in one call; the infos of all of them."""
        keep = []
        arr = (_Problem * len(problems))(*[_c_problem(p, keep) for p in problems])
        infos = (_Info * len(problems))()
        st = self._lib.tt_batch_run(self.handle, arr, len(problems), infos)
        if st == TT_ENUMERIC:
            raise TTError(st, "tt_batch_run", Job._info_dicts(infos))
        _check(st, "tt_batch_run")
        return Job._info_dicts(infos)

    def autotune(self, problems, reps=3):
        """tt_autotune: time the kernel variants of this job, record the fastest bit-identical one."""
        keep = []
        arr = (_Problem * len(problems))(*[_c_problem(p, keep) for p in problems])
        res = _TuneResult()
        _check(self._lib.tt_autotune(self.handle, arr, len(problems), reps, ctypes.byref(res)), "tt_autotune")
        return {f: getattr(res, f) for f, _ in _TuneResult._fields_}

    def server(self, max_bytes=1 << 30, max_active=256):
        return Server(self, max_bytes, max_active)

    def eval_points(self, p: Problem, idx_dev, out_dev, npts):
        """B at npts multi-indices; idx_dev / out_dev are device pointers (ints).

        out_dev holds npts doubles, or 2*npts ((hi, lo) pairs) for precision "dd"."""
        keep = []
        _check(self._lib.tt_eval_points(self.handle, ctypes.byref(_c_problem(p, keep)),
                                        ctypes.c_void_p(idx_dev), npts, ctypes.c_void_p(out_dev)),
               "tt_eval_points")

    def eval_fibers(self, p: Problem, pos, left_dev, r_left, right_dev, r_right, out_dev):
        keep = []
        _check(self._lib.tt_eval_fibers(self.handle, ctypes.byref(_c_problem(p, keep)), pos,
                                        ctypes.c_void_p(left_dev), r_left,
                                        ctypes.c_void_p(right_dev), r_right,
                                        ctypes.c_void_p(out_dev)), "tt_eval_fibers")


class Job:
    """A batch of integrals solved together (tt_cross_init ... tt_cross_free)."""

    def __init__(self, ctx: Context, problems):
        if isinstance(problems, Problem):
            problems = [problems]
        self.ctx, self._lib = ctx, ctx._lib
        self.problems = list(problems)
        keep = []
        arr = (_Problem * len(self.problems))(*[_c_problem(p, keep) for p in self.problems])
        handle = ctypes.c_void_p()
        _check(self._lib.tt_cross_init(ctx.handle, arr, len(self.problems), ctypes.byref(handle)),
               "tt_cross_init")
        self.handle = handle

    def free(self):
        if self.handle:
            self._lib.tt_cross_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def _infos(self):
        return (_Info * len(self.problems))()

    @staticmethod
    def _info_dicts(infos):
        return [dict(sweeps=i.sweeps, max_rank=i.max_rank, reason=STOP_REASONS.get(i.reason, i.reason),
                     err_flags=i.err_flags, evals=i.evals, value=i.value, rel_change=i.rel_change,
                     value_lo=i.value_lo, value_mant=i.value_mant, value_exp2=i.value_exp2,
                     recomputes=i.recomputes, value_scale=i.value_scale)
                for i in infos]

    def _checked_infos(self, status, infos, what):
        if status == TT_ENUMERIC:
            raise TTError(status, what, self._info_dicts(infos))
        return _check(status, what)

    def sweep(self, n=1):
        infos = self._infos()
        st = self._checked_infos(self._lib.tt_cross_sweep(self.handle, n, infos), infos, "tt_cross_sweep")
        return st == TT_CONVERGED, self._info_dicts(infos)

    def refresh(self):
        """tt_cross_refresh: one ALS maxvol refresh of the index sets (Alg. 3) at fixed ranks."""
        infos = self._infos()
        self._checked_infos(self._lib.tt_cross_refresh(self.handle, infos), infos, "tt_cross_refresh")
        return self._info_dicts(infos)

    def enqueue(self, n=1):
        """Enqueue n sweeps without waiting (capturable into a HIP graph)."""
        _check(self._lib.tt_cross_enqueue(self.handle, n), "tt_cross_enqueue")

    def run(self):
        """Sweep to the stopping rule; raises TTError (with .infos) if an integral stopped on an error."""
        infos = self._infos()
        self._checked_infos(self._lib.tt_cross_run(self.handle, infos), infos, "tt_cross_run")
        return self._info_dicts(infos)

    def values(self):
        vals = (ctypes.c_double * len(self.problems))()
        infos = self._infos()
        _check(self._lib.tt_cross_integrate(self.handle, vals, infos), "tt_cross_integrate")
        return list(vals), self._info_dicts(infos)

    def pivot_log(self, k):
        p = self.problems[k]
        nb = max(p.modes() - 1, 0)
        cap = max(1, nb * (p.max_sweeps if p.max_sweeps > 0 else 4 * p.rank_cap))
        buf = (_Pivot * cap)()
        written = ctypes.c_int64()
        _check(self._lib.tt_job_pivot_log(self.handle, k, buf, cap, ctypes.byref(written)),
               "tt_job_pivot_log")
        recs = [dict(row=r.row, col=r.col, accepted=bool(r.accepted), iters=r.iters, err=r.err,
                     value=r.value, col_fresh=bool(r.col_fresh)) for r in buf[:written.value]]
        return [recs[s * nb:(s + 1) * nb] for s in range(written.value // nb)] if nb else []

    def history(self, k):
        return self.history_dd(k)[0]

    def history_parts(self, k, parts=4):
        """[([components], exponent)]: the integral after the start and every sweep is
        sum(components) * 2^exponent (4 components of a quad-double job)."""
        p = self.problems[k]
        cap = (p.max_sweeps if p.max_sweeps > 0 else 4 * p.rank_cap) + 1
        vals = (ctypes.c_double * (cap * parts))()
        ex = (ctypes.c_int32 * cap)()
        n = ctypes.c_int64()
        _check(self._lib.tt_job_history_parts(self.handle, k, parts, vals, ex, cap, ctypes.byref(n)),
               "tt_job_history_parts")
        return [(list(vals[q * parts:(q + 1) * parts]), ex[q]) for q in range(n.value)]

    def nodes_parts(self, k, parts=4):
        """(t, w): the unscaled nodes and weights, `parts` components each."""
        n = self.problems[k].n
        t = (ctypes.c_double * (n * parts))()
        w = (ctypes.c_double * (n * parts))()
        _check(self._lib.tt_job_nodes_parts(self.handle, k, parts, t, w), "tt_job_nodes_parts")
        return ([list(t[i * parts:(i + 1) * parts]) for i in range(n)],
                [list(w[i * parts:(i + 1) * parts]) for i in range(n)])

    def history_dd(self, k):
        """(leading doubles, low doubles) of the integral after the start and every sweep."""
        p = self.problems[k]
        cap = (p.max_sweeps if p.max_sweeps > 0 else 4 * p.rank_cap) + 1
        buf = (ctypes.c_double * cap)()
        lo = (ctypes.c_double * cap)()
        written = ctypes.c_int64()
        _check(self._lib.tt_job_history(self.handle, k, buf, lo, None, cap, ctypes.byref(written)),
               "tt_job_history")
        return list(buf[:written.value]), list(lo[:written.value])

    def history_scaled(self, k):
        """[(mantissa, exponent)]: the integral after the start and every sweep is mantissa * 2^exponent."""
        p = self.problems[k]
        cap = (p.max_sweeps if p.max_sweeps > 0 else 4 * p.rank_cap) + 1
        buf = (ctypes.c_double * cap)()
        ex = (ctypes.c_int32 * cap)()
        written = ctypes.c_int64()
        _check(self._lib.tt_job_history(self.handle, k, buf, None, ex, cap, ctypes.byref(written)),
               "tt_job_history")
        return [(buf[q], ex[q]) for q in range(written.value)]

    def index_sets(self, k):
        """[(left rows, right rows)] per bond, each a list of tuples of node indices."""
        p = self.problems[k]
        m = p.modes()
        nb = max(m - 1, 0)
        if nb == 0:
            return []
        ranks = (ctypes.c_int32 * nb)()
        cap = nb * p.rank_cap * m
        nodes = (ctypes.c_int32 * cap)()
        written = ctypes.c_int64()
        _check(self._lib.tt_job_index_sets(self.handle, k, ranks, nodes, cap, ctypes.byref(written)),
               "tt_job_index_sets")
        out, pos = [], 0
        for b in range(nb):
            r = ranks[b]
            left = [tuple(nodes[pos + a * (b + 1): pos + (a + 1) * (b + 1)]) for a in range(r)]
            pos += r * (b + 1)
            w = m - b - 1
            right = [tuple(nodes[pos + a * w: pos + (a + 1) * w]) for a in range(r)]
            pos += r * w
            out.append((left, right))
        return out

    def phase_times(self, k):
        """(marks[sweep, row, 16], clock MHz) of the sweep kernel, or None if not profiled.

        Rows: the m-1 superblocks, then the m cores."""
        p = self.problems[k]
        nb = max(p.modes() - 1, 0)
        rows = nb + p.modes() if nb > 0 else 0
        ms = p.max_sweeps if p.max_sweeps > 0 else 4 * p.rank_cap
        cap = max(1, ms * rows * 16)
        buf = (ctypes.c_int64 * cap)()
        written = ctypes.c_int64()
        mhz = ctypes.c_double()
        _check(self._lib.tt_job_phase_times(self.handle, k, buf, cap, ctypes.byref(written),
                                            ctypes.byref(mhz)), "tt_job_phase_times")
        if written.value == 0:
            return None
        arr = np.array(buf[:written.value], dtype=np.int64).reshape(-1, rows, 16)
        return arr, mhz.value

    def core(self, k, c):
        """(F_c, C_c) of integral k at the current ranks as (r_{c-1} n) x r_c arrays (C_c None for the last core)."""
        p = self.problems[k]
        cap = p.rank_cap * p.n * p.rank_cap
        F = (ctypes.c_double * cap)()
        C = (ctypes.c_double * cap)()
        rows, cols = ctypes.c_int32(), ctypes.c_int32()
        _check(self._lib.tt_job_core(self.handle, k, c, F, C, cap, ctypes.byref(rows), ctypes.byref(cols)),
               "tt_job_core")
        nr, nc = rows.value, cols.value
        f = np.array(F[:nr * nc]).reshape(nr, nc)
        cc = np.array(C[:nr * nc]).reshape(nr, nc) if c < p.modes() - 1 else None
        return f, cc

    def nodes(self, k):
        """(t, w) rounded to double."""
        return self.nodes_dd(k)[:2]

    def nodes_dd(self, k):
        """(t, w, t_lo, w_lo): the device's double-double node and weight tables."""
        n = self.problems[k].n
        t, w, tl, wl = [(ctypes.c_double * n)() for _ in range(4)]
        _check(self._lib.tt_job_nodes(self.handle, k, t, w, tl, wl), "tt_job_nodes")
        return np.array(t[:]), np.array(w[:]), np.array(tl[:]), np.array(wl[:])


class Server:
    """Continuous-batching serving loop (tt_server_*): submit integrals as they arrive."""

    def __init__(self, ctx: Context, max_bytes=1 << 30, max_active=256):
        self.ctx, self._lib = ctx, ctx._lib
        handle = ctypes.c_void_p()
        _check(self._lib.tt_server_create(ctx.handle, max_bytes, max_active, ctypes.byref(handle)),
               "tt_server_create")
        self.handle = handle

    def submit(self, p: Problem):
        keep = []
        t = ctypes.c_uint64()
        _check(self._lib.tt_server_submit(self.handle, ctypes.byref(_c_problem(p, keep)), ctypes.byref(t)),
               "tt_server_submit")
        return t.value

    def _result(self, fn, ticket):
        info = _Info()
        lat = ctypes.c_double()
        st = _check(fn(self.handle, ticket, ctypes.byref(info), ctypes.byref(lat)), "tt_server result")
        if st == TT_PENDING:
            return None
        return Job._info_dicts([info])[0], lat.value

    def poll(self, ticket):
        """(info, latency_s) once done, else None."""
        return self._result(self._lib.tt_server_poll, ticket)

    def wait(self, ticket):
        return self._result(self._lib.tt_server_wait, ticket)

    def stats(self):
        st = _ServerStats()
        _check(self._lib.tt_server_get_stats(self.handle, ctypes.byref(st)), "tt_server_get_stats")
        return {f: getattr(st, f) for f, _ in _ServerStats._fields_}

    def close(self):
        if self.handle:
            self._lib.tt_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass
