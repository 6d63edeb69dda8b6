"""ctypes binding of the stmg C ABI (include/stmg.h).

Argument marshalling only: every step of the solve runs in the HIP library.
Device vectors are contiguous float64 torch tensors on the GPU; torch supplies
memory and the stream, nothing else. Loading fails loudly when the library
has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstmg.so")

STMG_OK, STMG_EINVAL, STMG_ENOMEM, STMG_ENOTCONV, STMG_ENUMERIC, STMG_EHIP, STMG_EAGAIN, STMG_ENOSYS = range(8)
FP64, FP32_REFINED = 0, 1
BC_DIRICHLET, BC_NEUMANN = 0, 1
NODAL_EXACT = 0
NODAL_CHEBYSHEV_MAX = 16
SLAB_EXACT = 0
SLAB_TWOGRID_MAX = 16
BCS = {"dirichlet": BC_DIRICHLET, "neumann": BC_NEUMANN}
SMOOTH_SAS, SMOOTH_S_ONLY, SMOOTH_SA, SMOOTH_AS, SMOOTH_SSA, SMOOTH_ASS, SMOOTH_SSAS, SMOOTH_SSASS = range(8)
SMOOTHERS = {"SAS": SMOOTH_SAS, "SS": SMOOTH_S_ONLY, "SA": SMOOTH_SA, "AS": SMOOTH_AS, "SSA": SMOOTH_SSA,
             "ASS": SMOOTH_ASS, "SSAS": SMOOTH_SSAS, "SSASS": SMOOTH_SSASS}
OP_RESIDUAL, OP_SMOOTH_S, OP_NODAL_A, OP_SAS, OP_SLAB_SOLVE, OP_RESTRICT, OP_PROLONG, OP_VCYCLE = range(8)
MAT_M, MAT_K, MAT_G, MAT_KN, MAT_PE = range(5)


class StmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"stmg error {code}: {msg}")
        self.code = code


class _Mesh(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("coords", C.POINTER(C.c_double)),
                ("n_tets", C.c_int32), ("tets", C.POINTER(C.c_int32)),
                ("vertex_parent", C.POINTER(C.c_int32)), ("tet_parent", C.POINTER(C.c_int32))]


class _Problem(C.Structure):
    _fields_ = [("n_meshes", C.c_int32), ("meshes", C.POINTER(_Mesh)),
                ("sigma", C.POINTER(C.c_double)), ("nu", C.POINTER(C.c_double)),
                ("T", C.c_double), ("Nt", C.c_int32), ("pt", C.c_int32), ("bc", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("omega", C.c_double), ("lambda_crit", C.c_double),
                ("allow_space_coarsening", C.c_int32), ("smoother", C.c_int32),
                ("precision", C.c_int32), ("rtol", C.c_double), ("max_cycles", C.c_int32),
                ("host_only", C.c_int32), ("stream_chunk", C.c_int32), ("row_schedule", C.c_int32),
                ("leaf_size", C.c_int32), ("gemm_rows", C.c_int32), ("factor_transpose", C.c_int32),
                ("gemm_splitk", C.c_int32), ("device_factor", C.c_int32), ("nodal", C.c_int32),
                ("graph", C.c_int32), ("slab", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("rel_res", C.c_double), ("setup_s", C.c_double),
                ("solve_s", C.c_double), ("res_history", C.POINTER(C.c_double))]


class Info(C.Structure):
    _fields_ = [("n_edges", C.c_int32), ("n_levels", C.c_int32), ("pt", C.c_int32),
                ("device_bytes", C.c_int64), ("factor_bytes", C.c_int64)]


class LevelInfo(C.Structure):
    _fields_ = [("mesh", C.c_int32), ("N", C.c_int32), ("tau", C.c_double), ("n_e", C.c_int32),
                ("n_v", C.c_int32), ("nnz_pattern", C.c_int64), ("factor_nnz_slab", C.c_int64),
                ("factor_nnz_nodal", C.c_int64), ("n_supernodes_slab", C.c_int32),
                ("lambda_", C.c_double), ("factor_nnz_slab_struct", C.c_int64),
                ("factor_nnz_nodal_struct", C.c_int64), ("slab_factor_mesh", C.c_int32),
                ("slab_steps", C.c_int32)]


class ServerOptions(C.Structure):
    _fields_ = [("hbm_budget", C.c_int64), ("max_active", C.c_int32), ("setup_threads", C.c_int32),
                ("batch", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("active", C.c_int64), ("pending", C.c_int64), ("p50_s", C.c_double), ("p99_s", C.c_double),
                ("mean_s", C.c_double), ("throughput_req_s", C.c_double), ("throughput_dofs", C.c_double),
                ("hbm_reserved", C.c_int64), ("hbm_peak", C.c_int64), ("hbm_budget", C.c_int64),
                ("batched_iterations", C.c_int64), ("batched_members", C.c_int64)]


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"stmg HIP library not built: {LIB_PATH} is missing "
                              "(run __graft_entry__.build() or python -m paper_1911_09548_amd.build)")
        # torch's HIP runtime must be the one the library binds to: stream
        # handles and device pointers come from torch. Importing torch first
        # makes the loader resolve the library's libamdhip64.so.7 to torch's
        # already-loaded copy instead of a second runtime.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.c_int32
        L.stmg_strerror.restype = C.c_char_p
        L.stmg_strerror.argtypes = [C.c_int]
        L.stmg_last_error_message.restype = C.c_char_p
        L.stmg_default_options.argtypes = [C.POINTER(Options)]
        L.stmg_setup.argtypes = [C.POINTER(_Problem), C.POINTER(Options), vp, C.POINTER(vp)]
        L.stmg_destroy.argtypes = [vp]
        L.stmg_info.argtypes = [vp, C.POINTER(Info)]
        L.stmg_level_info.argtypes = [vp, ip, C.POINTER(LevelInfo)]
        L.stmg_edges.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.POINTER(C.c_int32))]
        L.stmg_solve.argtypes = [vp, vp, vp, vp, vp, C.POINTER(Report)]
        L.stmg_load.argtypes = [vp, vp, vp, vp, dp]
        L.stmg_cycles.argtypes = [vp, ip, dp]
        L.stmg_store.argtypes = [vp, vp]
        L.stmg_residual.argtypes = [vp, vp, vp, vp, vp]
        L.stmg_residual_noalloc.argtypes = [vp, vp, vp, vp, vp]
        L.stmg_level_apply.argtypes = [vp, ip, ip, vp, vp, vp]
        L.stmg_export_matrix.argtypes = [vp, ip, ip, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                         C.POINTER(C.c_int64), vp, vp, vp]
        L.stmg_export_factor.argtypes = [vp, ip, ip] + [vp] * 11
        L.stmg_server_default_options.argtypes = [C.POINTER(ServerOptions)]
        L.stmg_server_create.argtypes = [C.POINTER(ServerOptions), C.POINTER(vp)]
        L.stmg_submit.argtypes = [vp, C.POINTER(_Problem), C.POINTER(Options), vp, vp, C.POINTER(C.c_uint64)]
        L.stmg_poll.argtypes = [vp, C.c_uint64, vp, C.POINTER(Report)]
        L.stmg_server_wait.argtypes = [vp, C.c_uint64, C.c_double]
        L.stmg_server_stats.argtypes = [vp, C.POINTER(ServerStats)]
        L.stmg_server_destroy.argtypes = [vp]
        L.stmg_profile.argtypes = [vp, ip]
        L.stmg_set_stream_tuning.argtypes = [vp, ip, ip]
        L.stmg_vcycle.argtypes = [vp, vp, vp]
        L.stmg_cycles_batched.argtypes = [C.POINTER(vp), ip, ip, dp]
        L.stmg_debug_fail_alloc.argtypes = [C.c_int64]
        L.stmg_debug_fail_alloc.restype = C.c_int64
        L.stmg_power_rate.argtypes = [vp, vp, ip, C.c_double, dp, dp, C.POINTER(C.c_int32)]
        L.stmg_profile_count.argtypes = [vp, C.POINTER(C.c_int32)]
        L.stmg_profile_get.argtypes = [vp, ip, C.c_char_p, ip, C.POINTER(C.c_int64), dp, dp, dp]
        for name in ("stmg_setup", "stmg_info", "stmg_level_info", "stmg_edges", "stmg_solve",
                     "stmg_load", "stmg_cycles", "stmg_store", "stmg_power_rate", "stmg_residual",
                     "stmg_residual_noalloc", "stmg_vcycle", "stmg_cycles_batched",
                     "stmg_level_apply", "stmg_export_matrix", "stmg_export_factor", "stmg_profile",
                     "stmg_profile_count", "stmg_profile_get", "stmg_set_stream_tuning", "stmg_server_create",
                     "stmg_submit", "stmg_poll", "stmg_server_wait", "stmg_server_stats"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def debug_fail_alloc(k):
    """Arm the k-th library allocation to fail (k <= 0 disarms); returns the
    allocations counted since the previous call."""
    return int(lib().stmg_debug_fail_alloc(int(k)))


def cycles_batched(solvers, n):
    """n iterations of several loaded solvers at once with merged solves;
    returns the [len(solvers)][n] relative residuals."""
    hs = (C.c_void_p * len(solvers))(*[s_._h.value for s_ in solvers])
    res = np.zeros((len(solvers), max(1, n)))
    _check(lib().stmg_cycles_batched(hs, len(solvers), n, res.ctypes.data_as(C.POINTER(C.c_double))))
    return res[:, :n]


def default_options(**kw) -> Options:
    o = Options()
    lib().stmg_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _check(rc, allow=()):
    if rc != STMG_OK and rc not in allow:
        L = lib()
        raise StmgError(rc, f"{L.stmg_strerror(rc).decode()}: {L.stmg_last_error_message().decode()}")
    return rc


def _ptr(t):
    """Device pointer of a contiguous float64 tensor (or None)."""
    if t is None:
        return None
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


def _marshal_problem(problem, keep):
    """Build the C problem struct; arrays are appended to `keep`."""
    meshes = (_Mesh * len(problem.levels))()
    for j, lev in enumerate(problem.levels):
        c = np.ascontiguousarray(lev.coords, dtype=np.float64)
        t = np.ascontiguousarray(lev.tets, dtype=np.int32)
        keep += [c, t]
        meshes[j].n_vertices = c.shape[0]
        meshes[j].coords = c.ctypes.data_as(C.POINTER(C.c_double))
        meshes[j].n_tets = t.shape[0]
        meshes[j].tets = t.ctypes.data_as(C.POINTER(C.c_int32))
        if j > 0:
            vp = np.ascontiguousarray(lev.vertex_parent, dtype=np.int32)
            tp = np.ascontiguousarray(lev.tet_parent, dtype=np.int32)
            keep += [vp, tp]
            meshes[j].vertex_parent = vp.ctypes.data_as(C.POINTER(C.c_int32))
            meshes[j].tet_parent = tp.ctypes.data_as(C.POINTER(C.c_int32))
    sig = np.ascontiguousarray(problem.sigma, dtype=np.float64)
    nu = np.ascontiguousarray(problem.nu, dtype=np.float64)
    keep += [sig, nu, meshes]
    return _Problem(len(problem.levels), meshes, sig.ctypes.data_as(C.POINTER(C.c_double)),
                    nu.ctypes.data_as(C.POINTER(C.c_double)), float(problem.T), int(problem.Nt),
                    int(problem.pt), BCS[getattr(problem, "bc", "dirichlet")])


class Server:
    """Continuous-batching request server (see stmg_server_* in include/stmg.h)."""

    def __init__(self, hbm_budget=0, max_active=16, setup_threads=4, batch=True):
        o = ServerOptions(int(hbm_budget), int(max_active), int(setup_threads), 1 if batch else 0)
        h = C.c_void_p()
        _check(lib().stmg_server_create(C.byref(o), C.byref(h)))
        self._h = h

    def submit(self, problem, rhs, u0=None, **opts):
        """rhs: host array [Nt][pt+1][n_edges] (float64); returns a ticket."""
        keep = []
        p = _marshal_problem(problem, keep)
        o = default_options(**opts)
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        u0 = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64)
        t = C.c_uint64()
        _check(lib().stmg_submit(self._h, C.byref(p), C.byref(o), C.c_void_p(rhs.ctypes.data),
                                 None if u0 is None else C.c_void_p(u0.ctypes.data), C.byref(t)))
        return t.value

    def wait(self, ticket, timeout=600.0):
        return lib().stmg_server_wait(self._h, ticket, float(timeout)) == STMG_OK

    def poll(self, ticket, shape=None):
        """(status, x or None, report); status STMG_EAGAIN while running."""
        x = np.zeros(shape, dtype=np.float64) if shape is not None else None
        rep = Report()
        rc = lib().stmg_poll(self._h, ticket, None if x is None else C.c_void_p(x.ctypes.data), C.byref(rep))
        if rc == STMG_EAGAIN:
            return rc, None, None
        return rc, x, dict(cycles=rep.cycles, rel_res=rep.rel_res, setup_s=rep.setup_s, solve_s=rep.solve_s)

    def stats(self):
        st = ServerStats()
        _check(lib().stmg_server_stats(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().stmg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """One space-time problem set up on the GPU (or host-only for inspection)."""

    def __init__(self, problem, stream=None, **opts):
        self._keep = []
        p = _marshal_problem(problem, self._keep)
        self.options = default_options(**opts)
        self.host_only = bool(self.options.host_only)
        if stream is None and not self.host_only:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        h = C.c_void_p()
        _check(lib().stmg_setup(C.byref(p), C.byref(self.options), C.c_void_p(stream or 0), C.byref(h)))
        self._h = h
        self.Nt, self.pt, self.q = int(problem.Nt), int(problem.pt), int(problem.pt) + 1
        self.info = Info()
        _check(lib().stmg_info(h, C.byref(self.info)))
        self.n_edges = self.info.n_edges

    def close(self):
        if getattr(self, "_h", None):
            lib().stmg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- inspection ------------------------------------------------------
    def level_info(self, level):
        li = LevelInfo()
        _check(lib().stmg_level_info(self._h, level, C.byref(li)))
        return li

    @property
    def n_levels(self):
        return self.info.n_levels

    def edges(self):
        n = C.c_int32()
        p = C.POINTER(C.c_int32)()
        _check(lib().stmg_edges(self._h, C.byref(n), C.byref(p)))
        return np.ctypeslib.as_array(p, shape=(n.value, 2)).copy()

    def export_matrix(self, level, which):
        import scipy.sparse as sp
        nr, ncl, nnz = C.c_int32(), C.c_int32(), C.c_int64()
        _check(lib().stmg_export_matrix(self._h, level, which, C.byref(nr), C.byref(ncl), C.byref(nnz),
                                        None, None, None))
        ptr = np.zeros(nr.value + 1, dtype=np.int64)
        col = np.zeros(nnz.value, dtype=np.int32)
        val = np.zeros(nnz.value, dtype=np.float64)
        _check(lib().stmg_export_matrix(self._h, level, which, C.byref(nr), C.byref(ncl), C.byref(nnz),
                                        C.c_void_p(ptr.ctypes.data), C.c_void_p(col.ctypes.data),
                                        C.c_void_p(val.ctypes.data)))
        return sp.csr_matrix((val, col, ptr), shape=(nr.value, ncl.value))

    def profile(self, enable=True):
        _check(lib().stmg_profile(self._h, 1 if enable else 0))

    def set_stream_tuning(self, stream_chunk=0, row_schedule=0):
        """Residual launch shape on the live handle (see the options of the same names)."""
        _check(lib().stmg_set_stream_tuning(self._h, stream_chunk, row_schedule))

    def profile_report(self):
        """Per-kernel launch statistics gathered since profile(True)."""
        n = C.c_int32()
        _check(lib().stmg_profile_count(self._h, C.byref(n)))
        out = []
        for i in range(n.value):
            name = C.create_string_buffer(128)
            la, ms, fl, by = C.c_int64(), C.c_double(), C.c_double(), C.c_double()
            _check(lib().stmg_profile_get(self._h, i, name, 128, C.byref(la), C.byref(ms), C.byref(fl),
                                          C.byref(by)))
            out.append(dict(kernel=name.value.decode(), launches=la.value, ms=ms.value, flops=fl.value,
                            bytes=by.value))
        return sorted(out, key=lambda d: -d["ms"])

    def export_factor(self, level, which):
        """Host copy of a factor (host factors, or a device handle's FP64 panels): dict of numpy arrays."""
        n, ns, nr, npan, cpx = C.c_int32(), C.c_int32(), C.c_int64(), C.c_int64(), C.c_int32()
        refs = [C.byref(x) for x in (n, ns, nr, npan, cpx)]
        _check(lib().stmg_export_factor(self._h, level, which, *refs, *([None] * 6)))
        out = dict(perm=np.zeros(n.value, np.int32), col0=np.zeros(ns.value + 1, np.int32),
                   rptr=np.zeros(ns.value + 1, np.int64), rows=np.zeros(nr.value, np.int32),
                   panel_off=np.zeros(ns.value + 1, np.int64),
                   panel=np.zeros(npan.value * (2 if cpx.value else 1), np.float64))
        ptrs = [C.c_void_p(out[k].ctypes.data) for k in ("perm", "col0", "rptr", "rows", "panel_off", "panel")]
        _check(lib().stmg_export_factor(self._h, level, which, *refs, *ptrs))
        if cpx.value:
            out["panel"] = out["panel"].view(np.complex128)
        out["complex"] = bool(cpx.value)
        return out

    # -- solving ---------------------------------------------------------
    def _full(self):
        import torch
        return torch.zeros((self.Nt, self.q, self.n_edges), dtype=torch.float64, device="cuda")

    def solve(self, rhs, u0=None, x0=None, out=None, allow_notconv=False):
        x = self._full() if out is None else out
        rep = Report()
        rc = lib().stmg_solve(self._h, _ptr(rhs), _ptr(u0), _ptr(x0), _ptr(x), C.byref(rep))
        _check(rc, allow=(STMG_ENOTCONV,) if allow_notconv else ())
        hist = [rep.res_history[i] for i in range(rep.cycles)]
        return x, dict(cycles=rep.cycles, rel_res=rep.rel_res, setup_s=rep.setup_s,
                       solve_s=rep.solve_s, history=hist, status=rc)

    def load(self, rhs, u0=None, x0=None):
        bn = C.c_double()
        _check(lib().stmg_load(self._h, _ptr(rhs), _ptr(u0), _ptr(x0), C.byref(bn)))
        return bn.value

    def cycles(self, n, want_residuals=True):
        res = np.zeros(max(1, n)) if want_residuals else None
        _check(lib().stmg_cycles(self._h, n, res.ctypes.data_as(C.POINTER(C.c_double))
                                 if want_residuals else None))
        return res[:n] if want_residuals else None

    def vcycle(self, rhs, x):
        """One V-cycle (or refinement step) on x in place (enqueued only)."""
        _check(lib().stmg_vcycle(self._h, _ptr(rhs), _ptr(x)))
        return x

    def power_rate(self, x0, max_cycles=200, underflow=1e-100):
        """Power iteration (section 5.1): V-cycles with zero right-hand side
        from the error x0 (full layout, device). Returns (largest reduction
        factor, list of per-cycle factors)."""
        rates = np.zeros(max_cycles)
        rate, done = C.c_double(), C.c_int32()
        _check(lib().stmg_power_rate(self._h, _ptr(x0), max_cycles, underflow, C.byref(rate),
                                     rates.ctypes.data_as(C.POINTER(C.c_double)), C.byref(done)))
        return rate.value, list(rates[:done.value])

    def store(self, out=None):
        x = self._full() if out is None else out
        _check(lib().stmg_store(self._h, _ptr(x)))
        return x

    def residual(self, x, rhs, u0=None):
        r = self._full()
        _check(lib().stmg_residual(self._h, _ptr(x), _ptr(rhs), _ptr(u0), _ptr(r)))
        return r

    def residual_noalloc(self, x, rhs, out, u0=None):
        """r = b - L x into `out` without device allocation (enqueued only)."""
        _check(lib().stmg_residual_noalloc(self._h, _ptr(x), _ptr(rhs), _ptr(u0), _ptr(out)))
        return out

    def level_apply(self, level, op, vin, vin2=None):
        import torch
        li = self.level_info(level)
        if op == OP_RESTRICT:
            lo = self.level_info(level + 1)
        elif op == OP_PROLONG:
            lo = self.level_info(level - 1)
        else:
            lo = li
        out = torch.zeros((lo.N, self.q, lo.n_e), dtype=torch.float64, device="cuda")
        _check(lib().stmg_level_apply(self._h, level, op, _ptr(vin), _ptr(vin2), _ptr(out)))
        return out
