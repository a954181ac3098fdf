"""Python binding of libcdcs.so (argument marshalling only).

Every step of the ADMM iteration runs in the library's HIP kernels; this
module converts instance records to the C structs of include/cdcs.h, calls
the entry points of the same names, and raises on negative return codes.
There is no CPU fallback: importing this module on a machine without the
built library, or calling the solver without a GPU, raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcdcs.so")

RUNNING, SOLVED, PRIMAL_INFEASIBLE, DUAL_INFEASIBLE, MAX_ITER = 0, 1, 2, 3, 4
STATUS_NAMES = {0: "running", 1: "solved", 2: "primal_infeasible", 3: "dual_infeasible", 4: "max_iter"}

_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_dp = C.POINTER(C.c_double)


class Problem(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("m", C.c_int32),
        ("c_nnz", C.c_int64), ("c_row", _i32p), ("c_col", _i32p), ("c_val", _dp),
        ("a_nnz", C.c_int64), ("a_con", _i32p), ("a_row", _i32p), ("a_col", _i32p), ("a_val", _dp),
        ("b", _dp),
        ("p", C.c_int32), ("clique_ptr", _i32p), ("clique_vtx", _i32p), ("clique_parent", _i32p),
    ]


class Settings(C.Structure):
    _fields_ = [("eps_tol", C.c_double), ("max_iter", C.c_int32), ("check_every", C.c_int32),
                ("timing", C.c_int32), ("use_graph", C.c_int32), ("eig_fp32", C.c_int32),
                ("autotune", C.c_int32), ("alpha", C.c_double), ("eig_warm", C.c_int32),
                ("method", C.c_int32), ("rho", C.c_double), ("jacobi_max", C.c_int32),
                ("band_min", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("iter", C.c_int32), ("status", C.c_int32),
                ("eps_p", C.c_double), ("eps_d", C.c_double), ("eps_g", C.c_double),
                ("obj_p", C.c_double), ("obj_d", C.c_double),
                ("tau", C.c_double), ("kappa", C.c_double), ("cx", C.c_double), ("by", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


ABI_VERSION = 6   # the layout of the structures above

SELF_DUAL, PRIMAL, DUAL = 0, 1, 2   # settings.method

EXPORTS = [
    "cdcs_default_settings", "cdcs_setup", "cdcs_setup_batch", "cdcs_iterate", "cdcs_solve",
    "cdcs_get_dims", "cdcs_get_entries", "cdcs_get_solution", "cdcs_get_certificate",
    "cdcs_get_state", "cdcs_set_state", "cdcs_get_phase_times", "cdcs_reset_phase_times",
    "cdcs_psd_project", "cdcs_psd_project_noalloc", "cdcs_adjoint", "cdcs_get_adjoint_info", "cdcs_get_tuning", "cdcs_last_error", "cdcs_abi_version",
    "cdcs_destroy",
]


class CDCSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cdcs error {code}: {msg}")
        self.code = code


_lib = None


def _hip_runtime():
    """The HIP runtime library the process shares with PyTorch-ROCm.

    torch ships its own libamdhip64.so; loading it (by path) before the
    solver library makes both use one runtime, so device pointers and
    streams from torch are valid in the solver.
    """
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec and spec.origin:
        p = os.path.join(os.path.dirname(spec.origin), "lib", "libamdhip64.so")
        if os.path.exists(p):
            return p
    return None


def load(path: str = LIB_PATH):
    """Load libcdcs.so and declare its signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_1611_01828_amd.build`")
    rt = _hip_runtime()
    if rt:
        C.CDLL(rt, mode=C.RTLD_GLOBAL)
    lib = C.CDLL(path)
    vp = C.c_void_p
    hp = C.POINTER(vp)
    lib.cdcs_default_settings.argtypes = [C.POINTER(Settings)]
    lib.cdcs_default_settings.restype = None
    lib.cdcs_setup.argtypes = [C.POINTER(Problem), C.POINTER(Settings), vp, hp]
    lib.cdcs_setup_batch.argtypes = [C.c_int32, C.POINTER(Problem), C.POINTER(Settings), vp, hp]
    lib.cdcs_iterate.argtypes = [vp, C.c_int32, C.POINTER(Info)]
    lib.cdcs_solve.argtypes = [vp, C.POINTER(Info)]
    lib.cdcs_get_dims.argtypes = [vp, C.c_int32, _i64p]
    lib.cdcs_get_entries.argtypes = [vp, C.c_int32, _i32p, _i32p]
    lib.cdcs_get_solution.argtypes = [vp, C.c_int32, vp, vp, vp, C.c_int32]
    lib.cdcs_get_certificate.argtypes = [vp, C.c_int32, vp, vp, C.c_int32]
    lib.cdcs_get_state.argtypes = [vp, C.c_int32, _dp, _dp]
    lib.cdcs_set_state.argtypes = [vp, C.c_int32, _dp, _dp]
    lib.cdcs_get_phase_times.argtypes = [vp, C.POINTER(C.c_char_p), _dp, _i64p, C.c_int32]
    lib.cdcs_get_tuning.argtypes = [vp, C.POINTER(C.c_int32), C.c_int32]
    lib.cdcs_reset_phase_times.argtypes = [vp]
    lib.cdcs_psd_project.argtypes = [C.c_int32, _i32p, _i64p, vp, vp, vp]
    lib.cdcs_psd_project_noalloc.argtypes = [C.c_int32, _i32p, _i64p, vp, vp, vp]
    lib.cdcs_get_adjoint_info.argtypes = [vp, _dp, _i32p]
    lib.cdcs_adjoint.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_int32, C.c_double, C.POINTER(C.c_int32)]
    lib.cdcs_last_error.restype = C.c_char_p
    lib.cdcs_last_error.argtypes = []
    lib.cdcs_abi_version.restype = C.c_int
    lib.cdcs_destroy.argtypes = [vp]
    lib.cdcs_destroy.restype = None
    for name in EXPORTS:
        if name not in ("cdcs_default_settings", "cdcs_last_error", "cdcs_destroy", "cdcs_abi_version"):
            getattr(lib, name).restype = C.c_int
    if lib.cdcs_abi_version() != ABI_VERSION:
        raise ImportError(f"{path} has ABI version {lib.cdcs_abi_version()}, this binding needs "
                          f"{ABI_VERSION}; rebuild with `python -m paper_1611_01828_amd.build`")
    _lib = lib
    return lib


def _check(rc):
    if rc < 0:
        raise CDCSError(rc, load().cdcs_last_error().decode())
    return rc


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


class _ProblemData:
    """Keeps the numpy arrays a Problem struct points to alive."""

    def __init__(self, inst):
        self.n, self.m = int(inst.n), int(inst.m)
        cr, cc, cv = inst.C
        self.cr = np.ascontiguousarray(cr, dtype=np.int32)
        self.cc = np.ascontiguousarray(cc, dtype=np.int32)
        self.cv = np.ascontiguousarray(cv, dtype=np.float64)
        con, ar, ac, av = inst.A
        self.acon = np.ascontiguousarray(con, dtype=np.int32)
        self.ar = np.ascontiguousarray(ar, dtype=np.int32)
        self.ac = np.ascontiguousarray(ac, dtype=np.int32)
        self.av = np.ascontiguousarray(av, dtype=np.float64)
        self.b = np.ascontiguousarray(inst.b, dtype=np.float64)
        cl = [np.asarray(c, dtype=np.int32) for c in inst.cliques]
        self.cptr = np.zeros(len(cl) + 1, dtype=np.int32)
        self.cptr[1:] = np.cumsum([len(c) for c in cl])
        self.cvtx = np.ascontiguousarray(np.concatenate(cl) if cl else np.zeros(0, np.int32), dtype=np.int32)
        par = getattr(inst, "parent", None)
        self.par = None if par is None else np.ascontiguousarray(par, dtype=np.int32)

    def struct(self):
        p = Problem()
        p.n, p.m = self.n, self.m
        p.c_nnz = len(self.cv)
        p.c_row, p.c_col, p.c_val = _ptr(self.cr, C.c_int32), _ptr(self.cc, C.c_int32), _ptr(self.cv, C.c_double)
        p.a_nnz = len(self.av)
        p.a_con, p.a_row = _ptr(self.acon, C.c_int32), _ptr(self.ar, C.c_int32)
        p.a_col, p.a_val = _ptr(self.ac, C.c_int32), _ptr(self.av, C.c_double)
        p.b = _ptr(self.b, C.c_double)
        p.p = len(self.cptr) - 1
        p.clique_ptr, p.clique_vtx = _ptr(self.cptr, C.c_int32), _ptr(self.cvtx, C.c_int32)
        p.clique_parent = _ptr(self.par, C.c_int32) if self.par is not None else None
        return p


def default_settings(**kw) -> Settings:
    s = Settings()
    load().cdcs_default_settings(C.byref(s))
    for k, v in kw.items():
        setattr(s, k, v)
    return s


class Solver:
    """A (batched) solve living on the GPU: the HSDE-ADMM (method = SELF_DUAL,
    the default) or the primal-only / dual-only ADMM (method = PRIMAL / DUAL)."""

    def __init__(self, instances, settings: Settings | None = None, stream=None, **kw):
        lib = load()
        if not isinstance(instances, (list, tuple)):
            instances = [instances]
        self.count = len(instances)
        data = [_ProblemData(i) for i in instances]
        arr = (Problem * self.count)(*[d.struct() for d in data])
        self.settings = settings or default_settings(**kw)
        h = C.c_void_p()
        st = C.c_void_p(stream) if stream else None
        _check(lib.cdcs_setup_batch(self.count, arr, C.byref(self.settings), st, C.byref(h)))
        self.h = h
        self._dims = []
        for i in range(self.count):
            d = (C.c_int64 * 4)()
            _check(lib.cdcs_get_dims(self.h, i, d))
            self._dims.append(tuple(int(x) for x in d))

    def close(self):
        if getattr(self, "h", None):
            load().cdcs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dims(self, i=0):
        """(nE, ns, m, p) of instance i."""
        return self._dims[i]

    def state_len(self, i=0):
        nE, ns, m, _ = self._dims[i]
        return nE + 2 * ns + m + 1

    def iterate(self, k=1):
        infos = (Info * self.count)()
        _check(load().cdcs_iterate(self.h, int(k), infos))
        return [x.as_dict() for x in infos]

    def solve(self):
        infos = (Info * self.count)()
        _check(load().cdcs_solve(self.h, infos))
        return [x.as_dict() for x in infos]

    def entries(self, i=0):
        nE = self._dims[i][0]
        r = np.empty(nE, np.int32)
        c = np.empty(nE, np.int32)
        _check(load().cdcs_get_entries(self.h, i, _ptr(r, C.c_int32), _ptr(c, C.c_int32)))
        return r, c

    def get_state(self, i=0):
        """(u, v~) of the self-dual method; (x, s, y), lam of the primal-only
        method; (x, z, y), (lam, v) of the dual-only method."""
        nE, ns, m, _ = self._dims[i]
        if self.settings.method == SELF_DUAL:
            u, vt = np.empty(self.state_len(i)), np.empty(self.state_len(i))
        else:
            u = np.empty(nE + ns + m)
            vt = np.empty(ns if self.settings.method == PRIMAL else 2 * ns)
        _check(load().cdcs_get_state(self.h, i, _ptr(u, C.c_double), _ptr(vt, C.c_double)))
        return u, vt

    def set_state(self, u, vt, i=0):
        u = np.ascontiguousarray(u, dtype=np.float64)
        vt = np.ascontiguousarray(vt, dtype=np.float64)
        _check(load().cdcs_set_state(self.h, i, _ptr(u, C.c_double), _ptr(vt, C.c_double)))

    def solution(self, i=0):
        nE, ns, m, _ = self._dims[i]
        X, y, Z = np.empty(nE), np.empty(m), np.empty(nE)
        _check(load().cdcs_get_solution(self.h, i, X.ctypes.data, y.ctypes.data, Z.ctypes.data, 0))
        return X, y, Z

    def certificate(self, i=0):
        nE, ns, m, _ = self._dims[i]
        y = np.full(m, np.nan)
        X = np.full(nE, np.nan)
        _check(load().cdcs_get_certificate(self.h, i, y.ctypes.data, X.ctypes.data, 0))
        return y, X

    def adjoint(self, dX, max_iter=20000, tol=1e-12):
        """dL/dc (svec over E', all instances concatenated) and dL/db for
        dL/dX = dX (numpy arrays on the host)."""
        NE = sum(d[0] for d in self._dims)
        M = sum(d[2] for d in self._dims)
        dX = np.ascontiguousarray(dX, dtype=np.float64)
        assert dX.shape == (NE,)
        dc = np.empty(NE)
        db = np.empty(M)
        it = C.c_int32()
        _check(load().cdcs_adjoint(self.h, dX.ctypes.data, dc.ctypes.data, db.ctypes.data, 0,
                                   int(max_iter), float(tol), C.byref(it)))
        return dc, db, it.value

    def adjoint_device(self, dX, dc, db, max_iter=20000, tol=1e-12):
        """As adjoint(), on torch CUDA tensors (float64)."""
        it = C.c_int32()
        _check(load().cdcs_adjoint(self.h, C.c_void_p(dX.data_ptr()), C.c_void_p(dc.data_ptr()),
                                   C.c_void_p(db.data_ptr()), 1, int(max_iter), float(tol), C.byref(it)))
        return it.value

    def adjoint_info(self):
        """Per instance of the last adjoint: (final relative residual, reason),
        reason 0 = within tol, 1 = stalled, 2 = iteration limit."""
        r = np.empty(self.count)
        why = np.empty(self.count, np.int32)
        _check(load().cdcs_get_adjoint_info(self.h, _ptr(r, C.c_double), _ptr(why, C.c_int32)))
        return r, why

    def phase_times(self):
        cap = 64
        names = (C.c_char_p * cap)()
        ms = (C.c_double * cap)()
        n = (C.c_int64 * cap)()
        k = _check(load().cdcs_get_phase_times(self.h, names, ms, n, cap))
        return {names[i].decode(): (ms[i], n[i]) for i in range(min(k, cap))}

    def reset_phase_times(self):
        _check(load().cdcs_reset_phase_times(self.h))

    def tuning(self):
        """Jacobi tile shape per clique-size bucket: list of dicts
        (kmax, threads, cliques, tuned)."""
        out = (C.c_int32 * 16)()
        n = _check(load().cdcs_get_tuning(self.h, out, 16))
        return [dict(kmax=out[4 * b], threads=out[4 * b + 1], cliques=out[4 * b + 2], tuned=bool(out[4 * b + 3]))
                for b in range(n)]


def psd_project(sizes, offsets, inp, out, stream=None):
    """Project packed blocks (torch CUDA tensors, float64) onto their PSD cones."""
    sizes = np.ascontiguousarray(sizes, dtype=np.int32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    _check(load().cdcs_psd_project(len(sizes), _ptr(sizes, C.c_int32), _ptr(offsets, C.c_int64),
                                   C.c_void_p(inp.data_ptr()), C.c_void_p(out.data_ptr()),
                                   C.c_void_p(stream) if stream else None))


def psd_project_noalloc(sizes, offsets, inp, out, stream=None):
    """psd_project through the entry point that allocates no device memory
    (its scratch is a fixed array in the library, shared by every call on a GPU)."""
    sizes = np.ascontiguousarray(sizes, dtype=np.int32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    _check(load().cdcs_psd_project_noalloc(len(sizes), _ptr(sizes, C.c_int32), _ptr(offsets, C.c_int64),
                                           C.c_void_p(inp.data_ptr()), C.c_void_p(out.data_ptr()),
                                           C.c_void_p(stream) if stream else None))
