"""ctypes binding of libcutbddc.so (include/cutbddc.h).

Argument marshalling only: every step of setup, factorisation and solve runs
in the library's HIP kernels.  Device buffers are torch tensors on the GPU;
the library reads and writes them through their data pointers on the
current torch stream.  There is no CPU fallback: without the built library
or a GPU the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcutbddc.so")

CB_OK = 0
CB_ERR_ARG = -1
CB_ERR_SINGULAR = -2
CB_ERR_NOT_SPD = -3
CB_ERR_NO_CONVERGENCE = -4
CB_ERR_DEVICE = -5
CB_ERR_STATE = -6
CB_ERR_OOM = -7
_NAMES = {0: "CB_OK", -1: "CB_ERR_ARG", -2: "CB_ERR_SINGULAR", -3: "CB_ERR_NOT_SPD",
          -4: "CB_ERR_NO_CONVERGENCE", -5: "CB_ERR_DEVICE", -6: "CB_ERR_STATE", -7: "CB_ERR_OOM"}


class CBError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class cb_problem(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("sub_cells", C.c_int32), ("n_balls", C.c_int32),
                ("ball_centres", C.POINTER(C.c_double)), ("ball_radii", C.POINTER(C.c_double)),
                ("kappa", C.POINTER(C.c_double)), ("weighting", C.c_int32), ("objects", C.c_int32),
                ("coarse_variant", C.c_int32), ("local_precision", C.c_int32),
                ("full_elements", C.c_int32), ("cut_boundary", C.c_int32)]


class cb_info(C.Structure):
    _fields_ = [("n_dof", C.c_int64), ("n_active", C.c_int64), ("n_cut", C.c_int64),
                ("n_cut_stored", C.c_int64),
                ("n_sub", C.c_int32), ("n_coarse", C.c_int32), ("n_objects", C.c_int32),
                ("n_iface", C.c_int32), ("max_local_dofs", C.c_int32),
                ("max_coarse_per_sub", C.c_int32), ("n_fp64_fallbacks", C.c_int32),
                ("factored", C.c_int32), ("sum_nI2", C.c_int64), ("sum_nG2", C.c_int64),
                ("sum_nI", C.c_int64), ("sum_nG", C.c_int64), ("flops_local_chol", C.c_double),
                ("t_integrate_ms", C.c_double),
                ("t_topology_ms", C.c_double), ("t_factor_ms", C.c_double),
                ("t_solve_ms", C.c_double), ("sum_nGnC", C.c_int64), ("n_nodes", C.c_int64),
                ("lanczos_lmin", C.c_double), ("lanczos_lmax", C.c_double),
                ("coarse_separator", C.c_int32), ("coarse_octant_max", C.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with paper_1703_06323_amd.build.build()")
    lib = C.CDLL(path)
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)
    lib.cb_setup.argtypes = [C.POINTER(cb_problem), vp, C.POINTER(vp)]
    lib.cb_factor.argtypes = [vp]
    lib.cb_solve.argtypes = [vp, vp, vp, C.c_double, C.c_int32, ip, dp]
    lib.cb_solve_rhs.argtypes = [vp, vp, vp, C.c_double, C.c_int32, ip, dp]
    lib.cb_grad.argtypes = [vp, vp, vp, vp, vp]
    lib.cb_apply_operator.argtypes = [vp, vp, vp]
    lib.cb_apply_preconditioner.argtypes = [vp, vp, vp]
    lib.cb_load.argtypes = [vp, vp, vp]
    lib.cb_query.argtypes = [vp, C.POINTER(cb_info)]
    lib.cb_pcg_history.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, vp, ip, dp, dp]
    lib.cb_lanczos_extremes.argtypes = [C.c_int32, vp, vp, dp, dp]
    lib.cb_manufactured_load.argtypes = [vp, dp, C.c_double, vp]
    lib.cb_manufactured_errors.argtypes = [vp, dp, C.c_double, vp, dp, dp]
    lib.cb_export_indexing.argtypes = [vp] + [vp] * 8
    lib.cb_export_problem_indexing.argtypes = [vp, C.c_int32] + [vp] * 8
    lib.cb_export_subdomains.argtypes = [vp, C.c_int32, vp, vp]
    lib.cb_export_cut_matrices.argtypes = [vp, vp, vp, vp]
    lib.cb_export_coarse.argtypes = [vp, vp]
    lib.cb_host_indexing.argtypes = [C.POINTER(cb_problem), vp, C.POINTER(cb_info)] + [vp] * 6
    lib.cb_profile.argtypes = [vp, C.c_int32]
    lib.cb_profile_time.argtypes = [vp, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.cb_profile_launches.argtypes = [vp, C.c_char_p, vp, C.c_int64, C.POINTER(C.c_int64)]
    lib.cb_time_kernel.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(C.c_double)]
    lib.cb_dense_spd_inverse.argtypes = [C.c_int32, C.c_int32, C.c_int32, vp, vp]
    lib.cb_setup_batch.argtypes = [C.POINTER(cb_problem), C.c_int32, vp, C.POINTER(vp)]
    lib.cb_solve_batch.argtypes = [vp, vp, vp, C.c_double, C.c_int32, ip, dp]
    lib.cb_query_problem.argtypes = [vp, C.c_int32, C.POINTER(cb_info)]
    lib.cb_last_error.restype = C.c_char_p
    lib.cb_destroy.argtypes = [vp]
    lib.cb_destroy.restype = None
    for name in ("cb_setup", "cb_factor", "cb_solve", "cb_solve_rhs", "cb_grad",
                 "cb_apply_operator", "cb_apply_preconditioner", "cb_load", "cb_query",
                 "cb_export_indexing", "cb_export_problem_indexing", "cb_export_subdomains",
                 "cb_export_cut_matrices", "cb_export_coarse",
                 "cb_dense_spd_inverse", "cb_profile", "cb_profile_time", "cb_host_indexing",
                 "cb_setup_batch", "cb_solve_batch", "cb_query_problem", "cb_profile_launches",
                 "cb_time_kernel"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(rc, allow=()):
    if rc != CB_OK and rc not in allow:
        raise CBError(rc, _lib.cb_last_error().decode())
    return rc


def _dptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Solver:
    """One cut-cube problem resident on the GPU.

    `problem` needs the attributes n, s, centres (n_b x 3), radii (n_b),
    kappa (n^3 or None), weighting, objects, coarse_variant,
    local_precision and full_elements."""

    def __init__(self, problem, stream=None):
        import torch
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("cutbddc needs a GPU")
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device())
        centres = np.ascontiguousarray(problem.centres, dtype=np.float64).reshape(-1)
        radii = np.ascontiguousarray(problem.radii, dtype=np.float64)
        kappa = None if problem.kappa is None else np.ascontiguousarray(problem.kappa, dtype=np.float64)
        self._keep = (centres, radii, kappa)
        P = C.POINTER(C.c_double)
        p = cb_problem(int(problem.n), int(problem.s), int(radii.size),
                       centres.ctypes.data_as(P), radii.ctypes.data_as(P),
                       kappa.ctypes.data_as(P) if kappa is not None else None,
                       int(problem.weighting), int(problem.objects), int(problem.coarse_variant),
                       int(problem.local_precision), int(problem.full_elements),
                       int(getattr(problem, "cut_boundary", 0)))
        st = torch.cuda.current_stream() if stream is None else stream
        self.stream = st
        ctx = C.c_void_p()
        _check(lib.cb_setup(C.byref(p), C.c_void_p(st.cuda_stream), C.byref(ctx)))
        self.ctx = ctx
        self.n = int(problem.n)
        self._n_dof = None

    def __del__(self):
        if getattr(self, "ctx", None) and _lib is not None:
            _lib.cb_destroy(self.ctx)
            self.ctx = None

    def close(self):
        self.__del__()

    # -- phases ------------------------------------------------------------
    def factor(self):
        _check(_lib.cb_factor(self.ctx))

    def info(self) -> dict:
        inf = cb_info()
        _check(_lib.cb_query(self.ctx, C.byref(inf)))
        return {k: getattr(inf, k) for k, _ in cb_info._fields_}

    @property
    def n_dof(self) -> int:
        # fixed at setup
        if self._n_dof is None:
            self._n_dof = int(self.info()["n_dof"])
        return self._n_dof

    def _vec(self, n):
        return self.torch.empty(n, dtype=self.torch.float64, device=self.device)

    def _f64(self, t):
        t = self.torch.as_tensor(t, dtype=self.torch.float64, device=self.device)
        return t.contiguous()

    def solve(self, f=None, rtol=1e-8, max_iter=1000, allow_no_convergence=False):
        """Returns (u [n_dof] cuda tensor, iterations, relative residual)."""
        u = self._vec(self.n_dof)
        it = C.c_int32(0)
        rel = C.c_double(0.0)
        fv = None if f is None else self._f64(f)
        rc = _lib.cb_solve(self.ctx, _dptr(fv), u.data_ptr(), float(rtol), int(max_iter),
                           C.byref(it), C.byref(rel))
        _check(rc, allow=(CB_ERR_NO_CONVERGENCE,) if allow_no_convergence else ())
        return u, int(it.value), float(rel.value)

    def solve_rhs(self, b, rtol=1e-8, max_iter=1000, allow_no_convergence=False):
        bv = self._f64(b)
        u = self._vec(self.n_dof)
        it = C.c_int32(0)
        rel = C.c_double(0.0)
        rc = _lib.cb_solve_rhs(self.ctx, bv.data_ptr(), u.data_ptr(), float(rtol), int(max_iter),
                               C.byref(it), C.byref(rel))
        _check(rc, allow=(CB_ERR_NO_CONVERGENCE,) if allow_no_convergence else ())
        return u, int(it.value), float(rel.value)

    def grad(self, u, lam):
        """(dJ/dtheta [n^3], dJ/df [(n+1)^3]) for the adjoint lam."""
        dth = self._vec(self.n ** 3)
        df = self._vec((self.n + 1) ** 3)
        _check(_lib.cb_grad(self.ctx, self._f64(u).data_ptr(), self._f64(lam).data_ptr(),
                            dth.data_ptr(), df.data_ptr()))
        return dth, df

    def apply_operator(self, x):
        y = self._vec(self.n_dof)
        _check(_lib.cb_apply_operator(self.ctx, self._f64(x).data_ptr(), y.data_ptr()))
        return y

    def apply_preconditioner(self, r):
        z = self._vec(self.n_dof)
        _check(_lib.cb_apply_preconditioner(self.ctx, self._f64(r).data_ptr(), z.data_ptr()))
        return z

    def load(self, f=None):
        b = self._vec(self.n_dof)
        fv = None if f is None else self._f64(f)
        _check(_lib.cb_load(self.ctx, _dptr(fv), b.data_ptr()))
        return b

    def pcg_history(self) -> dict:
        """The last solve's PCG record (cb_pcg_history)."""
        return _pcg_history(self.ctx, 0)

    def manufactured_load(self, x0=(0.0, 0.0, 0.0), k=5.0 * np.pi):
        """Load [n_dof] of the exact solution sin(k |x - x0|) (volume, surface
        data and the Dirichlet lift moved to the right)."""
        b = self._vec(self.n_dof)
        xv = (C.c_double * 3)(*[float(v) for v in x0])
        _check(_lib.cb_manufactured_load(self.ctx, xv, float(k), b.data_ptr()))
        return b

    def manufactured_errors(self, u, x0=(0.0, 0.0, 0.0), k=5.0 * np.pi):
        """(L2 error, H1-seminorm error) of u [n_dof] plus the lift."""
        xv = (C.c_double * 3)(*[float(v) for v in x0])
        l2 = C.c_double(0.0)
        h1 = C.c_double(0.0)
        _check(_lib.cb_manufactured_errors(self.ctx, xv, float(k), self._f64(u).data_ptr(), C.byref(l2), C.byref(h1)))
        return float(l2.value), float(h1.value)

    PROFILE_GROUPS = ("apply_interior", "apply_neumann", "apply_A", "coarse_gemv",
                      "local_cholesky", "local_inverse", "coarse_factor")

    def profile(self, enable=True):
        _check(_lib.cb_profile(self.ctx, 1 if enable else 0))

    def profile_times(self) -> dict:
        """{group: (total_ms, launches)} of the bracketed kernel groups."""
        return _profile_times(self.ctx, self.PROFILE_GROUPS)

    def time_kernel(self, which: str, reps: int = 20) -> float:
        """Average launch duration (ms) of "apply_interior" or "apply_neumann"
        over `reps` back-to-back launches (cb_time_kernel)."""
        code = {"apply_interior": 0, "apply_neumann": 1}[which]
        ms = C.c_double()
        _check(_lib.cb_time_kernel(self.ctx, code, int(reps), C.byref(ms)))
        return ms.value

    def profile_launches(self, name: str) -> np.ndarray:
        """Durations (ms) of every bracketed launch of one kernel group."""
        return _profile_launches(self.ctx, name)

    # -- host exports --------------------------------------------------------
    def export_indexing(self) -> dict:
        return _export_indexing(self.ctx, None, self.n, self.info())

    def export_subdomains(self):
        """(sub_ptr, sub_dofs): local DOFs of every subdomain, ascending."""
        return _export_subdomains(self.ctx, 0, int(self.info()["n_sub"]))

    def export_cut_matrices(self):
        n = int(self.info()["n_cut_stored"])
        K = np.zeros((max(n, 1), 36))
        M = np.zeros((max(n, 1), 36))
        cells = np.zeros(max(n, 1), np.int64)
        _check(_lib.cb_export_cut_matrices(self.ctx, K.ctypes.data_as(C.c_void_p),
                                           M.ctypes.data_as(C.c_void_p),
                                           cells.ctypes.data_as(C.c_void_p)))
        return K[:n], M[:n], cells[:n]

    def export_coarse(self) -> np.ndarray:
        nc = int(self.info()["n_coarse"])
        A = np.zeros((nc, nc))
        _check(_lib.cb_export_coarse(self.ctx, A.ctypes.data_as(C.c_void_p)))
        return A


class BatchSolver:
    """Many independent cut-cube problems in one context: setup, factor and
    PCG of all of them run as shared kernel launches (cb_setup_batch,
    cb_solve_batch).  The problems must share s and every option."""

    def __init__(self, problems, stream=None):
        import torch
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("cutbddc needs a GPU")
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device())
        n = len(problems)
        arr = (cb_problem * n)()
        self._keep = []
        Pd = C.POINTER(C.c_double)
        for k, problem in enumerate(problems):
            centres = np.ascontiguousarray(problem.centres, dtype=np.float64).reshape(-1)
            radii = np.ascontiguousarray(problem.radii, dtype=np.float64)
            kappa = None if problem.kappa is None else np.ascontiguousarray(problem.kappa, dtype=np.float64)
            self._keep.append((centres, radii, kappa))
            arr[k] = cb_problem(int(problem.n), int(problem.s), int(radii.size), centres.ctypes.data_as(Pd),
                                radii.ctypes.data_as(Pd), kappa.ctypes.data_as(Pd) if kappa is not None else None,
                                int(problem.weighting), int(problem.objects), int(problem.coarse_variant),
                                int(problem.local_precision), int(problem.full_elements),
                                int(getattr(problem, "cut_boundary", 0)))
        st = torch.cuda.current_stream() if stream is None else stream
        self.stream = st
        ctx = C.c_void_p()
        _check(lib.cb_setup_batch(arr, n, C.c_void_p(st.cuda_stream), C.byref(ctx)))
        self.ctx = ctx
        self.size = n
        self.ns = [int(p.n) for p in problems]

    def __del__(self):
        if getattr(self, "ctx", None) and _lib is not None:
            _lib.cb_destroy(self.ctx)
            self.ctx = None

    def close(self):
        self.__del__()

    def factor(self):
        _check(_lib.cb_factor(self.ctx))

    def info(self) -> dict:
        inf = cb_info()
        _check(_lib.cb_query(self.ctx, C.byref(inf)))
        return {k: getattr(inf, k) for k, _ in cb_info._fields_}

    def problem_info(self, k: int) -> dict:
        inf = cb_info()
        _check(_lib.cb_query_problem(self.ctx, int(k), C.byref(inf)))
        return {kk: getattr(inf, kk) for kk, _ in cb_info._fields_}

    def n_dofs(self):
        return [int(self.problem_info(k)["n_dof"]) for k in range(self.size)]

    def export_indexing(self, k: int) -> dict:
        return _export_indexing(self.ctx, int(k), self.ns[k], self.problem_info(k))

    def profile(self, enable=True):
        _check(_lib.cb_profile(self.ctx, 1 if enable else 0))

    def profile_launches(self, name: str) -> np.ndarray:
        return _profile_launches(self.ctx, name)

    def profile_times(self) -> dict:
        """{group: (total_ms, launches)} of the bracketed kernel groups."""
        return _profile_times(self.ctx, Solver.PROFILE_GROUPS)

    def pcg_history(self, k: int) -> dict:
        """The last solve's PCG record of problem k (cb_pcg_history)."""
        return _pcg_history(self.ctx, int(k))

    def export_subdomains(self, k: int):
        return _export_subdomains(self.ctx, int(k), int(self.problem_info(k)["n_sub"]))

    def solve(self, fs=None, rtol=1e-8, max_iter=1000, outputs=None, allow_no_convergence=False):
        """fs: list of cuda float64 tensors [(N_k+1)^3] (or None entries / None
        for f = 1).  Returns (list of u_k [n_dof_k], iterations [n],
        relative residuals [n])."""
        n = self.size
        if outputs is None:
            outputs = [self.torch.empty(d, dtype=self.torch.float64, device=self.device) for d in self.n_dofs()]
        fptr = (C.c_void_p * n)()
        keep = []
        if fs is not None:
            for k, f in enumerate(fs):
                if f is not None:
                    t = self.torch.as_tensor(f, dtype=self.torch.float64, device=self.device).contiguous()
                    keep.append(t)
                    fptr[k] = t.data_ptr()
        uptr = (C.c_void_p * n)(*[u.data_ptr() for u in outputs])
        it = np.zeros(n, np.int32)
        rel = np.zeros(n, np.float64)
        rc = _lib.cb_solve_batch(self.ctx, fptr if fs is not None else None, uptr, float(rtol), int(max_iter),
                                 it.ctypes.data_as(C.POINTER(C.c_int32)),
                                 rel.ctypes.data_as(C.POINTER(C.c_double)))
        _check(rc, allow=(CB_ERR_NO_CONVERGENCE,) if allow_no_convergence else ())
        return outputs, it, rel


def _pcg_history(ctx, k):
    n = C.c_int32(0)
    _check(_lib.cb_pcg_history(ctx, k, 0, None, None, None, C.byref(n), None, None))
    m = max(n.value, 1)
    a, b, r = np.zeros(m), np.zeros(m), np.zeros(m)
    lo, hi = C.c_double(0.0), C.c_double(0.0)
    _check(_lib.cb_pcg_history(ctx, k, m, a.ctypes.data_as(C.c_void_p), b.ctypes.data_as(C.c_void_p),
                               r.ctypes.data_as(C.c_void_p), C.byref(n), C.byref(lo), C.byref(hi)))
    k_ = n.value
    return {"alpha": a[:k_], "beta": b[:max(k_ - 1, 0)], "relres": r[:k_],
            "lambda_min": lo.value, "lambda_max": hi.value}


def lanczos_extremes(alpha, beta):
    """(lambda_min, lambda_max) of the Lanczos matrix of CG coefficients
    (cb_lanczos_extremes; host only)."""
    lib = load_library()
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    lo, hi = C.c_double(0.0), C.c_double(0.0)
    _check(lib.cb_lanczos_extremes(int(a.size), a.ctypes.data_as(C.c_void_p) if a.size else None,
                                   b.ctypes.data_as(C.c_void_p) if b.size else None, C.byref(lo), C.byref(hi)))
    return lo.value, hi.value


def _profile_times(ctx, groups):
    out = {}
    for name in groups:
        t = C.c_double(0.0)
        n = C.c_int64(0)
        _check(_lib.cb_profile_time(ctx, name.encode(), C.byref(t), C.byref(n)))
        if n.value:
            out[name] = (float(t.value), int(n.value))
    return out


def _profile_launches(ctx, name):
    n = C.c_int64(0)
    _check(_lib.cb_profile_launches(ctx, name.encode(), None, 0, C.byref(n)))
    out = np.zeros(n.value, np.float64)
    if n.value:
        _check(_lib.cb_profile_launches(ctx, name.encode(), out.ctypes.data_as(C.c_void_p), n.value, C.byref(n)))
    return out


_INDEX_KEYS = ("cell_status", "cell_count", "dof_node", "card", "obj_ptr", "obj_dofs", "obj_type",
               "coarse_of_obj")


def _export_indexing(ctx, k, n, inf) -> dict:
    """Integer indexing of problem k of a context (k None: the single-problem
    entry point)."""
    n3 = n ** 3
    out = {
        "cell_status": np.zeros(n3, np.uint8),
        "cell_count": np.zeros(n3, np.int32),
        "dof_node": np.zeros(inf["n_dof"], np.int64),
        "card": np.zeros(inf["n_dof"], np.int32),
        "obj_ptr": np.zeros(inf["n_objects"] + 1, np.int64),
        "obj_dofs": np.zeros(inf["n_iface"], np.int64),
        "obj_type": np.zeros(inf["n_objects"], np.int8),
        "coarse_of_obj": np.zeros(inf["n_objects"], np.int32),
    }
    args = [out[key].ctypes.data_as(C.c_void_p) for key in _INDEX_KEYS]
    if k is None:
        _check(_lib.cb_export_indexing(ctx, *args))
    else:
        _check(_lib.cb_export_problem_indexing(ctx, k, *args))
    return out


def _export_subdomains(ctx, k, n_sub):
    ptr = np.zeros(n_sub + 1, np.int64)
    _check(_lib.cb_export_subdomains(ctx, k, ptr.ctypes.data_as(C.c_void_p), None))
    dofs = np.zeros(max(int(ptr[-1]), 1), np.int64)
    _check(_lib.cb_export_subdomains(ctx, k, ptr.ctypes.data_as(C.c_void_p), dofs.ctypes.data_as(C.c_void_p)))
    return ptr, dofs[:int(ptr[-1])]


def _problem_struct(problem):
    centres = np.ascontiguousarray(problem.centres, dtype=np.float64).reshape(-1)
    radii = np.ascontiguousarray(problem.radii, dtype=np.float64)
    P = C.POINTER(C.c_double)
    p = cb_problem(int(problem.n), int(problem.s), int(radii.size), centres.ctypes.data_as(P),
                   radii.ctypes.data_as(P), None, int(problem.weighting), int(problem.objects),
                   int(problem.coarse_variant), int(problem.local_precision),
                   int(problem.full_elements), int(getattr(problem, "cut_boundary", 0)))
    return p, (centres, radii)


def host_indexing(problem, cell_count) -> dict:
    """Host-only indexing from given per-cell kept-point counts (no GPU)."""
    lib = load_library()
    p, keep = _problem_struct(problem)
    cnt = np.ascontiguousarray(cell_count, dtype=np.int32)
    inf = cb_info()
    _check(lib.cb_host_indexing(C.byref(p), cnt.ctypes.data_as(C.c_void_p), C.byref(inf),
                                None, None, None, None, None, None))
    out = {
        "dof_node": np.zeros(inf.n_dof, np.int64), "card": np.zeros(inf.n_dof, np.int32),
        "obj_ptr": np.zeros(inf.n_objects + 1, np.int64), "obj_dofs": np.zeros(inf.n_iface, np.int64),
        "obj_type": np.zeros(inf.n_objects, np.int8), "coarse_of_obj": np.zeros(inf.n_objects, np.int32),
    }
    _check(lib.cb_host_indexing(C.byref(p), cnt.ctypes.data_as(C.c_void_p), C.byref(inf),
                                *[out[k].ctypes.data_as(C.c_void_p) for k in
                                  ("dof_node", "card", "obj_ptr", "obj_dofs", "obj_type",
                                   "coarse_of_obj")]))
    out["n_coarse"] = int(inf.n_coarse)
    out["t_ms"] = float(inf.t_topology_ms)
    return out


def dense_spd_inverse(A: np.ndarray, precision: int = 0) -> np.ndarray:
    """Batched SPD inverse on the GPU (the factorisation building block)."""
    lib = load_library()
    A = np.ascontiguousarray(A, dtype=np.float64)
    if A.ndim == 2:
        A = A[None]
    out = np.zeros_like(A)
    _check(lib.cb_dense_spd_inverse(A.shape[1], A.shape[0], precision,
                                    A.ctypes.data_as(C.c_void_p), out.ctypes.data_as(C.c_void_p)))
    return out


def unpack36(P: np.ndarray) -> np.ndarray:
    """(n, 36) packed upper triangles -> (n, 8, 8) symmetric matrices."""
    out = np.zeros(P.shape[:-1] + (8, 8))
    k = 0
    for a in range(8):
        for b in range(a, 8):
            out[..., a, b] = P[..., k]
            out[..., b, a] = P[..., k]
            k += 1
    return out
