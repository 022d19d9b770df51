"""Whole-path oracle: discretise, build topology, factor BDDC, solve with PCG."""
from __future__ import annotations

import time

import numpy as np
import scipy.sparse.linalg as spla

from . import assemble, topology, bddc, pcg, adjoint


class OracleSolver:
    def __init__(self, problem, check_floating: bool = True):
        self.problem = problem
        t0 = time.perf_counter()
        self.d = assemble.discretise(problem, check_floating=check_floating)
        t1 = time.perf_counter()
        self.topo = topology.build(problem, self.d)
        t2 = time.perf_counter()
        self.M = bddc.BDDC(self.d, self.topo, stiffness=(problem.weighting == 1))
        t3 = time.perf_counter()
        self.times = {"integrate": t1 - t0, "topology": t2 - t1, "factor": t3 - t2}

    @property
    def n_dof(self):
        return self.d.n_dof

    def rhs(self, f_nodes=None):
        f = self.problem.f if f_nodes is None else f_nodes
        return assemble.load(self.d, f)

    def solve_rhs(self, b, rtol=1e-8, max_iter=1000):
        t0 = time.perf_counter()
        x, it, rel, al, be = pcg.pcg(lambda v: self.d.A @ v, self.M.apply, b,
                                     rtol=rtol, max_iter=max_iter)
        self.times["solve"] = time.perf_counter() - t0
        self.last_coeffs = (al, be)
        return x, it, rel

    def solve(self, f_nodes=None, rtol=1e-8, max_iter=1000):
        return self.solve_rhs(self.rhs(f_nodes), rtol=rtol, max_iter=max_iter)

    def direct(self, b):
        return spla.spsolve(self.d.A.tocsc(), b)

    def gradients(self, u, u_target, rtol=1e-8, max_iter=1000):
        lam, it, _ = self.solve_rhs(u - u_target, rtol=rtol, max_iter=max_iter)
        return adjoint.gradients(self.d, u, lam) + (lam, it)
