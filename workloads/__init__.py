"""Seeded synthetic cut-cube workloads.

This module only draws inputs: ball centres and radii, per-cell conductivity,
per-node source values and the loss target noise.  It holds none of the
solver's arithmetic, so both the CPU oracle and the HIP path can take their
inputs from here without sharing any method code.

Domain family: the unit cube minus a union of closed balls,
Omega = {x in (0,1)^3 : |x - c_i| > r_i for every ball i}, meshed by an
N x N x N Cartesian background grid and split into uniform blocks of s^3
cells (the paper builds subdomains by aggregating the active cells of a
Cartesian mesh, Sect. 2.1; its meshes use at most 512 cells per subdomain,
H/h = 8, Table 1).  The paper's own geometries (popcorn flake, spiral, ...)
are not defined in its text, so these seeded ball-packings stand in for them.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

# Option codes shared by both implementations (plain enums, no arithmetic).
W_CARDINALITY = 0
W_STIFFNESS = 1
OBJ_CEF = 0
OBJ_CE = 1
CV_STANDARD = 0
CV_V1 = 1
CV_V2 = 2
CUT_NEUMANN = 0
CUT_NITSCHE = 1
FP64 = 0
FP32_LOCAL = 1


@dataclass
class Problem:
    """One cut-cube Poisson problem: -div(kappa grad u) = f, u = 0 on the
    cube faces, homogeneous Neumann on the ball surfaces."""

    n: int                      # background cells per axis, h = 1/n
    s: int                      # subdomain block size in cells (divides n)
    centres: np.ndarray         # (n_b, 3) float64
    radii: np.ndarray           # (n_b,) float64
    kappa: Optional[np.ndarray] = None   # (n^3,) per-cell conductivity, lexicographic (x fastest); None = 1
    f: Optional[np.ndarray] = None       # ((n+1)^3,) nodal source values; None = 1
    weighting: int = W_STIFFNESS
    objects: int = OBJ_CEF
    coarse_variant: int = CV_V1
    local_precision: int = FP64
    full_elements: int = 0      # test flag: every active cell integrated as uncut
    cut_boundary: int = 0       # ball surfaces: 0 homogeneous Neumann, 1 homogeneous Dirichlet (Nitsche)
    name: str = ""

    def with_options(self, **kw) -> "Problem":
        return replace(self, **kw)

    @property
    def n_balls(self) -> int:
        return int(self.radii.shape[0])


def single_ball(n: int = 8, s: int = 4, shift_x: float = 0.0) -> Problem:
    """Unit cube minus the ball of radius 0.3 at (0.51, 0.52, 0.49); 8^3 cells
    in 2^3 subdomains of 4^3 cells; f = 1, kappa = 1.  `shift_x` moves the
    ball along x (the paper translates the background mesh by eps in [-h, h]
    instead, Sect. 5.2; moving the geometry is the same relative motion)."""
    c = np.array([[0.51 + shift_x, 0.52, 0.49]], dtype=np.float64)
    r = np.array([0.3], dtype=np.float64)
    return Problem(n=n, s=s, centres=c, radii=r, name=f"single_ball_n{n}_s{s}")


def eps_sweep_shifts(n: int = 8, count: int = 51) -> np.ndarray:
    """The count values eps_k = -h + 2h k/(count-1), k = 0..count-1 (Sect. 5.2
    uses 51 values in [-h, h])."""
    h = 1.0 / n
    k = np.arange(count, dtype=np.float64)
    return -h + 2.0 * h * k / (count - 1)


def uncut(n: int, s: int) -> Problem:
    """No balls: Omega is the whole cube (every cell interior)."""
    return Problem(n=n, s=s, centres=np.zeros((0, 3)), radii=np.zeros((0,)),
                   name=f"uncut_n{n}_s{s}")


def random_balls(n: int, s: int, n_balls: int, seed: int, *,
                 lognormal_kappa: bool = False, random_f: bool = True,
                 name: str = "") -> Problem:
    """Seeded cube-minus-balls problem.  Draw order: centres U(0.1,0.9)
    (n_balls x 3), radii U(0.05,0.12) (n_balls), then kappa = exp(N(0,1)) per
    cell if requested, then f ~ U(0,1) per grid node ((n+1)^3, lexicographic)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.1, 0.9, size=(n_balls, 3))
    r = rng.uniform(0.05, 0.12, size=(n_balls,))
    kappa = np.exp(rng.standard_normal(n ** 3)) if lognormal_kappa else None
    f = rng.uniform(0.0, 1.0, size=(n + 1) ** 3) if random_f else None
    return Problem(n=n, s=s, centres=c, radii=r, kappa=kappa, f=f,
                   name=name or f"balls{n_balls}_n{n}_s{s}_seed{seed}")


def cut_cube_64(seed: int = 1) -> Problem:
    """64^3 cells, 8^3 subdomains of 8^3 cells, 20 random balls, kappa = 1,
    f ~ U(0,1) per node."""
    return random_balls(64, 8, 20, seed, name="cut_cube_64_balls20")


def cut_cube_96_lognormal(seed: int = 2) -> Problem:
    """96^3 cells, 12^3 subdomains of 8^3 cells, 40 random balls,
    kappa = exp(N(0,1)) per cell, f ~ U(0,1) per node, FP32 local solves."""
    p = random_balls(96, 8, 40, seed, lognormal_kappa=True,
                     name="cut_cube_96_balls40_lognormal")
    return p.with_options(local_precision=FP32_LOCAL)


def operator_256(seed: int = 5) -> Problem:
    """256^3 cells, 32^3 subdomains of 8^3 cells, 200 balls with centres
    U(0.1,0.9)^3 then radii U(0.02,0.05), kappa = 1: the mesh whose operator
    working set (x, y, cell data: about 470 MB) exceeds the 256 MB MALL.
    Used for the operator apply only (its dense coarse problem would not
    fit)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.1, 0.9, size=(200, 3))
    r = rng.uniform(0.02, 0.05, size=(200,))
    return Problem(n=256, s=8, centres=c, radii=r, name="operator_256_balls200")


def batch_256(seed: int = 3, count: int = 256) -> List[Problem]:
    """`count` independent problems.  Per problem k, in order: N_k uniform from
    {16, 24, 32, 48}; n_b,k integer in [5, 30]; centres; radii; f.  kappa = 1,
    subdomains of 8^3 cells, FP32 local solves."""
    rng = np.random.default_rng(seed)
    out = []
    sizes = np.array([16, 24, 32, 48])
    for k in range(count):
        n = int(sizes[rng.integers(0, 4)])
        nb = int(rng.integers(5, 31))
        c = rng.uniform(0.1, 0.9, size=(nb, 3))
        r = rng.uniform(0.05, 0.12, size=(nb,))
        f = rng.uniform(0.0, 1.0, size=(n + 1) ** 3)
        out.append(Problem(n=n, s=8, centres=c, radii=r, f=f,
                           local_precision=FP32_LOCAL,
                           name=f"batch{k}_n{n}_balls{nb}"))
    return out


@dataclass
class GradientCase:
    problem: Problem            # kappa = exp(theta)
    theta: np.ndarray           # (n^3,) per-cell log-conductivity
    target_noise: np.ndarray    # ((n+1)^3,) N(0, 0.01^2) per grid node
    rng: np.random.Generator = field(repr=False, default=None)


def gradient_case(n: int = 64, s: int = 8, n_balls: int = 20,
                  seed: int = 4) -> GradientCase:
    """Differentiation workload.  Draw order: centres, radii (20 balls),
    theta ~ N(0, 0.5^2) per cell, f ~ U(0,1) per node, target noise
    N(0, 0.01^2) per grid node.  The returned generator continues the same
    stream (used to pick finite-difference cells)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.1, 0.9, size=(n_balls, 3))
    r = rng.uniform(0.05, 0.12, size=(n_balls,))
    theta = rng.normal(0.0, 0.5, size=n ** 3)
    f = rng.uniform(0.0, 1.0, size=(n + 1) ** 3)
    noise = rng.normal(0.0, 0.01, size=(n + 1) ** 3)
    p = Problem(n=n, s=s, centres=c, radii=r, kappa=np.exp(theta), f=f,
                name=f"gradient_n{n}_balls{n_balls}")
    return GradientCase(problem=p, theta=theta, target_noise=noise, rng=rng)
