"""Workload recipes: grid, constitutive parameters, boundary data, initial head.

The constitutive parameters are the ones the paper lists for its 1-D study and
Figure 1 (Haverkamp-type laws, Section 2).  Geometry, boundary data and the
K_s statistics of the larger workloads are this project's choices: a 64 cm
cube, initial head -61.5 cm, top face held at -20.7 cm (Dirichlet), the five
other faces no-flux.  The grid spacing is
h = L / (n + 1): the n unknowns per axis are the interior nodes of an
(n + 2)-node grid whose outermost nodes lie on the boundary (Section 2.1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

from .fields import lognormal_ks, uniform01

ARITH, UPSTREAM, HARMONIC, GEOMETRIC, INTEGRAL = 0, 1, 2, 3, 4
MEAN_NAMES = {"arith": ARITH, "upstream": UPSTREAM, "harmonic": HARMONIC, "geometric": GEOMETRIC,
              "integral": INTEGRAL}
NOFLUX, DIRICHLET = 0, 1
FP64, MIXED = 0, 1

KS0 = 0.00944          # cm/s
P_INIT = -61.5         # cm
P_TOP = -20.7          # cm
L_CUBE = 64.0          # cm


@dataclass
class Problem:
    nx: int
    ny: int
    nz: int
    hx: float
    hy: float
    hz: float
    alpha: float = 1.611e6
    beta: float = 3.96
    theta_s: float = 0.287
    theta_r: float = 0.075
    A: float = 1.175e6
    gamma: float = 4.74
    mean: int = ARITH
    # faces ordered -x, +x, -y, +y, -z (bottom), +z (top)
    bc_type: tuple = (NOFLUX, NOFLUX, NOFLUX, NOFLUX, NOFLUX, DIRICHLET)
    bc_value: tuple = (0.0, 0.0, 0.0, 0.0, 0.0, P_TOP)
    dt: float = 1.0
    # optional Dirichlet patch: boundary nodes of face patch_face whose two
    # tangential coordinates [cm] lie in [patch_lo, patch_hi] hold patch_value
    patch_face: int = -1
    patch_lo: tuple = (0.0, 0.0)
    patch_hi: tuple = (0.0, 0.0)
    patch_value: float = 0.0
    mean_vertical: int = -1             # mean on the z faces (-1: the same as mean)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


@dataclass
class Options:
    """Solver controls (Sections 3 and 6; unset constants are documented readings)."""
    fnormtol: float = 1e-8
    scsteptol: float = 2.220446049250313e-16 ** (2.0 / 3.0)
    max_newton: int = 200
    msbset: int = 10
    ls_alpha: float = 1e-4
    mxnewtstep: float = 0.0            # 0 -> 1000 * max(||p0||_2, 1)
    gmres_restart: int = 30
    eta: float = 1e-6
    gmres_maxit: int = 200
    amg_max_levels: int = 10
    amg_coarse_size: int = 512
    amg_sweeps: int = 3                # pairwise matching sweeps -> aggregates <= 2**sweeps
    coarse_dense_max: int = 4096
    coarse_l1_sweeps: int = 4
    amg_refresh: int = 1               # 1: every rebuild recomputes the coarse matrices (aggregates kept)
    precision: int = FP64
    gmres_reorth: float = 0.01          # second Gram-Schmidt pass only on severe cancellation
    aux_dflux: int = 0                  # 1: preconditioner diagonal takes the flux-derivative terms
    amg_smoothed: int = 0               # levels (from the finest) whose prolongator is smoothed (damped Jacobi on P_t)
    tile_kz: int = 0                    # planes per block of the tiled fine-level smoother (0: automatic)
    smoother: int = 0                   # 0: l1-Jacobi; 1: multicolour Gauss-Seidel on the finest level
    amg_aggregation: int = 0            # 0: pairwise matching sweeps; 1: decoupled greedy (VMB) aggregation
    amg_theta: float = 0.0              # strength threshold of the greedy aggregation (0: every coupling)
    amg_block: int = 4096               # rows per decoupled block of the greedy aggregation
    gmres_block: int = 10               # Arnoldi vectors per Gram-Schmidt round (1: classical; 2..10: s-step)
    gmres_shift: float = 0.65           # centre of the s-step basis shifts
    gmres_shift_span: float = 0.55      # half-width of the shift interval (Leja points; 0: one shift)


@dataclass
class Recipe:
    name: str
    problem: Problem
    options: Options
    nsteps: int
    ks_sigma: float
    ks_ell: tuple
    ks_seed: int
    description: str = ""
    extra: dict = field(default_factory=dict)

    def ks(self) -> np.ndarray:
        p = self.problem
        if self.ks_sigma == 0.0:
            return np.full(p.n, KS0, dtype=np.float64)
        return lognormal_ks((p.nx, p.ny, p.nz), KS0, self.ks_sigma, self.ks_ell, self.ks_seed)

    def p0(self) -> np.ndarray:
        return np.full(self.problem.n, P_INIT, dtype=np.float64)


def cube_problem(n: int, mean: int, dt: float, L: float = L_CUBE) -> Problem:
    h = L / (n + 1)
    return Problem(nx=n, ny=n, nz=n, hx=h, hy=h, hz=h, mean=mean, dt=dt)


def _c1(n: int = 16) -> Recipe:
    o = Options(amg_max_levels=2, precision=FP64)
    return Recipe("c1_16cube_fp64", cube_problem(n, HARMONIC, 1.0), o, 5, 0.0, (1, 1, 1), 0,
                  "16^3 homogeneous K_s, harmonic mean, dt=1 s, 5 steps, 2-level AMG, FP64")


def _c2(n: int = 128) -> Recipe:
    return Recipe("c2_128cube_fp64", cube_problem(n, ARITH, 10.0), Options(precision=FP64), 10,
                  2.0, (8.0, 8.0, 2.0), 20211202,
                  "128^3 lognormal K_s (sigma 2, l=8/8/2), arithmetic mean, dt=10 s, 10 steps, FP64")


def _c3(n: int = 256, precision: int = MIXED) -> Recipe:
    return Recipe("c3_256cube_mixed" if precision == MIXED else "c3_256cube_fp64",
                  cube_problem(n, UPSTREAM, 10.0), Options(precision=precision), 10,
                  2.5, (16.0, 16.0, 4.0), 20211203,
                  "256^3 lognormal K_s (sigma 2.5, l=16/16/4), upstream mean, dt=10 s, 10 steps")


def _c5(n: int = 512) -> Recipe:
    return Recipe("c5_512cube_mixed", cube_problem(n, HARMONIC, 30.0),
                  Options(precision=MIXED, amg_max_levels=5), 5,
                  3.0, (32.0, 32.0, 4.0), 20211205,
                  "512^3 lognormal K_s (sigma 3, l=32/32/4), harmonic mean, dt=30 s, 5 steps")


def _paper3d(n: int = 798, nz: int | None = None, precision: int = MIXED) -> Recipe:
    """The 3-D infiltration test of the paper's experiments (Section 6): the
    box [0,64] x [0,64] x [0,1] cm with 800 x 800 x 40 mesh points (798 x 798
    x 38 unknowns), upstream mean, head h_r on every face except a square of
    zero head in the middle of the top face (a/4 <= x, y <= 3a/4), initial
    head h_r, t in [0, 2] s with 10 time levels (9 steps of 2/9 s), GMRES(10)
    with eta = 1e-7.  The paper leaves h_r and the constitutive parameters of
    this test unstated: h_r = -61.5 cm and the Haverkamp parameters of its
    Fig. 1 with a homogeneous K_s are used.  GMRES rounds of 5 vectors (two
    per cycle of 10): the preconditioned spectrum of this thin grid reaches
    about 1.9, past the default shift interval, and rounds of 10 lose every
    twelfth round to vector-wise completion."""
    nz = nz if nz is not None else 38
    P = Problem(nx=n, ny=n, nz=nz, hx=64.0 / (n + 1), hy=64.0 / (n + 1), hz=1.0 / (nz + 1), mean=UPSTREAM,
                bc_type=(DIRICHLET,) * 6, bc_value=(P_INIT,) * 6, dt=2.0 / 9.0,
                patch_face=5, patch_lo=(16.0, 16.0), patch_hi=(48.0, 48.0), patch_value=0.0)
    o = Options(precision=precision, gmres_restart=10, eta=1e-7, gmres_block=5)
    return Recipe(f"paper3d_{n + 2}x{n + 2}x{nz + 2}", P, o, 9, 0.0, (1, 1, 1), 0,
                  "the paper's 3-D infiltration test: upstream mean, zero-head square on the top face")


RECIPES = {"c1": _c1, "c2": _c2, "c3": _c3, "c5": _c5, "paper3d": _paper3d}


def recipe(name: str, n: int | None = None, **kw) -> Recipe:
    """Build a named recipe; ``n`` changes the cube size and keeps every other
    statistic, the K_s correlation lengths in cells included (so a smaller
    grid sees the same local smoothness of the field as the full one)."""
    f = RECIPES[name]
    if n is None:
        return f(**kw)
    return f(n, **kw) if name != "c1" else f(n)


def serving_stream(count: int = 64, rate: float = 4.0, seed: int = 20211204,
                   sizes=(32, 48, 64, 80, 96), nsteps: int = 20):
    """The ensemble request stream: Poisson arrivals, random grid, field and mean."""
    reqs = []
    t = 0.0
    ctr = np.arange(6 * count, dtype=np.uint64)
    u = uniform01(seed, ctr).reshape(count, 6)
    for r in range(count):
        t += -math.log(u[r, 0]) / rate
        n = sizes[min(len(sizes) - 1, int(u[r, 1] * len(sizes)))]
        sigma = 1.0 + 2.0 * u[r, 2]
        mean = min(2, int(u[r, 3] * 3))
        ell = (n / 16.0, n / 16.0, max(1.0, n / 64.0))
        rec = Recipe(f"req{r}", cube_problem(n, mean, 10.0), Options(precision=MIXED), nsteps,
                     sigma, ell, seed * 1000 + r)
        reqs.append((t, rec))
    return reqs
