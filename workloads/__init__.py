"""Seeded synthetic workload definitions shared by the solver library's callers and the oracle.

This module holds inputs only: geometry of the coarse grid, the refinement recipe,
PDE coefficients, boundary parts, solver settings and random draws from seeded
generators.  It holds none of the method's arithmetic (no meshing, no assembly, no
multigrid).  Both the native problem generator and the oracle read a `Workload` and
build everything else on their own.

Shapes follow the paper's workloads: Q1 on axis-aligned boxes, adaptive refinement
with one level jump between neighbours (Sec. 2.2), scalar 2D transport-diffusion
(Sec. 5.1), 3D linear elasticity with nodal 3-vectors (Sec. 5.2; the paper's meshes
refined towards a face/edge/vertex, Table "table:ndofs"), and 4-component nodal
blocks of a 3D flow problem (pressure first, then velocity, Sec. 2.1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Tuple

import numpy as np

# ---------------------------------------------------------------------------
# refinement-round recipes (tuples, so that they are hashable and easy to pass to C)
#   ("uniform",)                          refine every leaf
#   ("band", cx, cy, r, delta)            refine every leaf whose closed box meets the open
#                                         annulus r-delta < |p-c| < r+delta (2D)
#   ("corner", axes_bitmask, thr)         refine every leaf of the current maximum depth whose
#                                         box lies in {x_a <= thr for every axis a in the mask}
# After every round the mesh is 2:1 balanced over shared vertices.
# ---------------------------------------------------------------------------

PDE_POISSON, PDE_TD, PDE_ELASTICITY, PDE_OSEEN = 0, 1, 2, 3
RHS_SINSIN, RHS_DISK, RHS_CONST, RHS_FIELD, RHS_NOISE, RHS_NONE, RHS_ELAST_MMS = 0, 1, 2, 3, 4, 5, 6
OUTER_IR, OUTER_FGMRES = 0, 1
COARSE_EXACT, COARSE_SMOOTH = 0, 1
SMOOTH_JACOBI, SMOOTH_CHEBYSHEV = 0, 1
PREC_FP64, PREC_FP32, PREC_FP32_F16VAL, PREC_FP32_BF16VAL = 0, 1, 2, 3


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    dim: int
    coarse: Tuple[int, ...]          # coarse cells per axis, (x, y[, z])
    h0: float                        # coarse cell edge length (cells are squares / cubes)
    rounds: Tuple[tuple, ...]        # refinement recipe, one entry per round
    pde: int
    block: int                       # components per node
    # PDE coefficients (unused ones stay at their defaults)
    eps: float = 1.0                 # diffusion (TD)
    bvec: Tuple[float, ...] = (0.0, 0.0)   # constant convection (TD)
    lam: float = 0.0                 # Lame lambda (elasticity)
    mu: float = 0.0                  # Lame mu (elasticity)
    nu: float = 0.0                  # viscosity (Oseen)
    dt: float = 1.0                  # time step (Oseen mass term 1/dt)
    pspg_alpha: float = 1.0          # pressure-stabilisation constant (Oseen)
    supg: bool = True                # streamline stabilisation of the TD operator
    mass_coef: float = 0.0           # coefficient c of a lumped mass term c * M_l in the operator
    t_end: float = 0.0               # time-dependent problems: end of the interval (0, t_end]
    # Dirichlet part: bitmask of faces (bit 2a = face x_a = 0, bit 2a+1 = face x_a = max)
    # and bitmask of constrained components on those faces
    dir_faces: int = 0
    dir_comps: int = 1
    rhs: int = RHS_NONE
    rhs_const: Tuple[float, ...] = ()
    # convection field / forcing coefficients (Oseen), see `oseen_fields`
    seed: int = 0
    # solver settings
    omega: float = 0.8
    nu1: int = 2
    nu2: int = 2
    outer: int = OUTER_IR
    gmres_m: int = 10
    rtol: float = 1e-8
    maxit: int = 200
    coarse_mode: int = COARSE_EXACT
    coarse_sweeps: int = 20
    # smoother of levels >= 1: damped (block-)Jacobi, or its Chebyshev acceleration on
    # [cheb_lo, cheb_hi] * lambda with lambda from power_its power-iteration steps
    smoother: int = SMOOTH_JACOBI
    cheb_lo: float = 0.15
    cheb_hi: float = 1.1
    power_its: int = 12
    # index (in the full coarsening hierarchy) of the level solved exactly; the paper allows
    # the coarse mesh to be the starting mesh or any finer one that balances multigrid work
    # against the cost of the direct solve (Sec. 2.2)
    coarse_level: int = 0

    @property
    def n_rounds(self) -> int:
        return len(self.rounds)

    def with_(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


ALL_FACES_2D = 0b1111
ALL_FACES_3D = 0b111111

# C2 annulus half-width, frozen so that the finest mesh has ~1.0e6 nodes after balancing
C2_DELTA = 0.062


def c1_poisson(rounds: int = 4) -> Workload:
    """2D Poisson on the unit square, 2x2 coarse cells; 4 uniform rounds give 33x33 nodes."""
    return Workload(name=f"poisson2d_u{rounds}", dim=2, coarse=(2, 2), h0=0.5,
                    rounds=(("uniform",),) * rounds, pde=PDE_POISSON, block=1,
                    dir_faces=ALL_FACES_2D, dir_comps=1, rhs=RHS_SINSIN,
                    omega=0.8, nu1=2, nu2=2, outer=OUTER_IR, rtol=1e-10)


def c2_td(band_rounds: int = 6, delta: float = C2_DELTA, uniform_rounds: int = 2) -> Workload:
    """2D transport-diffusion with streamline stabilisation on an annulus-refined mesh.

    eps = 1e-3, b = (1, 0.5), 8x8 coarse cells, 2 uniform rounds, then `band_rounds`
    rounds around the circle |p - (0.5, 0.5)| = 0.3; f = 1 inside the circle, u = 0 on
    the boundary; FGMRES(10) preconditioned by the V-cycle.
    """
    rounds = (("uniform",),) * uniform_rounds + (("band", 0.5, 0.5, 0.3, delta),) * band_rounds
    return Workload(name=f"td2d_u{uniform_rounds}b{band_rounds}", dim=2, coarse=(8, 8), h0=0.125,
                    rounds=rounds, pde=PDE_TD, block=1, eps=1e-3, bvec=(1.0, 0.5),
                    dir_faces=ALL_FACES_2D, dir_comps=1, rhs=RHS_DISK,
                    omega=0.8, nu1=2, nu2=2, outer=OUTER_FGMRES, gmres_m=10, rtol=1e-8)


def c3_elasticity(rounds: int = 6) -> Workload:
    """3D linear elasticity, lambda = 1, mu = 0.5, clamped at x = 0, body load (0,-1,0).

    2x2x2 coarse cubes; 6 uniform rounds give 129^3 nodes (3 components each)."""
    return Workload(name=f"elast3d_u{rounds}", dim=3, coarse=(2, 2, 2), h0=0.5,
                    rounds=(("uniform",),) * rounds, pde=PDE_ELASTICITY, block=3,
                    lam=1.0, mu=0.5, dir_faces=0b000001, dir_comps=0b111,
                    rhs=RHS_CONST, rhs_const=(0.0, -1.0, 0.0),
                    omega=0.6, nu1=2, nu2=2, outer=OUTER_FGMRES, rtol=1e-8)


def elasticity_mms(rounds: int = 3) -> Workload:
    """3D linear elasticity (lambda = 1, mu = 0.5) on the unit cube, clamped on every face,
    with the body load of the manufactured displacement
    u(x) = sin(pi x) sin(pi y) sin(pi z) * ELAST_MMS_DIR (used for the O(h^2) error check)."""
    return Workload(name=f"elast3d_mms_u{rounds}", dim=3, coarse=(2, 2, 2), h0=0.5,
                    rounds=(("uniform",),) * rounds, pde=PDE_ELASTICITY, block=3,
                    lam=1.0, mu=0.5, dir_faces=ALL_FACES_3D, dir_comps=0b111,
                    rhs=RHS_ELAST_MMS, omega=0.6, nu1=2, nu2=2, outer=OUTER_FGMRES, rtol=1e-10)


# direction of the manufactured elasticity displacement
ELAST_MMS_DIR = (1.0, -0.5, 0.75)


def td_time(n: int = 10, dt: float = 0.02, t_end: float = 2.0, coarse_level: int = 0) -> Workload:
    """The nonstationary transport-diffusion problem of Sec. 5.1: unit square, uniform mesh
    of width h = 2^-n ((2^n + 1)^2 nodes; 2x2 coarse cells and n - 1 uniform rounds),
    diffusion 0.01, convection b = (0, -1), backward Euler with step dt on (0, t_end]
    (100 steps by default), Dirichlet data of the exact solution td_exact on all sides.
    The operator of every level is M_l / dt + 0.01 K + C (lumped mass, Galerkin
    convection: the cell Peclet number |b| h / (2 * 0.01) is below 0.4 from n = 7 on)."""
    return Workload(name=f"tdtime_n{n}", dim=2, coarse=(2, 2), h0=0.5,
                    rounds=(("uniform",),) * (n - 1), pde=PDE_TD, block=1, eps=0.01,
                    bvec=(0.0, -1.0), supg=False, mass_coef=1.0 / dt, dt=dt, t_end=t_end,
                    dir_faces=ALL_FACES_2D, dir_comps=1, rhs=RHS_NONE,
                    omega=0.8, nu1=2, nu2=2, outer=OUTER_FGMRES, gmres_m=10, rtol=1e-8,
                    coarse_level=coarse_level)


def td_exact(t, x, y):
    """Exact solution of the Sec. 5.1 problem:
    theta = exp(-(m(t, x)^2 + m(t, y)^2) / 4), m(t, z) = 1/2 + cos(pi t / 2) / 4 - z."""
    c = 0.5 + 0.25 * np.cos(0.5 * np.pi * t)
    mx, my = c - x, c - y
    return np.exp(-0.25 * (mx * mx + my * my))


def td_source(t, x, y, diff=0.01, bvec=(0.0, -1.0)):
    """f = d_t theta - diff * lap theta + b . grad theta for theta = td_exact.
    With m_x = c - x, m_y = c - y, c(t) = 1/2 + cos(pi t / 2) / 4, theta = exp(-(m_x^2 +
    m_y^2) / 4): d_t theta = -theta (m_x + m_y) c' / 2 with c' = -pi sin(pi t / 2) / 8;
    d_x theta = theta m_x / 2, d_y theta = theta m_y / 2;
    lap theta = theta ((m_x^2 + m_y^2) / 4 - 1)."""
    c = 0.5 + 0.25 * np.cos(0.5 * np.pi * t)
    dc = -0.125 * np.pi * np.sin(0.5 * np.pi * t)
    mx, my = c - x, c - y
    th = np.exp(-0.25 * (mx * mx + my * my))
    dt_th = -0.5 * th * (mx + my) * dc
    lap = th * (0.25 * (mx * mx + my * my) - 1.0)
    return dt_th - diff * lap + bvec[0] * 0.5 * th * mx + bvec[1] * 0.5 * th * my


def c3_adaptive(kind: str, level: int) -> Workload:
    """The paper's adaptive cube meshes (Table 'table:ndofs'): 8^3 coarse cells, then
    `level-1` rounds refining the finest cells next to a face, an edge or a vertex,
    with C3's elasticity operator on top."""
    axes = {"face": 0b001, "edge": 0b011, "vertex": 0b111}[kind]
    rounds = tuple(("corner", axes, 2.0 ** (-k)) for k in range(1, level))
    return Workload(name=f"elast3d_{kind}{level}", dim=3, coarse=(8, 8, 8), h0=0.125,
                    rounds=rounds, pde=PDE_ELASTICITY, block=3, lam=1.0, mu=0.5,
                    dir_faces=0b000001, dir_comps=0b111, rhs=RHS_CONST,
                    rhs_const=(0.0, -1.0, 0.0), omega=0.6, nu1=2, nu2=2,
                    outer=OUTER_FGMRES, rtol=1e-8)


def c4_oseen(rounds: int = 5, tall: bool = False, seed: int = 0) -> Workload:
    """3D linearised flow step (Oseen): 1/dt mass + nu Laplace + beta.grad, equal-order
    Q1/Q1 with a pressure-gradient stabilisation; 4 components per node ordered
    (p, u, v, w).  No-slip on x=0, x=1, y=0, y=1, z=0; natural outflow on the top face.

    Cube: 2x2x2 coarse cubes (65^3 nodes at 5 rounds).  `tall=False` only; the
    129x129x65 box variant uses 2x2x1 coarse cubes of edge 0.5 with 6 rounds."""
    coarse = (2, 2, 1) if tall else (2, 2, 2)
    return Workload(name=f"oseen3d_{'b' if tall else ''}u{rounds}", dim=3, coarse=coarse, h0=0.5,
                    rounds=(("uniform",),) * rounds, pde=PDE_OSEEN, block=4,
                    nu=1e-3, dt=0.01, pspg_alpha=1.0, dir_faces=0b011111, dir_comps=0b1110,
                    rhs=RHS_FIELD, seed=seed, omega=0.6, nu1=2, nu2=2,
                    outer=OUTER_FGMRES, gmres_m=10, rtol=1e-8)


def oseen_fields(seed: int):
    """Coefficients of the seeded convection field beta = curl(psi) and velocity forcing.

    psi = sum_k a_k sin(2 pi kappa_k . x + phi_k) e_{j_k}, k = 1..8, so that
    beta(x) = scale * sum_k a_k 2 pi cos(2 pi kappa_k . x + phi_k) (kappa_k x e_{j_k});
    `scale` = 1 / sum_k |a_k| 2 pi |kappa_k x e_{j_k}| bounds max |beta| by 1.
    Forcing: f(x) = sum_m c_m sin(2 pi mu_m . x + varphi_m) e_{i_m}, m = 1..4.
    """
    rng = np.random.default_rng(seed)
    kappa = rng.integers(1, 3, size=(8, 3)).astype(np.float64)
    a = rng.standard_normal(8)
    phi = rng.uniform(0.0, 2.0 * math.pi, 8)
    j = rng.integers(0, 3, size=8)
    cross_norm = np.empty(8)
    for k in range(8):
        e = np.zeros(3)
        e[j[k]] = 1.0
        cross_norm[k] = np.linalg.norm(np.cross(kappa[k], e))
    scale = 1.0 / float(np.sum(np.abs(a) * 2.0 * math.pi * cross_norm))
    fk = rng.integers(1, 3, size=(4, 3)).astype(np.float64)
    fc = rng.standard_normal(4)
    fphi = rng.uniform(0.0, 2.0 * math.pi, 4)
    fi = rng.integers(0, 3, size=4)
    return dict(kappa=kappa, a=a, phi=phi, j=j.astype(np.int32), scale=scale,
                fk=fk, fc=fc, fphi=fphi, fi=fi.astype(np.int32))


def batch_problems(n_problems: int = 64, base_seed: int = 1000, max_levels: int = 9,
                   min_levels: int = 4):
    """Independent 2D transport-diffusion problems of uneven size (seeded draws).

    Problem k uses numpy.random.default_rng(base_seed + k): eps = 10^U[-4,-1],
    b = (cos t, sin t) with t ~ U[0, 2pi), L ~ U{min..max} levels, u ~ U{1..L-1}
    uniform rounds, the remaining L-1-u rounds refine an annulus with centre
    ~ U[0.3,0.7]^2, radius ~ U[0.15,0.35] and half-width ~ U[0.02,0.1].

    Jacobi damping 0.6: with 0.8 the V-cycle of the most convection-dominated members
    (Peclet numbers in the hundreds on the coarse levels) amplifies some error modes and
    FGMRES(10) stalls on 6 of the 64 default problems; 0.6 converges on all of them."""
    out = []
    for k in range(n_problems):
        rng = np.random.default_rng(base_seed + k)
        eps = 10.0 ** rng.uniform(-4.0, -1.0)
        t = rng.uniform(0.0, 2.0 * math.pi)
        L = int(rng.integers(min_levels, max_levels + 1))
        u = int(rng.integers(1, L))
        cx, cy = rng.uniform(0.3, 0.7, 2)
        r = rng.uniform(0.15, 0.35)
        delta = rng.uniform(0.02, 0.1)
        rounds = (("uniform",),) * u + (("band", float(cx), float(cy), float(r), float(delta)),) * (L - 1 - u)
        out.append(Workload(name=f"batch{k}", dim=2, coarse=(8, 8), h0=0.125, rounds=rounds,
                            pde=PDE_TD, block=1, eps=float(eps),
                            bvec=(math.cos(t), math.sin(t)), dir_faces=ALL_FACES_2D,
                            dir_comps=1, rhs=RHS_NOISE, seed=base_seed + k, omega=0.6,
                            outer=OUTER_FGMRES, gmres_m=10, rtol=1e-8))
    return out


def noise(seed: int, n: int, nrhs: int = 1) -> np.ndarray:
    """Seeded N(0,1) samples, shape (n, nrhs)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 77]))
    return rng.standard_normal((n, nrhs))


def weyl_vec(n: int) -> np.ndarray:
    """Start vector of the smoother's power iteration: frac(i g) - 1/2 for i = 0 .. n-1,
    g = (sqrt(5) - 1) / 2 (Weyl's equidistributed sequence), every operation exact or
    correctly rounded in FP64 so that any implementation of the definition agrees."""
    t = np.arange(n, dtype=np.float64) * 0.61803398874989484820
    return t - np.floor(t) - 0.5


def rand_vec(seed: int, n: int) -> np.ndarray:
    """Seeded U[-1,1) test vector used by kernel-level parity tests."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 31]))
    return rng.uniform(-1.0, 1.0, n)


def by_name(name: str) -> Workload:
    table = {
        "c1": c1_poisson(),
        "c2": c2_td().with_(coarse_level=3),
        "c3": c3_elasticity().with_(coarse_level=2),
        "c4": c4_oseen().with_(coarse_level=2),
        "c4b": c4_oseen(rounds=6, tall=True).with_(coarse_level=2),
        "c3f": c3_adaptive("face", 6),
    }
    return table[name]
