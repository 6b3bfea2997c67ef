"""Seeded synthetic workloads for the Parareal exponential-integrator Q1 FEM.

This module only *describes* problem instances: domains, grid sizes, the
parameters of a separable forcing, the initial value, the time slicing and the
Runge--Kutta stage nodes.  It holds none of the method's arithmetic (no
quadrature, no transforms, no phi functions, no time stepping); each consumer
(the FP64 CPU oracle and the HIP library binding) evaluates these descriptors
with code of its own.

Problem statement (paper, Section 1, eq. (1.1) and Section 2, eq. (2.1)):
    u_t = D * Laplace(u) + f(t, x)   on a box Omega in R^d, t0 <= t <= t0 + T,
    u = 0 on the boundary,  u(t0) = u0.

Separable descriptors used throughout
-------------------------------------
A forcing (or an initial value, or an exact solution) is a list of ``Term``:

    term(t, x) = amp * tau(t) * prod_a X_a(x_a)

    tau(t)  = exp(alpha*t) * cos(omega*t + phase) * (p0 + p1 t + p2 t^2 + p3 t^3)
    X_a(x)  = (q0 + q1 x + q2 x^2) * sin(kappa*x + phase)

A pure polynomial space factor uses kappa = 0, phase = pi/2 (sin = 1).  For an
initial value the time factor is ignored.

Random draws (numpy PCG64, ``numpy.random.default_rng(seed)``) happen in a
fixed order: first the stage nodes, then for each forcing mode m the per-axis
wavenumbers, the amplitude and the angular frequency.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

PI = math.pi


@dataclass(frozen=True)
class TimeFactor:
    alpha: float = 0.0
    omega: float = 0.0
    phase: float = 0.0
    poly: Tuple[float, float, float, float] = (1.0, 0.0, 0.0, 0.0)


@dataclass(frozen=True)
class SpaceFactor:
    kappa: float = 0.0
    phase: float = PI / 2
    poly: Tuple[float, float, float] = (1.0, 0.0, 0.0)


@dataclass(frozen=True)
class Term:
    amp: float
    time: TimeFactor
    space: Tuple[SpaceFactor, ...]


@dataclass(frozen=True)
class MovingHat:
    """A moving hat source amp tau(t) max(1 - |x_axis - c(t)| / width, 0)
    prod_{b != axis} X_b(x_b), c(t) = c0 + c1 sin(omega t + phase) (the
    oscillating source of the paper's Example 5.4).  space[axis] is unused."""
    amp: float
    axis: int
    width: float
    c0: float
    c1: float = 0.0
    omega: float = 0.0
    phase: float = 0.0
    time: TimeFactor = TimeFactor()
    space: Tuple[SpaceFactor, ...] = ()


def sine_factor(k: int, lo: float, hi: float) -> SpaceFactor:
    """sin(k*pi*(x - lo)/(hi - lo)): the k-th Dirichlet sine on [lo, hi]."""
    kappa = k * PI / (hi - lo)
    return SpaceFactor(kappa=kappa, phase=-kappa * lo)


def poly_factor(q0: float, q1: float = 0.0, q2: float = 0.0) -> SpaceFactor:
    return SpaceFactor(kappa=0.0, phase=PI / 2, poly=(q0, q1, q2))


@dataclass
class Problem:
    name: str
    dim: int
    n: Tuple[int, ...]            # interior Q1 nodes per axis (elements - 1)
    lo: Tuple[float, ...]
    hi: Tuple[float, ...]
    D: float
    t0: float
    T: float
    forcing: List[Term]
    u0: List[Term]                # time factors ignored
    N: int                        # coarse slices
    J: int                        # fine steps per slice (M in the paper)
    c_fine: Tuple[float, ...]     # q stage nodes of F
    c_coarse: Tuple[float, ...]   # p stage nodes of G
    precision: str = "fp64"       # "fp64" or "split_bf16" (FP32 state)
    K_max: int = 8
    tol: float = 1e-8
    exact: Optional[List[Term]] = None
    seed: Optional[int] = None
    notes: str = ""
    # Dirichlet data u = g on the boundary (separable terms with time
    # factors); empty: homogeneous data
    boundary: List[Term] = field(default_factory=list)
    # moving hat sources added to the forcing (not separable in t and x)
    moving: List[MovingHat] = field(default_factory=list)
    # per axis: periodic (n nodes per period) instead of Dirichlet; empty:
    # all Dirichlet
    periodic: Tuple[bool, ...] = ()

    @property
    def q(self) -> int:
        return len(self.c_fine)

    @property
    def p(self) -> int:
        return len(self.c_coarse)

    @property
    def dof(self) -> int:
        return int(np.prod(self.n))

    @property
    def dT(self) -> float:
        return self.T / self.N

    @property
    def dt(self) -> float:
        return self.T / (self.N * self.J)

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


# --------------------------------------------------------------------------
# stage nodes
# --------------------------------------------------------------------------

def uniform_nodes(s: int) -> Tuple[float, ...]:
    """c_i = (i-1)/s, i = 1..s: the equispaced nodes used by the paper's
    experiments (Section 5.1)."""
    return tuple(i / s for i in range(s))


def random_nodes(rng: np.random.Generator, s: int, min_gap: float = 0.05) -> Tuple[float, ...]:
    """s sorted U(0,1) nodes, redrawn while two of them are closer than
    ``min_gap`` (close nodes blow up the Lagrange basis)."""
    while True:
        c = np.sort(rng.uniform(0.0, 1.0, s))
        if s == 1 or np.min(np.diff(c)) >= min_gap:
            return tuple(float(x) for x in c)


def _sine_modes(rng, n_modes, dims_lohi, omega_lo, omega_hi, kmax=32):
    terms = []
    for _ in range(n_modes):
        ks = rng.integers(1, kmax + 1, len(dims_lohi))
        amp = float(rng.normal())
        omega = float(rng.uniform(omega_lo, omega_hi))
        space = tuple(sine_factor(int(k), lo, hi) for k, (lo, hi) in zip(ks, dims_lohi))
        terms.append(Term(amp, TimeFactor(omega=omega), space))
    return terms


# --------------------------------------------------------------------------
# the five benchmark configurations
# --------------------------------------------------------------------------

def config(i: int, seed: Optional[int] = None) -> Problem:
    """The five synthetic workloads (1D check case, 2D FP64, 3D split-BF16,
    2D learned-G, 3D learned-G + mixed precision)."""
    if seed is None:
        seed = 1000 + i
    rng = np.random.default_rng(seed)
    if i == 1:
        c = random_nodes(rng, 2)
        k = int(rng.integers(1, 5))
        D = 1.0
        sf = sine_factor(k, 0.0, 1.0)
        f = [Term(D * k * k * PI * PI - 1.0, TimeFactor(alpha=-1.0), (sf,))]
        return Problem("cfg1-1d-63", 1, (63,), (0.0,), (1.0,), D, 0.0, 1.0, f,
                       [Term(1.0, TimeFactor(), (sf,))], 8, 16, c, c, "fp64", 8, 1e-8,
                       exact=[Term(1.0, TimeFactor(alpha=-1.0), (sf,))], seed=seed,
                       notes=f"k={k}")
    if i == 2:
        c = random_nodes(rng, 3)
        box = [(0.0, 1.0), (0.0, 1.0)]
        f = _sine_modes(rng, 8, box, 1.0, 20.0)
        return Problem("cfg2-2d-255", 2, (255, 255), (0.0, 0.0), (1.0, 1.0), 0.1, 0.0, 2.0,
                       f, [], 64, 32, c, c, "fp64", 8, 1e-8, seed=seed)
    if i == 3:
        c = random_nodes(rng, 3)
        box = [(0.0, 1.0), (0.0, 2.0), (0.0, 1.0)]
        f = _sine_modes(rng, 16, box, 1.0, 20.0)
        return Problem("cfg3-3d-127x255x127", 3, (127, 255, 127), (0.0, 0.0, 0.0),
                       (1.0, 2.0, 1.0), 0.05, 0.0, 1.0, f, [], 128, 16, c, c,
                       "split_bf16", 8, 1e-5, seed=seed)
    if i == 4:
        c = random_nodes(rng, 4)
        box = [(0.0, 1.0), (0.0, 1.0)]
        f = _sine_modes(rng, 12, box, 5.0, 50.0)
        return Problem("cfg4-2d-511-learned", 2, (511, 511), (0.0, 0.0), (1.0, 1.0), 0.01,
                       0.0, 4.0, f, [], 256, 32, c, c, "fp64", 8, 1e-8, seed=seed)
    if i == 5:
        c = random_nodes(rng, 4)
        box = [(0.0, 1.0)] * 3
        f = _sine_modes(rng, 24, box, 2.0, 40.0)
        return Problem("cfg5-3d-255-learned", 3, (255, 255, 255), (0.0,) * 3, (1.0,) * 3,
                       0.02, 0.0, 2.0, f, [], 64, 32, c, c, "split_bf16", 8, 1e-5, seed=seed)
    raise ValueError(f"no configuration {i}")


def random_forcing(seed: int, dim: int, n_modes: int, lohi: Sequence[Tuple[float, float]],
                   omega_lo: float, omega_hi: float, kmax: int = 32) -> List[Term]:
    """A seeded sine-mode forcing of the same family as the configurations
    (used for training pairs of the learned coarse correction)."""
    rng = np.random.default_rng(seed)
    return _sine_modes(rng, n_modes, list(lohi)[:dim], omega_lo, omega_hi, kmax)


def shrink(p: Problem, n: Sequence[int], N: Optional[int] = None, J: Optional[int] = None) -> Problem:
    """The same forcing and time stepping on a different grid / slicing (used
    to build small parity cases that still span several tiles)."""
    kw = dict(n=tuple(n))
    if N is not None:
        kw["N"] = N
    if J is not None:
        kw["J"] = J
    return p.with_(**kw)


# --------------------------------------------------------------------------
# the paper's worked examples (Section 5.1)
# --------------------------------------------------------------------------

def example_5_1(n_elems: int, N: int, M: int, s_fine: int, s_coarse: Optional[int] = None) -> Problem:
    """1D: u_t = u_xx + (2 + x(1-x)) e^t on [0,1], u = x(1-x) e^t, T = 1."""
    sc = s_fine if s_coarse is None else s_coarse
    xx = poly_factor(0.0, 1.0, -1.0)
    f = [Term(2.0, TimeFactor(alpha=1.0), (poly_factor(1.0),)),
         Term(1.0, TimeFactor(alpha=1.0), (xx,))]
    return Problem(f"ex5.1-{n_elems}", 1, (n_elems - 1,), (0.0,), (1.0,), 1.0, 0.0, 1.0, f,
                   [Term(1.0, TimeFactor(), (xx,))], N, M, uniform_nodes(s_fine),
                   uniform_nodes(sc), "fp64", 64, 0.0,
                   exact=[Term(1.0, TimeFactor(alpha=1.0), (xx,))])


def example_5_2(nx: int, ny: int, N: int, M: int, s_fine: int, s_coarse: Optional[int] = None) -> Problem:
    """2D on [1/4,5/4]x[1/8,5/8], D = 1, T = 0.6,
    u = e^{-4 pi^2 t} sin(pi(x-1/4)) sin(2 pi(y-1/8))."""
    sc = s_fine if s_coarse is None else s_coarse
    sx = SpaceFactor(kappa=PI, phase=-PI / 4)
    sy = SpaceFactor(kappa=2 * PI, phase=-2 * PI / 8)
    decay = TimeFactor(alpha=-4 * PI * PI)
    f = [Term(PI * PI, decay, (sx, sy))]
    return Problem(f"ex5.2-{nx}x{ny}", 2, (nx - 1, ny - 1), (0.25, 0.125), (1.25, 0.625), 1.0,
                   0.0, 0.6, f, [Term(1.0, TimeFactor(), (sx, sy))], N, M,
                   uniform_nodes(s_fine), uniform_nodes(sc), "fp64", 64, 0.0,
                   exact=[Term(1.0, decay, (sx, sy))])


def example_5_4(alpha: float, freq: float, n_elems: int = 1024, N: int = 4, M: int = 16,
                s_fine: int = 2, s_coarse: Optional[int] = None) -> Problem:
    """1D oscillating source on [0, 1], T = 1: u_t = alpha u_xx + g, u0 =
    4x(1 - x), homogeneous Dirichlet data, g a hat of half-width w = 0.05 and
    height 100 sqrt(alpha) centred at c(t) = 0.5 + (0.5 - w) sin(2 pi f t);
    N x M = 4 x 16, N_x = 1024 elements, iterated 4 times (the paper shows
    figures only)."""
    sc = s_fine if s_coarse is None else s_coarse
    w = 0.05
    hat = MovingHat(100.0 * math.sqrt(alpha), 0, w, 0.5, 0.5 - w, 2.0 * PI * freq, 0.0,
                    TimeFactor(), (SpaceFactor(),))
    return Problem(f"ex5.4-a{alpha:g}-f{freq:g}", 1, (n_elems - 1,), (0.0,), (1.0,), alpha, 0.0,
                   1.0, [], [Term(1.0, TimeFactor(), (poly_factor(0.0, 4.0, -4.0),))], N, M,
                   uniform_nodes(s_fine), uniform_nodes(sc), "fp64", 4, 0.0, moving=[hat])


def example_5_3(nx: int, N: int, M: int, s_fine: int, s_coarse: Optional[int] = None) -> Problem:
    """3D on [0,1/4]x[1/8,3/8]x[0,1/4], D = 1/8, T = 0.4,
    u = e^{-4 pi^2 t} sin(4pi(x-1/4)) sin(4pi(y-1/8)) sin(4pi(z-1/2))."""
    sc = s_fine if s_coarse is None else s_coarse
    sx = SpaceFactor(kappa=4 * PI, phase=-PI)
    sy = SpaceFactor(kappa=4 * PI, phase=-PI / 2)
    sz = SpaceFactor(kappa=4 * PI, phase=-2 * PI)
    decay = TimeFactor(alpha=-4 * PI * PI)
    f = [Term(2 * PI * PI, decay, (sx, sy, sz))]
    return Problem(f"ex5.3-{nx}", 3, (nx - 1,) * 3, (0.0, 0.125, 0.0), (0.25, 0.375, 0.25),
                   0.125, 0.0, 0.4, f, [Term(1.0, TimeFactor(), (sx, sy, sz))], N, M,
                   uniform_nodes(s_fine), uniform_nodes(sc), "fp64", 64, 0.0,
                   exact=[Term(1.0, decay, (sx, sy, sz))])


def tiny_problem(dim: int, n: Sequence[int], seed: int = 7, n_modes: int = 3, s: int = 3,
                 N: int = 4, J: int = 3, D: float = 0.1, T: float = 0.5,
                 u0_modes: int = 1, precision: str = "fp64") -> Problem:
    """A small seeded problem with a random sine-mode forcing and a random
    sine-mode initial value: the parity workhorse for ragged grids."""
    rng = np.random.default_rng(seed)
    c = random_nodes(rng, s)
    box = [(0.0, 1.0 + 0.25 * a) for a in range(dim)]
    kmax = max(1, min(n))
    f = _sine_modes(rng, n_modes, box, 1.0, 20.0, kmax=kmax)
    u0 = []
    for _ in range(u0_modes):
        ks = rng.integers(1, kmax + 1, dim)
        u0.append(Term(float(rng.normal()), TimeFactor(),
                       tuple(sine_factor(int(k), lo, hi) for k, (lo, hi) in zip(ks, box))))
    return Problem(f"tiny-{dim}d-" + "x".join(map(str, n)), dim, tuple(n),
                   tuple(lo for lo, _ in box), tuple(hi for _, hi in box), D, 0.0, T, f, u0,
                   N, J, c, c, precision, 8, 1e-8, seed=seed)
