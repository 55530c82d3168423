"""Seeded synthetic multi-period AC OPF instances.

The public cases the paper benchmarks (IEEE-30/118, PEGASE-1354/9241 with
generated load profiles, Table 2 and the paragraph after it) are not
available, so every workload here is a seeded synthetic grid with the same
structure: a meshed transmission network (spanning tree plus random extra
lines), one generator per generator bus, bus loads that follow a scaled
periodic profile over the horizon (the paper's load recipe: a perturbed,
scaled periodic function), and an evaluation point, multipliers and
condensation weights drawn inside the bounds.

This module only draws numbers.  It holds none of the model's arithmetic
(no power flow, no derivative, no KKT algebra) so that both the CPU oracle
and the HIP path can consume its arrays without sharing any of the method.

The variable vector ``x`` and constraint vector ``c`` use the library's
canonical period-major layout (0-based):

    x = concat_t [vm(N) | va(N) | pg(G) | qg(G) | pf(B) | qf(B) | pt(B) | qt(B)]
    c = concat_t [balP(N) | balQ(N) | ref(1) | cpf(B) | cqf(B) | cpt(B) |
                  cqt(B) | thf(B) | tht(B) | ang(B)]  followed by the ramp
        rows ramp[(t-1)*G + g] for t = 1..T-1.

Only the sizes of those blocks are needed to draw vectors of the right
length; the draw order below is part of the recipe and fixed.
"""
from __future__ import annotations

import math
import dataclasses
from dataclasses import dataclass

import numpy as np

SEEDS = {"tiny": 1, "mid": 2, "paper": 3}
BATCH_SEED0 = 4000
ADJOINT_SEED0 = 5000

SHAPES = {
    "tiny": dict(N=14, B=20, G=5, T=4),
    "mid": dict(N=2000, B=3200, G=400, T=24),
    "paper": dict(N=10000, B=13000, G=2000, T=168),
}


@dataclass
class Network:
    """One instance: topology, per-element data and the load profile."""

    N: int
    B: int
    G: int
    T: int
    ref_bus: int
    vmin: np.ndarray
    vmax: np.ndarray
    f_bus: np.ndarray
    t_bus: np.ndarray
    r: np.ndarray
    x: np.ndarray
    b_charge: np.ndarray
    rate: np.ndarray
    angmin: np.ndarray
    angmax: np.ndarray
    tap: np.ndarray
    shift: np.ndarray
    gen_bus: np.ndarray
    c2: np.ndarray
    c1: np.ndarray
    c0: np.ndarray
    pmin: np.ndarray
    pmax: np.ndarray
    qmin: np.ndarray
    qmax: np.ndarray
    ramp: np.ndarray
    pd: np.ndarray  # (T, N) period-major
    qd: np.ndarray  # (T, N)

    @property
    def n_period(self) -> int:
        return 2 * self.N + 2 * self.G + 4 * self.B

    @property
    def m_period(self) -> int:
        return 2 * self.N + 7 * self.B + 1

    @property
    def n(self) -> int:
        return self.T * self.n_period

    @property
    def m(self) -> int:
        return self.T * self.m_period + self.G * (self.T - 1)


def make_network(N: int, B: int, G: int, T: int, seed: int, rng=None) -> Network:
    """Draw a network in the fixed order: tree, extra lines, line data,
    generators, loads.  ``rng`` may be passed to continue an existing stream
    (the batched recipe draws the shape first from the same stream)."""
    if N < 2 or B < N - 1 or G < 1 or G > N or T < 1:
        raise ValueError("need N >= 2, B >= N-1, 1 <= G <= N, T >= 1")
    if B > N * (N - 1) // 2:
        raise ValueError("too many lines for a simple graph")
    if rng is None:
        rng = np.random.default_rng(seed)
    # 1. spanning tree: bus i (i >= 1) hangs off a uniformly drawn earlier bus
    parent = rng.integers(0, np.arange(1, N)) if N > 1 else np.zeros(0, np.int64)
    f = list(parent.astype(np.int64))
    t = list(range(1, N))
    seen = {(min(a, b), max(a, b)) for a, b in zip(f, t)}
    # 2. extra lines between distinct, not yet connected bus pairs
    while len(f) < B:
        u, v = rng.integers(0, N, 2)
        u, v = int(u), int(v)
        key = (min(u, v), max(u, v))
        if u == v or key in seen:
            continue
        seen.add(key)
        f.append(u)
        t.append(v)
    f_bus = np.asarray(f, dtype=np.int32)
    t_bus = np.asarray(t, dtype=np.int32)
    # 3. line data (per unit)
    r = rng.uniform(0.001, 0.05, B)
    x = rng.uniform(0.01, 0.3, B)
    b_charge = rng.uniform(0.0, 0.1, B)
    rate = rng.uniform(0.5, 3.0, B)
    angmin = np.full(B, -math.pi / 6)
    angmax = np.full(B, math.pi / 6)
    tap = np.ones(B)
    shift = np.zeros(B)
    # 4. generators, one per generator bus
    gen_bus = rng.choice(N, G, replace=False).astype(np.int32)
    ref_bus = int(gen_bus[0])
    c2 = rng.uniform(0.0, 0.1, G)
    c1 = rng.uniform(10.0, 40.0, G)
    c0 = np.zeros(G)
    pmin = np.zeros(G)
    pmax = rng.uniform(1.0, 5.0, G)
    qmax = 0.5 * pmax
    qmin = -qmax
    ramp = np.full(G, 0.2)
    vmin = np.full(N, 0.9)
    vmax = np.full(N, 1.1)
    # 5. loads: per-bus base times a diurnal factor over 0-based periods
    base = rng.uniform(0.0, 1.0, N)
    factor = 0.7 + 0.3 * np.sin(2.0 * math.pi * np.arange(T) / 24.0)
    pd = np.ascontiguousarray(factor[:, None] * base[None, :])
    qd = 0.3 * pd
    return Network(N, B, G, T, ref_bus, vmin, vmax, f_bus, t_bus, r, x, b_charge,
                   rate, angmin, angmax, tap, shift, gen_bus, c2, c1, c0, pmin,
                   pmax, qmin, qmax, ramp, pd, qd)


def config_network(name: str) -> Network:
    s = SHAPES[name]
    return make_network(s["N"], s["B"], s["G"], s["T"], SEEDS[name])


def cap_load(net: Network, frac: float) -> Network:
    """The same network with every period's real and reactive loads scaled
    by one factor, chosen so that the peak period's total real load is at
    most ``frac`` of the total generation capacity (sum of pmax).  With the
    random ratings and limits of the draws, the single-period problems of
    the heavier periods have no feasible point that either the interior-point
    loop or a general constrained solver finds; capped loads give instances
    a whole solve can finish."""
    s = min(1.0, frac * float(net.pmax.sum()) / float(net.pd.sum(axis=1).max()))
    return dataclasses.replace(net, pd=net.pd * s, qd=net.qd * s)


def batched_shape(rng) -> tuple[int, int, int, int]:
    """Uneven batch member: N log-uniform on [100, 5000], B = 1.4N,
    G = 0.2N, T uniform on {6..48}."""
    N = int(round(math.exp(rng.uniform(math.log(100), math.log(5000)))))
    B = int(round(1.4 * N))
    G = int(round(0.2 * N))
    T = int(rng.integers(6, 49))
    return N, B, G, T


def batched_networks(k: int = 64, seed0: int = BATCH_SEED0) -> list[Network]:
    nets = []
    for i in range(k):
        rng = np.random.default_rng(seed0 + i)
        N, B, G, T = batched_shape(rng)
        nets.append(make_network(N, B, G, T, seed0 + i, rng=rng))
    return nets


def adjoint_networks(k: int = 16, seed0: int = ADJOINT_SEED0) -> list[Network]:
    s = SHAPES["mid"]
    return [make_network(s["N"], s["B"], s["G"], s["T"], seed0 + i) for i in range(k)]


@dataclass
class Point:
    """Evaluation data: primal point, multipliers, objective weight and the
    condensation weights (caller-side diagonals of the condensed matrix)."""

    x: np.ndarray
    lam: np.ndarray
    sigma: float
    diag_x: np.ndarray
    dcon: np.ndarray


def make_point(net: Network, seed: int, stress: bool = False) -> Point:
    """Draw x inside the bounds, multipliers ~ N(0,1), and log-uniform
    weights on [1e-4, 1e4].  ``stress`` draws angles on [-pi, pi]."""
    rng = np.random.default_rng(10_000 + seed)
    N, B, G, T = net.N, net.B, net.G, net.T
    vm = rng.uniform(0.9, 1.1, (T, N))
    va = rng.uniform(-math.pi, math.pi, (T, N)) if stress else rng.uniform(-0.5, 0.5, (T, N))
    pg = rng.uniform(net.pmin, net.pmax, (T, G))
    qg = rng.uniform(net.qmin, net.qmax, (T, G))
    flows = [rng.uniform(-net.rate, net.rate, (T, B)) for _ in range(4)]
    x = np.concatenate([vm, va, pg, qg] + flows, axis=1).reshape(-1)
    lam = rng.standard_normal(net.m)
    diag_x = 10.0 ** rng.uniform(-4.0, 4.0, net.n)
    dcon = 10.0 ** rng.uniform(-4.0, 4.0, net.m)
    return Point(np.ascontiguousarray(x), lam, 1.0, diag_x, dcon)


@dataclass
class IpmState:
    """An iterate of the lifted interior-point method: primal x, slacks s of
    the relaxed rows c(x) - s = 0, multipliers y of those rows, bound
    multipliers (zl, zu of x, vl, vu of s), the bounds themselves (+-inf =
    absent), the barrier parameter and the two regularisations."""

    x: np.ndarray
    s: np.ndarray
    y: np.ndarray
    zl: np.ndarray
    zu: np.ndarray
    vl: np.ndarray
    vu: np.ndarray
    xl: np.ndarray
    xu: np.ndarray
    sl: np.ndarray
    su: np.ndarray
    mu: float
    delta_w: float
    delta_c: float


def _interior(rng, lo, hi):
    """One value strictly inside each [lo, hi] (either side may be infinite)."""
    fl, fu = np.isfinite(lo), np.isfinite(hi)
    u = rng.uniform(0.05, 0.95, lo.shape)
    e = np.exp(rng.uniform(-3.0, 1.0, lo.shape))
    z = rng.standard_normal(lo.shape)
    out = np.where(fl & fu, np.where(fl & fu, lo, 0.0) + u * np.where(fl & fu, hi - lo, 0.0), z)
    out = np.where(fl & ~fu, np.where(fl, lo, 0.0) + e, out)
    out = np.where(~fl & fu, np.where(fu, hi, 0.0) - e, out)
    return out


def make_ipm_state(xl, xu, cl, cu, seed: int, eps: float = 1e-4) -> IpmState:
    """Draw an interior iterate for the given variable and row bounds.

    Slack bounds are the row bounds with equality rows widened to +-eps (the
    relaxation width is the solver's choice); x and s lie strictly inside
    their bounds (free entries ~ N(0, 1)); each multiplier of a finite bound
    is log-uniform on [1e-3, 1e1], 0 where the bound is absent; y ~ N(0, 1);
    mu = 0.1, delta_w = 1e-4, delta_c = 1e-6."""
    rng = np.random.default_rng(20_000 + seed)
    xl, xu = np.asarray(xl, dtype=np.float64), np.asarray(xu, dtype=np.float64)
    cl, cu = np.asarray(cl, dtype=np.float64), np.asarray(cu, dtype=np.float64)
    eq = cl == cu
    sl = np.where(eq, cl - eps, cl)
    su = np.where(eq, cu + eps, cu)
    x = _interior(rng, xl, xu)
    s = _interior(rng, sl, su)
    mult = lambda b: np.where(np.isfinite(b), 10.0 ** rng.uniform(-3.0, 1.0, b.shape), 0.0)
    zl, zu, vl, vu = mult(xl), mult(xu), mult(sl), mult(su)
    y = rng.standard_normal(cl.shape)
    return IpmState(x, s, y, zl, zu, vl, vu, xl, xu, sl, su, 0.1, 1e-4, 1e-6)
