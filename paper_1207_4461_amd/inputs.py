"""Seeded synthetic inputs for the QBX hot path.

This module only *creates data*: panel node coordinates sampled from analytic
curves, smooth random densities, random cotangents and the Green's-identity
density pair.  It contains none of the QBX arithmetic (no upsampling, no
weights, no centers, no expansions) and is the only code shared by the CPU
oracle's tests and the GPU path.

Geometry follows the paper's test setup (Section 4.1 "Four test geometries"):
closed counter-clockwise curves gamma(t), t in [0, 2*pi), split into panels
that are equispaced in the parameter, with 16 Gauss-Legendre nodes per panel.
The curve shapes (ellipse, star-shaped "starfish" families, random smooth
star shapes) are the synthetic stand-ins of the workloads listed below.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Dict, List, Optional, Tuple

import numpy as np

Q_NODES = 16  # nodes per panel on the target (Nystrom) grid, Section 4.1

S_KIND = 1
D_KIND = 2
EXTERIOR = 1
INTERIOR = -1
BOTH = 0


# --------------------------------------------------------------------------
# curves: gamma(t) and gamma'(t) for t in [0, 2*pi), counter-clockwise
# --------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Curve:
    """A star-shaped curve r(t)*(cos t, sin t) or an ellipse (a cos t, b sin t)."""

    kind: str                      # "ellipse" or "star"
    a: float = 1.0                 # ellipse semi-axis along x
    b: float = 1.0                 # ellipse semi-axis along y
    modes: Tuple[Tuple[int, float, float], ...] = ()   # star: (m, amplitude, phase)

    def point(self, t: np.ndarray) -> np.ndarray:
        t = np.asarray(t, dtype=np.float64)
        if self.kind == "ellipse":
            return np.stack([self.a * np.cos(t), self.b * np.sin(t)], axis=-1)
        r = np.ones_like(t)
        for m, amp, ph in self.modes:
            r = r + amp * np.cos(m * t + ph)
        return np.stack([r * np.cos(t), r * np.sin(t)], axis=-1)

    def deriv(self, t: np.ndarray) -> np.ndarray:
        t = np.asarray(t, dtype=np.float64)
        if self.kind == "ellipse":
            return np.stack([-self.a * np.sin(t), self.b * np.cos(t)], axis=-1)
        r = np.ones_like(t)
        dr = np.zeros_like(t)
        for m, amp, ph in self.modes:
            r = r + amp * np.cos(m * t + ph)
            dr = dr - amp * m * np.sin(m * t + ph)
        return np.stack([dr * np.cos(t) - r * np.sin(t),
                         dr * np.sin(t) + r * np.cos(t)], axis=-1)


def ellipse(a: float, b: float) -> Curve:
    return Curve("ellipse", a=a, b=b)


def star(*modes: Tuple[int, float, float]) -> Curve:
    return Curve("star", modes=tuple((int(m), float(a), float(p)) for m, a, p in modes))


def gl16_parameters() -> np.ndarray:
    """The 16 Gauss-Legendre abscissae on [-1, 1], ascending (input placement only)."""
    x, _ = np.polynomial.legendre.leggauss(Q_NODES)
    return x


def panel_parameters(n_panels: int) -> np.ndarray:
    """Curve parameter t of every node: [n_panels, 16], panels equispaced in t."""
    tau = gl16_parameters()
    dt = 2.0 * math.pi / n_panels
    t0 = dt * np.arange(n_panels, dtype=np.float64)
    return t0[:, None] + 0.5 * (tau[None, :] + 1.0) * dt


def panel_nodes(curve: Curve, n_panels: int) -> np.ndarray:
    """Node coordinates [n_panels, 16, 2] (float64, C-contiguous)."""
    return np.ascontiguousarray(curve.point(panel_parameters(n_panels)))


# --------------------------------------------------------------------------
# densities and cotangents
# --------------------------------------------------------------------------
def smooth_density(rng: np.random.Generator, t: np.ndarray, max_mode: int = 5) -> np.ndarray:
    """sigma(t) = sum_{m=0..max_mode} c_m e^{imt}, Re c_m, Im c_m iid N(0,1)/(1+m^2)."""
    m = np.arange(max_mode + 1)
    c = (rng.standard_normal(max_mode + 1) + 1j * rng.standard_normal(max_mode + 1)) / (1.0 + m**2)
    tt = np.asarray(t, dtype=np.float64).reshape(-1)
    return np.exp(1j * np.outer(tt, m)) @ c


def complex_normal(rng: np.random.Generator, shape) -> np.ndarray:
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def green_pair(curve: Curve, n_panels: int, k: float, x0=(3.0, 1.0)) -> Tuple[np.ndarray, np.ndarray]:
    """u = H0(k|x - x0|) and du/dn = -k H1(k|x-x0|) (x-x0).n/|x-x0| at the nodes.

    The normal is the exact outward unit normal of the analytic curve; x0 lies
    outside the curve.  Returned flat in node order [n_panels*16], complex128.
    """
    from scipy.special import hankel1

    t = panel_parameters(n_panels).reshape(-1)
    x = curve.point(t)
    d = curve.deriv(t)
    nrm = np.stack([d[:, 1], -d[:, 0]], axis=-1)
    nrm /= np.linalg.norm(nrm, axis=-1, keepdims=True)
    dx = x - np.asarray(x0, dtype=np.float64)[None, :]
    rho = np.linalg.norm(dx, axis=-1)
    u = hankel1(0, k * rho)
    dudn = -k * hankel1(1, k * rho) * np.sum(dx * nrm, axis=-1) / rho
    return u.astype(np.complex128), dudn.astype(np.complex128)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    """One contour with its QBX parameters and inputs (all numpy, host)."""

    name: str
    curve: Curve
    n_panels: int
    k: float
    p: int
    r: float
    oversample: int
    side: int
    kind: int
    nodes: np.ndarray                 # [P, 16, 2] float64
    density: np.ndarray               # [n_kinds, P*16] complex128 (S first, then D)
    cotangent: Optional[np.ndarray] = None   # [n_sides, n_kinds, P*16] complex128

    @property
    def n_kinds(self) -> int:
        return (1 if self.kind & S_KIND else 0) + (1 if self.kind & D_KIND else 0)

    @property
    def n_sides(self) -> int:
        return 2 if self.side == BOTH else 1

    @property
    def n_targets(self) -> int:
        return self.n_panels * Q_NODES

    @property
    def n_sources(self) -> int:
        return self.n_panels * Q_NODES * self.oversample

    @property
    def n_centers(self) -> int:
        return self.n_targets * self.n_sides


def _densities(rng, t, n_kinds, max_mode):
    return np.stack([smooth_density(rng, t, max_mode) for _ in range(n_kinds)])


def make_problem(name: str, curve: Curve, n_panels: int, k: float, p: int, side: int, kind: int,
                 seed: int, r: float = 0.5, oversample: int = 4, max_mode: int = 5,
                 with_cotangent: bool = False) -> Problem:
    rng = np.random.default_rng(seed)
    t = panel_parameters(n_panels).reshape(-1)
    prob = Problem(name=name, curve=curve, n_panels=n_panels, k=float(k), p=int(p), r=float(r),
                   oversample=int(oversample), side=int(side), kind=int(kind),
                   nodes=panel_nodes(curve, n_panels), density=None)  # type: ignore[arg-type]
    prob.density = _densities(rng, t, prob.n_kinds, max_mode)
    if with_cotangent:
        prob.cotangent = complex_normal(rng, (prob.n_sides, prob.n_kinds, prob.n_targets))
    return prob


# The five workloads (sizes, shapes and parameters of the paper's tests scaled to
# one MI355X).  Curves are in t in [0, 2*pi).
def ellipse32(seed: int = 0) -> Problem:
    """Ellipse (1, 0.5), 32 panels, k=10, p=8, exterior, S only."""
    return make_problem("ellipse-32", ellipse(1.0, 0.5), 32, 10.0, 8, EXTERIOR, S_KIND, seed,
                        with_cotangent=True)


def star256(seed: int = 1) -> Problem:
    """Starfish 1+0.25cos5t, 256 panels, k=20, p=12, both sides, S and D."""
    return make_problem("starfish5-256", star((5, 0.25, 0.0)), 256, 20.0, 12, BOTH,
                        S_KIND | D_KIND, seed, with_cotangent=True)


def star256_green(seed: int = 1, x0=(3.0, 1.0)) -> Problem:
    """star256's geometry with the Green's-identity pair: S density du/dn, D density u."""
    prob = star256(seed)
    u, dudn = green_pair(prob.curve, prob.n_panels, prob.k, x0)
    prob.density = np.stack([dudn, u])
    return prob


def star1024(seed: int = 2) -> Problem:
    """Starfish 1+0.3cos7t, 1024 panels, k=40, p=16, exterior, S, fwd+bwd."""
    return make_problem("starfish7-1024", star((7, 0.3, 0.0)), 1024, 40.0, 16, EXTERIOR, S_KIND,
                        seed, with_cotangent=True)


def star4096(seed: int = 4) -> Problem:
    """Starfish 1+0.25cos5t+0.05cos13t, 4096 panels, k=100, p=20, both sides, S+D."""
    return make_problem("starfish5-13-4096", star((5, 0.25, 0.0), (13, 0.05, 0.0)), 4096, 100.0,
                        20, BOTH, S_KIND | D_KIND, seed, max_mode=60, with_cotangent=True)


def paper80(seed: int = 5) -> Problem:
    """The size of the paper's one timing (Section 5: a single-layer apply at p = 5, 7680
    sources, 1280 targets): the Section 4.1 starfish r = 1 + sin(5t)/4 in 80 panels,
    oversample 6 (Section 4.1's factor), one side, k = 0.5 (the value of Section 4's
    operator tests; the timing sentence gives none)."""
    return make_problem("starfish5-80-sec5", star((5, 0.25, -0.5 * math.pi)), 80, 0.5, 5,
                        EXTERIOR, S_KIND, seed, oversample=6, with_cotangent=True)


def random64(seed: int = 3, n_contours: int = 64) -> List[Problem]:
    """64 random star contours r = 1 + sum_{m=2..8} a_m cos(mt+phi_m), a_m~U(0,.05),
    phi_m~U(0,2pi); panels ~U{16..512}; k~U(5,50); p in {8,12,16}; S or D (prob 1/2);
    exterior centers.  Everything is drawn from one generator."""
    rng = np.random.default_rng(seed)
    out = []
    for c in range(n_contours):
        amps = rng.uniform(0.0, 0.05, size=7)
        phis = rng.uniform(0.0, 2.0 * math.pi, size=7)
        curve = star(*[(m, a, ph) for m, a, ph in zip(range(2, 9), amps, phis)])
        n_panels = int(rng.integers(16, 513))
        k = float(rng.uniform(5.0, 50.0))
        p = int(rng.choice([8, 12, 16]))
        kind = S_KIND if rng.uniform() < 0.5 else D_KIND
        sub_seed = int(rng.integers(0, 2**31 - 1))
        out.append(make_problem(f"random-{c}", curve, n_panels, k, p, EXTERIOR, kind, sub_seed,
                                with_cotangent=True))
    return out


@dataclasses.dataclass
class ExplicitProblem:
    """Sources and expansion centers given directly (no panels)."""

    k: float
    p: int
    kind: int
    src_xy: np.ndarray     # [n_src, 2]
    src_nu: np.ndarray     # [n_src, 2] normals (not unit: lengths in [0.5, 1.5])
    src_q: np.ndarray      # [n_kinds, n_src] complex weighted densities
    ctr_xy: np.ndarray     # [n_ctr, 2]
    ctr_r: np.ndarray      # [n_ctr]
    ctr_theta: np.ndarray  # [n_ctr]
    cotangent: np.ndarray  # [n_kinds, n_ctr] complex


def explicit_problem(n_src: int, n_ctr: int, k: float, p: int, kind: int,
                     seed: int) -> ExplicitProblem:
    """Sources at random parameters on the curve r = 1 + 0.1 cos 3t with random
    normals, centers at radius 0.5 with radii in [0.05, 0.25] (every source stays
    at least 0.4 from every center), random target directions."""
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(0.0, 2.0 * math.pi, n_src))
    r = 1.0 + 0.1 * np.cos(3.0 * t)
    src_xy = np.stack([r * np.cos(t), r * np.sin(t)], axis=1)
    ang = rng.uniform(0.0, 2.0 * math.pi, n_src)
    ln = rng.uniform(0.5, 1.5, n_src)
    src_nu = np.stack([ln * np.cos(ang), ln * np.sin(ang)], axis=1)
    nk = (1 if kind & S_KIND else 0) + (1 if kind & D_KIND else 0)
    src_q = complex_normal(rng, (nk, n_src)) * (2.0 * math.pi / n_src)
    phi = rng.uniform(0.0, 2.0 * math.pi, n_ctr)
    ctr_xy = 0.5 * np.stack([np.cos(phi), np.sin(phi)], axis=1)
    ctr_r = rng.uniform(0.05, 0.25, n_ctr)
    ctr_theta = rng.uniform(-math.pi, math.pi, n_ctr)
    cot = complex_normal(rng, (nk, n_ctr))
    return ExplicitProblem(float(k), int(p), int(kind), src_xy, src_nu, src_q, ctr_xy, ctr_r,
                           ctr_theta, cot)


def small(name: str = "small", n_panels: int = 6, k: float = 3.0, p: int = 5, side: int = BOTH,
          kind: int = S_KIND | D_KIND, seed: int = 11, oversample: int = 4,
          curve: Optional[Curve] = None, r: float = 0.5) -> Problem:
    """A tiny problem for dense checks (defaults: starfish-like, 6 panels)."""
    if curve is None:
        curve = star((3, 0.15, 0.3))
    return make_problem(name, curve, n_panels, k, p, side, kind, seed, r=r, oversample=oversample,
                        with_cotangent=True)


CONFIGS: Dict[str, Callable[..., object]] = {
    "ellipse32": ellipse32, "star256": star256, "star1024": star1024, "random64": random64,
    "star4096": star4096, "paper80": paper80,
}
