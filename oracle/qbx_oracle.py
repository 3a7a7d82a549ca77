"""CPU FP64 oracle for Quadrature by Expansion (QBX), 2D Helmholtz S and D.

TEST INFRASTRUCTURE ONLY.  Nothing in the product imports this module; only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may call it.  It shares no code with the HIP path.

It follows the paper (Kloeckner, Barnett, Greengard, O'Neil, "Quadrature by
Expansion: A New Method for the Evaluation of Layer Potentials") step by step,
in plain PyTorch CPU ops (float64 / complex128) so that autograd gives exact
gradients of the discrete map:

* Section 4.1: each panel carries a 16-term Legendre expansion of x(tau),
  y(tau), obtained from the 16 Gauss-Legendre node values by GL quadrature
  (a discrete Legendre transform).
* Section 3.4.2: the density is interpolated from the target (Nystrom) grid to
  the finer source grid; the source grid is the q_s = 16*oversample point GL
  rule on the same panel (Section 4.1, "q = 6*16").  Weights are
  w = omega*|dX/dtau|, normals n = (y', -x')/|X'| (outward for counter-
  clockwise curves, Section 3.2), and the panel length h_m = sum of w.
* Section 3.3, step 4(a): center c = x + s*r*h_m*n, s=+1 exterior, -1
  interior, radius R = r*h_m (r = 1/2 in the paper).
* Section 2, eq. (graf-coefficient) and Section 3.2 eq. (graf-coefficient-dlp):
  a_l = sum_j w_j sigma_j H_l(k rho_j) e^{-i l theta_j}, l=-p..p, and the
  double-layer variant with the source normal derivative of
  H_l(k|x'-c|) e^{-i l theta'}, taken by the polar chain rule with
  H_l' = H_{l-1} - (l/z) H_l (DLMF 10.6.2).
  (The paper writes e^{+i l theta'} here and e^{-i l theta} at evaluation; the
  index change l -> -l gives the convention used here, which is identical.)
* Section 3.3, step 4(c): u = (i/4) sum_l a_l J_l(k|x-c|) e^{i l theta}, the
  i/4 of the Helmholtz kernel (i/4) H_0 (Section 1) applied at evaluation.
* Section 3.2: both one-sided limits are returned; the principal value of D is
  their average (eq. dlp-twosided).
* Section 3.2: target derivatives by analytic differentiation of the local
  expansion (``evaluate_gradient``, ``layer_potential_gradient``), through the
  ladder relations of the regular waves J_l e^{i l theta} in x and y; their
  on-surface values (principal value of grad S, finite part of grad D) from
  the one-sided limits by the jump relations (``gradient_principal_value``).
* Section 4.3: the Dirichlet problem by the combined-field representation,
  with S and D as two-sided averages (Section 3.5), solved densely
  (``dirichlet_solve``) and evaluated off the curve (``representation``).
* Section 5: the near/far split (``layer_potential_split``): QBX only for
  sources on panels near the target's panel, the smooth rule applied directly
  at the target for all others; and one stored local expansion serving several
  nearby targets (``expansion_coefficients``, ``evaluate_expansions``).

Two modes:
* ``mode="dense"``: every order l evaluated by its own library call
  (scipy.special.hankel1 / h1vp / jv); numpy; tiny inputs only.
* ``mode="fast"``: H_0, H_1 from the library, higher orders by the upward
  recurrence H_{l+1} = (2l/z) H_l - H_{l-1} (DLMF 10.6.1); J_l from the
  library.  Differentiable (torch autograd) for the adjoint.

Layout conventions shared with the boundary: density [n_kinds][P*16] (S
first, then D), output [n_sides][n_kinds][P*16] with the exterior limit first
when both sides are requested.
"""
from __future__ import annotations

import math
from typing import Dict, Optional, Sequence, Tuple

import numpy as np
import scipy.special as sps
import torch

Q = 16
S_KIND = 1
D_KIND = 2
EXTERIOR = 1
INTERIOR = -1
BOTH = 0

_F64 = torch.float64
_C128 = torch.complex128


# ---------------------------------------------------------------------------
# special functions: library calls, wrapped so autograd can differentiate them
# ---------------------------------------------------------------------------
class _Hankel1(torch.autograd.Function):
    """H^(1)_n(x) for real x > 0 (scipy); derivative (H_{n-1} - H_{n+1})/2 (DLMF 10.6.1)."""

    @staticmethod
    def forward(ctx, x, n):
        ctx.save_for_backward(x)
        ctx.n = n
        return torch.from_numpy(np.asarray(sps.hankel1(n, x.detach().numpy()), dtype=np.complex128))

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        n = ctx.n
        d = hankel1(n - 1, x) - hankel1(n + 1, x)
        return torch.real(torch.conj(g) * 0.5 * d), None


class _BesselJ(torch.autograd.Function):
    """J_n(x) (scipy); derivative (J_{n-1} - J_{n+1})/2 (DLMF 10.6.1)."""

    @staticmethod
    def forward(ctx, x, n):
        ctx.save_for_backward(x)
        ctx.n = n
        return torch.from_numpy(np.asarray(sps.jv(n, x.detach().numpy()), dtype=np.float64))

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        n = ctx.n
        return g * 0.5 * (besselj(n - 1, x) - besselj(n + 1, x)), None


def hankel1(n: int, x: torch.Tensor) -> torch.Tensor:
    return _Hankel1.apply(x, int(n))


def besselj(n: int, x: torch.Tensor) -> torch.Tensor:
    return _BesselJ.apply(x, int(n))


# ---------------------------------------------------------------------------
# Section 4.1: Legendre panel representation; Section 3.4.2: source grid
# ---------------------------------------------------------------------------
def gauss_legendre(n: int) -> Tuple[np.ndarray, np.ndarray]:
    """n-point Gauss-Legendre nodes (ascending) and weights on [-1, 1].

    Nodes from numpy; weights from their defining Christoffel-Darboux form
    w_i = 1 / sum_{j<n} (j + 1/2) P_j(x_i)^2 (a sum of positive terms, accurate to
    rounding; numpy's own weights lose ~1e-12 relative at the ends for n >= 64)."""
    x, _ = np.polynomial.legendre.leggauss(n)
    P = np.polynomial.legendre.legvander(x, n - 1)
    w = 1.0 / np.sum((np.arange(n) + 0.5)[None, :] * P * P, axis=1)
    return x, w


def _legendre_transform(n: int = Q) -> np.ndarray:
    """T[m, a]: Legendre coefficient m of the series through the n GL node values.

    c_m = (2m+1)/2 * sum_a omega_a X_a P_m(tau_a) (GL quadrature of the
    Legendre projection, as in Section 4.1)."""
    tau, om = gauss_legendre(n)
    P = np.polynomial.legendre.legvander(tau, n - 1)          # [a, m] = P_m(tau_a)
    return ((2.0 * np.arange(n) + 1.0) / 2.0)[:, None] * (P * om[:, None]).T


def _legendre_eval(tau: np.ndarray, n: int = Q) -> Tuple[np.ndarray, np.ndarray]:
    """E[b, m] = P_m(tau_b) and E'[b, m] = P_m'(tau_b), m < n."""
    E = np.polynomial.legendre.legvander(tau, n - 1)
    Ed = np.zeros_like(E)
    for m in range(n):
        e = np.zeros(n)
        e[m] = 1.0
        Ed[:, m] = np.polynomial.legendre.legval(tau, np.polynomial.legendre.legder(e))
    return E, Ed


def interpolation_matrices(oversample: int) -> Dict[str, torch.Tensor]:
    """Linear maps from the 16 node values of a panel to the source grid.

    Returns value map V [q_s,16], tau-derivative map Vd [q_s,16], the
    tau-derivative at the 16 nodes themselves Dn [16,16], and the source GL
    weights omega [q_s]."""
    qs = Q * oversample
    T = _legendre_transform(Q)
    tau_s, om_s = gauss_legendre(qs)
    E, Ed = _legendre_eval(tau_s, Q)
    tau_t, _ = gauss_legendre(Q)
    _, Edt = _legendre_eval(tau_t, Q)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(_F64)
    return {"V": t(E @ T), "Vd": t(Ed @ T), "Dn": t(Edt @ T), "omega": t(om_s)}


def source_grid(nodes: torch.Tensor, oversample: int) -> Dict[str, torch.Tensor]:
    """Oversampled source grid of every panel (Section 3.4.2, Section 4.1).

    nodes: [P, 16, 2] float64.  Returns flat source arrays of length P*q_s
    (x, y, w, nx, ny), the panel lengths h [P] and the target normals [P*16, 2]."""
    M = interpolation_matrices(oversample)
    P = nodes.shape[0]
    Xs = torch.einsum("bq,pqd->pbd", M["V"], nodes)            # [P, qs, 2]
    dXs = torch.einsum("bq,pqd->pbd", M["Vd"], nodes)
    speed = torch.sqrt(dXs[..., 0] ** 2 + dXs[..., 1] ** 2)
    w = M["omega"][None, :] * speed                              # arc-length weights
    h = w.sum(dim=1)                                             # panel length
    n_src = torch.stack([dXs[..., 1], -dXs[..., 0]], dim=-1) / speed[..., None]
    dXt = torch.einsum("aq,pqd->pad", M["Dn"], nodes)           # tangent at targets
    n_tgt = torch.stack([dXt[..., 1], -dXt[..., 0]], dim=-1)
    n_tgt = n_tgt / torch.sqrt(n_tgt[..., 0] ** 2 + n_tgt[..., 1] ** 2)[..., None]
    return {
        "x": Xs[..., 0].reshape(-1), "y": Xs[..., 1].reshape(-1), "w": w.reshape(-1),
        "nx": n_src[..., 0].reshape(-1), "ny": n_src[..., 1].reshape(-1),
        "h": h, "n_tgt": n_tgt.reshape(P * Q, 2), "V": M["V"],
    }


def interpolate_density(density: torch.Tensor, oversample: int) -> torch.Tensor:
    """Density on the source grid from its 16 node values per panel (Section 3.4.2).

    density: [..., P*16] complex -> [..., P*q_s] complex."""
    V = interpolation_matrices(oversample)["V"].to(_C128)
    lead = density.shape[:-1]
    d = density.reshape(*lead, -1, Q)
    return torch.einsum("bq,...pq->...pb", V, d).reshape(*lead, -1)


# ---------------------------------------------------------------------------
# Section 3.3 step 4(a): expansion centers
# ---------------------------------------------------------------------------
def expansion_centers(nodes: torch.Tensor, h: torch.Tensor, n_tgt: torch.Tensor, r: float,
                      side: int, center_rule: str = "h") -> Dict[str, torch.Tensor]:
    """c = x + side*R*n (side=+1 exterior, -1 interior) with R = r*h_m, or with
    R = r*sqrt(h_m) for center_rule="sqrt" (Section 3.1 names r = sqrt(h) as the choice
    that makes the error vanish as h -> 0 at fixed p); theta = arg(x - c)."""
    x = nodes.reshape(-1, 2)
    hr = torch.sqrt(h) if center_rule == "sqrt" else h
    R = (r * hr)[:, None].expand(-1, Q).reshape(-1)
    c = x + float(side) * R[:, None] * n_tgt
    d = x - c
    return {"cx": c[:, 0], "cy": c[:, 1], "R": R, "theta": torch.atan2(d[:, 1], d[:, 0])}


# ---------------------------------------------------------------------------
# Section 2 / 3.2: expansion coefficients a_l, l = -p..p
# ---------------------------------------------------------------------------
def _hankel_orders_fast(z: torch.Tensor, lmax: int):
    """H_0..H_lmax at z by the upward recurrence from library H_0, H_1."""
    H = [hankel1(0, z), hankel1(1, z)]
    for l in range(1, lmax):
        H.append((2.0 * l / z) * H[l] - H[l - 1])
    return H[: lmax + 1]


def _coefficients_chunk(src, dens, cx, cy, k, p, kind, mode):
    """a[kind] [C, 2p+1] for one chunk of centers, summing over every source."""
    vx = src["x"][None, :] - cx[:, None]
    vy = src["y"][None, :] - cy[:, None]
    rho = torch.sqrt(vx * vx + vy * vy)
    theta = torch.atan2(vy, vx)
    z = k * rho
    out = {}
    need_d = bool(kind & D_KIND)
    if mode == "fast":
        H = _hankel_orders_fast(z, p + 1)
        Hd = [-H[1]] + [H[l - 1] - (l / z) * H[l] for l in range(1, p + 1)]

        def Hl(L):
            s = 1.0 if L >= 0 or (-L) % 2 == 0 else -1.0
            return s * H[abs(L)]

        def Hdl(L):
            s = 1.0 if L >= 0 or (-L) % 2 == 0 else -1.0
            return s * Hd[abs(L)]
    else:
        zn = z.detach().numpy()
        cache_h, cache_d = {}, {}

        def Hl(L):
            if L not in cache_h:
                cache_h[L] = torch.from_numpy(np.asarray(sps.hankel1(L, zn)))
            return cache_h[L]

        def Hdl(L):
            if L not in cache_d:
                cache_d[L] = torch.from_numpy(np.asarray(sps.h1vp(L, zn)))
            return cache_d[L]

    if need_d:
        # n . v_hat and n . theta_hat for every pair (source normal n_j)
        n_v = (src["nx"][None, :] * vx + src["ny"][None, :] * vy) / rho
        n_t = (-src["nx"][None, :] * vy + src["ny"][None, :] * vx) / rho
    coefs_s, coefs_d = [], []
    for L in range(-p, p + 1):
        phase = torch.exp(-1j * L * theta)
        if kind & S_KIND:
            f = Hl(L) * phase
            coefs_s.append((f * dens["S"][None, :]).sum(dim=1))
        if need_d:
            g = (k * Hdl(L) * n_v - (1j * L / rho) * Hl(L) * n_t) * phase
            coefs_d.append((g * dens["D"][None, :]).sum(dim=1))
    if kind & S_KIND:
        out["S"] = torch.stack(coefs_s, dim=1)
    if need_d:
        out["D"] = torch.stack(coefs_d, dim=1)
    return out


def coefficients(src, dens, ctr, k, p, kind, mode="fast", chunk_pairs=1 << 21):
    """Coefficients a_l for every center (dict kind -> [C, 2p+1] complex)."""
    C = ctr["cx"].shape[0]
    N = src["x"].shape[0]
    step = max(1, chunk_pairs // max(N, 1))
    parts = []
    for c0 in range(0, C, step):
        sl = slice(c0, min(C, c0 + step))
        parts.append(_coefficients_chunk(src, dens, ctr["cx"][sl], ctr["cy"][sl], k, p, kind, mode))
    return {key: torch.cat([q[key] for q in parts], dim=0) for key in parts[0]}


# ---------------------------------------------------------------------------
# Section 3.3 step 4(c): evaluate the local expansion at the target
# ---------------------------------------------------------------------------
def evaluate(a: torch.Tensor, R: torch.Tensor, theta: torch.Tensor, k: float, p: int,
             mode: str = "fast") -> torch.Tensor:
    """u = (i/4) sum_{l=-p}^{p} a_l J_l(kR) e^{i l theta}."""
    x = k * R
    u = torch.zeros(a.shape[0], dtype=_C128)
    for L in range(-p, p + 1):
        if mode == "fast":
            J = besselj(abs(L), x) * (1.0 if L >= 0 or (-L) % 2 == 0 else -1.0)
        else:
            J = torch.from_numpy(np.asarray(sps.jv(L, x.detach().numpy())))
        u = u + a[:, L + p] * J * torch.exp(1j * L * theta)
    return 0.25j * u


def evaluate_gradient(a: torch.Tensor, R: torch.Tensor, theta: torch.Tensor, k: float, p: int,
                      mode: str = "fast") -> torch.Tensor:
    """Target gradient of the local expansion at x = c + R e^{i theta} (Section 3.2:
    derivatives with respect to the target by analytic differentiation of the local
    Bessel expansion).  With the regular waves beta_l(v) = J_l(k|v|) e^{i l arg v},
    the ladder relations (DLMF 10.6.1, written in x and y) are
        d/dx beta_l = (k/2)(beta_{l-1} - beta_{l+1}),
        d/dy beta_l = (ik/2)(beta_{l-1} + beta_{l+1}),
    so for u = (i/4) sum_{|l|<=p} a_l beta_l
        grad u = (i/4)(k/2) sum_l a_l (beta_{l-1} - beta_{l+1}, i (beta_{l-1} + beta_{l+1})).
    Returns [C, 2] complex (du/dx, du/dy)."""
    x = k * R
    beta = {}
    for L in range(-p - 1, p + 2):
        if mode == "fast":
            J = besselj(abs(L), x) * (1.0 if L >= 0 or (-L) % 2 == 0 else -1.0)
        else:
            J = torch.from_numpy(np.asarray(sps.jv(L, x.detach().numpy())))
        beta[L] = J * torch.exp(1j * L * theta)
    gx = torch.zeros(a.shape[0], dtype=_C128)
    gy = torch.zeros(a.shape[0], dtype=_C128)
    for L in range(-p, p + 1):
        gx = gx + a[:, L + p] * (beta[L - 1] - beta[L + 1])
        gy = gy + a[:, L + p] * 1j * (beta[L - 1] + beta[L + 1])
    return 0.25j * 0.5 * k * torch.stack([gx, gy], dim=1)


# ---------------------------------------------------------------------------
# top level
# ---------------------------------------------------------------------------
def _as_t(a, dtype):
    if isinstance(a, torch.Tensor):
        return a.to(dtype)
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype)


def sides_of(side: int) -> Sequence[int]:
    return (EXTERIOR, INTERIOR) if side == BOTH else (side,)


def kinds_of(kind: int) -> Sequence[str]:
    return tuple(k for k, bit in (("S", S_KIND), ("D", D_KIND)) if kind & bit)


def layer_potential(nodes, density, k: float, p: int, r: float = 0.5, oversample: int = 4,
                    side: int = EXTERIOR, kind: int = S_KIND, targets=None, mode: str = "fast",
                    return_aux: bool = False, dipole: str = "normal", center_rule: str = "h"):
    """One-sided QBX limits at the targets.

    nodes [P,16,2] float64, density [n_kinds, P*16] complex128 (S first, then D).
    ``targets``: optional index array into the P*16 targets (sampled evaluation).
    ``dipole="tangential"``: the D slot computes the tangential dipole R of eq. riesz-def,
    the source derivative along the unit tangent t = (x', y')/|x'| (counter-clockwise)
    in place of the normal.  ``center_rule``: see ``expansion_centers``.
    Returns u [n_sides, n_kinds, T] complex128 (exterior first for BOTH)."""
    nodes = _as_t(nodes, _F64)
    density = _as_t(density, _C128)
    kinds = kinds_of(kind)
    src = source_grid(nodes, oversample)
    if dipole == "tangential":
        src = dict(src, nx=-src["ny"], ny=src["nx"])
    fine = interpolate_density(density, oversample)
    dens = {}
    for i, kk in enumerate(kinds):
        dens[kk] = src["w"].to(_C128) * fine[i]
    outs, aux = [], {}
    for s in sides_of(side):
        ctr = expansion_centers(nodes, src["h"], src["n_tgt"], r, s, center_rule)
        if targets is not None:
            idx = torch.as_tensor(np.asarray(targets), dtype=torch.long)
            ctr = {key: val[idx] for key, val in ctr.items()}
        a = coefficients(src, dens, ctr, k, p, kind, mode)
        us = [evaluate(a[kk], ctr["R"], ctr["theta"], k, p, mode) for kk in kinds]
        outs.append(torch.stack(us))
        aux[s] = {"ctr": ctr, "a": a}
    u = torch.stack(outs)
    if return_aux:
        return u, {"src": src, "sides": aux}
    return u


def layer_potential_gradient(nodes, density, k: float, p: int, r: float = 0.5,
                             oversample: int = 4, side: int = EXTERIOR, kind: int = S_KIND,
                             targets=None, mode: str = "fast"):
    """One-sided QBX limits of the target gradient and of the normal derivative
    (S' = n . grad S, D' = n . grad D, as defined at the start of Section 4), from
    the same coefficients as ``layer_potential``.

    Returns (grad [n_sides, n_kinds, T, 2] complex, dn [n_sides, n_kinds, T] complex),
    exterior first for BOTH; n is the outward unit normal at the target."""
    nodes = _as_t(nodes, _F64)
    density = _as_t(density, _C128)
    kinds = kinds_of(kind)
    src = source_grid(nodes, oversample)
    fine = interpolate_density(density, oversample)
    dens = {kk: src["w"].to(_C128) * fine[i] for i, kk in enumerate(kinds)}
    n_tgt = src["n_tgt"]
    if targets is not None:
        idx = torch.as_tensor(np.asarray(targets), dtype=torch.long)
        n_tgt = n_tgt[idx]
    grads = []
    for s in sides_of(side):
        ctr = expansion_centers(nodes, src["h"], src["n_tgt"], r, s)
        if targets is not None:
            ctr = {key: val[idx] for key, val in ctr.items()}
        a = coefficients(src, dens, ctr, k, p, kind, mode)
        grads.append(torch.stack([evaluate_gradient(a[kk], ctr["R"], ctr["theta"], k, p, mode)
                                  for kk in kinds]))
    g = torch.stack(grads)
    dn = g[..., 0] * n_tgt[:, 0].to(_C128) + g[..., 1] * n_tgt[:, 1].to(_C128)
    return g, dn


def target_frame(nodes):
    """Per target: the outward unit normal n (the centers' normal: the 16-node
    derivative rotated, Section 3.2), the unit tangent t with n = (t_2, -t_1) as
    Section 3.2 assumes, i.e. t = (-n_2, n_1), the counter-clockwise direction, and
    the speed |dX/dtau|.  Returns (n [T, 2], t [T, 2], speed [T])."""
    nodes = _as_t(nodes, _F64)
    Dn = interpolation_matrices(1)["Dn"]
    dX = torch.einsum("aq,pqd->pad", Dn, nodes).reshape(-1, 2)
    speed = torch.sqrt(dX[:, 0] ** 2 + dX[:, 1] ** 2)
    n = torch.stack([dX[:, 1], -dX[:, 0]], dim=-1) / speed[:, None]
    t = torch.stack([-n[:, 1], n[:, 0]], dim=-1)
    return n, t, speed


def arclength_derivative(nodes, density):
    """d sigma / ds at the targets: the derivative in the panel parameter of the
    degree-15 interpolant through the 16 node values (the same 16-node derivative
    as the geometry), over the speed |dX/dtau|.  density [..., T] -> [..., T]."""
    nodes = _as_t(nodes, _F64)
    density = _as_t(density, _C128)
    Dn = interpolation_matrices(1)["Dn"].to(_C128)
    lead = density.shape[:-1]
    d = torch.einsum("aq,...pq->...pa", Dn, density.reshape(*lead, -1, Q)).reshape(*lead, -1)
    return d / target_frame(nodes)[2].to(_C128)


def gradient_principal_value(nodes, density, grad, dn, side: int, kind: int):
    """On-surface derivatives from QBX's one-sided limits, by the jump relations of
    Section 3.2 (x on the curve, + the exterior, - the interior):

      grad S(x)  = grad S(x^+-) +- (1/2) n sigma(x)     (principal value),
      d_i D(x)   = d_i D(x^+-)  -+ (1/2) t_i dsigma/ds (finite part, eq. dlpderiv),

    so S' = n . grad S jumps by sigma/2 from each side and D' = n . grad D has no
    jump.  side = BOTH: the average of the two one-sided limits (the two-sided form
    that eq. dlp-twosided uses for D); otherwise the one given limit minus its jump.
    grad [n_sides, n_kinds, T, 2], dn [n_sides, n_kinds, T] (either may be None),
    density [n_kinds, T] (S density first).  Returns (grad [n_kinds, T, 2],
    dn [n_kinds, T])."""
    kinds = kinds_of(kind)
    g = None if grad is None else _as_t(grad, _C128)
    d = None if dn is None else _as_t(dn, _C128)
    if side == BOTH:
        return (None if g is None else 0.5 * (g[0] + g[1]),
                None if d is None else 0.5 * (d[0] + d[1]))
    s = 1.0 if side == EXTERIOR else -1.0
    n, t, _ = target_frame(nodes)
    density = _as_t(density, _C128)
    g_out, d_out = [], []
    for ki, kk in enumerate(kinds):
        if kk == "S":
            sig = density[ki]
            if g is not None:
                g_out.append(g[0, ki] + s * 0.5 * n.to(_C128) * sig[:, None])
            if d is not None:
                d_out.append(d[0, ki] + s * 0.5 * sig)
        else:
            dmu = arclength_derivative(nodes, density[ki])
            if g is not None:
                g_out.append(g[0, ki] - s * 0.5 * t.to(_C128) * dmu[:, None])
            if d is not None:
                d_out.append(d[0, ki])
    return (None if g is None else torch.stack(g_out),
            None if d is None else torch.stack(d_out))


# ---------------------------------------------------------------------------
# Section 5: direct evaluation for distant panels, QBX for the near ones
# ---------------------------------------------------------------------------
def panel_bounds(nodes) -> Tuple[np.ndarray, np.ndarray]:
    """Per panel: b_m, the mean of its 16 nodes (added in node order, then times
    1/16), and rad2_m = max_a |X_{m,a} - b_m|^2.  Returns (b [P, 2], rad2 [P])."""
    X = np.asarray(nodes.detach().numpy() if isinstance(nodes, torch.Tensor) else nodes,
                   dtype=np.float64)
    sx, sy = X[:, 0, 0].copy(), X[:, 0, 1].copy()
    for a in range(1, Q):
        sx = sx + X[:, a, 0]
        sy = sy + X[:, a, 1]
    bx, by = sx * 0.0625, sy * 0.0625
    dx = X[:, :, 0] - bx[:, None]
    dy = X[:, :, 1] - by[:, None]
    rad2 = (dx * dx + dy * dy).max(axis=1)
    return np.stack([bx, by], axis=1), rad2


def near_panels(nodes, gamma: float) -> np.ndarray:
    """near[m, m'] (bool [P, P]): source panel m' is near target panel m when
    |b_m - b_m'|^2 < gamma^2 max(rad2_m, rad2_m') (no fused multiply-add anywhere,
    so any IEEE double implementation takes the same decisions)."""
    b, rad2 = panel_bounds(nodes)
    g2 = float(gamma) * float(gamma)
    dx = b[:, None, 0] - b[None, :, 0]
    dy = b[:, None, 1] - b[None, :, 1]
    return (dx * dx + dy * dy) < g2 * np.maximum(rad2[:, None], rad2[None, :])


def nystrom_grid(nodes: torch.Tensor, density: torch.Tensor, kinds) -> Tuple[dict, dict]:
    """The Nystrom (target) grid as a source grid: the 16 nodes of each panel with
    their own 16-point Gauss-Legendre rule, w = omega |X'(tau)|, the outward normals
    n = (y', -x')/|X'| at the nodes (the derivative of the 16-node interpolant), and
    the node densities weighted, w sigma (no interpolation).  The far sums of the
    near/far split take this grid: away from a panel its 16-point rule is as
    accurate as the oversampled one (Section 3.4.2 oversamples only for the
    expansion coefficients)."""
    _, om = gauss_legendre(Q)
    Dn = interpolation_matrices(1)["Dn"]
    dX = torch.einsum("aq,pqd->pad", Dn, nodes)
    speed = torch.sqrt(dX[..., 0] ** 2 + dX[..., 1] ** 2)
    w = torch.from_numpy(om)[None, :] * speed
    src = {"x": nodes[..., 0].reshape(-1), "y": nodes[..., 1].reshape(-1),
           "w": w.reshape(-1),
           "nx": (dX[..., 1] / speed).reshape(-1), "ny": (-dX[..., 0] / speed).reshape(-1)}
    dens = {kk: src["w"].to(_C128) * density[i] for i, kk in enumerate(kinds)}
    return src, dens


def direct_sum(src, dens, tx, ty, k: float, kind: int, sel) -> Dict[str, torch.Tensor]:
    """Smooth-rule sums over the sources ``sel`` at the targets (tx, ty) [C], without
    the i/4: S: sum_j w_j sigma_j H_0(k rho_j); D: sum_j w_j mu_j dH_0(k|x - x'_j|)/dn'_j
    = sum_j w_j mu_j k H_1(k rho_j) (x - x'_j).n_j / rho_j.  sel: [C, N] bool."""
    dx = tx[:, None] - src["x"][None, :]
    dy = ty[:, None] - src["y"][None, :]
    # rho of an excluded pair may be 0: evaluate there at 1 and drop the term (the
    # square root is taken after the choice, so its derivative stays finite)
    rho = torch.sqrt(torch.where(sel, dx * dx + dy * dy, torch.ones_like(dx)))
    z = k * rho
    out = {}
    if kind & S_KIND:
        out["S"] = torch.where(sel, hankel1(0, z) * dens["S"][None, :], 0.0).sum(dim=1)
    if kind & D_KIND:
        ndot = (dx * src["nx"][None, :] + dy * src["ny"][None, :]) / rho
        term = k * hankel1(1, z) * ndot * dens["D"][None, :]
        out["D"] = torch.where(sel, term, 0.0).sum(dim=1)
    return out


def direct_gradient(src, dens, tx, ty, k: float, kind: int, sel) -> Dict[str, torch.Tensor]:
    """Target gradients of ``direct_sum`` (without the i/4), [C, 2] per kind, by the chain
    rule with u = (x - x')/rho, f = u.n' and H_0' = -H_1, H_1' = H_0 - H_1/z (DLMF 10.6.2):
    S: grad H_0(k rho) = -k H_1 u;
    D: grad [k H_1 f] = k [k H_0 f u + (H_1/rho)(n' - 2 f u)]."""
    dx = tx[:, None] - src["x"][None, :]
    dy = ty[:, None] - src["y"][None, :]
    rho = torch.where(sel, torch.sqrt(dx * dx + dy * dy), torch.ones_like(dx))
    ux, uy = dx / rho, dy / rho
    z = k * rho
    H0, H1 = hankel1(0, z), hankel1(1, z)
    out = {}
    if kind & S_KIND:
        q = torch.where(sel, -k * H1 * dens["S"][None, :], 0.0)
        out["S"] = torch.stack([(q * ux).sum(dim=1), (q * uy).sum(dim=1)], dim=1)
    if kind & D_KIND:
        nx, ny = src["nx"][None, :], src["ny"][None, :]
        f = ux * nx + uy * ny
        a = torch.where(sel, k * k * H0 * f * dens["D"][None, :], 0.0)
        b = torch.where(sel, k * (H1 / rho) * dens["D"][None, :], 0.0)
        gx = a * ux + b * (nx - 2 * f * ux)
        gy = a * uy + b * (ny - 2 * f * uy)
        out["D"] = torch.stack([gx.sum(dim=1), gy.sum(dim=1)], dim=1)
    return out


def layer_potential_split_gradient(nodes, density, k: float, p: int, r: float = 0.5,
                                   oversample: int = 4, side: int = EXTERIOR,
                                   kind: int = S_KIND, gamma: float = 6.0, targets=None,
                                   mode: str = "fast"):
    """Target derivatives with the near/far split (Sections 3.2 and 5): the local
    expansion of the near sources differentiated as in ``layer_potential_gradient``,
    plus (i/4) ``direct_gradient`` of the others.  Returns (grad [n_sides, n_kinds, T, 2],
    dn [n_sides, n_kinds, T]) as ``layer_potential_gradient``."""
    nodes = _as_t(nodes, _F64)
    density = _as_t(density, _C128)
    kinds = kinds_of(kind)
    P = nodes.shape[0]
    src = source_grid(nodes, oversample)
    qs = Q * oversample
    fine = interpolate_density(density, oversample)
    dens = {kk: src["w"].to(_C128) * fine[i] for i, kk in enumerate(kinds)}
    near = near_panels(nodes, gamma)
    tidx = np.arange(P * Q) if targets is None else np.asarray(targets, dtype=np.int64)
    xy = nodes.reshape(-1, 2)
    src_panel = np.arange(P * qs) // qs
    nsrc, ndens = nystrom_grid(nodes, density, kinds)
    node_panel = np.arange(P * Q) // Q
    sides = sides_of(side)
    ctrs = [expansion_centers(nodes, src["h"], src["n_tgt"], r, s) for s in sides]
    g = torch.zeros(len(sides), len(kinds), len(tidx), 2, dtype=_C128)
    for m in np.unique(tidx // Q):
        rows = np.nonzero(tidx // Q == m)[0]
        ti = torch.as_tensor(tidx[rows], dtype=torch.long)
        near_src = near[m][src_panel]
        ni = torch.as_tensor(np.nonzero(near_src)[0], dtype=torch.long)
        sub = {key: src[key][ni] for key in ("x", "y", "nx", "ny")}
        dsub = {kk: dens[kk][ni] for kk in kinds}
        far = torch.as_tensor(np.broadcast_to(~near[m][node_panel],
                                              (len(rows), node_panel.size)).copy())
        dg = direct_gradient(nsrc, ndens, xy[ti, 0], xy[ti, 1], k, kind, far)
        for si in range(len(sides)):
            ctr = {key: val[ti] for key, val in ctrs[si].items()}
            a = coefficients(sub, dsub, ctr, k, p, kind, mode)
            for i, kk in enumerate(kinds):
                g[si, i, torch.as_tensor(rows)] = (
                    evaluate_gradient(a[kk], ctr["R"], ctr["theta"], k, p, mode) + 0.25j * dg[kk])
    n_tgt = src["n_tgt"][torch.as_tensor(tidx, dtype=torch.long)]
    dn = g[..., 0] * n_tgt[:, 0].to(_C128) + g[..., 1] * n_tgt[:, 1].to(_C128)
    return g, dn


def layer_potential_split(nodes, density, k: float, p: int, r: float = 0.5, oversample: int = 4,
                          side: int = EXTERIOR, kind: int = S_KIND, gamma: float = 6.0,
                          targets=None, mode: str = "fast"):
    """One-sided limits with the near/far split of Section 5: for the targets of
    panel m, the sources of panels near m (``near_panels``) enter through the QBX
    expansion about each target's center (coefficients summed over those sources
    only, evaluated as in ``layer_potential``), and every other panel through its
    own 16-point rule on the Nystrom grid (``nystrom_grid``) applied directly at
    the target, (i/4) ``direct_sum``.  Same arguments and layout as
    ``layer_potential``.

    The near sources alone form an open patch whose ends lie about gamma*rad from
    the target; their local expansion converges like (R/d_end)^(p+1), so the split
    adds an error of that size to the QBX error (gamma = 6 suits p = 20; p = 10
    needs gamma near 16 for 1e-12)."""
    nodes = _as_t(nodes, _F64)
    density = _as_t(density, _C128)
    kinds = kinds_of(kind)
    P = nodes.shape[0]
    src = source_grid(nodes, oversample)
    qs = Q * oversample
    fine = interpolate_density(density, oversample)
    dens = {kk: src["w"].to(_C128) * fine[i] for i, kk in enumerate(kinds)}
    near = near_panels(nodes, gamma)
    tidx = np.arange(P * Q) if targets is None else np.asarray(targets, dtype=np.int64)
    xy = nodes.reshape(-1, 2)
    src_panel = np.arange(P * qs) // qs
    nsrc, ndens = nystrom_grid(nodes, density, kinds)
    node_panel = np.arange(P * Q) // Q
    sides = sides_of(side)
    ctrs = [expansion_centers(nodes, src["h"], src["n_tgt"], r, s) for s in sides]
    u = torch.zeros(len(sides), len(kinds), len(tidx), dtype=_C128)
    for m in np.unique(tidx // Q):
        rows = np.nonzero(tidx // Q == m)[0]
        ti = torch.as_tensor(tidx[rows], dtype=torch.long)
        near_src = near[m][src_panel]
        ni = torch.as_tensor(np.nonzero(near_src)[0], dtype=torch.long)
        sub = {key: src[key][ni] for key in ("x", "y", "nx", "ny")}
        dsub = {kk: dens[kk][ni] for kk in kinds}
        far = torch.as_tensor(np.broadcast_to(~near[m][node_panel],
                                              (len(rows), node_panel.size)).copy())
        dsum = direct_sum(nsrc, ndens, xy[ti, 0], xy[ti, 1], k, kind, far)   # both sides
        for si in range(len(sides)):
            ctr = {key: val[ti] for key, val in ctrs[si].items()}
            a = coefficients(sub, dsub, ctr, k, p, kind, mode)
            for i, kk in enumerate(kinds):
                u[si, i, torch.as_tensor(rows)] = (evaluate(a[kk], ctr["R"], ctr["theta"], k, p, mode)
                                                   + 0.25j * dsum[kk])
    return u


def split_vjp(nodes, density, k: float, p: int, r: float, oversample: int, side: int, kind: int,
              cotangent, gamma: float = 6.0):
    """Gradients of L = Re sum conj(g) u, u = ``layer_potential_split``, with respect to the
    density [n_kinds, P*16] (complex, PyTorch convention) and the nodes [P, 16, 2]: autograd
    through the split's own steps (source grid, weights, normals, centers, the QBX
    coefficients of the near sources, the direct rule at the targets for the far ones).
    The near relation is piecewise constant in the nodes and enters as a fixed choice.
    Small inputs only (the whole graph is kept)."""
    X = torch.tensor(np.asarray(nodes, dtype=np.float64), requires_grad=True)
    d = torch.tensor(np.asarray(density, dtype=np.complex128), requires_grad=True)
    u = layer_potential_split(X, d, k, p, r, oversample, side, kind, gamma=gamma)
    g = torch.as_tensor(np.asarray(cotangent, dtype=np.complex128))
    torch.real(torch.sum(torch.conj(g) * u)).backward()
    return d.grad.detach().numpy(), X.grad.detach().numpy()


def split_loss(nodes, density, k, p, r, oversample, side, kind, cotangent, gamma=6.0) -> float:
    """L = Re sum conj(g) u for u = ``layer_potential_split`` (the scalar of ``split_vjp``)."""
    with torch.no_grad():
        u = layer_potential_split(nodes, density, k, p, r, oversample, side, kind,
                                  gamma=gamma).numpy()
    return float(np.real(np.sum(np.conj(np.asarray(cotangent)) * u)))


def apply_explicit(src_xy, src_nu, src_q, ctr_xy, ctr_r, ctr_theta, k: float, p: int,
                   kind: int, mode: str = "fast") -> torch.Tensor:
    """The same expansion for sources and centers given directly (no panels):
    coefficients of Section 2, eq. graf-coefficient (S) and Section 3.2, eq.
    graf-coefficient-dlp (D, the source factor differentiated along the given normal,
    linear in it), evaluated at x_i = c_i + R_i e^{i theta_i} (Section 3.3 step 4(c)).
    src_q [n_kinds, n_src] are the weighted densities.  Returns [n_kinds, n_ctr].
    Differentiable in every argument (autograd)."""
    src_xy = _as_t(src_xy, _F64)
    src_q = _as_t(src_q, _C128)
    ctr_xy = _as_t(ctr_xy, _F64)
    ctr_r = _as_t(ctr_r, _F64)
    ctr_theta = _as_t(ctr_theta, _F64)
    kinds = kinds_of(kind)
    nu = _as_t(src_nu, _F64) if src_nu is not None else torch.zeros_like(src_xy)
    src = {"x": src_xy[:, 0], "y": src_xy[:, 1], "nx": nu[:, 0], "ny": nu[:, 1]}
    dens = {kk: src_q[i] for i, kk in enumerate(kinds)}
    ctr = {"cx": ctr_xy[:, 0], "cy": ctr_xy[:, 1]}
    a = coefficients(src, dens, ctr, k, p, kind, mode)
    return torch.stack([evaluate(a[kk], ctr_r, ctr_theta, k, p, mode) for kk in kinds])


def apply_explicit_vjp(src_xy, src_nu, src_q, ctr_xy, ctr_r, ctr_theta, k: float, p: int,
                       kind: int, cotangent) -> Dict[str, np.ndarray]:
    """Gradients of L = Re sum conj(g) out of apply_explicit (autograd; complex
    inputs in the PyTorch convention dL/dRe + i dL/dIm)."""
    leaves = {
        "src_xy": _as_t(src_xy, _F64).clone().requires_grad_(True),
        "src_nu": (_as_t(src_nu, _F64) if src_nu is not None
                   else torch.zeros(np.shape(src_xy), dtype=_F64)).clone().requires_grad_(True),
        "q": _as_t(src_q, _C128).clone().requires_grad_(True),
        "ctr_xy": _as_t(ctr_xy, _F64).clone().requires_grad_(True),
        "ctr_r": _as_t(ctr_r, _F64).clone().requires_grad_(True),
        "ctr_theta": _as_t(ctr_theta, _F64).clone().requires_grad_(True),
    }
    out = apply_explicit(leaves["src_xy"], leaves["src_nu"], leaves["q"], leaves["ctr_xy"],
                         leaves["ctr_r"], leaves["ctr_theta"], k, p, kind)
    g = _as_t(cotangent, _C128)
    torch.real(torch.conj(g) * out).sum().backward()
    return {key: (val.grad.numpy() if val.grad is not None else np.zeros(tuple(val.shape)))
            for key, val in leaves.items()}


# ---------------------------------------------------------------------------
# Section 5: one local expansion for several nearby targets.  The coefficients of
# eq. graf-coefficient (and eq. graf-coefficient-dlp) are formed once per center and
# stored; any target inside a center's disk is then evaluated from them by Section 3.3
# step 4(c) with its own distance and angle from the center.
# ---------------------------------------------------------------------------
def expansion_coefficients(nodes, density, k: float, p: int, r: float = 0.5,
                           oversample: int = 4, side: int = EXTERIOR, kind: int = S_KIND,
                           mode: str = "fast", centers=None):
    """Local expansion coefficients a_l, l = -p..p, of every center of the contour (the
    centers of ``layer_potential``, exterior ones first for BOTH), without the i/4.
    ``centers``: optional index array into those centers (sampled evaluation).
    Returns (a [n_kinds, n_centers, 2p+1] complex, centers [n_centers, 2], radii
    [n_centers])."""
    nodes = _as_t(nodes, _F64)
    density = _as_t(density, _C128)
    kinds = kinds_of(kind)
    src = source_grid(nodes, oversample)
    fine = interpolate_density(density, oversample)
    dens = {kk: src["w"].to(_C128) * fine[i] for i, kk in enumerate(kinds)}
    parts = [expansion_centers(nodes, src["h"], src["n_tgt"], r, s) for s in sides_of(side)]
    ctr = {key: torch.cat([c[key] for c in parts]) for key in parts[0]}
    if centers is not None:
        idx = torch.as_tensor(np.asarray(centers), dtype=torch.long)
        ctr = {key: val[idx] for key, val in ctr.items()}
    a = coefficients(src, dens, ctr, k, p, kind, mode)
    return (torch.stack([a[kk] for kk in kinds]), torch.stack([ctr["cx"], ctr["cy"]], dim=-1),
            ctr["R"])


def evaluate_expansions(coef, centers, targets, center_index, k: float, p: int,
                        mode: str = "fast") -> torch.Tensor:
    """u(x_t) = (i/4) sum_{l=-p..p} a_l J_l(k|x_t - c|) e^{i l arg(x_t - c)} with c the
    center ``center_index[t]`` (Section 3.3 step 4(c) at a target of the caller's
    choice inside the center's disk).  coef [n_kinds, n_centers, 2p+1]; returns
    [n_kinds, n_targets]."""
    coef = _as_t(coef, _C128)
    centers = _as_t(centers, _F64)
    targets = _as_t(targets, _F64)
    idx = torch.as_tensor(np.asarray(center_index), dtype=torch.long)
    d = targets - centers[idx]
    R = torch.sqrt(d[:, 0] ** 2 + d[:, 1] ** 2)
    theta = torch.atan2(d[:, 1], d[:, 0])
    return torch.stack([evaluate(coef[i, idx], R, theta, k, p, mode)
                        for i in range(coef.shape[0])])


def assign_centers(centers, radii, targets, slack: float = 1.0) -> np.ndarray:
    """For every target, the nearest center whose disk holds it (|x - c| <= slack R),
    or -1 if no disk does."""
    c = np.asarray(centers, dtype=np.float64)
    R = np.asarray(radii, dtype=np.float64)
    t = np.asarray(targets, dtype=np.float64)
    d2 = (t[:, None, 0] - c[None, :, 0]) ** 2 + (t[:, None, 1] - c[None, :, 1]) ** 2
    inside = d2 <= (slack * R[None, :]) ** 2
    d2 = np.where(inside, d2, np.inf)
    best = np.argmin(d2, axis=1)
    return np.where(np.isfinite(d2[np.arange(len(t)), best]), best, -1)


def qbx_matrix(nodes, k: float, p: int, r: float = 0.5, oversample: int = 4, side: int = EXTERIOR,
               kind_name: str = "S") -> np.ndarray:
    """Dense QBX operator A [T, P*16] (targets x coarse density) for one side and kind.

    A = K diag(w) U: K_ij = (i/4) sum_{|l|<=p} J_l(kR_i) e^{il theta_i} G_l(x'_j - c_i), the
    regularized kernel of Section 2 (eq. qbx-kernel), with G_l = H_l(k rho) e^{-il theta'}
    for S and its source-normal derivative (library derivative h1vp) for D, every order a
    separate library call; w the source weights; U the block-diagonal 16 -> q_s
    interpolation of Section 3.4.2.  Tiny inputs only."""
    with torch.no_grad():
        nodes = _as_t(nodes, _F64)
        src = source_grid(nodes, oversample)
        ctr = expansion_centers(nodes, src["h"], src["n_tgt"], r, side)
        vx = (src["x"][None, :] - ctr["cx"][:, None]).numpy()
        vy = (src["y"][None, :] - ctr["cy"][:, None]).numpy()
        rho = np.hypot(vx, vy)
        th = np.arctan2(vy, vx)
        z = k * rho
        kR = (k * ctr["R"]).numpy()[:, None]
        tht = ctr["theta"].numpy()[:, None]
        nx, ny = src["nx"].numpy()[None, :], src["ny"].numpy()[None, :]
        K = np.zeros(rho.shape, dtype=np.complex128)
        for L in range(-p, p + 1):
            beta = sps.jv(L, kR) * np.exp(1j * L * tht)
            if kind_name == "S":
                G = sps.hankel1(L, z) * np.exp(-1j * L * th)
            else:
                n_v = (nx * vx + ny * vy) / rho
                n_t = (-nx * vy + ny * vx) / rho
                G = (k * sps.h1vp(L, z) * n_v - (1j * L / rho) * sps.hankel1(L, z) * n_t) * np.exp(-1j * L * th)
            K += beta * G
        K *= 0.25j * src["w"].numpy()[None, :]
        V = src["V"].numpy()
        P = nodes.shape[0]
        U = np.kron(np.eye(P), V)
        return K @ U


# ---------------------------------------------------------------------------
# Section 4.3: the Dirichlet problem by the combined-field representation
# ---------------------------------------------------------------------------
def dirichlet_matrix(nodes, k: float, p: int, r: float = 0.5, oversample: int = 4,
                     side: int = EXTERIOR, alpha: complex = 1j) -> np.ndarray:
    """The Nystrom matrix of eq. dirichlet-inteq, -+ I/2 + alpha S - D (upper sign: the
    exterior problem), with S and D the principal values taken as the averages of the two
    one-sided QBX limits (eq. dlp-twosided).  Section 3.5: the one-sided QBX limit of D
    damps high-frequency densities but not the sigma/2 of its jump, so only the
    two-sided average keeps the discrete spectrum clustering like the continuous one
    (and GMRES converging below the discretization error).  [T, T], tiny inputs only."""
    S = 0.5 * (qbx_matrix(nodes, k, p, r, oversample, EXTERIOR, "S")
               + qbx_matrix(nodes, k, p, r, oversample, INTERIOR, "S"))
    D = 0.5 * (qbx_matrix(nodes, k, p, r, oversample, EXTERIOR, "D")
               + qbx_matrix(nodes, k, p, r, oversample, INTERIOR, "D"))
    half = -0.5 if side == EXTERIOR else 0.5
    return half * np.eye(S.shape[0]) + alpha * S - D


def dirichlet_solve(nodes, f, k: float, p: int, r: float = 0.5, oversample: int = 4,
                    side: int = EXTERIOR, alpha: complex = 1j) -> np.ndarray:
    """sigma [T] at the nodes solving (-+ I/2 + alpha S - D) sigma = f by a dense direct
    solve (the discrete solution that the paper's GMRES iteration converges to)."""
    A = dirichlet_matrix(nodes, k, p, r, oversample, side, alpha)
    return np.linalg.solve(A, np.asarray(f, dtype=np.complex128))


def representation(nodes, sigma, k: float, points, oversample: int = 4,
                   alpha: complex = 1j) -> np.ndarray:
    """u(y) = -D sigma(y) + alpha S sigma(y) at points y [n, 2] away from the curve, by the
    smooth source rule (Section 4.3 evaluates the representation at observation
    points inside the domain)."""
    nodes = _as_t(nodes, _F64)
    src = source_grid(nodes, oversample)
    q = src["w"].to(_C128) * interpolate_density(_as_t(sigma, _C128)[None], oversample)[0]
    pts = torch.as_tensor(np.asarray(points, dtype=np.float64))
    sel = torch.ones(pts.shape[0], q.shape[0], dtype=torch.bool)
    d = direct_sum(src, {"S": q, "D": q}, pts[:, 0], pts[:, 1], k, S_KIND | D_KIND, sel)
    return (0.25j * (alpha * d["S"] - d["D"])).numpy()


# ---------------------------------------------------------------------------
# adjoint: gradients of L = Re <g, u> by autograd through the steps above
# ---------------------------------------------------------------------------
def vjp(nodes, density, k: float, p: int, r: float, oversample: int, side: int, kind: int,
        cotangent, panels=None, chunk_pairs: int = 1 << 20):
    """Gradients of L = Re sum conj(g) u with respect to density [n_kinds, P*16] (complex,
    PyTorch convention dL/dRe + i dL/dIm) and nodes [P, 16, 2].

    With ``panels`` (indices), only those panels' gradients are exact: the loss is
    restricted to the pairs that touch them (their centers against every source, plus
    every other center against their sources), which has the same gradient on them.
    Work is split into center chunks, each rebuilt and back-propagated on its own."""
    nodes_np = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64))
    dens_np = np.ascontiguousarray(np.asarray(density, dtype=np.complex128))
    g_np = np.asarray(cotangent, dtype=np.complex128)
    P = nodes_np.shape[0]
    T = P * Q
    qs = Q * oversample
    kinds = kinds_of(kind)
    g_nodes = torch.zeros(P, Q, 2, dtype=_F64)
    g_dens = torch.zeros(len(kinds), T, dtype=_C128)
    all_src = np.arange(P * qs)
    if panels is None:
        groups = [(np.arange(T), all_src)]
    else:
        pm = np.zeros(P, dtype=bool)
        pm[np.asarray(panels)] = True
        tgt_in = np.repeat(pm, Q)
        src_in = np.repeat(pm, qs)
        groups = [(np.nonzero(tgt_in)[0], all_src), (np.nonzero(~tgt_in)[0], np.nonzero(src_in)[0])]
    for si, s in enumerate(sides_of(side)):
        for tgt_idx, src_idx in groups:
            if len(tgt_idx) == 0 or len(src_idx) == 0:
                continue
            step = max(1, chunk_pairs // len(src_idx))
            for c0 in range(0, len(tgt_idx), step):
                sel = torch.as_tensor(tgt_idx[c0:c0 + step], dtype=torch.long)
                sidx = torch.as_tensor(src_idx, dtype=torch.long)
                X = torch.from_numpy(nodes_np).clone().requires_grad_(True)
                Dn = torch.from_numpy(dens_np).clone().requires_grad_(True)
                src = source_grid(X, oversample)
                fine = interpolate_density(Dn, oversample)
                srcs = {key: src[key][sidx] for key in ("x", "y", "nx", "ny", "w")}
                dens = {kk: srcs["w"].to(_C128) * fine[i][sidx] for i, kk in enumerate(kinds)}
                ctr = expansion_centers(X, src["h"], src["n_tgt"], r, s)
                ctr = {key: val[sel] for key, val in ctr.items()}
                a = coefficients(srcs, dens, ctr, k, p, kind, "fast", chunk_pairs)
                L = torch.zeros((), dtype=_F64)
                for ki, kk in enumerate(kinds):
                    u = evaluate(a[kk], ctr["R"], ctr["theta"], k, p, "fast")
                    g = torch.from_numpy(g_np[si, ki][sel.numpy()])
                    L = L + torch.real(torch.conj(g) * u).sum()
                L.backward()
                g_nodes += X.grad
                g_dens += Dn.grad
    return g_dens.numpy(), g_nodes.numpy()


def loss(nodes, density, k, p, r, oversample, side, kind, cotangent) -> float:
    """L = Re sum conj(g) u (the scalar whose gradients ``vjp`` returns)."""
    with torch.no_grad():
        u = layer_potential(nodes, density, k, p, r, oversample, side, kind).numpy()
    return float(np.real(np.sum(np.conj(np.asarray(cotangent)) * u)))
