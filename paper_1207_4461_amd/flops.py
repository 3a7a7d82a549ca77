"""Algorithmic FP64 operation counts of the pair kernels, per (center, source) pair.

Counting rule: add, sub, mul = 1; fused multiply-add = 2; sqrt, reciprocal square
root, divide and rint = 1 each, however the kernel computes them (the kernels refine
a hardware reciprocal square root by a third-order step; that step is not counted).
The counts follow the kernels' formulas for the common branch (every lane of the
wavefront at z = k*rho >= 80: the asymptotic seed with the shortest fits), line by
line:

forward pair (one center, one source, order p):
  geometry      v = x'-c (2), rho = sqrt(vx^2+vy^2) (4), 1/rho (1), cos/sin of
                theta_i - theta' (8), z and 1/z (2)                        = 17
  D geometry    cos/sin(theta_i - arg nu) (6)
  seed H0, H1   80/z and (80/z)^2 (2), 4 interleaved degree-3 polynomials (26),
                Q scaling (2), phase: rounding by 1.5*2^52 and a two-part reduction
                by 2 pi/1024 (7), degree-2 sin/cos polynomials in r^2 (11), times
                the table entry (6), 1/sqrt(z) and the amplitude (3: the table holds
                sqrt(2/pi)), rotation by P + iQ (12)                         =  69
                (waves with a lane at 60 <= z < 80 run degree-4 fits, 78; at
                20 <= z < 60 degree 6, 96; at 10 <= z < 20 degree 9, 123; the long
                fits of 6 <= z < 10 cost 150: so the counts are lower bounds)
  recurrence    per order: H_{l+1} (4) + 2l/z (1)                            =  5
  S per order   J_l cos(l D) (1) + accumulate (4) + Chebyshev cos (2)        =  7
  D per order   J_{l+1} cos(lD+psi) - J_{l-1} cos(lD-psi) (3) + accumulate (4)
                + two Chebyshev sequences (4)                                = 11
  accumulation  w sigma K (8 per kind)

Totals (derived in flops_forward_pair below):
  S:   95 + 12 p         D:   114 + 16 p        S+D: 128 + 23 p
"""
from __future__ import annotations

SEED = 69   # H_0, H_1 on the common branch (see above)


def flops_forward_pair(p: int, kind: int) -> int:
    """FP64 flops per (center, source) pair of the forward pair kernel."""
    S = bool(kind & 1)
    D = bool(kind & 2)
    outer = 2 + 4 + 1 + 4 + 4 + 2          # v, rho, 1/rho, cos D, sin D, z, 1/z
    if D:
        outer += 6                          # cos psi, sin psi
    outer += 8 * (int(S) + int(D))          # w*density*K accumulation
    seed = SEED
    setup = 2                               # 2/z, 2 cos D
    if S:
        setup += 2 + 4                      # H0 J0 term, final 2*sum + term
    if D:
        setup += 3 + 6                      # H0 J1 cos psi term, cos(D +- psi)
    lmax = p + 1 if D else p
    orders = 0
    for l in range(1, lmax + 1):
        if S and l <= p:
            orders += 5
        if D:
            orders += 7 if l <= p - 1 else 5
        if l < lmax:
            orders += 5 + (2 if S else 0) + (4 if D else 0)
    return outer + seed + setup + orders


def interactions(n_centers: int, n_sources: int, kind: int) -> int:
    """Source-center interactions: centers x sources x operators."""
    return n_centers * n_sources * (2 if kind == 3 else 1)


def _pair_sums_flops(p: int, kind: int) -> int:
    """pair_sums() of the forward with tape: seed, recurrences and the complex
    derivative sums K, K_rho, K_theta', K_R, K_theta."""
    S = bool(kind & 1)
    D = bool(kind & 2)
    lmax = p + 1 if D else p
    f = SEED + 2 + (12 if D else 0)           # seed, 2/z and 2 cos D, cos/sin(D +- psi)
    for l in range(1, lmax + 1):
        f += 6 + 1                              # H_{l+1}, H_{l-1} - H_{l+1}, 2l/z
        if S:
            f += 4                              # Chebyshev cos, sin
            if l <= p:
                f += 20                         # K, K_rho, K_theta', K_R
        if D:
            f += 8                              # four Chebyshev sequences
            up = l <= p - 1
            f += (3 if up else 1) + 8           # J_{l+1} a - J_{l-1} b; K, K_rho
            f += (1 if up else 0) + 1 + 2 + 4   # l (J_{l+1} sa - J_{l-1} sb); K_theta'
            f += (3 if up else 1) + 4 + 3 + 4   # K_R; K_theta
    if S:
        f += 24
    if D:
        f += 34
    return f


def _proj_sums_flops(p: int, kind: int, fused: bool) -> int:
    """pair_sums_proj(): K complex, the derivative sums over the real sequences
    Re(w H_l) (one per kind)."""
    S = bool(kind & 1)
    D = bool(kind & 2)
    lmax = p + 1 if D else p
    f = SEED + 2 + (12 if D else 0)
    f += 6 * (int(S) + int(D))                  # Re(w H_0), Re(w H_1) per kind
    for l in range(1, lmax + 1):
        f += 5                                  # H_{l+1} (complex), 2l/z
        if S:
            f += 2 + 4                          # Re(w_S H_{l+1}); Chebyshev cos, sin
            if l <= p:
                # f = J c; K (4); K_rho (sub, fma); K_theta' (l J s, fma); K_R (Jd c, fma)
                f += 1 + 4 + 3 + 4 + (3 if fused else 0)
        if D:
            up = l <= p - 1
            f += 2 + 8                          # Re(w_D H_{l+1}); four Chebyshev sequences
            # f (3 or 1); K (4); K_rho (3); sA, sB (2 or 1); K_theta' (4); K_psi (3)
            f += (3 if up else 1) + 4 + 3 + (2 if up else 1) + 4 + 3
            if fused:
                f += 5 if up else 3             # K_R
    if S:
        f += 6 + 3 + 1 + (4 if fused else 0)
    if D:
        f += 2 + 6 + 5 + 1 + 3 + (5 if fused else 0)
    return f


def flops_tape_pair(p: int, kind: int) -> int:
    """Forward-with-tape pair kernel (center-major): u and the per-center tape."""
    S = bool(kind & 1)
    D = bool(kind & 2)
    outer = 17 + (6 if D else 0)
    outer += 56 * (int(S) + int(D))             # grad_v combination + 5 weighted sums
    return outer + _pair_sums_flops(p, kind)


def _proj_outer(kind: int) -> int:
    S = bool(kind & 1)
    D = bool(kind & 2)
    nk = int(S) + int(D)
    outer = 17 + (6 if D else 0)                # geometry (and the normal's angle)
    outer += 6 * nk                             # w = G q per kind
    outer += 8 * nk                             # conj(G K) per kind
    outer += 2 * (nk - 1) + 1 + 6 + 2           # sum over kinds, grad_v, accumulate
    outer += 1 if D else 0                      # K_psi
    return outer


def flops_adjoint_pair(p: int, kind: int) -> int:
    """Source-major adjoint pair kernel: density, source-position and normal sums."""
    return _proj_outer(kind) + _proj_sums_flops(p, kind, False)


def flops_fused_pair(p: int, kind: int) -> int:
    """Fused adjoint pair kernel: the source-side sums as the source-major pass,
    plus Re w K_R and Re w K_theta for the center side (K_theta = -K_theta' for
    S, K_psi - K_theta' for D)."""
    S = bool(kind & 1)
    D = bool(kind & 2)
    center = (1 if D else 0) + (2 if S and D else 0)
    return _proj_outer(kind) + center + _proj_sums_flops(p, kind, True)


def flops_grad_pair(p: int, kind: int) -> int:
    """Target-derivative pair kernel: the sums of q K_R and q K_theta per kind.  The
    order-weighted values lJ_l = l J_l come from a per-center table, so K_theta costs one
    multiply per term and kind less than with l applied in the pair."""
    S = bool(kind & 1)
    D = bool(kind & 2)
    lmax = p + 1 if D else p
    f = 17 + (6 if D else 0)                    # geometry (and the normal's angle)
    f += 16 * (int(S) + int(D))                 # two complex MACs with q per kind
    f += SEED + 2 + (12 if D else 0)            # seed, 2/z and 2 cos D, cos/sin(D +- psi)
    for l in range(1, lmax + 1):
        if S and l <= p:
            f += 5 + 5                          # K_R (Jd c, MAC); K_theta (lJ s, MAC)
        if D:
            up = l <= p - 1
            f += (7 if up else 5) + (7 if up else 5)   # K_R; K_theta from lJ_{l-+1}
        if l < lmax:
            f += 5 + (4 if S else 0) + (8 if D else 0)   # H_{l+1} and 2l/z; Chebyshev
    if S:
        f += 10
    if D:
        f += 20
    return f


def flops_far_pair(kind: int) -> int:
    """Far pass of the split forward, per (target, source) pair on a far panel (its
    density adjoint has the same count, with the cotangent weight in place of q):
    x - x' (2), rho (4), 1/rho (1), z (1; 80/z is the seed's first multiply, of 1/rho),
    seed H0, H1 on the branch a panel takes when every lane is past k rho >= 80 (69);
    S: w sigma H_0 (8); D: (x - x').n'/rho (4), w mu times it (2), times H_1 (8).
    S: 85, D: 91, S+D: 99.  Panels with a lane nearer run longer fits (9 flops more
    at z >= 60, 27 at z >= 20), so the count is a lower bound."""
    f = 2 + 4 + 1 + 1 + SEED
    if kind & 1:
        f += 8
    if kind & 2:
        f += 4 + 2 + 8
    return f


def near_panel_counts(nodes, gamma: float):
    """Per target panel, the number of source panels the split counts as near:
    |b_m - b_m'|^2 < gamma^2 max(rad2_m, rad2_m'), b the mean of the panel's 16
    nodes and rad2 its largest squared node distance from b (the relation the
    kernels test)."""
    import numpy as np

    X = np.asarray(nodes, dtype=np.float64)
    sx, sy = X[:, 0, 0].copy(), X[:, 0, 1].copy()
    for a in range(1, X.shape[1]):
        sx = sx + X[:, a, 0]
        sy = sy + X[:, a, 1]
    bx, by = sx * 0.0625, sy * 0.0625
    dx, dy = X[:, :, 0] - bx[:, None], X[:, :, 1] - by[:, None]
    rad2 = (dx * dx + dy * dy).max(axis=1)
    ex, ey = bx[:, None] - bx[None, :], by[:, None] - by[None, :]
    g2 = float(gamma) * float(gamma)
    return ((ex * ex + ey * ey) < g2 * np.maximum(rad2[:, None], rad2[None, :])).sum(axis=1)


def split_pairs(nodes, oversample: int, n_sides: int, gamma: float):
    """(center-source pairs of the near pass, target-source pairs of the far pass).

    Near panels lend their q_s = 16 * oversample upsampled sources to each center;
    far panels their 16 nodes (the far rule is the panel's own 16-point rule), the
    pair taken once for both sides.
    """
    cnt = near_panel_counts(nodes, gamma)
    P, qs = len(cnt), 16 * oversample
    near = int(cnt.sum()) * 16 * n_sides * qs
    far = int((P - cnt).sum()) * 16 * 16
    return near, far
