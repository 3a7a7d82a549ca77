"""Bars for stored expansion coefficients (imported by tests, not collected).

The coefficient a_l is a quadrature sum whose terms q_j H_l(k rho_j) e^{-il theta_j}
grow like (2/(k rho_j))^l while the sum does not: at l = p its rounding error is
eps times up to 1e13 times its size, in the oracle as much as on the GPU (scipy's
Hankel functions move it as far).  Two checks use that:
  * per element, |a - a_ref| <= 1e-13 B_l + 4 delta G_l, with B_l the sum of the
    terms' moduli (the rounding bound of the sum, ~450 eps of it; for D the
    ladder's (k/2)(B_{l-1} + B_{l+1})), delta the distance between the two sides'
    centers (each places them from the nodes with its own rounding) and G_l the
    bound on the terms' gradient in the center, (k/2)(B_{l-1} + B_{l+1}) for S
    (the ladder for H_l e^{-il theta}) and (k/2)^2 (B_{l-2} + 2 B_l + B_{l+2}) for D;
  * in the disk-weighted norm max |a_l - a_ref_l| s_l / max |a_ref_l| s_l <= 1e-11,
    s_l the largest |J_l(k t)| for t in [0, R]: the size each order can have in the
    potential anywhere inside the center's disk.
"""
import sys

import numpy as np
import scipy.special as sps
import torch

from oracle import qbx_oracle as O

DISK_TOL = 1e-11
ROUND_FACTOR = 1e-13
SENS_FACTOR = 4.0


def term_bounds(pb, centers):
    """B[kind][c, m] = sum_j |q_j| |H_m(k |x'_j - c|)|, m = 0..p+2, with q = w sigma (S) or
    w mu (D, |nu| = 1) on the oracle's source grid."""
    nodes = torch.as_tensor(np.asarray(pb.nodes))
    src = O.source_grid(nodes, pb.oversample)
    fine = O.interpolate_density(torch.as_tensor(np.asarray(pb.density)), pb.oversample)
    w = src["w"].numpy()
    x, y = src["x"].numpy(), src["y"].numpy()
    C = np.asarray(centers)
    rho = np.hypot(x[None, :] - C[:, 0:1], y[None, :] - C[:, 1:2])
    H = np.stack([np.abs(sps.hankel1(m, pb.k * rho)) for m in range(pb.p + 3)], -1)
    return [np.einsum("j,cjm->cm", np.abs(w * fine[i].numpy()), H) for i in range(fine.shape[0])]


def disk_weight(R, k, p):
    """s[c, l + p] = max over t in [0, R_c] of |J_l(k t)| (sampled finely)."""
    t = np.linspace(0.0, 1.0, 257)
    s = np.stack([np.abs(sps.jv(l, k * np.asarray(R)[:, None] * t[None, :])).max(1)
                  for l in range(p + 1)], -1)
    return np.concatenate([s[:, :0:-1], s], -1)


def check_coefficients(a, ref, pb, centers, radii, delta=0.0):
    """Both coefficient bars for every kind; ``delta``: the largest distance between the
    centers of ``a`` and those of ``ref``.  Returns the disk-weighted errors."""
    B = term_bounds(pb, centers)
    s = disk_weight(radii, pb.k, pb.p)
    kinds = {1: "S", 2: "D", 3: "SD"}[pb.kind]
    p, errs = pb.p, []
    for ki, kn in enumerate(kinds):
        Bk, h = B[ki], 0.5 * pb.k
        if kn == "S":
            rnd = np.stack([Bk[:, abs(l)] for l in range(-p, p + 1)], -1)
            sens = np.stack([h * (Bk[:, abs(l - 1)] + Bk[:, abs(l + 1)])
                             for l in range(-p, p + 1)], -1)
        else:
            rnd = np.stack([h * (Bk[:, abs(l - 1)] + Bk[:, abs(l + 1)])
                            for l in range(-p, p + 1)], -1)
            sens = np.stack([h * h * (Bk[:, abs(l - 2)] + 2 * Bk[:, abs(l)] + Bk[:, abs(l + 2)])
                             for l in range(-p, p + 1)], -1)
        bound = ROUND_FACTOR * rnd + SENS_FACTOR * delta * sens
        d = np.abs(a[ki] - ref[ki])
        worst = float((d / bound).max())
        e = float((d * s).max() / (np.abs(ref[ki]) * s).max())
        print(f"  coefficients {kn}: disk-weighted {e:.3e}, worst / rounding bound {worst:.3e}",
              file=sys.stderr, flush=True)
        assert worst <= 1.0
        assert e <= DISK_TOL
        errs.append(e)
    return errs
