"""Pins of the oracle's Dirichlet solve (Section 4.3: the combined-field representation
u = -D sigma + alpha S sigma, eq. dirichlet-inteq, Nystrom at the nodes, S and D as
two-sided averages per Section 3.5) against exact
solutions it does not produce: fields of point charges (H_0 sources) placed outside the
domain, evaluated at observation points inside it.  The error falls under refinement;
planted mistakes (the D term's sign, the sign of sigma/2) are caught."""
import numpy as np
import scipy.special as sps

from oracle import qbx_oracle as O
from paper_1207_4461_amd import inputs as I

K = 3.0
CASES = {
    # side: (charges (x, y, strength) outside the domain, observation points inside it)
    I.EXTERIOR: ([(0.1, 0.2, 1.0), (-0.3, 0.1, 0.5 - 0.2j)],
                 [(2.0, 0.5), (-1.5, 1.7), (0.3, -2.2)]),
    I.INTERIOR: ([(2.5, 0.3, 1.0), (-1.0, 2.4, 0.7j)],
                 [(0.1, 0.1), (-0.3, 0.2), (0.2, -0.3)]),
}


def charges_field(pts, charges, k=K):
    pts = np.asarray(pts, dtype=np.float64)
    u = np.zeros(len(pts), dtype=np.complex128)
    for cx, cy, c in charges:
        u += c * sps.hankel1(0, k * np.hypot(pts[:, 0] - cx, pts[:, 1] - cy))
    return u


def solve_error(side, P, p, oversample=2):
    charges, obs = CASES[side]
    nodes = I.panel_nodes(I.ellipse(1.0, 0.6), P)
    f = charges_field(nodes.reshape(-1, 2), charges)
    sigma = O.dirichlet_solve(nodes, f, K, p, oversample=oversample, side=side)
    u = O.representation(nodes, sigma, K, np.asarray(obs), oversample=oversample)
    ex = charges_field(obs, charges)
    return float(np.abs(u - ex).max() / np.abs(ex).max())


def test_point_charges_exterior_and_interior():
    for side, bound, bound8 in ((I.EXTERIOR, 3e-5, 1e-6), (I.INTERIOR, 1e-4, 5e-6)):
        e8, e12 = solve_error(side, 8, 6), solve_error(side, 12, 6)
        assert e12 < bound and e8 > 5 * e12, (side, e8, e12)
        assert solve_error(side, 12, 8) < bound8


def test_planted_dirichlet_mistakes_are_caught(monkeypatch):
    orig = O.dirichlet_matrix

    def d_sign(nodes, k, p, r=0.5, oversample=4, side=1, alpha=1j):
        return orig(nodes, k, p, r, oversample, side, alpha) + 2 * O.qbx_matrix(
            nodes, k, p, r, oversample, side, "D")

    def wrong_side(nodes, k, p, r=0.5, oversample=4, side=1, alpha=1j):
        return orig(nodes, k, p, r, oversample, -side, alpha)

    for bad in (d_sign, wrong_side):
        monkeypatch.setattr(O, "dirichlet_matrix", bad)
        try:
            assert solve_error(I.EXTERIOR, 8, 6) > 1e-2, bad.__name__
        finally:
            monkeypatch.setattr(O, "dirichlet_matrix", orig)
