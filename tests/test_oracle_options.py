"""Pins of the oracle's forward options against facts its code does not produce:

* the tangential dipole R of eq. riesz-def (``dipole="tangential"``): on the unit circle
  R e^{imt} = (pi m / 2) J_m(k) H_m(k) e^{imt} on both sides, and on any closed curve
  R sigma = -S[d sigma / ds] (integration by parts), with d sigma/ds taken analytically;
* the center rule R = r sqrt(h) of Section 3.1 (``center_rule="sqrt"``): centers on the
  unit circle at |c - x| = r sqrt(2 pi / P) along the exact normal, Green's identity, and
  the closed form of S on the circle;
* planted mistakes (a reversed tangent, the h rule in place of sqrt(h)) are caught.
"""
import numpy as np
import scipy.special as sps
import torch

from oracle import qbx_oracle as O
from paper_1207_4461_amd import inputs as I


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def _circle_R(P=16, k=3.0, p=10, m=3):
    nodes = I.panel_nodes(I.ellipse(1.0, 1.0), P)
    t = I.panel_parameters(P).reshape(-1)
    dens = np.exp(1j * m * t)
    u = O.layer_potential(nodes, np.stack([dens]), k, p, side=I.BOTH, kind=2,
                          dipole="tangential").numpy()
    return u, 0.5 * np.pi * m * sps.jv(m, k) * sps.hankel1(m, k) * dens


def test_tangential_dipole_circle_closed_form():
    u, ref = _circle_R()
    assert rel(u[1, 0], ref) < 1e-11 and rel(u[0, 0], ref) < 1e-6


def test_tangential_dipole_is_minus_S_of_the_arc_derivative():
    curve = I.star((5, 0.25, 0.0))
    errs = []
    for P in (24, 36):
        nodes = I.panel_nodes(curve, P)
        t = I.panel_parameters(P).reshape(-1)
        d = curve.deriv(t)
        speed = np.hypot(d[:, 0], d[:, 1])
        sig = np.exp(2j * t) + 0.3 * np.exp(-5j * t)
        dsig = (2j * np.exp(2j * t) - 1.5j * np.exp(-5j * t)) / speed
        R = O.layer_potential(nodes, np.stack([sig]), 5.0, 12, side=I.BOTH, kind=2,
                              dipole="tangential").numpy()
        S = O.layer_potential(nodes, np.stack([dsig]), 5.0, 12, side=I.BOTH, kind=1).numpy()
        errs.append(max(rel(R[0, 0], -S[0, 0]), rel(R[1, 0], -S[1, 0])))
    assert errs[1] < 1e-10 and errs[0] > 20 * errs[1]


def test_sqrt_center_rule_places_centers_exactly():
    P, r = 20, 0.5
    nodes = I.panel_nodes(I.ellipse(1.0, 1.0), P)
    x = nodes.reshape(-1, 2)
    dens = np.ones((1, P * 16), dtype=np.complex128)
    _, aux = O.layer_potential(nodes, dens, 2.0, 4, r, 4, I.BOTH, 1, return_aux=True,
                               center_rule="sqrt")
    R = r * np.sqrt(2 * np.pi / P)            # arc length of an equal-parameter panel
    for s, sg in ((I.EXTERIOR, 1.0), (I.INTERIOR, -1.0)):
        c = aux["sides"][s]["ctr"]
        cxy = np.stack([c["cx"].numpy(), c["cy"].numpy()], axis=1)
        assert np.abs(cxy - x * (1 + sg * R)).max() < 1e-13      # the normal of the circle is x
        assert np.abs(c["R"].numpy() - R).max() < 1e-13


def test_sqrt_center_rule_green_identity_and_circle():
    curve = I.star((5, 0.25, 0.0))
    P, k, p = 40, 5.0, 10
    nodes = I.panel_nodes(curve, P)
    u, dudn = I.green_pair(curve, P, k)
    v = O.layer_potential(nodes, np.stack([dudn, u]), k, p, side=I.BOTH, kind=3,
                          center_rule="sqrt").numpy()
    sc = np.abs(u).max()
    assert np.abs(v[1, 0] - v[1, 1] - u).max() / sc < 1e-6
    assert np.abs(v[0, 0] - v[0, 1]).max() / sc < 1e-6
    Pc, m = 32, 3
    nodes = I.panel_nodes(I.ellipse(1.0, 1.0), Pc)
    t = I.panel_parameters(Pc).reshape(-1)
    dens = np.exp(1j * m * t)
    w = O.layer_potential(nodes, np.stack([dens]), 3.0, 10, side=I.INTERIOR, kind=1,
                          center_rule="sqrt").numpy()
    assert rel(w[0, 0], 0.5j * np.pi * sps.jv(m, 3.0) * sps.hankel1(m, 3.0) * dens) < 1e-11


def test_planted_option_mistakes_are_caught(monkeypatch):
    orig_grid, orig_ctr = O.source_grid, O.expansion_centers

    def reversed_tangent(nodes, oversample):
        g = orig_grid(nodes, oversample)
        return dict(g, nx=-g["nx"], ny=-g["ny"])

    monkeypatch.setattr(O, "source_grid", reversed_tangent)
    u, ref = _circle_R()
    assert rel(u[1, 0], ref) > 1e-2
    monkeypatch.setattr(O, "source_grid", orig_grid)

    def h_rule(nodes, h, n_tgt, r, side, center_rule="h"):
        return orig_ctr(nodes, h, n_tgt, r, side, "h")

    monkeypatch.setattr(O, "expansion_centers", h_rule)
    try:
        test_sqrt_center_rule_places_centers_exactly()
        caught = False
    except AssertionError:
        caught = True
    monkeypatch.setattr(O, "expansion_centers", orig_ctr)
    assert caught
