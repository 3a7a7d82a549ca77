"""Pins of the oracle's near/far split (Section 5: direct evaluation for distant
panel interactions, QBX for the near neighbours) against facts its code does not
produce by itself:

* with every panel near, the split is the plain QBX result (itself pinned by the
  Wronskian, Graf brute force and Green's identity);
* for distant panels the direct smooth rule and the QBX expansion agree pair by
  pair up to the expansion's truncation, so the split matches plain QBX at high p
  to far below the QBX error, and the gap closes as gamma grows;
* closed forms on the unit circle for density e^{imt}, with the near patch wide
  enough that its ends do not limit the expansion ((R/d_end)^(p+1) < 1e-12);
* Green's representation identity S[du/dn] - D^-[u] = u and S[du/dn] - D^+[u] = 0;
* the near relation: symmetric, every panel near itself, and on a circle the
  count per panel from the chord-length formula.

The mutation test at the end plants plausible mistakes in the split and checks that
a pin catches each.
"""
import math

import numpy as np
import pytest
import scipy.special as sps
import torch

from oracle import qbx_oracle as O
from paper_1207_4461_amd import inputs as I


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def split(pb, gamma, **kw):
    return O.layer_potential_split(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side,
                                   pb.kind, gamma=gamma, **kw).numpy()


def qbx(pb, **kw):
    return O.layer_potential(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side,
                             pb.kind, **kw).numpy()


def test_all_near_is_plain_qbx():
    pb = I.small(n_panels=7, p=6, k=4.0, kind=3, side=I.BOTH)
    assert O.near_panels(pb.nodes, 1e150).all()
    assert rel(split(pb, 1e150), qbx(pb)) < 1e-15


def test_split_matches_qbx_to_truncation():
    """p = 20: the far sources' QBX truncation is far below 1e-11, so the split and
    plain QBX agree; at smaller gamma (sources closer to the centers) the gap grows."""
    pb = I.small(n_panels=28, p=20, k=5.0, kind=3, side=I.BOTH)
    ref = qbx(pb)
    gaps = []
    for gamma in (4.0, 6.0, 10.0):
        near = O.near_panels(pb.nodes, gamma)
        assert 0 < near.sum() < near.size
        gaps.append(rel(split(pb, gamma), ref))
    assert gaps[0] < 1e-12 and gaps[1] < 1e-13 and gaps[2] < 1e-13
    assert gaps[0] > 10 * max(gaps[1], gaps[2])


def _circle(P, k, p, m, gamma):
    nodes = I.panel_nodes(I.ellipse(1.0, 1.0), P)
    t = I.panel_parameters(P).reshape(-1)
    dens = np.exp(1j * m * t)
    u = O.layer_potential_split(nodes, np.stack([dens, dens]), k, p, 0.5, 4, I.BOTH, 3,
                                gamma=gamma).numpy()
    return dens, u


def test_split_circle_closed_forms():
    """Unit circle, density e^{imt}: S = (i pi/2) J_m(k) H_m(k) e^{imt} on both sides,
    D^- = (i pi k/2) J_m(k) H_m'(k) e^{imt}, D^+ = (i pi k/2) J_m'(k) H_m(k) e^{imt}."""
    P, k, p, m = 48, 3.0, 10, 3
    assert not O.near_panels(I.panel_nodes(I.ellipse(1.0, 1.0), P), 16.0).all()
    dens, u = _circle(P, k, p, m, 16.0)
    S = 0.5j * np.pi * sps.jv(m, k) * sps.hankel1(m, k) * dens
    Dm = 0.5j * np.pi * k * sps.jv(m, k) * sps.h1vp(m, k) * dens
    Dp = 0.5j * np.pi * k * sps.jvp(m, k) * sps.hankel1(m, k) * dens
    assert rel(u[0, 0], S) < 1e-10 and rel(u[1, 0], S) < 1e-10
    assert rel(u[1, 1], Dm) < 1e-10 and rel(u[0, 1], Dp) < 1e-10


def _green(P, k, p, gamma, x0=(3.0, 1.0)):
    curve = I.star((5, 0.25, 0.0))
    nodes = I.panel_nodes(curve, P)
    u, dudn = I.green_pair(curve, P, k, x0)
    v = O.layer_potential_split(nodes, np.stack([dudn, u]), k, p, 0.5, 4, I.BOTH, 3,
                                gamma=gamma).numpy()
    sc = np.abs(u).max()
    return np.abs(v[1, 0] - v[1, 1] - u).max() / sc, np.abs(v[0, 0] - v[0, 1]).max() / sc


def test_split_green_identity():
    for P in (30, 45):
        e_in, e_out = _green(P, 5.0, 20, 6.0)
        assert e_in < 1e-8 and e_out < 1e-8, (P, e_in, e_out)


def test_patch_end_error_model():
    """At p = 10 the near patch's ends limit the expansion: the split's gap to plain
    QBX falls with gamma roughly like gamma^-(p+1), from about 1e-9 at gamma = 6."""
    pb = I.small(n_panels=36, p=10, k=3.0, kind=3, side=I.INTERIOR)
    ref = qbx(pb)
    g6, g16 = rel(split(pb, 6.0), ref), rel(split(pb, 16.0), ref)
    assert 1e-11 < g6 < 1e-7 and g16 < 1e-11 and g6 / g16 > (16 / 6) ** 6


def test_near_relation_on_circle():
    """Equal panels on the unit circle: b_m lie on a circle of radius |b|, so panel
    m' is near m when 2|b| sin(pi d / P) < gamma rad, d the index distance."""
    P = 64
    nodes = I.panel_nodes(I.ellipse(1.0, 1.0), P)
    b, rad2 = O.panel_bounds(nodes)
    bn, rad = float(np.hypot(*b[0])), math.sqrt(float(rad2.max()))
    for gamma in (1.0, 3.7, 6.0, 11.3):
        near = O.near_panels(nodes, gamma)
        assert (near == near.T).all() and near.diagonal().all()
        d = np.arange(P)
        dist = 2 * bn * np.sin(np.pi * np.minimum(d, P - d) / P)
        # no chord within 1e-9 of the threshold, so rounding cannot decide
        assert np.abs(dist - gamma * rad).min() > 1e-9
        expect = int((dist < gamma * rad).sum())
        assert (near.sum(axis=1) == expect).all(), (gamma, expect)


def test_planted_split_mistakes_are_caught(monkeypatch):
    pb = I.small(n_panels=24, p=8, k=5.0, kind=3, side=I.BOTH)
    ref = qbx(pb)
    assert rel(split(pb, 6.0), ref) < 1e-7
    orig_near, orig_direct = O.near_panels, O.direct_sum

    def swapped(nodes, gamma):
        return ~orig_near(nodes, gamma)

    def d_sign(src, dens, tx, ty, k, kind, sel):
        out = orig_direct(src, dens, tx, ty, k, kind, sel)
        out["D"] = -out["D"]
        return out

    def no_k(src, dens, tx, ty, k, kind, sel):
        out = orig_direct(src, dens, tx, ty, k, kind, sel)
        out["D"] = out["D"] / k
        return out

    def h1_for_h0(src, dens, tx, ty, k, kind, sel):
        out = orig_direct(src, dens, tx, ty, k, kind, sel)
        d2 = dict(dens)
        d2["D"] = dens["S"]
        out["S"] = orig_direct(src, d2, tx, ty, k, 2, sel)["D"]
        return out

    for name, attr, bad in (("swapped", "near_panels", swapped), ("d_sign", "direct_sum", d_sign),
                            ("no_k", "direct_sum", no_k), ("h1_for_h0", "direct_sum", h1_for_h0)):
        monkeypatch.setattr(O, attr, bad)
        try:
            # a swapped relation puts each target's own node among the direct sources:
            # the sum is not finite, which is caught as well
            assert not rel(split(pb, 6.0), ref) <= 1e-4, name
        finally:
            monkeypatch.setattr(O, attr, orig_near if attr == "near_panels" else orig_direct)


def _direct_setup():
    pb = I.small(n_panels=12, p=8, k=5.0, kind=3, side=I.BOTH)
    src = O.source_grid(torch.as_tensor(pb.nodes), 4)
    fine = O.interpolate_density(torch.as_tensor(pb.density), 4)
    dens = {"S": src["w"].to(torch.complex128) * fine[0],
            "D": src["w"].to(torch.complex128) * fine[1]}
    tx = torch.tensor([3.0, -2.5, 0.2], dtype=torch.float64)
    ty = torch.tensor([0.4, 1.7, -2.9], dtype=torch.float64)
    sel = torch.ones(3, src["x"].shape[0], dtype=torch.bool)
    return pb, src, dens, tx, ty, sel


def test_direct_gradient_is_the_derivative_of_the_direct_sum():
    """Fourth-order central differences of direct_sum at points off the curve."""
    pb, src, dens, tx, ty, sel = _direct_setup()
    gd = O.direct_gradient(src, dens, tx, ty, pb.k, 3, sel)
    h = 1e-4
    for kk in ("S", "D"):
        fd = []
        for ex, ey in ((1.0, 0.0), (0.0, 1.0)):
            f = lambda s: O.direct_sum(src, dens, tx + s * ex, ty + s * ey, pb.k, 3, sel)[kk]
            fd.append(((8 * (f(h) - f(-h)) - (f(2 * h) - f(-2 * h))) / (12 * h)).numpy())
        assert rel(np.stack(fd, axis=1), gd[kk].numpy()) < 1e-9, kk


def test_split_gradient_matches_qbx_gradient():
    """p = 20: the far sources' truncation is negligible, so the split's target
    derivatives match the plain QBX ones; the planted sign mistake in the D term of the
    direct gradient is caught."""
    pb = I.small(n_panels=28, p=20, k=5.0, kind=3, side=I.BOTH)
    g0, dn0 = O.layer_potential_gradient(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample,
                                         pb.side, pb.kind)
    g1, dn1 = O.layer_potential_split_gradient(pb.nodes, pb.density, pb.k, pb.p, pb.r,
                                               pb.oversample, pb.side, pb.kind, gamma=6.0)
    assert rel(g1.numpy(), g0.numpy()) < 1e-13 and rel(dn1.numpy(), dn0.numpy()) < 1e-13


def test_planted_direct_gradient_mistake_is_caught(monkeypatch):
    pb, src, dens, tx, ty, sel = _direct_setup()
    orig = O.hankel1

    def swapped(n, x):             # H_0 and H_1 exchanged inside the gradient
        return orig(1 - n, x) if n in (0, 1) else orig(n, x)

    good = O.direct_gradient(src, dens, tx, ty, pb.k, 3, sel)["D"]
    monkeypatch.setattr(O, "hankel1", swapped)
    bad = O.direct_gradient(src, dens, tx, ty, pb.k, 3, sel)["D"]
    monkeypatch.setattr(O, "hankel1", orig)
    assert rel(bad.numpy(), good.numpy()) > 1e-2


# ---------------------------------------------------------------------------
# node gradient of the split (split_vjp: autograd through the split's steps)
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def split_tiny():
    pb = I.small(n_panels=8, p=6, k=4.0, kind=3, side=I.BOTH, oversample=2)
    gamma = 2.0   # three near panels per panel, five far
    gd, gn = O.split_vjp(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side,
                         pb.kind, pb.cotangent, gamma)
    return pb, gamma, gd, gn


def _split_L(pb, gamma, X):
    return O.split_loss(X, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                        pb.cotangent, gamma)


def test_split_node_gradient_central_differences(split_tiny):
    pb, gamma, _, gn = split_tiny
    assert (O.near_panels(pb.nodes, gamma).sum(1) < pb.n_panels).all()
    rng = np.random.default_rng(5)
    for _ in range(3):
        E = rng.standard_normal(pb.nodes.shape)
        fd = lambda h: (_split_L(pb, gamma, pb.nodes + h * E)
                        - _split_L(pb, gamma, pb.nodes - h * E)) / (2 * h)
        rich = (4.0 * fd(1e-6) - fd(2e-6)) / 3.0
        an = float(np.sum(gn * E))
        assert abs(rich - an) <= 1e-7 * abs(an)
    for (m, a, d) in [(0, 0, 0), (3, 8, 1), (7, 15, 0)]:
        E = np.zeros_like(pb.nodes)
        E[m, a, d] = 1.0
        h = 1e-6
        fd = (_split_L(pb, gamma, pb.nodes + h * E) - _split_L(pb, gamma, pb.nodes - h * E)) / (2 * h)
        assert abs(fd - gn[m, a, d]) <= 1e-6 * max(1.0, abs(gn[m, a, d]))


def test_split_gradient_with_every_panel_near_is_the_qbx_gradient():
    pb = I.small(n_panels=6, p=6, k=4.0, kind=3, side=I.BOTH, oversample=2)
    gd, gn = O.split_vjp(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side,
                         pb.kind, pb.cotangent, 1e3)
    rd, rn = O.vjp(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                   pb.cotangent)
    assert rel(gn, rn) < 1e-12 and rel(gd, rd) < 1e-12


def test_split_gradient_invariances(split_tiny):
    pb, gamma, gd, gn = split_tiny
    scale = np.abs(gn).sum()
    assert np.abs(gn.sum(axis=(0, 1))).max() < 1e-13 * scale
    torque = np.sum(pb.nodes[..., 0] * gn[..., 1] - pb.nodes[..., 1] * gn[..., 0])
    assert abs(torque) < 1e-13 * scale * np.abs(pb.nodes).max()
    L = _split_L(pb, gamma, pb.nodes)
    assert abs(np.real(np.vdot(gd, pb.density)) - L) < 1e-13 * abs(L)


def test_planted_split_gradient_mistake_is_caught(split_tiny, monkeypatch):
    """The far rule with its target held fixed (the target's own motion dropped)."""
    pb, gamma, _, gn = split_tiny
    orig = O.direct_sum

    def frozen_target(src, dens, tx, ty, k, kind, sel):
        return orig(src, dens, tx.detach(), ty.detach(), k, kind, sel)

    monkeypatch.setattr(O, "direct_sum", frozen_target)
    _, bad = O.split_vjp(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side,
                         pb.kind, pb.cotangent, gamma)
    assert rel(bad, gn) > 1e-3


def test_nystrom_grid_closed_forms():
    """The far sources (``nystrom_grid``): the nodes' own 16-point rule gives the
    ellipse's area by the divergence theorem (oint x n_x ds = oint y n_y ds = area
    pi a b), the closed curve's oint n ds = 0, and the perimeter 4 a E(1 - b^2/a^2);
    its weighted densities are w sigma at the nodes."""
    a, b, P = 2.0, 1.0, 24
    curve = I.ellipse(a, b)
    nodes = torch.from_numpy(I.panel_nodes(curve, P))
    sig = torch.arange(P * 16, dtype=torch.float64).to(torch.complex128) * (1 + 2j)
    src, dens = O.nystrom_grid(nodes, sig[None, :], ("S",))
    w = src["w"].numpy()
    area = math.pi * a * b
    assert abs((w * src["x"].numpy() * src["nx"].numpy()).sum() - area) < 1e-13 * area
    assert abs((w * src["y"].numpy() * src["ny"].numpy()).sum() - area) < 1e-13 * area
    assert abs((w * src["nx"].numpy()).sum()) < 1e-13 and abs((w * src["ny"].numpy()).sum()) < 1e-13
    per = 4 * a * sps.ellipe(1 - (b / a) ** 2)   # the complete elliptic integral E(m)
    assert abs(w.sum() - per) < 1e-12 * per
    assert np.allclose(src["x"].numpy(), nodes[..., 0].reshape(-1).numpy(), rtol=0, atol=0)
    assert torch.equal(dens["S"], src["w"].to(torch.complex128) * sig)
    # unit normals, outward on a counter-clockwise curve: n . x > 0 on the ellipse
    n2 = src["nx"] ** 2 + src["ny"] ** 2
    assert float((n2 - 1).abs().max()) < 1e-15
    assert bool(((src["nx"] * src["x"] + src["ny"] * src["y"]) > 0).all())
