"""Pins of the oracle's target derivatives (Section 3.2: derivatives with respect to
the target by analytic differentiation of the local Bessel expansion; S' and D' as
defined at the start of Section 4) against facts the oracle's ladder formula does not produce
by itself:

* central differences (Richardson-extrapolated) of the oracle's own evaluation of the
  same local expansion at displaced targets, with the center and coefficients fixed;
* closed forms on the unit circle for density e^{imt}: the one-sided normal
  derivatives of S and D and the tangential derivative i m u;
* the jump relations of Section 3.2 (grad S^+ - grad S^- = -n sigma; D' continuous);
* Green's representation identity, differentiated: grad S^-[du/dn] - grad D^-[u] =
  grad u and grad S^+[du/dn] - grad D^+[u] = 0 for u = H0(k|x-x0|), x0 outside.

The mutation test at the end plants plausible mistakes in the oracle's gradient and
checks that a pin catches each.
"""
import numpy as np
import scipy.special as sps
import torch

from oracle import qbx_oracle as O
from paper_1207_4461_amd import inputs as I


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def _circle(P, k, p, m):
    nodes = I.panel_nodes(I.ellipse(1.0, 1.0), P)
    t = I.panel_parameters(P).reshape(-1)
    dens = np.exp(1j * m * t)
    g, dn = O.layer_potential_gradient(nodes, np.stack([dens, dens]), k, p, side=I.BOTH, kind=3)
    u = O.layer_potential(nodes, np.stack([dens, dens]), k, p, side=I.BOTH, kind=3).numpy()
    return t, dens, g.numpy(), dn.numpy(), u


def test_gradient_circle_closed_forms():
    """Unit circle, density e^{imt}.  Inside, S = (i pi/2) J_m(kr) H_m(k) e^{imt} and
    D = (i pi k/2) J_m(kr) H_m'(k) e^{imt}; outside, J_m(k) H_m(kr) and J_m'(k) H_m(kr).
    The radial derivatives at r = 1 give S'^- = (i pi k/2) J_m' H_m, S'^+ = (i pi k/2) J_m H_m',
    D'^- = D'^+ = (i pi k^2/2) J_m' H_m'; the tangential derivative is i m u."""
    P, k, p, m = 16, 3.0, 10, 3
    t, dens, g, dn, u = _circle(P, k, p, m)
    Sm = 0.5j * np.pi * k * sps.jvp(m, k) * sps.hankel1(m, k) * dens
    Sp = 0.5j * np.pi * k * sps.jv(m, k) * sps.h1vp(m, k) * dens
    Dd = 0.5j * np.pi * k * k * sps.jvp(m, k) * sps.h1vp(m, k) * dens
    # exterior limits carry the QBX error of this resolution, interior ones are exact
    assert rel(dn[0, 0], Sp) < 1e-5 and rel(dn[1, 0], Sm) < 1e-11
    assert rel(dn[0, 1], Dd) < 1e-5 and rel(dn[1, 1], Dd) < 1e-11
    # tangential derivative: t = (-sin t, cos t) at the point (cos t, sin t)
    tx, ty = -np.sin(t), np.cos(t)
    for si in range(2):
        for ki in range(2):
            dt = g[si, ki, :, 0] * tx + g[si, ki, :, 1] * ty
            assert rel(dt, 1j * m * u[si, ki]) < 1e-5
    # Section 3.2 jumps: grad S^+ - grad S^- = -n sigma, so S'^- - S'^+ = sigma;
    # grad D^+ - grad D^- = t dsigma/ds = t (i m sigma): no normal part
    assert rel(dn[1, 0] - dn[0, 0], dens) < 1e-5
    assert np.abs(dn[0, 1] - dn[1, 1]).max() / np.abs(Dd).max() < 1e-5


def _fd_gradient(a, cx, cy, tx, ty, k, p, h):
    """Central differences of the oracle's evaluation of one local expansion at
    displaced targets (fixed center and coefficients), Richardson-extrapolated."""
    def u_at(x, y):
        dx, dy = torch.as_tensor(x - cx), torch.as_tensor(y - cy)
        return O.evaluate(a, torch.hypot(dx, dy), torch.atan2(dy, dx), k, p).numpy()

    def D(step):
        out = []
        for ex, ey in ((1.0, 0.0), (0.0, 1.0)):
            up = u_at(tx + step * ex, ty + step * ey)
            um = u_at(tx - step * ex, ty - step * ey)
            out.append((up - um) / (2 * step))
        return np.stack(out, axis=-1)

    return (4.0 * D(h / 2) - D(h)) / 3.0


def test_gradient_is_the_derivative_of_the_local_expansion():
    pb = I.small(n_panels=8, p=7, k=4.0, kind=3, side=I.BOTH)
    u, aux = O.layer_potential(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side,
                               pb.kind, return_aux=True)
    g, _ = O.layer_potential_gradient(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample,
                                      pb.side, pb.kind)
    g = g.numpy()
    xy = pb.nodes.reshape(-1, 2)
    sel = np.array([0, 5, 17, 40, 77, 127])
    for si, s in enumerate(O.sides_of(pb.side)):
        ctr, a = aux["sides"][s]["ctr"], aux["sides"][s]["a"]
        for ki, kk in enumerate(O.kinds_of(pb.kind)):
            fd = _fd_gradient(a[kk][sel], ctr["cx"][sel].numpy(), ctr["cy"][sel].numpy(),
                              xy[sel, 0], xy[sel, 1], pb.k, pb.p, 2e-3 * ctr["R"][sel].numpy())
            assert rel(g[si, ki, sel], fd) < 1e-8, (s, kk)


def _green_gradient(P, k, p, x0=(3.0, 1.0)):
    curve = I.star((5, 0.25, 0.0))
    nodes = I.panel_nodes(curve, P)
    u, dudn = I.green_pair(curve, P, k, x0)
    g, _ = O.layer_potential_gradient(nodes, np.stack([dudn, u]), k, p, side=I.BOTH, kind=3)
    xy = nodes.reshape(-1, 2)
    d = xy - np.asarray(x0)
    rr = np.hypot(d[:, 0], d[:, 1])
    grad_u = (-k * sps.hankel1(1, k * rr) / rr)[:, None] * d
    return g.numpy(), grad_u


def test_gradient_green_identity_on_starfish():
    """grad S^-[du/dn] - grad D^-[u] = grad u and grad S^+[du/dn] - grad D^+[u] = 0 on the
    curve, for u = H0(k|x-x0|) with x0 outside; the error falls under refinement."""
    errs = []
    for P in (20, 30):
        g, grad_u = _green_gradient(P, 5.0, 8)
        sc = np.abs(grad_u).max()
        interior = g[1, 0] - g[1, 1]
        exterior = g[0, 0] - g[0, 1]
        errs.append(np.abs(interior - grad_u).max() / sc)
        assert np.abs(exterior).max() / sc < 1e-6
    assert errs[1] < 1e-6 and errs[0] > 5 * errs[1]


def test_planted_gradient_mistakes_are_caught(monkeypatch):
    orig = O.evaluate_gradient

    def flipped_ladder(a, R, theta, k, p, mode="fast"):
        g = orig(a, R, theta, k, p, mode)
        return g * torch.tensor([-1.0, 1.0], dtype=torch.float64)   # beta_{l+1} - beta_{l-1} in d/dx
    def dropped_half(a, R, theta, k, p, mode="fast"):
        return 2.0 * orig(a, R, theta, k, p, mode)
    def swapped_components(a, R, theta, k, p, mode="fast"):
        return orig(a, R, theta, k, p, mode)[:, [1, 0]]
    for bad in (flipped_ladder, dropped_half, swapped_components):
        monkeypatch.setattr(O, "evaluate_gradient", bad)
        t, dens, g, dn, u = _circle(16, 3.0, 10, 3)
        Sm = 0.5j * np.pi * 3.0 * sps.jvp(3, 3.0) * sps.hankel1(3, 3.0) * dens
        assert rel(dn[1, 0], Sm) > 1e-3, bad.__name__
        monkeypatch.setattr(O, "evaluate_gradient", orig)


# ---------------------------------------------------------------------------
# on-surface derivatives from the one-sided limits (Section 3.2 jump relations)
# ---------------------------------------------------------------------------
def _circle_pv_closed_forms(t, dens, k, m):
    """Unit circle, density e^{imt}: grad S principal value and grad D finite part.
    S'_pv = (S'^+ + S'^-)/2 = (i pi k/4)(J_m' H_m + J_m H_m'), the tangential
    derivative of S is i m S with S = (i pi/2) J_m H_m; D' = (i pi k^2/2) J_m' H_m' has
    no jump and the finite-part tangential derivative is i m D_pv with
    D_pv = (D^+ + D^-)/2 = (i pi k/4)(J_m' H_m + J_m H_m')."""
    j, jp = sps.jv(m, k), sps.jvp(m, k)
    h, hp = sps.hankel1(m, k), sps.h1vp(m, k)
    S = 0.5j * np.pi * j * h * dens
    Sn = 0.25j * np.pi * k * (jp * h + j * hp) * dens
    Dpv = 0.25j * np.pi * k * (jp * h + j * hp) * dens
    Dn = 0.5j * np.pi * k * k * jp * hp * dens
    n = np.stack([np.cos(t), np.sin(t)], -1)
    tt = np.stack([-np.sin(t), np.cos(t)], -1)
    gS = Sn[:, None] * n + (1j * m * S)[:, None] * tt
    gD = Dn[:, None] * n + (1j * m * Dpv)[:, None] * tt
    return gS, gD, Sn, Dn


def _pv_on_circle(side, P=16, k=3.0, p=10, m=3):
    nodes = I.panel_nodes(I.ellipse(1.0, 1.0), P)
    t = I.panel_parameters(P).reshape(-1)
    dens = np.exp(1j * m * t)
    d2 = np.stack([dens, dens])
    g, dn = O.layer_potential_gradient(nodes, d2, k, p, side=side, kind=3)
    gp, dp = O.gradient_principal_value(nodes, d2, g, dn, side, 3)
    return t, dens, gp.numpy(), dp.numpy()


def test_gradient_principal_value_circle_closed_forms():
    """From either one-sided limit alone (the jump subtracted) or from their average,
    the unit circle's closed forms: interior limits are exact at this resolution, the
    exterior ones carry the QBX error."""
    k, m = 3.0, 3
    for side, tol in ((I.INTERIOR, 1e-10), (I.EXTERIOR, 1e-5), (I.BOTH, 1e-5)):
        t, dens, gp, dp = _pv_on_circle(side, k=k, m=m)
        gS, gD, Sn, Dn = _circle_pv_closed_forms(t, dens, k, m)
        e = (rel(gp[0], gS), rel(gp[1], gD), rel(dp[0], Sn), rel(dp[1], Dn))
        assert max(e) < tol, (side, e)


def test_gradient_principal_value_sides_agree_on_starfish():
    """The exterior and the interior fix-ups give the same on-surface values: each
    subtracts its own side's jump, so they differ by the QBX error of the one-sided
    derivatives only.  D' has no jump and is not changed by the fix-up, so the gap
    between its two raw limits measures that error; every fixed-up quantity's gap
    stays within a small factor of it and falls with it under refinement, while the
    raw one-sided limits of the others differ by O(1)."""
    curve = I.star((5, 0.25, 0.0))
    gaps = []
    for P in (40, 64):
        nodes = I.panel_nodes(curve, P)
        t = I.panel_parameters(P).reshape(-1)
        rng = np.random.default_rng(7)
        dens = np.stack([I.smooth_density(rng, t), I.smooth_density(rng, t)])
        g, dn = O.layer_potential_gradient(nodes, dens, 4.0, 10, side=I.BOTH, kind=3)
        ge, de = O.gradient_principal_value(nodes, dens, g[:1], dn[:1], I.EXTERIOR, 3)
        gi, di = O.gradient_principal_value(nodes, dens, g[1:], dn[1:], I.INTERIOR, 3)
        ga, da = O.gradient_principal_value(nodes, dens, g, dn, I.BOTH, 3)
        qbx_err = rel(dn[0, 1].numpy(), dn[1, 1].numpy())          # D': no jump
        gap = max(rel(ge[0].numpy(), gi[0].numpy()), rel(ge[1].numpy(), gi[1].numpy()),
                  rel(de[0].numpy(), di[0].numpy()))
        assert gap < 5 * qbx_err, (P, gap, qbx_err)
        assert rel(ga.numpy(), ge.numpy()) < 5 * qbx_err
        assert rel(g[0, 0].numpy(), g[1, 0].numpy()) > 0.05      # raw S limits: O(1) apart
        assert rel(dn[0, 0].numpy(), dn[1, 0].numpy()) > 0.05
        gaps.append(gap)
    assert gaps[1] < 2e-4 and gaps[0] > 5 * gaps[1], gaps


def test_planted_principal_value_mistakes_are_caught(monkeypatch):
    """A reversed tangent, d sigma/dtau in place of d sigma/ds and the other side's
    jump each break the circle's closed forms."""
    k, m = 3.0, 3
    orig_frame, orig_ds = O.target_frame, O.arclength_derivative

    def reversed_tangent(nodes):
        n, tt, sp = orig_frame(nodes)
        return n, -tt, sp

    def tau_derivative(nodes, density):
        return orig_ds(nodes, density) * orig_frame(nodes)[2].to(torch.complex128)

    for name, patch in (("target_frame", reversed_tangent),
                        ("arclength_derivative", tau_derivative)):
        monkeypatch.setattr(O, name, patch)
        t, dens, gp, dp = _pv_on_circle(I.INTERIOR, k=k, m=m)
        gS, gD, Sn, Dn = _circle_pv_closed_forms(t, dens, k, m)
        assert rel(gp[1], gD) > 1e-2, name
        monkeypatch.setattr(O, name, {"target_frame": orig_frame,
                                      "arclength_derivative": orig_ds}[name])
    # the interior limits with the exterior's jumps
    P = 16
    nodes = I.panel_nodes(I.ellipse(1.0, 1.0), P)
    t = I.panel_parameters(P).reshape(-1)
    dens = np.exp(1j * m * t)
    d2 = np.stack([dens, dens])
    g, dn = O.layer_potential_gradient(nodes, d2, k, 10, side=I.INTERIOR, kind=3)
    gp, dp = O.gradient_principal_value(nodes, d2, g, dn, I.EXTERIOR, 3)
    gS, gD, Sn, Dn = _circle_pv_closed_forms(t, dens, k, m)
    assert rel(dp.numpy()[0], Sn) > 1e-1 and rel(gp.numpy()[1], gD) > 1e-1
