"""GPU tests of the Dirichlet solve (qbx_solve_dirichlet through the C ABI; Section 4.3,
eq. dirichlet-inteq): the GMRES solution against the oracle's dense direct solve of the
same Nystrom system (bar 1e-11 relative max-norm), and end to end against exact fields
of point charges, with the representation u = -D sigma + alpha S sigma evaluated off the
curve on the GPU (qbx_apply_explicit, the nodes' own 16-point rule as sources)."""
import sys

import numpy as np
import pytest
import scipy.special as sps
import torch

from oracle import qbx_oracle as O
from paper_1207_4461_amd import inputs as I

pytestmark = pytest.mark.gpu
TOL = 1e-11


@pytest.fixture(scope="module")
def Q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1207_4461_amd import qbx
    return qbx


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


EXT = ([(0.1, 0.2, 1.0), (-0.3, 0.1, 0.5 - 0.2j)], [(2.0, 0.5), (-1.5, 1.7), (0.3, -2.2)])
INT = ([(2.5, 0.3, 1.0), (-1.0, 2.4, 0.7j)], [(0.1, 0.1), (-0.3, 0.2), (0.2, -0.3)])


def charges_field(pts, charges, k):
    pts = np.asarray(pts, dtype=np.float64)
    u = np.zeros(len(pts), dtype=np.complex128)
    for cx, cy, c in charges:
        u += c * sps.hankel1(0, k * np.hypot(pts[:, 0] - cx, pts[:, 1] - cy))
    return u


@pytest.mark.parametrize("side,P,p,os_", [(I.EXTERIOR, 8, 6, 2), (I.INTERIOR, 12, 8, 2),
                                          (I.EXTERIOR, 10, 4, 1), (I.INTERIOR, 9, 10, 3)])
def test_solve_matches_oracle_dense_solve(Q, side, P, p, os_):
    k = 3.0
    charges, _ = EXT if side == I.EXTERIOR else INT
    nodes = I.panel_nodes(I.ellipse(1.0, 0.6), P)
    f = charges_field(nodes.reshape(-1, 2), charges, k)
    ref = O.dirichlet_solve(nodes, f, k, p, oversample=os_, side=side)
    sig, it, res = Q.solve_dirichlet(dev(nodes), dev(f), k, p, oversample=os_, side=side)
    e = rel(sig.cpu().numpy(), ref)
    say(f"  side {side} P={P} p={p} os={os_}: {it} products, residual {res:.2e}, vs oracle {e:.2e}")
    assert res < 1e-13 and e <= TOL


def node_rule(curve, P):
    """The nodes' own 16-point rule from the analytic curve: weights and unit normals."""
    t = I.panel_parameters(P).reshape(-1)
    d = curve.deriv(t)
    speed = np.hypot(d[:, 0], d[:, 1])
    _, om = np.polynomial.legendre.leggauss(16)
    w = np.tile(om, P) * (np.pi / P) * speed
    n = np.stack([d[:, 1], -d[:, 0]], axis=1) / speed[:, None]
    return w, n


def evaluate_off_curve(Q, nodes, sigma, w, n, k, pts, alpha=1j):
    """u = -D sigma + alpha S sigma at pts, as local expansions about centers a small
    step from each point (the smooth rule of the nodes as explicit sources)."""
    src = dev(nodes.reshape(-1, 2))
    q = torch.as_tensor(w, device="cuda") * sigma
    eps = 1e-3
    pts = np.asarray(pts, dtype=np.float64)
    ctr = dev(pts - np.array([eps, 0.0]))
    R = torch.full((len(pts),), eps, dtype=torch.float64, device="cuda")
    e = torch.ones(len(pts), dtype=torch.complex128, device="cuda")
    out = Q.apply_explicit(src, dev(n), torch.stack([q, q]), ctr, R, e, k, 8, kind=3)
    return (alpha * out[0] - out[1]).cpu().numpy()


@pytest.mark.parametrize("side,gamma", [(I.EXTERIOR, 0.0), (I.INTERIOR, 0.0), (I.EXTERIOR, 6.0)])
def test_point_charges_end_to_end(Q, side, gamma):
    """Starfish 1 + 0.25 cos 5t, 256 panels, k = 20, p = 12 (the star256 geometry):
    Dirichlet data of point charges outside the domain, solved to 1e-14 and evaluated
    at observation points inside it, against the exact field."""
    curve, P, k, p = I.star((5, 0.25, 0.0)), 256, 20.0, 12
    charges, obs = EXT if side == I.EXTERIOR else INT
    nodes = I.panel_nodes(curve, P)
    f = charges_field(nodes.reshape(-1, 2), charges, k)
    sig, it, res = Q.solve_dirichlet(dev(nodes), dev(f), k, p, side=side, gamma=gamma)
    sig2, it2, _ = Q.solve_dirichlet(dev(nodes), dev(f), k, p, side=side, gamma=gamma)
    assert torch.equal(sig, sig2) and it == it2
    w, n = node_rule(curve, P)
    u = evaluate_off_curve(Q, nodes, sig, w, n, k, obs)
    e = rel(u, charges_field(obs, charges, k))
    say(f"  side {side} gamma {gamma}: {it} products, residual {res:.2e}, field error {e:.2e}")
    assert res < 1e-13 and it < 200 and e < 1e-9


def test_split_products_give_the_same_solution(Q):
    curve, P, k, p = I.star((5, 0.25, 0.0)), 64, 5.0, 20
    charges, _ = EXT
    nodes = I.panel_nodes(curve, P)
    f = charges_field(nodes.reshape(-1, 2), charges, k)
    a, _, _ = Q.solve_dirichlet(dev(nodes), dev(f), k, p)
    b, _, _ = Q.solve_dirichlet(dev(nodes), dev(f), k, p, gamma=1e150)    # every panel near
    c, _, _ = Q.solve_dirichlet(dev(nodes), dev(f), k, p, gamma=6.0)
    ea, ec = rel(b.cpu().numpy(), a.cpu().numpy()), rel(c.cpu().numpy(), a.cpu().numpy())
    say(f"  all-near split vs plain {ea:.2e}; gamma 6 vs plain {ec:.2e}")
    assert ea < 1e-12 and ec < 1e-10


@pytest.mark.parametrize("side,P,p,os_", [(I.EXTERIOR, 8, 6, 2), (I.INTERIOR, 12, 8, 2)])
def test_adjoint_solve_matches_oracle_dense_solve(Q, side, P, p, os_):
    """lambda = A^-H g against the dense solve with the oracle's matrix conjugate-transposed."""
    k = 3.0
    nodes = I.panel_nodes(I.ellipse(1.0, 0.6), P)
    rng = np.random.default_rng(7)
    g = rng.standard_normal(P * 16) + 1j * rng.standard_normal(P * 16)
    A = O.dirichlet_matrix(nodes, k, p, oversample=os_, side=side)
    ref = np.linalg.solve(A.conj().T, g)
    lam, it, res = Q.solve_dirichlet_adjoint(dev(nodes), dev(g), k, p, oversample=os_, side=side)
    e = rel(lam.cpu().numpy(), ref)
    say(f"  side {side} P={P} p={p}: {it} products, residual {res:.2e}, vs oracle {e:.2e}")
    assert res < 1e-13 and e <= TOL


def test_differentiable_solve_gradients(Q):
    """Gradient for f by gradcheck (fast mode); for the nodes against a central difference
    of L = Re <g, sigma(x)> along a smooth deformation, with f held fixed."""
    curve, P, k, p = I.star((5, 0.25, 0.0)), 10, 3.0, 8
    X = I.panel_nodes(curve, P)
    nodes = dev(X)
    f = dev(charges_field(X.reshape(-1, 2), EXT[0], k))
    fn = lambda F: Q.dirichlet_solve_apply(nodes, F, k, p, oversample=2)
    assert torch.autograd.gradcheck(fn, (f.clone().requires_grad_(True),), eps=1e-6, atol=1e-7,
                                    rtol=1e-6, fast_mode=True)
    rng = np.random.default_rng(11)
    g = dev(rng.standard_normal(P * 16) + 1j * rng.standard_normal(P * 16))
    xn = nodes.clone().requires_grad_(True)
    L = torch.real(torch.sum(torch.conj(g) * Q.dirichlet_solve_apply(xn, f, k, p, oversample=2)))
    L.backward()
    t = I.panel_parameters(P)
    E = np.stack([np.sin(3 * t), np.cos(2 * t)], -1)

    def Lof(Y):
        s, _, _ = Q.solve_dirichlet(dev(Y), f, k, p, oversample=2)
        return float(torch.real(torch.sum(torch.conj(g) * s)))

    h = 1e-6
    fd = (Lof(X + h * E) - Lof(X - h * E)) / (2 * h)
    an = float(torch.sum(xn.grad * dev(E)))
    say(f"  directional derivative: FD {fd:.12e} adjoint {an:.12e}")
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_solve_node_gradient_entry_matches_its_definition(Q):
    """qbx_solve_dirichlet_node_gradient against -grad_x Re <lam, A(x) sigma> formed
    from the layer potentials' node adjoint with the cotangents written out here."""
    curve, P, k, p = I.star((5, 0.25, 0.0)), 12, 4.0, 8
    nodes = dev(I.panel_nodes(curve, P))
    rng = np.random.default_rng(8)
    T = P * 16
    sig = dev(rng.standard_normal(T) + 1j * rng.standard_normal(T))
    lam = dev(rng.standard_normal(T) + 1j * rng.standard_normal(T))
    alpha = 0.3 + 1.1j
    for gamma in (0.0, 4.0):
        gn = Q.solve_dirichlet_node_gradient(nodes, sig, lam, k, p, oversample=2, side=I.INTERIOR,
                                             alpha=alpha, gamma=gamma).cpu().numpy()
        cs, cd = (0.5 * np.conj(alpha)) * lam, -0.5 * lam
        cot = torch.stack([torch.stack([cs, cd]), torch.stack([cs, cd])]).contiguous()
        dens = torch.stack([sig, sig]).contiguous()
        if gamma > 0:
            _, ref = Q.layer_potential_split_vjp(nodes, dens, cot, k, p, 0.5, 2, I.BOTH, 3,
                                                 gamma=gamma, want_nodes=True, want_density=False)
        else:
            _, ref = Q.layer_potential_vjp(nodes, dens, cot, k, p, 0.5, 2, I.BOTH, 3,
                                           want_density=False)
        e = rel(gn, -ref.cpu().numpy())
        say(f"  gamma {gamma}: entry vs written-out cotangents {e:.2e}")
        assert e < 1e-13


def test_differentiable_solve_with_split_products(Q):
    curve, P, k, p = I.star((5, 0.25, 0.0)), 64, 5.0, 20
    nodes = dev(I.panel_nodes(curve, P))
    f = dev(charges_field(I.panel_nodes(curve, P).reshape(-1, 2), EXT[0], k))
    rng = np.random.default_rng(2)
    g = dev(rng.standard_normal(P * 16) + 1j * rng.standard_normal(P * 16))
    a, _, _ = Q.solve_dirichlet_adjoint(nodes, g, k, p)
    b, _, _ = Q.solve_dirichlet_adjoint(nodes, g, k, p, gamma=6.0)
    e = rel(b.cpu().numpy(), a.cpu().numpy())
    say(f"  adjoint solve, split products vs plain: {e:.2e}")
    assert e < 1e-10
    # node gradient with split products: against the plain products' and a central
    # difference of the split solve along a smooth deformation
    X = I.panel_nodes(curve, P)
    grads = []
    for gam in (0.0, 6.0):
        xn = nodes.clone().requires_grad_(True)
        L = torch.real(torch.sum(torch.conj(g) * Q.dirichlet_solve_apply(xn, f, k, p, gamma=gam)))
        L.backward()
        grads.append(xn.grad.cpu().numpy())
    e = rel(grads[1], grads[0])
    say(f"  node gradient, split products vs plain: {e:.2e}")
    assert e < 1e-9
    t = I.panel_parameters(P)
    E = np.stack([np.sin(3 * t), np.cos(2 * t)], -1)

    def Lof(Y):
        s_, _, _ = Q.solve_dirichlet(dev(Y), f, k, p, gamma=6.0)
        return float(torch.real(torch.sum(torch.conj(g) * s_)))

    h = 1e-6
    fd = (Lof(X + h * E) - Lof(X - h * E)) / (2 * h)
    an = float(np.sum(grads[1] * E))
    say(f"  split directional derivative: FD {fd:.12e} adjoint {an:.12e}")
    assert abs(fd - an) <= 1e-6 * abs(an)
