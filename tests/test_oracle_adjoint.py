"""Pins of the oracle's adjoint (autograd through the oracle's steps).

* density gradient = A^H g with A the dense QBX matrix built by per-order library
  calls (a different code path: scipy per order, unit-vector columns);
* node gradient vs central finite differences of L = Re <g, u>;
* exact invariances: translation (sum of node gradients = 0) and rotation
  (sum of x cross grad = 0) of the discrete map;
* the restricted-loss variant used for sampled checks at full size equals the
  full gradient on the panels it covers.
"""
import numpy as np
import pytest

from oracle import qbx_oracle as O
from paper_1207_4461_amd import inputs as I


@pytest.fixture(scope="module")
def tiny():
    pb = I.small(n_panels=5, p=6, k=4.0)
    gd, gn = O.vjp(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                   pb.cotangent)
    return pb, gd, gn


def test_density_gradient_is_dense_transpose(tiny):
    pb, gd, _ = tiny
    for ki, kname in enumerate(("S", "D")):
        ref = 0
        for si, s in enumerate((I.EXTERIOR, I.INTERIOR)):
            A = O.qbx_matrix(pb.nodes, pb.k, pb.p, pb.r, pb.oversample, s, kname)
            ref = ref + A.conj().T @ pb.cotangent[si, ki]
        assert np.abs(gd[ki] - ref).max() / np.abs(ref).max() < 1e-13


def test_node_gradient_central_differences(tiny):
    pb, _, gn = tiny
    rng = np.random.default_rng(3)
    L = lambda X: O.loss(X, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                         pb.cotangent)
    for _ in range(3):
        E = rng.standard_normal(pb.nodes.shape)
        fd = lambda h: (L(pb.nodes + h * E) - L(pb.nodes - h * E)) / (2 * h)
        rich = (4.0 * fd(1e-6) - fd(2e-6)) / 3.0          # O(h^4) Richardson step
        an = float(np.sum(gn * E))
        assert abs(rich - an) <= 1e-7 * abs(an)
    # one node coordinate at a time on a panel edge and the middle
    for (m, a, d) in [(0, 0, 0), (2, 7, 1), (4, 15, 1)]:
        E = np.zeros_like(pb.nodes)
        E[m, a, d] = 1.0
        h = 1e-6
        fd = (L(pb.nodes + h * E) - L(pb.nodes - h * E)) / (2 * h)
        assert abs(fd - gn[m, a, d]) <= 1e-6 * max(1.0, abs(gn[m, a, d]))


def test_gradient_invariances(tiny):
    pb, gd, gn = tiny
    scale = np.abs(gn).sum()
    assert np.abs(gn.sum(axis=(0, 1))).max() < 1e-13 * scale
    torque = np.sum(pb.nodes[..., 0] * gn[..., 1] - pb.nodes[..., 1] * gn[..., 0])
    assert abs(torque) < 1e-13 * scale * np.abs(pb.nodes).max()
    # dot-product test: L = Re <grad_density, density> (L is linear in the density)
    L = O.loss(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
               pb.cotangent)
    assert abs(np.real(np.vdot(gd, pb.density)) - L) < 1e-13 * abs(L)


def test_restricted_gradient_matches_full(tiny):
    pb, gd, gn = tiny
    sel = [1, 3]
    gd2, gn2 = O.vjp(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                     pb.cotangent, panels=sel)
    assert np.abs(gn2[sel] - gn[sel]).max() < 1e-13 * np.abs(gn).max()
    a = gd2.reshape(2, -1, 16)[:, sel]
    b = gd.reshape(2, -1, 16)[:, sel]
    assert np.abs(a - b).max() < 1e-13 * np.abs(gd).max()
