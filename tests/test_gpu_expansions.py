"""GPU parity of the stored local expansions (Section 5: one expansion serving several
nearby targets) through the C ABI: qbx_expansion_coefficients against the oracle's
coefficients, qbx_evaluate_expansions against the oracle's evaluation at points
inside the disks, qbx_assign_centers against the oracle's rule on the same centers,
and checks on the GPU alone (self-evaluation equals the one-sided limits; Green's
representation off the curve).

Coefficients are held to the bars of expansion_bars.py; evaluated potentials and
centers to plain relative max-norm bars."""
import sys

import numpy as np
import pytest
import scipy.special as sps
import torch

from oracle import qbx_oracle as O
from paper_1207_4461_amd import inputs as I

from expansion_bars import check_coefficients

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


def center_gap(C, ref):
    """Largest distance between the two sides' centers, at least 4 ulps of the
    coordinates (the source grids differ by about that much)."""
    C, ref = np.asarray(C), np.asarray(ref)
    return max(float(np.hypot(*(C - ref).T).max()), 4 * np.spacing(np.abs(ref).max()))


def disk_targets(C, R, ci, rng, lo=0.2, hi=0.9):
    ang = rng.uniform(0, 2 * np.pi, len(ci))
    rr = rng.uniform(lo, hi, len(ci))
    return C[ci] + (rr * R[ci])[:, None] * np.stack([np.cos(ang), np.sin(ang)], -1)


CASES = [
    dict(name="S-ext-p0", n_panels=5, p=0, kind=1, side=1),
    dict(name="S-int-p5", n_panels=6, p=5, kind=1, side=-1),
    dict(name="D-ext-p3", n_panels=5, p=3, kind=2, side=1),
    dict(name="SD-both-p7", n_panels=7, p=7, kind=3, side=0),
    dict(name="SD-both-p12-os3", n_panels=6, p=12, kind=3, side=0, oversample=3, k=7.0),
    dict(name="SD-int-p24-os1", n_panels=9, p=24, kind=3, side=-1, oversample=1, k=2.0),
]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_expansions_small_against_oracle(Q, case):
    c = dict(case)
    name = c.pop("name")
    pb = I.small(name=name, **c)
    say(f"case {name}: P={pb.n_panels} p={pb.p} kind={pb.kind} side={pb.side} os={pb.oversample}")
    ra, rC, rR = O.expansion_coefficients(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample,
                                          pb.side, pb.kind)
    ra, rC, rR = ra.numpy(), rC.numpy(), rR.numpy()
    a, Cg, Rg = Q.expansion_coefficients(dev(pb.nodes), dev(pb.density), pb.k, pb.p, pb.r,
                                         pb.oversample, pb.side, pb.kind)
    a, Cg, Rg = a.cpu().numpy(), Cg.cpu().numpy(), Rg.cpu().numpy()
    # both sides differentiate the same 16-node interpolant through different formulas
    # (a 16 x 16 differentiation matrix against Legendre series); its norm ~1e2 lets
    # rounding reach ~1e-13 of the coordinates
    assert rel(Cg, rC) < 1e-12 and rel(Rg, rR) < 1e-12
    check_coefficients(a, ra, pb, rC, rR, center_gap(Cg, rC))
    # targets inside the disks of every third center, assigned on the GPU
    rng = np.random.default_rng(7)
    ci = np.arange(0, len(Cg), 3)
    tg = disk_targets(Cg, Rg, ci, rng)
    idx = Q.assign_centers(dev(Cg), dev(Rg), dev(tg)).cpu().numpy()
    assert np.array_equal(idx, O.assign_centers(Cg, Rg, tg))
    assert (idx >= 0).all()
    u = Q.evaluate_expansions(dev(a), dev(Cg), dev(tg), dev(idx.astype(np.int32)), pb.k, pb.p,
                              pb.kind).cpu().numpy()
    ref = O.evaluate_expansions(ra, rC, tg, idx, pb.k, pb.p).numpy()
    for ki in range(u.shape[0]):
        e = rel(u[ki], ref[ki])
        say(f"  evaluation kind {ki}: {e:.3e}")
        assert e <= TOL


def test_self_evaluation_is_the_layer_potential_on_gpu(Q):
    """Each center's expansion at its own target gives qbx_layer_potential's limit."""
    pb = I.small(n_panels=11, p=9, k=5.0, kind=3, side=I.BOTH)
    nodes, dens = dev(pb.nodes), dev(pb.density)
    a, Cg, Rg = Q.expansion_coefficients(nodes, dens, pb.k, pb.p, pb.r, pb.oversample, pb.side,
                                         pb.kind)
    tg = torch.cat([nodes.reshape(-1, 2)] * 2)
    idx = torch.arange(tg.shape[0], dtype=torch.int32, device="cuda")
    v = Q.evaluate_expansions(a, Cg, tg, idx, pb.k, pb.p, pb.kind).cpu().numpy()
    u = Q.layer_potential(nodes, dens, pb.k, pb.p, pb.r, pb.oversample, pb.side,
                          pb.kind).cpu().numpy()
    T = pb.n_targets
    for si in range(2):
        for ki in range(2):
            e = rel(v[ki, si * T:(si + 1) * T], u[si, ki])
            say(f"  side {si} kind {ki}: {e:.3e}")
            assert e < 1e-12


@pytest.mark.parametrize("cfg,n", [("star256", 40), ("star1024", 20)])
def test_expansions_full_size_sampled(Q, cfg, n):
    pb = getattr(I, cfg)()
    Mc = pb.n_centers
    sel = np.unique(np.concatenate([[0, Mc - 1],
                                    np.random.default_rng(9).choice(Mc, n, replace=False)]))
    say(f"{cfg}: {Mc} centers, {len(sel)} sampled")
    a, Cg, Rg = Q.expansion_coefficients(dev(pb.nodes), dev(pb.density), pb.k, pb.p, pb.r,
                                         pb.oversample, pb.side, pb.kind)
    a = a.cpu().numpy()[:, sel]
    ra, rC, rR = O.expansion_coefficients(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample,
                                          pb.side, pb.kind, centers=sel)
    ra, rC, rR = ra.numpy(), rC.numpy(), rR.numpy()
    Cs = Cg.cpu().numpy()[sel]
    assert rel(Cs, rC) < 1e-12 and rel(Rg.cpu().numpy()[sel], rR) < 1e-12
    check_coefficients(a, ra, pb, rC, rR, center_gap(Cs, rC))
    tg = disk_targets(Cg.cpu().numpy(), Rg.cpu().numpy(), sel, np.random.default_rng(2))
    v = Q.evaluate_expansions(dev(a), dev(Cg.cpu().numpy()[sel]), dev(tg),
                              dev(np.arange(len(sel), dtype=np.int32)), pb.k, pb.p,
                              pb.kind).cpu().numpy()
    ref = O.evaluate_expansions(ra, rC, tg, np.arange(len(sel)), pb.k, pb.p).numpy()
    for ki in range(v.shape[0]):
        e = rel(v[ki], ref[ki])
        say(f"  evaluation kind {ki}: {e:.3e}")
        assert e <= TOL


def test_green_representation_off_the_curve_on_gpu(Q):
    """S[du/dn] - D[u] = u in interior disks and 0 in exterior ones, for u = H_0(k|x - x0|),
    computed on the GPU alone."""
    curve = I.star((5, 0.25, 0.0))
    P, k, p, x0 = 40, 5.0, 10, (3.0, 1.0)
    nodes = I.panel_nodes(curve, P)
    u, dudn = I.green_pair(curve, P, k, x0)
    a, Cg, Rg = Q.expansion_coefficients(dev(nodes), dev(np.stack([dudn, u])), k, p, 0.5, 4,
                                         I.BOTH, 3)
    C, R = Cg.cpu().numpy(), Rg.cpu().numpy()
    T = P * 16
    ci = np.arange(0, 2 * T, 3)
    tg = disk_targets(C, R, ci, np.random.default_rng(0), 0.5, 0.7)
    idx = Q.assign_centers(Cg, Rg, dev(tg)).cpu().numpy()
    v = Q.evaluate_expansions(a, Cg, dev(tg), dev(idx.astype(np.int32)), k, p, 3).cpu().numpy()
    rep = v[0] - v[1]
    uex = sps.hankel1(0, k * np.hypot(tg[:, 0] - x0[0], tg[:, 1] - x0[1]))
    inside = idx >= T
    sc = np.abs(uex).max()
    e_in = np.abs(rep[inside] - uex[inside]).max() / sc
    e_out = np.abs(rep[~inside]).max() / sc
    say(f"  interior {e_in:.2e} exterior {e_out:.2e}")
    assert e_in < 1e-12 and e_out < 1e-12
