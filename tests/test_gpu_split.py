"""GPU parity of the near/far split forward (qbx_layer_potential_split, through the
C ABI) against the oracle's split (Section 5), and its relation to the plain QBX
forward.  Bar: 1e-11 relative max-norm per output array against the oracle.  The
near/far decisions are bit-identical on both sides (same IEEE formula, no fused
multiply-add), so the two sides sum the same pairs by the same rule."""
import sys

import numpy as np
import pytest
import torch

from oracle import qbx_oracle as O
from paper_1207_4461_amd import inputs as I
from parity_helpers import bar, ulp_perturbed

pytestmark = pytest.mark.gpu
TOL = 1e-11
NODE_TOL = 1e-10   # node gradients, as for the plain adjoint


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


def gpu_split(Q, pb, gamma):
    u = Q.layer_potential_split(dev(pb.nodes), dev(pb.density), pb.k, pb.p, pb.r, pb.oversample,
                                pb.side, pb.kind, gamma=gamma)
    torch.cuda.synchronize()
    return u.cpu().numpy()


CASES = [
    dict(name="S-ext-p4-g3", n_panels=9, p=4, kind=1, side=1, gamma=3.0),
    dict(name="D-int-p6-g4", n_panels=10, p=6, kind=2, side=-1, gamma=4.0),
    dict(name="SD-both-p0-g2", n_panels=7, p=0, kind=3, side=0, gamma=2.0),
    dict(name="SD-both-p12-g6", n_panels=13, p=12, kind=3, side=0, gamma=6.0),
    dict(name="SD-both-p20-os1-g6", n_panels=11, p=20, kind=3, side=0, oversample=1, gamma=6.0),
    dict(name="SD-both-p9-os3-g5", n_panels=9, p=9, kind=3, side=0, oversample=3, k=7.0, gamma=5.0),
    dict(name="SD-both-p3-P3-g1", n_panels=3, p=3, kind=3, side=0, gamma=1.0),
    dict(name="S-ext-p24-os2-g0.5", n_panels=8, p=24, kind=1, side=1, oversample=2, k=2.0,
         gamma=0.5),
    dict(name="SD-both-p5-allnear", n_panels=6, p=5, kind=3, side=0, gamma=1e150),
]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_split_small_elementwise(Q, case):
    c = dict(case)
    name, gamma = c.pop("name"), c.pop("gamma")
    pb = I.small(name=name, **c)
    near = O.near_panels(pb.nodes, gamma)
    say(f"case {name}: P={pb.n_panels} p={pb.p} kind={pb.kind} side={pb.side} os={pb.oversample}"
        f" gamma={gamma}: near panels per panel {near.sum(axis=1).min()}..{near.sum(axis=1).max()}")
    ref = O.layer_potential_split(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side,
                                  pb.kind, gamma=gamma).numpy()
    u = gpu_split(Q, pb, gamma)
    for si in range(ref.shape[0]):
        for ki in range(ref.shape[1]):
            e = rel(u[si, ki], ref[si, ki])
            say(f"  side {si} kind {ki}: {e:.3e}")
            assert e <= TOL


def test_split_all_near_is_the_plain_forward(Q):
    pb = I.small(n_panels=9, p=11, k=6.0, kind=3, side=I.BOTH)
    u = gpu_split(Q, pb, 1e150)
    v = Q.layer_potential(dev(pb.nodes), dev(pb.density), pb.k, pb.p, pb.r, pb.oversample, pb.side,
                          pb.kind).cpu().numpy()
    e = rel(u, v)
    say(f"  all-near split vs plain forward {e:.2e}")
    assert e < 1e-13


def test_split_scan_path_when_lists_overflow(Q):
    """72 panels, every one near every other: the near lists (64 entries) overflow and
    the near passes scan all panels instead.  Forward, derivatives and both adjoints
    then equal the plain (unsplit) results."""
    pb = I.small(n_panels=72, p=6, k=5.0, kind=3, side=I.BOTH)
    nodes, dens, cot = dev(pb.nodes), dev(pb.density), dev(pb.cotangent)
    args = (pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind)
    g = 1e150
    e_f = rel(Q.layer_potential_split(nodes, dens, *args, gamma=g).cpu().numpy(),
              Q.layer_potential(nodes, dens, *args).cpu().numpy())
    a_g, a_n = Q.layer_potential_split_gradient(nodes, dens, *args, gamma=g)
    b_g, b_n = Q.layer_potential_gradient(nodes, dens, *args)
    e_g = max(rel(a_g.cpu().numpy(), b_g.cpu().numpy()), rel(a_n.cpu().numpy(), b_n.cpu().numpy()))
    sd = Q.layer_potential_split_vjp(nodes, dens, cot, *args, gamma=g)
    sd2, sn = Q.layer_potential_split_vjp(nodes, dens, cot, *args, gamma=g, want_nodes=True)
    pd, pn = Q.layer_potential_vjp(nodes, dens, cot, *args)
    e_d = max(rel(sd.cpu().numpy(), pd.cpu().numpy()), rel(sd2.cpu().numpy(), pd.cpu().numpy()))
    e_n = rel(sn.cpu().numpy(), pn.cpu().numpy())
    say(f"  overflowing lists: forward {e_f:.1e} derivatives {e_g:.1e} density adjoint {e_d:.1e}"
        f" node adjoint {e_n:.1e}")
    assert e_f < 1e-13 and e_g < 1e-13 and e_d < 1e-13 and e_n < 1e-12


@pytest.mark.parametrize("cfg,n", [("star256", 24), ("star1024", 16), ("star4096", 5)])
def test_split_full_size_sampled(Q, cfg, n):
    """The workloads at full size (gamma = 6) on sampled targets against the oracle,
    and the whole output against the plain QBX forward on the GPU (they differ by the
    far panels' rule, 16 nodes against the oversampled grid, the far sources' QBX
    truncation and the near patch's end effect only)."""
    pb = getattr(I, cfg)()
    idx = np.unique(np.concatenate([[0, pb.n_targets - 1],
                                    np.random.default_rng(9).choice(pb.n_targets, n, replace=False)]))
    near = O.near_panels(pb.nodes, 6.0)
    say(f"{cfg}: P={pb.n_panels} p={pb.p} kind={pb.kind} side={pb.side}, {len(idx)} targets, "
        f"near panels per panel {near.sum(axis=1).min()}..{near.sum(axis=1).max()}")
    u = gpu_split(Q, pb, 6.0)
    u2 = gpu_split(Q, pb, 6.0)
    assert np.array_equal(u, u2)                      # fixed summation order
    ref = O.layer_potential_split(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side,
                                  pb.kind, gamma=6.0, targets=idx).numpy()
    e = rel(u[:, :, idx], ref)
    v = Q.layer_potential(dev(pb.nodes), dev(pb.density), pb.k, pb.p, pb.r, pb.oversample, pb.side,
                          pb.kind).cpu().numpy()
    gap = rel(u, v)
    say(f"  vs oracle split {e:.3e}; vs plain QBX forward {gap:.3e}")
    assert e <= TOL
    assert gap < 1e-8


def test_split_green_identity_on_gpu(Q):
    curve = I.star((5, 0.25, 0.0))
    P, k, p, x0 = 45, 5.0, 20, (3.0, 1.0)
    nodes = I.panel_nodes(curve, P)
    u, dudn = I.green_pair(curve, P, k, x0)
    v = Q.layer_potential_split(dev(nodes), dev(np.stack([dudn, u])), k, p, 0.5, 4, I.BOTH, 3,
                                gamma=6.0).cpu().numpy()
    sc = np.abs(u).max()
    e_in = np.abs(v[1, 0] - v[1, 1] - u).max() / sc
    e_out = np.abs(v[0, 0] - v[0, 1]).max() / sc
    say(f"  interior {e_in:.3e} exterior {e_out:.3e}")
    assert e_in < 1e-8 and e_out < 1e-8


def oracle_split_density_grad(pb, gamma):
    dens = torch.tensor(pb.density, dtype=torch.complex128, requires_grad=True)
    u = O.layer_potential_split(pb.nodes, dens, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                                gamma=gamma)
    L = torch.real(torch.sum(torch.conj(torch.as_tensor(pb.cotangent)) * u))
    L.backward()
    return dens.grad.numpy()


ADJ_CASES = [
    dict(name="S-ext-p4-g3", n_panels=9, p=4, kind=1, side=1, gamma=3.0),
    dict(name="D-int-p6-g4", n_panels=10, p=6, kind=2, side=-1, gamma=4.0),
    dict(name="SD-both-p12-g6", n_panels=13, p=12, kind=3, side=0, gamma=6.0),
    dict(name="SD-both-p20-os1-g6", n_panels=11, p=20, kind=3, side=0, oversample=1, gamma=6.0),
    dict(name="SD-both-p9-os3-g5", n_panels=9, p=9, kind=3, side=0, oversample=3, k=7.0, gamma=5.0),
    dict(name="SD-both-p3-P3-g1", n_panels=3, p=3, kind=3, side=0, gamma=1.0),
]


@pytest.mark.parametrize("case", ADJ_CASES, ids=[c["name"] for c in ADJ_CASES])
def test_split_density_adjoint_small(Q, case):
    c = dict(case)
    name, gamma = c.pop("name"), c.pop("gamma")
    pb = I.small(name=name, **c)
    ref = oracle_split_density_grad(pb, gamma)
    gd = Q.layer_potential_split_vjp(dev(pb.nodes), dev(pb.density), dev(pb.cotangent), pb.k,
                                     pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                                     gamma=gamma).cpu().numpy()
    e = rel(gd, ref)
    say(f"  {name}: density gradient vs oracle autograd {e:.3e}")
    assert e <= TOL


def test_split_density_adjoint_all_near_is_the_plain_adjoint(Q):
    pb = I.small(n_panels=9, p=11, k=6.0, kind=3, side=I.BOTH)
    a = Q.layer_potential_split_vjp(dev(pb.nodes), dev(pb.density), dev(pb.cotangent), pb.k, pb.p,
                                    pb.r, pb.oversample, pb.side, pb.kind, gamma=1e150)
    b, _ = Q.layer_potential_vjp(dev(pb.nodes), dev(pb.density), dev(pb.cotangent), pb.k, pb.p,
                                 pb.r, pb.oversample, pb.side, pb.kind, want_nodes=False)
    e = rel(a.cpu().numpy(), b.cpu().numpy())
    say(f"  all-near split adjoint vs plain adjoint {e:.2e}")
    assert e < 1e-13


@pytest.mark.parametrize("cfg", ["star1024", "star4096"])
def test_split_density_adjoint_dot_product(Q, cfg):
    """<g, A sigma> = <A^H g, sigma> for the split operator at full size."""
    pb = getattr(I, cfg)()
    nodes, dens = dev(pb.nodes), dev(pb.density)
    rng = np.random.default_rng(3)
    g = dev(rng.standard_normal((pb.n_sides, pb.n_kinds, pb.n_targets))
            + 1j * rng.standard_normal((pb.n_sides, pb.n_kinds, pb.n_targets)))
    args = (pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind)
    u = Q.layer_potential_split(nodes, dens, *args, gamma=6.0)
    gd = Q.layer_potential_split_vjp(nodes, dens, g, *args, gamma=6.0)
    lhs = complex(torch.sum(torch.conj(g) * u))
    rhs = complex(torch.sum(torch.conj(gd) * dens))
    e = abs(lhs - rhs) / abs(lhs)
    say(f"  {cfg}: <g, A s> {lhs:.12e}  <A^H g, s> {rhs:.12e}  rel {e:.2e}")
    assert e < 1e-12


@pytest.mark.parametrize("case", ADJ_CASES, ids=[c["name"] for c in ADJ_CASES])
def test_split_node_adjoint_small(Q, case):
    """Density and node gradients of the split against the oracle's autograd through
    its split (split_vjp), element by element."""
    c = dict(case)
    name, gamma = c.pop("name"), c.pop("gamma")
    pb = I.small(name=name, **c)
    rd, rn = O.split_vjp(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side,
                         pb.kind, pb.cotangent, gamma)
    gd, gn = Q.layer_potential_split_vjp(dev(pb.nodes), dev(pb.density), dev(pb.cotangent),
                                         pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                                         gamma=gamma, want_nodes=True)
    ed, en = rel(gd.cpu().numpy(), rd), rel(gn.cpu().numpy(), rn)
    _, gn_only = Q.layer_potential_split_vjp(dev(pb.nodes), dev(pb.density), dev(pb.cotangent),
                                             pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                                             gamma=gamma, want_nodes=True, want_density=False)
    say(f"  {name}: density {ed:.3e}, nodes {en:.3e} vs oracle autograd")
    assert ed <= TOL and en <= NODE_TOL
    assert torch.equal(gn_only, gn)


def test_split_node_adjoint_all_near_is_the_plain_adjoint(Q):
    pb = I.small(n_panels=9, p=11, k=6.0, kind=3, side=I.BOTH)
    args = (pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind)
    nodes, dens, cot = dev(pb.nodes), dev(pb.density), dev(pb.cotangent)
    a_d, a_n = Q.layer_potential_split_vjp(nodes, dens, cot, *args, gamma=1e150, want_nodes=True)
    b_d, b_n = Q.layer_potential_vjp(nodes, dens, cot, *args)
    ed = rel(a_d.cpu().numpy(), b_d.cpu().numpy())
    en = rel(a_n.cpu().numpy(), b_n.cpu().numpy())
    say(f"  all-near split vs plain adjoint: density {ed:.2e}, nodes {en:.2e}")
    assert ed < 1e-13 and en < 1e-12


@pytest.mark.parametrize("cfg", ["star256", "star1024"])
def test_split_node_adjoint_full_size(Q, cfg):
    """At full size: translation and rotation invariance of the node gradient, the
    dot-product identity for the density, and a Richardson central difference of the
    split forward along a smooth deformation (the near relation checked unchanged)."""
    pb = getattr(I, cfg)()
    nodes, dens = dev(pb.nodes), dev(pb.density)
    rng = np.random.default_rng(4)
    gc = rng.standard_normal((pb.n_sides, pb.n_kinds, pb.n_targets)) \
        + 1j * rng.standard_normal((pb.n_sides, pb.n_kinds, pb.n_targets))
    g = dev(gc)
    args = (pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind)
    gamma = 6.0
    gd, gn = Q.layer_potential_split_vjp(nodes, dens, g, *args, gamma=gamma, want_nodes=True)
    gn = gn.cpu().numpy()
    scale = np.abs(gn).sum()
    trans = np.abs(gn.sum(axis=(0, 1))).max() / scale
    torque = abs(np.sum(pb.nodes[..., 0] * gn[..., 1] - pb.nodes[..., 1] * gn[..., 0])) / (
        scale * np.abs(pb.nodes).max())
    u = Q.layer_potential_split(nodes, dens, *args, gamma=gamma)
    lhs = float(torch.real(torch.sum(torch.conj(g) * u)))
    rhs = float(torch.real(torch.sum(torch.conj(gd) * dens)))
    t = I.panel_parameters(pb.n_panels)
    E = np.stack([np.sin(3 * t), np.cos(2 * t)], -1)

    def L(h):
        X = pb.nodes + h * E
        v = Q.layer_potential_split(dev(X), dens, *args, gamma=gamma)
        return float(torch.real(torch.sum(torch.conj(g) * v)))

    near0 = O.near_panels(pb.nodes, gamma)
    for h in (-2e-5, 2e-5):
        assert np.array_equal(O.near_panels(pb.nodes + h * E, gamma), near0)
    fd = lambda h: (L(h) - L(-h)) / (2 * h)
    rich = (4.0 * fd(5e-6) - fd(1e-5)) / 3.0
    an = float(np.sum(gn * E))
    say(f"  {cfg}: translation {trans:.1e} rotation {torque:.1e} dot {abs(lhs - rhs) / abs(lhs):.1e}"
        f" FD {rich:.10e} adjoint {an:.10e} ({abs(rich - an) / abs(an):.1e})")
    assert trans < 1e-12 and torque < 1e-12
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    assert abs(rich - an) <= 1e-6 * abs(an)


def test_split_autograd_function(Q):
    pb = I.small(n_panels=10, p=8, k=4.0, kind=3, side=I.BOTH)
    nodes = dev(pb.nodes)
    dens = dev(pb.density).requires_grad_(True)
    u = Q.qbx_apply(nodes, dens, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind, gamma=4.0)
    L = torch.real(torch.sum(torch.conj(dev(pb.cotangent)) * u))
    L.backward()
    ref = oracle_split_density_grad(pb, 4.0)
    assert rel(dens.grad.cpu().numpy(), ref) <= TOL
    f = lambda Dn: Q.qbx_apply(nodes, Dn, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                               gamma=4.0)
    assert torch.autograd.gradcheck(f, (dens.detach().clone().requires_grad_(True),),
                                    eps=1e-7, atol=1e-6, rtol=1e-5)
    # the nodes too
    xn = nodes.clone().requires_grad_(True)
    u = Q.qbx_apply(xn, dens.detach(), pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                    gamma=4.0)
    torch.real(torch.sum(torch.conj(dev(pb.cotangent)) * u)).backward()
    _, rn = O.split_vjp(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                        pb.cotangent, 4.0)
    e = rel(xn.grad.cpu().numpy(), rn)
    say(f"  qbx_apply(gamma) node gradient vs oracle autograd {e:.3e}")
    assert e <= NODE_TOL


GRAD_CASES = [
    dict(name="S-ext-p4-g3", n_panels=9, p=4, kind=1, side=1, gamma=3.0),
    dict(name="D-int-p6-g4", n_panels=10, p=6, kind=2, side=-1, gamma=4.0),
    dict(name="SD-both-p12-g6", n_panels=13, p=12, kind=3, side=0, gamma=6.0),
    dict(name="SD-both-p20-os1-g6", n_panels=11, p=20, kind=3, side=0, oversample=1, gamma=6.0),
    dict(name="SD-both-p9-os3-g5", n_panels=9, p=9, kind=3, side=0, oversample=3, k=7.0, gamma=5.0),
    dict(name="SD-both-p3-P3-g1", n_panels=3, p=3, kind=3, side=0, gamma=1.0),
]


@pytest.mark.parametrize("case", GRAD_CASES, ids=[c["name"] for c in GRAD_CASES])
def test_split_gradient_small(Q, case):
    c = dict(case)
    name, gamma = c.pop("name"), c.pop("gamma")
    pb = I.small(name=name, **c)
    rg, rdn = O.layer_potential_split_gradient(pb.nodes, pb.density, pb.k, pb.p, pb.r,
                                               pb.oversample, pb.side, pb.kind, gamma=gamma)
    g, dn = Q.layer_potential_split_gradient(dev(pb.nodes), dev(pb.density), pb.k, pb.p, pb.r,
                                             pb.oversample, pb.side, pb.kind, gamma=gamma)
    g, dn = g.cpu().numpy(), dn.cpu().numpy()
    for si in range(rg.shape[0]):
        for ki in range(rg.shape[1]):
            eg, ed = rel(g[si, ki], rg[si, ki].numpy()), rel(dn[si, ki], rdn[si, ki].numpy())
            say(f"  {name} side {si} kind {ki}: grad {eg:.3e}  n.grad {ed:.3e}")
            assert eg <= TOL and ed <= TOL
    _, dn2 = Q.layer_potential_split_gradient(dev(pb.nodes), dev(pb.density), pb.k, pb.p, pb.r,
                                              pb.oversample, pb.side, pb.kind, gamma=gamma,
                                              want_grad=False)
    assert np.array_equal(dn2.cpu().numpy(), dn)


def test_split_gradient_star4096(Q):
    pb = I.star4096()
    idx = np.unique(np.concatenate([[0, pb.n_targets - 1],
                                    np.random.default_rng(12).choice(pb.n_targets, 5,
                                                                     replace=False)]))
    rg, rdn = O.layer_potential_split_gradient(pb.nodes, pb.density, pb.k, pb.p, pb.r,
                                               pb.oversample, pb.side, pb.kind, gamma=6.0,
                                               targets=idx)
    g, dn = Q.layer_potential_split_gradient(dev(pb.nodes), dev(pb.density), pb.k, pb.p, pb.r,
                                             pb.oversample, pb.side, pb.kind, gamma=6.0)
    g0, dn0 = Q.layer_potential_gradient(dev(pb.nodes), dev(pb.density), pb.k, pb.p, pb.r,
                                         pb.oversample, pb.side, pb.kind)
    g, dn = g.cpu().numpy(), dn.cpu().numpy()
    # the bar: 1e-11, or a few times each array's change under one ulp on every node
    # coordinate (parity_helpers), about 5e-10 for the D derivatives at this size
    g1, dn1 = Q.layer_potential_split_gradient(dev(ulp_perturbed(pb.nodes)), dev(pb.density),
                                               pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                                               gamma=6.0)
    g1, dn1 = g1.cpu().numpy(), dn1.cpu().numpy()
    rg, rdn = rg.numpy(), rdn.numpy()
    for si in range(rg.shape[0]):
        for ki in range(rg.shape[1]):
            eg, ed = rel(g[si, ki, idx], rg[si, ki]), rel(dn[si, ki, idx], rdn[si, ki])
            bg = bar(TOL, rel(g1[si, ki], g[si, ki]))
            bd = bar(TOL, rel(dn1[si, ki], dn[si, ki]))
            say(f"  star4096 side {si} kind {ki}: vs oracle grad {eg:.3e} (bar {bg:.2e}) "
                f"n.grad {ed:.3e} (bar {bd:.2e})")
            assert eg <= bg and ed <= bd
    gap = max(rel(g, g0.cpu().numpy()), rel(dn, dn0.cpu().numpy()))
    say(f"  star4096: vs plain QBX derivatives {gap:.3e}")
    assert gap < 1e-10
