"""GPU parity of the hand-written adjoint (through the C ABI) against the oracle.

Density gradients are compared with the oracle's (autograd of the paper's steps,
itself pinned to the dense transposed QBX matrix) at <= 1e-11 relative max-norm;
node gradients at <= 1e-10 (derivatives amplify rounding by ~1/h).  Full-size
workloads: sampled panels through the oracle's restricted gradient, plus
size-independent properties (linearity / dot-product, translation and rotation
invariance, central differences of the GPU forward).
"""
import dataclasses
import sys

import numpy as np
import pytest
import torch

from oracle import qbx_oracle as O
from paper_1207_4461_amd import inputs as I
from parity_helpers import bar, rel, star4096_golden, ulp_perturbed

pytestmark = pytest.mark.gpu
TOL_D = 1e-11
TOL_N = 1e-10


@pytest.fixture(scope="module")
def Q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1207_4461_amd import qbx
    return qbx


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_vjp(Q, pb, tape=None):
    gd, gn = Q.layer_potential_vjp(dev(pb.nodes), dev(pb.density), dev(pb.cotangent), pb.k, pb.p,
                                   pb.r, pb.oversample, pb.side, pb.kind, tape=tape)
    torch.cuda.synchronize()
    return gd.cpu().numpy(), gn.cpu().numpy()


CASES = [
    dict(name="S-ext-p4", n_panels=5, p=4, kind=1, side=1),
    dict(name="S-int-p0", n_panels=4, p=0, kind=1, side=-1),
    dict(name="D-ext-p3", n_panels=5, p=3, kind=2, side=1),
    dict(name="SD-both-p0", n_panels=4, p=0, kind=3, side=0),
    dict(name="D-both-p1", n_panels=4, p=1, kind=2, side=0),
    dict(name="SD-both-p6", n_panels=6, p=6, kind=3, side=0),
    dict(name="SD-both-p12-os2", n_panels=5, p=12, kind=3, side=0, oversample=2, k=7.0),
    dict(name="SD-both-p20-os3", n_panels=4, p=20, kind=3, side=0, oversample=3, k=2.0),
]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_adjoint_small_elementwise(Q, case):
    c = dict(case)
    name = c.pop("name")
    pb = I.small(name=name, **c)
    say(f"case {name}: P={pb.n_panels} p={pb.p} kind={pb.kind} side={pb.side} os={pb.oversample}")
    rd, rn = O.vjp(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                   pb.cotangent)
    gd, gn = gpu_vjp(Q, pb)
    ed, en = rel(gd, rd), rel(gn, rn)
    say(f"  grad density {ed:.3e}  grad nodes {en:.3e}")
    assert ed <= TOL_D and en <= TOL_N


def test_tape_forward_matches_forward_and_reuse(Q):
    pb = I.small(n_panels=7, p=9, kind=3, side=0)
    nodes, dens = dev(pb.nodes), dev(pb.density)
    u0 = Q.layer_potential(nodes, dens, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind)
    tape = torch.empty(Q.tape_bytes(pb.n_panels, pb.p, pb.side, pb.kind), dtype=torch.uint8,
                       device="cuda")
    u1 = Q.layer_potential(nodes, dens, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                           tape=tape)
    torch.cuda.synchronize()
    assert rel(u1.cpu().numpy(), u0.cpu().numpy()) < 1e-14
    # without a tape the adjoint is the fused pass: the same sums in another order
    a = gpu_vjp(Q, pb)
    b = gpu_vjp(Q, pb, tape=tape)
    assert rel(a[0], b[0]) < 1e-13 and rel(a[1], b[1]) < 1e-12


def test_autograd_function_and_gradcheck(Q):
    pb = I.small(n_panels=4, p=3, k=3.0, kind=3, side=0)
    nodes = dev(pb.nodes).requires_grad_(True)
    dens = dev(pb.density).requires_grad_(True)
    u = Q.qbx_apply(nodes, dens, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind)
    g = dev(pb.cotangent)
    L = torch.real(torch.sum(torch.conj(g) * u))
    L.backward()
    rd, rn = O.vjp(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                   pb.cotangent)
    assert rel(dens.grad.cpu().numpy(), rd) < TOL_D
    assert rel(nodes.grad.cpu().numpy(), rn) < TOL_N
    f = lambda X, Dn: Q.qbx_apply(X, Dn, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind)
    assert torch.autograd.gradcheck(f, (nodes.detach().clone().requires_grad_(True),
                                        dens.detach().clone().requires_grad_(True)),
                                    eps=1e-7, atol=1e-6, rtol=1e-5)


def _panels(pb, n, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([[0, pb.n_panels - 1], rng.choice(pb.n_panels, n, replace=False)]))


def check_star4096_panels(gd, gn, sens, n_kinds, what, tol_d=TOL_D, tol_n=TOL_N):
    """Element-wise parity of full star4096 gradients with the stored oracle values on
    three panels.  sens: the same gradients' change under one ulp on every node
    coordinate ({"density": [per kind], "nodes": x}); the bars are the plain ones or
    a few times that sensitivity, whichever is larger."""
    sel, rd, rn = star4096_golden()
    a = gd.reshape(n_kinds, -1, 16)[:, sel]
    en = rel(gn[sel], rn)
    bn = bar(tol_n, sens["nodes"])
    say(f"  {what}: star4096 panels {sel.tolist()}: grad nodes {en:.3e} (one-ulp "
        f"sensitivity {sens['nodes']:.2e}, bar {bn:.2e})")
    assert en <= bn
    for ki in range(n_kinds):
        ed = rel(a[ki], rd[ki])
        bd = bar(tol_d, sens["density"][ki])
        say(f"    kind {ki}: grad density {ed:.3e} (one-ulp sensitivity "
            f"{sens['density'][ki]:.2e}, bar {bd:.2e})")
        assert ed <= bd


def ulp_sensitivity(Q, pb, gd, gn, **kw):
    """How far one ulp on every node coordinate moves the GPU gradients."""
    pert = dataclasses.replace(pb, nodes=ulp_perturbed(pb.nodes))
    gd1, gn1 = gpu_vjp(Q, pert, **kw)
    nk = pb.n_kinds
    return {"density": [rel(gd1.reshape(nk, -1)[k], gd.reshape(nk, -1)[k]) for k in range(nk)],
            "nodes": rel(gn1, gn)}


def test_adjoint_star4096_sampled_panels(Q):
    """The fused adjoint at the bench workload's full size (4096 panels, tile height
    1024 under the default partial-sum bound, so every tile runs four sub-blocks),
    element by element on three panels against the oracle (bars: see parity_helpers;
    the S density gradient and the node gradient meet the plain bars)."""
    pb = I.star4096()
    say(f"star4096: P={pb.n_panels} p={pb.p} kind={pb.kind} side={pb.side}")
    gd, gn = gpu_vjp(Q, pb)
    sens = ulp_sensitivity(Q, pb, gd, gn)
    check_star4096_panels(gd, gn, sens, pb.n_kinds, "default tuning")
    sel, rd, rn = star4096_golden()
    assert rel(gd.reshape(2, -1, 16)[0, sel], rd[0]) <= TOL_D
    assert rel(gn[sel], rn) <= TOL_N


def test_adjoint_star4096_identical_geometry(Q):
    """The adjoint's pair terms at star4096 with the geometry's rounding taken out: the
    oracle's source grid and centers (both sides) go through qbx_apply_explicit_adjoint
    and through the oracle's autograd of the same expansions, for the 64 sources of the
    last panel against every center.  The gradients for the weighted densities, the
    source points and normals (all centers summed) and the center data meet the plain
    bars."""
    pb = I.star4096()
    X = torch.from_numpy(pb.nodes)
    src = O.source_grid(X, pb.oversample)
    fine = O.interpolate_density(torch.from_numpy(pb.density), pb.oversample)
    q = src["w"].to(torch.complex128)[None] * fine
    m = pb.n_panels - 1
    sidx = torch.arange(m * 64, m * 64 + 64)
    src_xy = torch.stack([src["x"], src["y"]], -1)[sidx].contiguous()
    src_nu = torch.stack([src["nx"], src["ny"]], -1)[sidx].contiguous()
    qs = q[:, sidx].contiguous()
    parts = [O.expansion_centers(X, src["h"], src["n_tgt"], pb.r, s) for s in (1, -1)]
    cx, cy, R, th = [torch.cat([c[key] for c in parts]) for key in ("cx", "cy", "R", "theta")]
    cot = np.stack([np.concatenate([pb.cotangent[0, kk], pb.cotangent[1, kk]])
                    for kk in range(pb.n_kinds)])
    ref = {"q": 0.0, "src_xy": 0.0, "src_nu": 0.0}
    r_ctr = {"ctr_xy": [], "ctr_r": [], "ctr_theta": []}
    step = 8192
    for c0 in range(0, len(cx), step):
        sl = slice(c0, c0 + step)
        g = O.apply_explicit_vjp(src_xy, src_nu, qs, torch.stack([cx[sl], cy[sl]], -1), R[sl],
                                 th[sl], pb.k, pb.p, pb.kind, cot[:, sl])
        for key in ref:
            ref[key] = ref[key] + g[key]
        for key in r_ctr:
            r_ctr[key].append(g[key])
    r_ctr = {key: np.concatenate(v) for key, v in r_ctr.items()}
    ctr_dir = torch.exp(1j * th.to(torch.complex128))
    gg = Q.apply_explicit_vjp(dev(src_xy), dev(src_nu), dev(qs), dev(torch.stack([cx, cy], -1)),
                              dev(R), dev(ctr_dir), dev(cot), pb.k, pb.p, pb.kind)
    gg = {key: v.cpu().numpy() for key, v in gg.items()}
    errs = {key: rel(gg[key], ref[key]) for key in ref}
    errs.update({key: rel(gg[key], r_ctr[key]) for key in r_ctr})
    say(f"  identical geometry, panel {m}'s sources x all centers: "
        + ", ".join(f"{key} {v:.2e}" for key, v in errs.items()))
    for ki in range(pb.n_kinds):
        e = rel(gg["q"][ki], ref["q"][ki])
        say(f"    kind {ki}: grad q {e:.2e}")
        assert e <= TOL_D
    assert max(errs.values()) <= TOL_N


def _tile_height(Mc, N, kind, budget):
    slots = (2 if kind == 3 else 1) + 1 + (1 if kind & 2 else 0)
    h = 256
    while h < Mc and -(-Mc // h) * slots * N * 16 > budget:
        h *= 2
    return min(h, Mc)


@pytest.mark.parametrize("case,budgets", [
    (dict(n_panels=40, p=9, k=6.0, kind=3, side=0), (600000.0, 400000.0, 200000.0)),
    (dict(n_panels=40, p=14, k=9.0, kind=2, side=-1, oversample=4), (300000.0, 4096.0)),
    (dict(n_panels=23, p=5, k=4.0, kind=1, side=1, oversample=3), (40000.0,)),
])
def test_fused_adjoint_tall_tiles(Q, case, budgets):
    """Tiles taller than one 256-center sub-block (the path a small partial-sum bound,
    or the star4096 workload under the default one, takes): the wave owning a chunk
    adds each sub-block's source sums into its row in turn.  Element-wise against the
    oracle for tile heights 512, 1024 and the whole center set (a ragged last
    sub-block), with one and with several source blocks."""
    pb = I.small(**case)
    rd, rn = O.vjp(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                   pb.cotangent)
    before = Q.get_tuning()
    try:
        for budget in budgets:
            h = _tile_height(pb.n_centers, pb.n_sources, pb.kind, budget)
            assert h > 256
            for ft in (256, 1 << 22):
                Q.set_tuning(fused_part_bytes=budget, fused_tiles=ft)
                gd, gn = gpu_vjp(Q, pb)
                ed, en = rel(gd, rd), rel(gn, rn)
                say(f"  budget {budget:.0f} (tile height {h} of {pb.n_centers} centers) "
                    f"fused_tiles {ft}: grad density {ed:.3e}  grad nodes {en:.3e}")
                assert ed <= TOL_D and en <= TOL_N
    finally:
        Q.set_tuning(**before)


@pytest.mark.parametrize("cfg,n", [("star256", 3), ("star1024", 2)])
def test_adjoint_full_size_sampled_panels(Q, cfg, n):
    pb = getattr(I, cfg)()
    sel = _panels(pb, n, 11)
    say(f"{cfg}: P={pb.n_panels} p={pb.p} sampled panels {sel.tolist()}")
    gd, gn = gpu_vjp(Q, pb)
    rd, rn = O.vjp(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                   pb.cotangent, panels=sel)
    nk = pb.n_kinds
    a = gd.reshape(nk, -1, 16)[:, sel]
    b = rd.reshape(nk, -1, 16)[:, sel]
    ed = rel(a, b)
    en = rel(gn[sel], rn[sel])
    say(f"  grad density {ed:.3e}  grad nodes {en:.3e}")
    assert ed <= TOL_D and en <= TOL_N


@pytest.mark.parametrize("cfg", ["star1024", "star4096"])
def test_adjoint_full_size_properties(Q, cfg):
    """Linearity (dot-product test), translation and rotation invariance of the node
    gradient, and a central difference of the GPU forward along a smooth deformation."""
    pb = getattr(I, cfg)()
    say(f"{cfg}: P={pb.n_panels} p={pb.p} kind={pb.kind} side={pb.side}")
    nodes, dens, g = dev(pb.nodes), dev(pb.density), dev(pb.cotangent)
    u = Q.layer_potential(nodes, dens, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind)
    L = float(torch.real(torch.sum(torch.conj(g) * u)))
    gd, gn = Q.layer_potential_vjp(nodes, dens, g, pb.k, pb.p, pb.r, pb.oversample, pb.side,
                                   pb.kind)
    Ld = float(torch.real(torch.sum(torch.conj(gd) * dens)))
    say(f"  dot product: L {L:.15e}  <grad, density> {Ld:.15e}")
    assert abs(L - Ld) <= 1e-12 * abs(L)
    gnn = gn.cpu().numpy()
    scale = np.abs(gnn).sum()
    tr = np.abs(gnn.sum(axis=(0, 1))).max() / scale
    torque = abs(np.sum(pb.nodes[..., 0] * gnn[..., 1] - pb.nodes[..., 1] * gnn[..., 0])) / scale
    say(f"  translation {tr:.3e} rotation {torque:.3e}")
    assert tr < 1e-12 and torque < 1e-12
    # smooth deformation: X -> X + eps * (sin 3t, cos 2t)
    t = I.panel_parameters(pb.n_panels)
    E = np.stack([np.sin(3 * t), np.cos(2 * t)], -1)
    def Lof(X):
        uu = Q.layer_potential(dev(X), dens, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind)
        return float(torch.real(torch.sum(torch.conj(g) * uu)))
    h = 1e-6
    fd = (Lof(pb.nodes + h * E) - Lof(pb.nodes - h * E)) / (2 * h)
    an = float(np.sum(gnn * E))
    say(f"  directional derivative: FD {fd:.12e} adjoint {an:.12e}")
    assert abs(fd - an) <= 1e-6 * abs(an)


@pytest.mark.parametrize("case", [dict(n_panels=12, p=9, k=5.0, kind=3, side=0),
                                  dict(n_panels=9, p=0, k=3.0, kind=2, side=-1),
                                  dict(n_panels=40, p=16, k=12.0, kind=1, side=1)])
def test_fused_adjoint_matches_tape_path(Q, case):
    """Without a tape the adjoint is one fused pass; with a tape it is the
    source-major pass plus the tape's center sums; density-only skips the center
    side.  All three give the same gradients (to summation order) and match the
    oracle."""
    pb = I.small(**case)
    nodes, dens = dev(pb.nodes), dev(pb.density)
    cot = dev(pb.cotangent)
    args = (pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind)
    tape = torch.empty(Q.tape_bytes(pb.n_panels, pb.p, pb.side, pb.kind), dtype=torch.uint8,
                       device="cuda")
    Q.layer_potential(nodes, dens, *args, tape=tape)
    gd_t, gn_t = Q.layer_potential_vjp(nodes, dens, cot, *args, tape=tape)
    gd_f, gn_f = Q.layer_potential_vjp(nodes, dens, cot, *args)
    gd_d, gn_d = Q.layer_potential_vjp(nodes, dens, cot, *args, want_nodes=False)
    assert gn_d is None
    rd, rn = O.vjp(pb.nodes, pb.density, *args, pb.cotangent)
    e = [rel(gd_f.cpu().numpy(), gd_t.cpu().numpy()), rel(gn_f.cpu().numpy(), gn_t.cpu().numpy()),
         rel(gd_d.cpu().numpy(), gd_t.cpu().numpy()), rel(gd_f.cpu().numpy(), rd),
         rel(gn_f.cpu().numpy(), rn)]
    say(f"  fused vs tape: density {e[0]:.2e} nodes {e[1]:.2e}; density-only {e[2]:.2e}; "
        f"fused vs oracle {e[3]:.2e} {e[4]:.2e}")
    assert e[0] < 1e-13 and e[1] < 1e-12 and e[2] < 1e-13 and e[3] < 1e-11 and e[4] < 1e-10


def test_fused_adjoint_is_bitwise_deterministic(Q):
    pb = I.small(n_panels=20, p=11, k=6.0, kind=3, side=0)
    a = gpu_vjp(Q, pb)
    b = gpu_vjp(Q, pb)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_fused_adjoint_tile_shapes(Q):
    """The fused pass at the extreme tile targets (one source block per center
    block, and one 64-source chunk per tile) gives the oracle's gradients."""
    pb = I.small(n_panels=30, p=8, k=4.0, kind=3, side=0)
    rd, rn = O.vjp(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                   pb.cotangent)
    before = Q.get_tuning()
    try:
        for ft in (256, 1 << 22):
            Q.set_tuning(fused_tiles=ft)
            gd, gn = gpu_vjp(Q, pb)
            ed, en = rel(gd, rd), rel(gn, rn)
            say(f"  fused_tiles={ft}: grad density {ed:.3e}  grad nodes {en:.3e}")
            assert ed <= TOL_D and en <= TOL_N
    finally:
        Q.set_tuning(**before)
