"""GPU tests of the batched persistent launch: every contour of a batch must give what
the per-contour entry points give (same formulas, same kernels' bodies) and what the
oracle gives; the batch of the random-contour workload is checked in full against the
per-contour path and on sampled targets against the oracle."""
import sys

import numpy as np
import pytest
import torch

from oracle import qbx_oracle as O
from paper_1207_4461_amd import inputs as I

pytestmark = pytest.mark.gpu


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


def mixed_batch():
    specs = [dict(n_panels=5, p=4, kind=1, side=1, k=3.0), dict(n_panels=7, p=9, kind=2, side=0, k=5.0),
             dict(n_panels=4, p=0, kind=3, side=-1, k=2.0), dict(n_panels=9, p=12, kind=3, side=0, k=7.0),
             dict(n_panels=6, p=24, kind=1, side=0, k=1.5), dict(n_panels=6, p=16, kind=2, side=1, k=9.0)]
    return [I.small(name=f"b{i}", seed=30 + i, **s) for i, s in enumerate(specs)]


def per_contour_forward(Q, pb):
    return Q.layer_potential(dev(pb.nodes), dev(pb.density), pb.k, pb.p, pb.r, pb.oversample,
                             pb.side, pb.kind).cpu().numpy()


def test_batched_forward_matches_per_contour_and_oracle(Q):
    pbs = mixed_batch()
    B = Q.Batch(pbs, oversample=4)
    outs = [o.cpu().numpy() for o in B.split_out(B.forward())]
    outs_t = [o.cpu().numpy() for o in B.split_out(B.forward(with_tape=True))]
    for pb, u, ut in zip(pbs, outs, outs_t):
        ref = O.layer_potential(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side,
                                pb.kind).numpy()
        e1, e2 = rel(u, per_contour_forward(Q, pb)), rel(u, ref)
        say(f"  {pb.name} p={pb.p} kind={pb.kind} side={pb.side}: vs per-contour {e1:.2e} vs oracle {e2:.2e}")
        assert e1 < 1e-13 and e2 < 1e-11
        assert rel(ut, u) < 1e-14


def test_batched_adjoint_matches_per_contour_and_oracle(Q):
    pbs = mixed_batch()
    B = Q.Batch(pbs, oversample=4)
    cot = B.pack_out([pb.cotangent for pb in pbs])
    B.forward(with_tape=True)
    gd_t, gn_t = B.adjoint(cot, use_tape=True)
    gd, gn = B.adjoint(cot, use_tape=False)          # the fused pass
    gd2, gn2 = B.adjoint(cot, use_tape=False)
    assert torch.equal(gd, gd2) and torch.equal(gn, gn2)
    et = (rel(gd.cpu().numpy(), gd_t.cpu().numpy()), rel(gn.cpu().numpy(), gn_t.cpu().numpy()))
    say(f"  batched fused vs tape: density {et[0]:.2e} nodes {et[1]:.2e}")
    assert et[0] < 1e-13 and et[1] < 1e-12
    for pb, a, x in zip(pbs, B.split_density(gd), B.split_nodes(gn)):
        rd, rn = O.vjp(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                       pb.cotangent)
        pd, pn = Q.layer_potential_vjp(dev(pb.nodes), dev(pb.density), dev(pb.cotangent), pb.k,
                                       pb.p, pb.r, pb.oversample, pb.side, pb.kind)
        a, x = a.cpu().numpy(), x.cpu().numpy()
        ed, en = rel(a, rd), rel(x, rn)
        say(f"  {pb.name}: density {ed:.2e} nodes {en:.2e} (vs per-contour "
            f"{rel(a, pd.cpu().numpy()):.2e}, {rel(x, pn.cpu().numpy()):.2e})")
        assert ed < 1e-11 and en < 1e-10
        assert rel(a, pd.cpu().numpy()) < 1e-12 and rel(x, pn.cpu().numpy()) < 1e-11


def test_batched_fused_tile_depths(Q):
    """The batched fused pass at the extreme tile depths (1 and 64 source chunks
    per tile) gives the per-contour gradients."""
    pbs = mixed_batch()
    B = Q.Batch(pbs, oversample=4)
    cot = B.pack_out([pb.cotangent for pb in pbs])
    ref = [Q.layer_potential_vjp(dev(pb.nodes), dev(pb.density), dev(pb.cotangent), pb.k, pb.p,
                                 pb.r, pb.oversample, pb.side, pb.kind) for pb in pbs]
    before = Q.get_tuning()
    try:
        for depth in (1, 64):
            Q.set_tuning(batch_fused_chunks=depth)
            gd, gn = B.adjoint(cot, use_tape=False)
            ed = max(rel(a.cpu().numpy(), r[0].cpu().numpy()) for a, r in zip(B.split_density(gd), ref))
            en = max(rel(x.cpu().numpy(), r[1].cpu().numpy()) for x, r in zip(B.split_nodes(gn), ref))
            say(f"  depth {depth}: density {ed:.2e} nodes {en:.2e}")
            assert ed < 1e-12 and en < 1e-11
    finally:
        Q.set_tuning(**before)


def test_batched_fused_tall_tiles(Q):
    """The batched fused pass with tiles taller than one 256-center sub-block (a small
    partial-sum bound): 512 centers, and the whole center set with a ragged last
    sub-block, against the oracle."""
    specs = [dict(n_panels=20, p=10, kind=3, side=0, k=6.0),
             dict(n_panels=33, p=7, kind=1, side=1, k=4.0),
             dict(n_panels=9, p=12, kind=2, side=0, k=7.0)]
    pbs = [I.small(name=f"t{i}", seed=50 + i, **c) for i, c in enumerate(specs)]
    refs = [O.vjp(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                  pb.cotangent) for pb in pbs]
    before = Q.get_tuning()
    try:
        for budget in (200000.0, 4096.0):
            Q.set_tuning(fused_part_bytes=budget)
            B = Q.Batch(pbs, oversample=4)
            cot = B.pack_out([pb.cotangent for pb in pbs])
            gd, gn = B.adjoint(cot, use_tape=False)
            for pb, a, x, (rd, rn) in zip(pbs, B.split_density(gd), B.split_nodes(gn), refs):
                ed, en = rel(a.cpu().numpy(), rd), rel(x.cpu().numpy(), rn)
                say(f"  budget {budget:.0f} {pb.name} ({pb.n_centers} centers): density "
                    f"{ed:.2e} nodes {en:.2e}")
                assert ed < 1e-11 and en < 1e-10
    finally:
        Q.set_tuning(**before)


def test_random64_batch_full(Q):
    pbs = I.random64()
    B = Q.Batch(pbs, oversample=4)
    out = B.forward(with_tape=True)
    outs = B.split_out(out)
    cot = B.pack_out([pb.cotangent for pb in pbs])
    gd, gn = B.adjoint(cot, use_tape=True)
    gdf, gnf = B.adjoint(cot, use_tape=False)        # the fused pass, as timed
    worst_f = worst_d = worst_n = 0.0
    for i, pb in enumerate(pbs):
        u = outs[i].cpu().numpy()
        worst_f = max(worst_f, rel(u, per_contour_forward(Q, pb)))
        pd, pn = Q.layer_potential_vjp(dev(pb.nodes), dev(pb.density), dev(pb.cotangent), pb.k,
                                       pb.p, pb.r, pb.oversample, pb.side, pb.kind)
        pd, pn = pd.cpu().numpy(), pn.cpu().numpy()
        for a, b in ((gd, gn), (gdf, gnf)):
            worst_d = max(worst_d, rel(B.split_density(a)[i].cpu().numpy(), pd))
            worst_n = max(worst_n, rel(B.split_nodes(b)[i].cpu().numpy(), pn))
    say(f"  random64 batch (tape and fused) vs per-contour: forward {worst_f:.2e} "
        f"grad density {worst_d:.2e} grad nodes {worst_n:.2e}")
    assert worst_f < 1e-13 and worst_d < 1e-12 and worst_n < 1e-11
    # oracle on sampled targets of three contours (smallest, largest, one D)
    order = np.argsort([pb.n_panels for pb in pbs])
    dpick = next(i for i in range(len(pbs)) if pbs[i].kind == 2)
    for i in sorted({int(order[0]), int(order[-1]), dpick}):
        pb = pbs[i]
        idx = np.unique(np.random.default_rng(i).choice(pb.n_targets, 12, replace=False))
        ref = O.layer_potential(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side,
                                pb.kind, targets=idx).numpy()
        e = rel(outs[i].cpu().numpy()[:, :, idx], ref)
        say(f"  contour {i} (P={pb.n_panels}, p={pb.p}, kind={pb.kind}, k={pb.k:.1f}): oracle {e:.2e}")
        assert e < 1e-11


def test_batched_autotune_keeps_results(Q):
    """The autotuner only changes launch shapes: results after tuning match the
    per-contour path as before, and the installed tuning is the one returned."""
    pbs = mixed_batch()
    B = Q.Batch(pbs, oversample=4)
    before = Q.get_tuning()
    try:
        tuned = B.autotune(passes=1)
        say(f"  tuned: {tuned}")
        assert Q.get_tuning() == tuned
        assert tuned["batch_adjoint_tasks"] in [2048 << i for i in range(8)]
        assert tuned["batch_grid_scale"] in (0.5, 1.0, 2.0, 4.0)
        assert tuned["batch_fused_chunks"] in (4, 8, 16, 32)
        outs = [o.cpu().numpy() for o in B.split_out(B.forward(with_tape=True))]
        cot = B.pack_out([pb.cotangent for pb in pbs])
        gd, gn = B.adjoint(cot, use_tape=True)
        for pb, u, g1, g2 in zip(pbs, outs, B.split_density(gd), B.split_nodes(gn)):
            assert rel(u, per_contour_forward(Q, pb)) < 1e-13
            rd, rn = Q.layer_potential_vjp(dev(pb.nodes), dev(pb.density), dev(pb.cotangent), pb.k,
                                           pb.p, pb.r, pb.oversample, pb.side, pb.kind)
            assert rel(g1.cpu().numpy(), rd.cpu().numpy()) < 1e-12
            assert rel(g2.cpu().numpy(), rn.cpu().numpy()) < 1e-11
    finally:
        Q.set_tuning(**before)
