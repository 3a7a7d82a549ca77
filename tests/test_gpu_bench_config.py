"""Parity at full size in the launch configuration bench.py times: the autotuner
installs the shapes it picks for the timed passes (forward and fused adjoint), and
the results are then checked against the oracle on sampled targets (star4096) and
against one launch per contour (random64, the batched launch)."""
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


def test_star4096_in_bench_configuration(Q):
    pb = I.star4096()
    nodes, dens, cot = dev(pb.nodes), dev(pb.density), dev(pb.cotangent)
    args = (pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind)
    before = Q.get_tuning()
    try:
        tuned = Q.autotune(nodes, dens, *args, passes=1, fields=Q.TUNE_FORWARD | Q.TUNE_FUSED)
        say(f"  tuned: {tuned}")
        u = Q.layer_potential(nodes, dens, *args).cpu().numpy()
        idx = np.unique(np.concatenate([[0, pb.n_targets - 1],
                                        np.random.default_rng(9).choice(pb.n_targets, 10,
                                                                        replace=False)]))
        ref = O.layer_potential(pb.nodes, pb.density, *args, targets=idx).numpy()
        e = rel(u[:, :, idx], ref)
        say(f"  forward at {len(idx)} sampled targets: {e:.3e}")
        assert e <= 1e-11
        # the fused adjoint in the same shapes: the dot-product identity at full size
        gd, gn = Q.layer_potential_vjp(nodes, dens, cot, *args)
        L = float(np.real(np.sum(np.conj(pb.cotangent) * u)))
        Ld = float(torch.real(torch.sum(torch.conj(gd) * dens)))
        say(f"  dot product: {abs(L - Ld) / abs(L):.3e}")
        assert abs(L - Ld) <= 1e-12 * abs(L)
        # and element by element on three panels against the oracle's stored gradients
        from test_gpu_adjoint import check_star4096_panels, ulp_sensitivity
        gd, gn = gd.cpu().numpy(), gn.cpu().numpy()
        check_star4096_panels(gd, gn, ulp_sensitivity(Q, pb, gd, gn), pb.n_kinds,
                              "bench tuning")
    finally:
        Q.set_tuning(**before)


def test_random64_in_bench_configuration(Q):
    pbs = I.random64()
    B = Q.Batch(pbs, oversample=4)
    before = Q.get_tuning()
    try:
        tuned = B.autotune(passes=1, fields=Q.TUNE_FORWARD | Q.TUNE_FUSED)
        say(f"  tuned: {tuned}")
        outs = B.split_out(B.forward())
        cot = B.pack_out([pb.cotangent for pb in pbs])
        gd, gn = B.adjoint(cot, use_tape=False)
        worst = [0.0, 0.0, 0.0]
        for i in (0, 17, 31, 63):
            pb = pbs[i]
            u = Q.layer_potential(dev(pb.nodes), dev(pb.density), pb.k, pb.p, pb.r, pb.oversample,
                                  pb.side, pb.kind).cpu().numpy()
            pd, pn = Q.layer_potential_vjp(dev(pb.nodes), dev(pb.density), dev(pb.cotangent), pb.k,
                                           pb.p, pb.r, pb.oversample, pb.side, pb.kind)
            worst[0] = max(worst[0], rel(outs[i].cpu().numpy(), u))
            worst[1] = max(worst[1], rel(B.split_density(gd)[i].cpu().numpy(), pd.cpu().numpy()))
            worst[2] = max(worst[2], rel(B.split_nodes(gn)[i].cpu().numpy(), pn.cpu().numpy()))
        say(f"  batched vs per contour: {worst}")
        assert worst[0] < 1e-13 and worst[1] < 1e-12 and worst[2] < 1e-11
    finally:
        Q.set_tuning(**before)
