"""The flop model behind every TFLOP/s figure (paper_1207_4461_amd/flops.py): its per-pair
counts equal the closed forms its docstring derives, the direct-pass counts are fixed, and
the split's pair counts add up to the workload's pairs at the two extremes of gamma."""
import numpy as np

from paper_1207_4461_amd import flops as F
from paper_1207_4461_amd import inputs as I


def test_forward_counts_follow_the_closed_forms():
    for p in range(1, 40):
        assert F.flops_forward_pair(p, 1) == 95 + 12 * p
        assert F.flops_forward_pair(p, 2) == 114 + 16 * p
        assert F.flops_forward_pair(p, 3) == 128 + 23 * p


def test_counts_grow_with_the_order_and_fuse_below_the_sum():
    for kind in (1, 2, 3):
        for fn in (F.flops_forward_pair, F.flops_tape_pair, F.flops_adjoint_pair,
                   F.flops_fused_pair, F.flops_grad_pair):
            c = [fn(p, kind) for p in range(0, 30)]
            assert all(b > a for a, b in zip(c, c[1:])), fn.__name__
    for p in (4, 12, 20):
        # S and D in one pass share the geometry and the seed
        for fn in (F.flops_forward_pair, F.flops_fused_pair):
            assert fn(p, 3) < fn(p, 1) + fn(p, 2)


def test_direct_pass_counts():
    assert (F.flops_far_pair(1), F.flops_far_pair(2), F.flops_far_pair(3)) == (85, 91, 99)
    assert F.interactions(10, 7, 3) == 140 and F.interactions(10, 7, 1) == 70


def test_split_pair_counts_at_the_extremes():
    P, os_ = 12, 2
    nodes = I.panel_nodes(I.star((5, 0.25, 0.0)), P)
    qs = 16 * os_
    near, far = F.split_pairs(nodes, os_, 2, 1e150)          # every panel near
    assert (near, far) == (2 * 16 * P * qs * P, 0)
    cnt = F.near_panel_counts(nodes, 1e-9)                    # each panel near only itself
    assert np.array_equal(cnt, np.ones(P, dtype=cnt.dtype))
    near, far = F.split_pairs(nodes, os_, 2, 1e-9)
    # far panels lend their 16 nodes, whatever the oversampling
    assert (near, far) == (2 * 16 * qs * P, (P - 1) * 16 * 16 * P)
