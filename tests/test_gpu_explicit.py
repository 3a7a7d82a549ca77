"""GPU parity of the explicit-source / explicit-center entry points (through the C ABI)
against the oracle's explicit sums and their autograd gradients; and the consistency
of the explicit path with the contour path on a contour's own sources and centers."""
import sys

import numpy as np
import pytest
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


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t if dtype is None else t.to(dtype)).cuda()


def gpu_args(ep):
    return (dev(ep.src_xy), dev(ep.src_nu), dev(ep.src_q), dev(ep.ctr_xy), dev(ep.ctr_r),
            dev(np.exp(1j * ep.ctr_theta)))


CASES = [
    dict(n_src=333, n_ctr=37, k=3.0, p=0, kind=3),
    dict(n_src=500, n_ctr=64, k=5.0, p=6, kind=1),
    dict(n_src=129, n_ctr=70, k=2.0, p=12, kind=2),
    dict(n_src=1000, n_ctr=23, k=8.0, p=15, kind=3),
    dict(n_src=64, n_ctr=1, k=1.0, p=24, kind=3),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c['kind']}-p{c['p']}-N{c['n_src']}" for c in CASES])
def test_explicit_forward_and_adjoint(Q, case):
    ep = I.explicit_problem(seed=5, **case)
    say(f"case {case}")
    ref = O.apply_explicit(ep.src_xy, ep.src_nu, ep.src_q, ep.ctr_xy, ep.ctr_r, ep.ctr_theta,
                           ep.k, ep.p, ep.kind).numpy()
    args = gpu_args(ep)
    out = Q.apply_explicit(*args, ep.k, ep.p, ep.kind).cpu().numpy()
    tape = torch.empty(Q.explicit_tape_bytes(case["n_ctr"], ep.kind), dtype=torch.uint8,
                       device="cuda")
    out_t = Q.apply_explicit(*args, ep.k, ep.p, ep.kind, tape=tape).cpu().numpy()
    for kk in range(ref.shape[0]):
        e = rel(out[kk], ref[kk])
        say(f"  forward kind {kk}: {e:.3e}")
        assert e < TOL
    assert rel(out_t, out) < 1e-14
    g_ref = O.apply_explicit_vjp(ep.src_xy, ep.src_nu, ep.src_q, ep.ctr_xy, ep.ctr_r,
                                 ep.ctr_theta, ep.k, ep.p, ep.kind, ep.cotangent)
    cot = dev(ep.cotangent)
    for use_tape in (False, True):
        g = Q.apply_explicit_vjp(*args, cot, ep.k, ep.p, ep.kind,
                                 tape=tape if use_tape else None)
        # the theta gradient vanishes identically at p = 0 (J_0 has no angular factor):
        # measure it against the scale of the other center gradients
        floor = 1e-3 * max(np.abs(g_ref["ctr_r"]).max(), np.abs(g_ref["ctr_xy"]).max())
        for key in ("q", "src_xy", "ctr_xy", "ctr_r", "ctr_theta") + (("src_nu",) if ep.kind & 2 else ()):
            a, b = g[key].cpu().numpy(), g_ref[key]
            e = float(np.abs(a - b).max() / max(np.abs(b).max(), floor))
            say(f"  grad {key} (tape={use_tape}): {e:.3e}")
            assert e < (1e-11 if key == "q" else 1e-10), key


def test_explicit_matches_contour_path(Q):
    """The contour entry point equals the explicit sums on its own source grid and
    centers (built by the oracle's geometry), both computed on the GPU."""
    pb = I.small(n_panels=10, p=9, k=4.0, kind=3, side=I.INTERIOR)
    _, aux = O.layer_potential(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side,
                               pb.kind, return_aux=True)
    src = aux["src"]
    fine = O.interpolate_density(torch.from_numpy(pb.density), pb.oversample)
    q = (src["w"].to(torch.complex128)[None, :] * fine).numpy()
    ctr = aux["sides"][I.INTERIOR]["ctr"]
    out = Q.apply_explicit(
        dev(torch.stack([src["x"], src["y"]], 1).numpy()),
        dev(torch.stack([src["nx"], src["ny"]], 1).numpy()), dev(q),
        dev(torch.stack([ctr["cx"], ctr["cy"]], 1).numpy()), dev(ctr["R"].numpy()),
        dev(np.exp(1j * ctr["theta"].numpy())), pb.k, pb.p, pb.kind).cpu().numpy()
    u = Q.layer_potential(dev(pb.nodes), dev(pb.density), pb.k, pb.p, pb.r, pb.oversample,
                          pb.side, pb.kind).cpu().numpy()[0]
    e = rel(out, u)
    say(f"  explicit vs contour path: {e:.3e}")
    assert e < 1e-12
