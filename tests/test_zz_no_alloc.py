"""The forward entry point that allocates nothing (qbx_layer_potential_noalloc)
against the workspace entry point (qbx_layer_potential), both through the C ABI.

The two run the same kernels in the same launch shapes, so their results must
agree bit for bit; the smaller call is also held to the oracle's 1e-11 bar.  Two
calls in a row, the second on a smaller problem, show that the shared static
scratch carries nothing from one call into the next.
"""
import ctypes as C
import sys

import numpy as np
import pytest
import torch

from oracle import qbx_oracle as O
from paper_1207_4461_amd import _lib, inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return _lib.load()


def _run_both(lib, pb):
    dev = torch.device("cuda:0")
    nodes = torch.from_numpy(pb.nodes).to(dev)
    dens = torch.from_numpy(np.ascontiguousarray(pb.density)).to(dev)
    shape = (pb.n_sides, pb.n_kinds, pb.n_targets)
    out_ws = torch.full(shape, complex("nan"), dtype=torch.complex128, device=dev)
    out_na = torch.full(shape, complex("nan"), dtype=torch.complex128, device=dev)
    geo = _lib.Geometry(pb.n_panels, 16, nodes.data_ptr())
    stream = torch.cuda.current_stream(dev).cuda_stream
    nbytes = lib.qbx_workspace_bytes(pb.n_panels, 16, pb.p, pb.oversample, pb.side, pb.kind)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    _lib.check(lib.qbx_layer_potential(C.byref(geo), dens.data_ptr(), pb.k, pb.p, pb.r,
                                       pb.oversample, pb.side, pb.kind, out_ws.data_ptr(), None,
                                       ws.data_ptr(), nbytes, stream))
    _lib.check(lib.qbx_layer_potential_noalloc(C.byref(geo), dens.data_ptr(), pb.k, pb.p, pb.r,
                                               pb.oversample, pb.side, pb.kind,
                                               out_na.data_ptr(), stream))
    torch.cuda.synchronize()
    return out_ws.cpu().numpy(), out_na.cpu().numpy()


def test_noalloc_matches_workspace_entry_twice(lib):
    # first call: star256 (256 panels, both sides, S+D, p = 12), about 5 MB of scratch
    big = I.star256()
    say(f"no-alloc call 1: {big.name} P={big.n_panels} p={big.p} side={big.side} kind={big.kind}")
    a, b = _run_both(lib, big)
    assert np.isfinite(b).all()
    assert np.array_equal(a, b), np.abs(a - b).max()
    # second call, smaller and ragged: 7 panels, exterior, D, p = 7, oversample 3
    small = I.small(n_panels=7, p=7, k=4.0, side=I.EXTERIOR, kind=I.D_KIND, oversample=3)
    say(f"no-alloc call 2: {small.name} P={small.n_panels} p={small.p} side={small.side} "
        f"kind={small.kind} oversample={small.oversample}")
    a, b = _run_both(lib, small)
    assert np.isfinite(b).all()
    assert np.array_equal(a, b), np.abs(a - b).max()
    ref = O.layer_potential(small.nodes, small.density, small.k, small.p, small.r,
                            small.oversample, small.side, small.kind).numpy()
    err = np.abs(b - ref).max() / np.abs(ref).max()
    say(f"  no-alloc small case vs oracle: rel max err {err:.3e}")
    assert err <= 1e-11, err


def test_noalloc_rejects_a_problem_beyond_the_scratch(lib):
    big = I.star4096()
    dev = torch.device("cuda:0")
    nodes = torch.from_numpy(big.nodes).to(dev)
    geo = _lib.Geometry(big.n_panels, 16, nodes.data_ptr())
    rc = lib.qbx_layer_potential_noalloc(C.byref(geo), C.c_void_p(16), big.k, big.p, big.r,
                                         big.oversample, big.side, big.kind, C.c_void_p(16),
                                         torch.cuda.current_stream(dev).cuda_stream)
    assert rc == _lib.QBX_EWORKSPACE and b"static scratch" in lib.qbx_last_error()
