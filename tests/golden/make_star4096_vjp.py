"""Write star4096_vjp_panels.json: the oracle's gradients of L = Re <g, u> with
respect to the density and the node coordinates on three panels of the star4096
workload (4096 panels, k = 100, p = 20, both sides, S+D, oversample 4), for the
GPU adjoint's element-wise parity test at that size.

It calls only the oracle (its restricted gradient, exact on the named panels)
and the seeded input generator.  Run from the repository root:

    python tests/golden/make_star4096_vjp.py

It takes a few minutes on eight cores.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import qbx_oracle as O  # noqa: E402
from paper_1207_4461_amd import inputs as I  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "star4096_vjp_panels.json")


def panels(pb):
    """The first and last panel, and one interior panel drawn from a fixed seed."""
    inner = int(np.random.default_rng(4096).integers(1, pb.n_panels - 1))
    return [0, inner, pb.n_panels - 1]


def main():
    pb = I.star4096()
    sel = panels(pb)
    t0 = time.perf_counter()
    gd, gn = O.vjp(pb.nodes, pb.density, pb.k, pb.p, pb.r, pb.oversample, pb.side, pb.kind,
                   pb.cotangent, panels=sel)
    dt = time.perf_counter() - t0
    nk = pb.n_kinds
    d = gd.reshape(nk, pb.n_panels, 16)[:, sel]
    n = gn[sel]
    rec = {
        "workload": "star4096",
        "what": "oracle.vjp restricted to the listed panels: grad_density [n_kinds][panel][16] "
                "complex (re, im), grad_nodes [panel][16][2]",
        "n_panels": pb.n_panels, "k": pb.k, "p": pb.p, "r": pb.r, "oversample": pb.oversample,
        "side": pb.side, "kind": pb.kind, "panels": sel,
        "grad_density_re": np.real(d).tolist(), "grad_density_im": np.imag(d).tolist(),
        "grad_nodes": n.tolist(),
        "oracle_seconds": round(dt, 1),
    }
    with open(OUT, "w") as fh:
        json.dump(rec, fh, indent=0)
        fh.write("\n")
    print(f"wrote {OUT} ({dt:.1f} s)")


if __name__ == "__main__":
    main()
