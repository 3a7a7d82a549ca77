"""Shared pieces of the full-size GPU parity tests (imported by tests, not collected).

At the star4096 workload (4096 panels, k = 100, p = 20, centers at distance
R = h/2 ~ 8e-4 from the curve) some outputs are ill-conditioned in the input
nodes: moving every node coordinate by one ulp moves the D density gradient by
about 2e-11 of its largest value and the target derivatives of D by about
5e-10.  The oracle and the GPU build the source grid, normals and centers from
the same nodes with different rounding (a few ulps), so their results can agree
only to a few times that sensitivity.  The end-to-end bars at that size are
therefore max(bar, SENS_FACTOR x the sensitivity measured in the test itself);
the kernels' own terms are held to the plain bar by the identical-geometry
tests, which give both sides the oracle's geometry.
"""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SENS_FACTOR = 4.0


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def ulp_perturbed(nodes, seed=1):
    """Every coordinate moved by one ulp, up or down at random (seeded)."""
    sgn = np.random.default_rng(seed).choice([-1.0, 1.0], size=np.shape(nodes))
    return np.where(sgn > 0, np.nextafter(nodes, np.inf), np.nextafter(nodes, -np.inf))


def bar(tol, sensitivity):
    return max(tol, SENS_FACTOR * sensitivity)


def star4096_golden():
    """The oracle's gradients on three star4096 panels (tests/golden/make_star4096_vjp.py):
    (panels, grad_density [n_kinds][3][16] complex, grad_nodes [3][16][2])."""
    with open(os.path.join(GOLDEN, "star4096_vjp_panels.json")) as fh:
        g = json.load(fh)
    gd = np.asarray(g["grad_density_re"]) + 1j * np.asarray(g["grad_density_im"])
    return np.asarray(g["panels"]), gd, np.asarray(g["grad_nodes"])
