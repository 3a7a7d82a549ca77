"""PyTorch-facing API of libqbx: tensors in, tensors out, on torch's current stream.

Every step of the computation runs in the HIP library; this module only checks
tensor shapes/dtypes/devices, allocates outputs and workspaces with torch, and
passes raw device pointers through the C ABI (include/qbx.h).
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Tuple

import torch

from . import _lib

S = _lib.QBX_S
D = _lib.QBX_D
SD = _lib.QBX_S | _lib.QBX_D
INTERIOR = _lib.QBX_INTERIOR
EXTERIOR = _lib.QBX_EXTERIOR
BOTH = _lib.QBX_BOTH
Q = _lib.QBX_Q


def n_kinds(kind: int) -> int:
    return 2 if kind == SD else 1


def n_sides(side: int) -> int:
    return 2 if side == BOTH else 1


def _stream(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _need(t: torch.Tensor, name: str, dtype, shape) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def workspace_bytes(n_panels: int, p: int, oversample: int = 4, side: int = EXTERIOR,
                    kind: int = S) -> int:
    n = _lib.load().qbx_workspace_bytes(n_panels, Q, p, oversample, side, kind)
    if n == 0:
        raise _lib.QBXError(_lib.QBX_EINVAL, "invalid problem parameters")
    return int(n)


def tape_bytes(n_panels: int, p: int, side: int = EXTERIOR, kind: int = S) -> int:
    return int(_lib.load().qbx_tape_bytes(n_panels, Q, p, side, kind))


def _workspace(nbytes: int, device, workspace: Optional[torch.Tensor]) -> torch.Tensor:
    if workspace is not None:
        if workspace.device != device or workspace.dtype != torch.uint8:
            raise ValueError("workspace must be a uint8 tensor on the nodes' device")
        if workspace.numel() < nbytes:
            raise ValueError(f"workspace holds {workspace.numel()} bytes, {nbytes} needed")
        return workspace
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def layer_potential(nodes: torch.Tensor, density: torch.Tensor, k: float, p: int, r: float = 0.5,
                    oversample: int = 4, side: int = EXTERIOR, kind: int = S,
                    tape: Optional[torch.Tensor] = None,
                    workspace: Optional[torch.Tensor] = None, dipole: str = "normal",
                    center_rule: str = "h") -> torch.Tensor:
    """One-sided QBX limits, out[n_sides, n_kinds, 16*P] complex128 (exterior first).
    dipole="tangential": the D slot is the tangential dipole R; center_rule="sqrt":
    center distance r sqrt(h) (both through qbx_layer_potential_ext, forward only)."""
    if dipole not in ("normal", "tangential") or center_rule not in ("h", "sqrt"):
        raise ValueError("dipole must be 'normal' or 'tangential', center_rule 'h' or 'sqrt'")
    if dipole != "normal" or center_rule != "h":
        if tape is not None:
            raise ValueError("a tape is only written with the default options")
        return _layer_potential_ext(nodes, density, k, p, r, oversample, side, kind, workspace,
                                    int(dipole == "tangential"), int(center_rule == "sqrt"))
    lib = _lib.load()
    P = int(nodes.shape[0]) if nodes.dim() == 3 else -1
    _need(nodes, "nodes", torch.float64, (P, Q, 2))
    nk = n_kinds(kind)
    _need(density, "density", torch.complex128, (nk, P * Q))
    dev = nodes.device
    out = torch.empty((n_sides(side), nk, P * Q), dtype=torch.complex128, device=dev)
    ws = _workspace(workspace_bytes(P, p, oversample, side, kind), dev, workspace)
    tp = None
    if tape is not None:
        need = tape_bytes(P, p, side, kind)
        if tape.device != dev or tape.numel() * tape.element_size() < need:
            raise ValueError("tape too small or on the wrong device")
        tp = tape.data_ptr()
    geo = _lib.Geometry(P, Q, nodes.data_ptr())
    rc = lib.qbx_layer_potential(C.byref(geo), density.data_ptr(), float(k), int(p), float(r),
                                 int(oversample), int(side), int(kind), out.data_ptr(), tp,
                                 ws.data_ptr(), ws.numel(), _stream(dev))
    _lib.check(rc)
    return out


def layer_potential_noalloc(nodes: torch.Tensor, density: torch.Tensor, k: float, p: int,
                            r: float = 0.5, oversample: int = 4, side: int = EXTERIOR,
                            kind: int = S, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """The plain forward of layer_potential through qbx_layer_potential_noalloc: no
    workspace; the library's static device scratch (shared by every call on the
    device: calls that overlap on one GPU race).  Pass `out` to allocate nothing
    here either."""
    lib = _lib.load()
    P = int(nodes.shape[0]) if nodes.dim() == 3 else -1
    _need(nodes, "nodes", torch.float64, (P, Q, 2))
    nk = n_kinds(kind)
    _need(density, "density", torch.complex128, (nk, P * Q))
    dev = nodes.device
    shape = (n_sides(side), nk, P * Q)
    if out is None:
        out = torch.empty(shape, dtype=torch.complex128, device=dev)
    else:
        _need(out, "out", torch.complex128, shape)
        if out.device != dev:
            raise ValueError("out must be on the nodes' device")
    geo = _lib.Geometry(P, Q, nodes.data_ptr())
    with torch.cuda.device(dev):
        rc = lib.qbx_layer_potential_noalloc(C.byref(geo), density.data_ptr(), float(k), int(p),
                                             float(r), int(oversample), int(side), int(kind),
                                             out.data_ptr(), _stream(dev))
    _lib.check(rc)
    return out


def expansion_coefficients(nodes: torch.Tensor, density: torch.Tensor, k: float, p: int,
                           r: float = 0.5, oversample: int = 4, side: int = EXTERIOR,
                           kind: int = S, workspace: Optional[torch.Tensor] = None):
    """qbx_expansion_coefficients: the stored local expansions of every center,
    (coef [n_kinds, Mc, 2p+1] complex128 without the i/4, centers [Mc, 2], radii [Mc])."""
    lib = _lib.load()
    P = int(nodes.shape[0]) if nodes.dim() == 3 else -1
    _need(nodes, "nodes", torch.float64, (P, Q, 2))
    nk = n_kinds(kind)
    _need(density, "density", torch.complex128, (nk, P * Q))
    dev = nodes.device
    Mc = n_sides(side) * P * Q
    coef = torch.empty((nk, Mc, 2 * p + 1), dtype=torch.complex128, device=dev)
    ctr = torch.empty((Mc, 2), dtype=torch.float64, device=dev)
    rad = torch.empty(Mc, dtype=torch.float64, device=dev)
    nbytes = int(lib.qbx_expansion_workspace_bytes(P, Q, int(p), int(oversample), int(side),
                                                   int(kind)))
    if nbytes == 0:
        raise _lib.QBXError(_lib.QBX_EINVAL, "invalid problem parameters")
    ws = _workspace(nbytes, dev, workspace)
    geo = _lib.Geometry(P, Q, nodes.data_ptr())
    _lib.check(lib.qbx_expansion_coefficients(C.byref(geo), density.data_ptr(), float(k), int(p),
                                              float(r), int(oversample), int(side), int(kind),
                                              coef.data_ptr(), ctr.data_ptr(), rad.data_ptr(),
                                              ws.data_ptr(), ws.numel(), _stream(dev)))
    return coef, ctr, rad


def evaluate_expansions(coef: torch.Tensor, centers: torch.Tensor, targets: torch.Tensor,
                        center_index: torch.Tensor, k: float, p: int, kind: int = S
                        ) -> torch.Tensor:
    """qbx_evaluate_expansions: [n_kinds, n_targets] complex128, each target from the
    expansion of center_index[t] (int32)."""
    lib = _lib.load()
    nk = n_kinds(kind)
    Mc = int(centers.shape[0])
    _need(coef, "coef", torch.complex128, (nk, Mc, 2 * p + 1))
    _need(centers, "centers", torch.float64, (Mc, 2))
    nt = int(targets.shape[0])
    _need(targets, "targets", torch.float64, (nt, 2))
    _need(center_index, "center_index", torch.int32, (nt,))
    out = torch.empty((nk, nt), dtype=torch.complex128, device=coef.device)
    _lib.check(lib.qbx_evaluate_expansions(Mc, centers.data_ptr(), coef.data_ptr(), float(k),
                                           int(p), int(kind), nt, targets.data_ptr(),
                                           center_index.data_ptr(), out.data_ptr(),
                                           _stream(coef.device)))
    return out


def assign_centers(centers: torch.Tensor, radii: torch.Tensor, targets: torch.Tensor,
                   slack: float = 1.0) -> torch.Tensor:
    """qbx_assign_centers: per target, the nearest center whose disk (radius x slack)
    holds it, or -1 (int32)."""
    lib = _lib.load()
    Mc = int(centers.shape[0])
    _need(centers, "centers", torch.float64, (Mc, 2))
    _need(radii, "radii", torch.float64, (Mc,))
    nt = int(targets.shape[0])
    _need(targets, "targets", torch.float64, (nt, 2))
    idx = torch.empty(nt, dtype=torch.int32, device=centers.device)
    _lib.check(lib.qbx_assign_centers(Mc, centers.data_ptr(), radii.data_ptr(), nt,
                                      targets.data_ptr(), float(slack), idx.data_ptr(),
                                      _stream(centers.device)))
    return idx


def _layer_potential_ext(nodes, density, k, p, r, oversample, side, kind, workspace, dipole,
                         center_rule):
    lib = _lib.load()
    P = int(nodes.shape[0]) if nodes.dim() == 3 else -1
    _need(nodes, "nodes", torch.float64, (P, Q, 2))
    nk = n_kinds(kind)
    _need(density, "density", torch.complex128, (nk, P * Q))
    dev = nodes.device
    out = torch.empty((n_sides(side), nk, P * Q), dtype=torch.complex128, device=dev)
    ws = _workspace(workspace_bytes(P, p, oversample, side, kind), dev, workspace)
    geo = _lib.Geometry(P, Q, nodes.data_ptr())
    opt = _lib.ForwardOptions(dipole, center_rule)
    _lib.check(lib.qbx_layer_potential_ext(C.byref(geo), density.data_ptr(), float(k), int(p),
                                           float(r), int(oversample), int(side), int(kind),
                                           C.byref(opt), out.data_ptr(), ws.data_ptr(),
                                           ws.numel(), _stream(dev)))
    return out


def layer_potential_split(nodes: torch.Tensor, density: torch.Tensor, k: float, p: int,
                          r: float = 0.5, oversample: int = 4, side: int = EXTERIOR, kind: int = S,
                          gamma: float = 6.0,
                          workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Near/far split forward (qbx_layer_potential_split): QBX for the sources of
    panels within gamma panel radii of the target's panel, the smooth rule applied
    directly for all others.  out[n_sides, n_kinds, 16*P] complex128, exterior
    first.  Its adjoint (density and nodes) is layer_potential_split_vjp, and qbx_apply
    with gamma is the differentiable form."""
    lib = _lib.load()
    P = int(nodes.shape[0]) if nodes.dim() == 3 else -1
    _need(nodes, "nodes", torch.float64, (P, Q, 2))
    nk = n_kinds(kind)
    _need(density, "density", torch.complex128, (nk, P * Q))
    dev = nodes.device
    out = torch.empty((n_sides(side), nk, P * Q), dtype=torch.complex128, device=dev)
    ws = _workspace(workspace_bytes(P, p, oversample, side, kind), dev, workspace)
    geo = _lib.Geometry(P, Q, nodes.data_ptr())
    rc = lib.qbx_layer_potential_split(C.byref(geo), density.data_ptr(), float(k), int(p),
                                       float(r), int(oversample), int(side), int(kind),
                                       float(gamma), out.data_ptr(), ws.data_ptr(), ws.numel(),
                                       _stream(dev))
    _lib.check(rc)
    return out


def layer_potential_split_gradient(nodes: torch.Tensor, density: torch.Tensor, k: float, p: int,
                                   r: float = 0.5, oversample: int = 4, side: int = EXTERIOR,
                                   kind: int = S, gamma: float = 6.0, want_grad: bool = True,
                                   want_dn: bool = True,
                                   workspace: Optional[torch.Tensor] = None):
    """Target derivatives with the near/far split (qbx_layer_potential_split_gradient):
    (grad, dn) as layer_potential_gradient."""
    lib = _lib.load()
    P = int(nodes.shape[0]) if nodes.dim() == 3 else -1
    _need(nodes, "nodes", torch.float64, (P, Q, 2))
    nk = n_kinds(kind)
    _need(density, "density", torch.complex128, (nk, P * Q))
    dev = nodes.device
    shape = (n_sides(side), nk, P * Q)
    grad = torch.empty(shape + (2,), dtype=torch.complex128, device=dev) if want_grad else None
    dn = torch.empty(shape, dtype=torch.complex128, device=dev) if want_dn else None
    ws = _workspace(workspace_bytes(P, p, oversample, side, kind), dev, workspace)
    geo = _lib.Geometry(P, Q, nodes.data_ptr())
    _lib.check(lib.qbx_layer_potential_split_gradient(
        C.byref(geo), density.data_ptr(), float(k), int(p), float(r), int(oversample), int(side),
        int(kind), float(gamma), grad.data_ptr() if grad is not None else None,
        dn.data_ptr() if dn is not None else None, ws.data_ptr(), ws.numel(), _stream(dev)))
    return grad, dn


def layer_potential_split_vjp(nodes: torch.Tensor, density: torch.Tensor,
                              cotangent: torch.Tensor, k: float, p: int, r: float = 0.5,
                              oversample: int = 4, side: int = EXTERIOR, kind: int = S,
                              gamma: float = 6.0, want_nodes: bool = False,
                              want_density: bool = True,
                              workspace: Optional[torch.Tensor] = None):
    """Gradients of L = Re <cotangent, layer_potential_split(...)>
    (qbx_layer_potential_split_adjoint).  Returns the density gradient [n_kinds, 16P]
    complex128, or with want_nodes the pair (density gradient or None, node gradient
    [P, 16, 2])."""
    lib = _lib.load()
    P = int(nodes.shape[0]) if nodes.dim() == 3 else -1
    _need(nodes, "nodes", torch.float64, (P, Q, 2))
    nk = n_kinds(kind)
    _need(density, "density", torch.complex128, (nk, P * Q))
    _need(cotangent, "cotangent", torch.complex128, (n_sides(side), nk, P * Q))
    dev = nodes.device
    gd = torch.empty((nk, P * Q), dtype=torch.complex128, device=dev) if (
        want_density or not want_nodes) else None
    gn = torch.empty((P, Q, 2), dtype=torch.float64, device=dev) if want_nodes else None
    ws = _workspace(workspace_bytes(P, p, oversample, side, kind), dev, workspace)
    geo = _lib.Geometry(P, Q, nodes.data_ptr())
    _lib.check(lib.qbx_layer_potential_split_adjoint(
        C.byref(geo), density.data_ptr(), float(k), int(p), float(r), int(oversample), int(side),
        int(kind), float(gamma), cotangent.data_ptr(), gd.data_ptr() if gd is not None else None,
        gn.data_ptr() if gn is not None else None, ws.data_ptr(), ws.numel(), _stream(dev)))
    return (gd, gn) if want_nodes else gd


def solve_workspace_bytes(n_panels: int, p: int, oversample: int, side: int, restart: int) -> int:
    n = _lib.load().qbx_solve_workspace_bytes(n_panels, Q, p, oversample, side, restart)
    if n == 0:
        raise ValueError("invalid solve parameters")
    return n


def _solve(fn, nodes, rhs, k, p, r, oversample, side, alpha, gamma, tol, restart, max_iter,
           workspace):
    lib = _lib.load()
    P = int(nodes.shape[0]) if nodes.dim() == 3 else -1
    _need(nodes, "nodes", torch.float64, (P, Q, 2))
    _need(rhs, "right-hand side", torch.complex128, (P * Q,))
    dev = nodes.device
    x = torch.empty(P * Q, dtype=torch.complex128, device=dev)
    ws = _workspace(solve_workspace_bytes(P, p, oversample, side, restart), dev, workspace)
    geo = _lib.Geometry(P, Q, nodes.data_ptr())
    it, res = C.c_int(), C.c_double()
    a = complex(alpha)
    _lib.check(getattr(lib, fn)(C.byref(geo), rhs.data_ptr(), float(k), int(p), float(r),
                                int(oversample), int(side), a.real, a.imag, float(gamma),
                                float(tol), int(restart), int(max_iter), x.data_ptr(),
                                C.byref(it), C.byref(res), ws.data_ptr(), ws.numel(),
                                _stream(dev)))
    return x, it.value, res.value


def solve_dirichlet(nodes: torch.Tensor, f: torch.Tensor, k: float, p: int, r: float = 0.5,
                    oversample: int = 4, side: int = EXTERIOR, alpha: complex = 1j,
                    gamma: float = 0.0, tol: float = 1e-14, restart: int = 100,
                    max_iter: int = 1000, workspace: Optional[torch.Tensor] = None):
    """Dirichlet problem by the combined-field representation u = -D sigma + alpha S sigma
    (qbx_solve_dirichlet): sigma [16P] complex128 with (-+ 1/2 + alpha S - D) sigma = f
    for the EXTERIOR or INTERIOR problem, by GMRES on the sqrt(w)-scaled system; gamma > 0
    uses the near/far split for the products.  Returns (sigma, iterations, residual)."""
    return _solve("qbx_solve_dirichlet", nodes, f, k, p, r, oversample, side, alpha, gamma, tol,
                  restart, max_iter, workspace)


def solve_dirichlet_adjoint(nodes: torch.Tensor, g: torch.Tensor, k: float, p: int,
                            r: float = 0.5, oversample: int = 4, side: int = EXTERIOR,
                            alpha: complex = 1j, gamma: float = 0.0, tol: float = 1e-14,
                            restart: int = 100, max_iter: int = 1000,
                            workspace: Optional[torch.Tensor] = None):
    """lambda = A^-H g for the operator of solve_dirichlet (qbx_solve_dirichlet_adjoint).
    Returns (lambda, iterations, residual)."""
    return _solve("qbx_solve_dirichlet_adjoint", nodes, g, k, p, r, oversample, side, alpha,
                  gamma, tol, restart, max_iter, workspace)


def solve_dirichlet_node_gradient(nodes: torch.Tensor, sigma: torch.Tensor, lam: torch.Tensor,
                                  k: float, p: int, r: float = 0.5, oversample: int = 4,
                                  side: int = EXTERIOR, alpha: complex = 1j, gamma: float = 0.0,
                                  workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """-grad_nodes Re <lam, A(nodes) sigma> with sigma held fixed
    (qbx_solve_dirichlet_node_gradient): the node part of the gradient through the
    solve, with lam from solve_dirichlet_adjoint.  Returns [P, 16, 2]."""
    lib = _lib.load()
    P = int(nodes.shape[0]) if nodes.dim() == 3 else -1
    _need(nodes, "nodes", torch.float64, (P, Q, 2))
    _need(sigma, "sigma", torch.complex128, (P * Q,))
    _need(lam, "lam", torch.complex128, (P * Q,))
    dev = nodes.device
    nbytes = lib.qbx_solve_node_gradient_workspace_bytes(P, Q, int(p), int(oversample))
    if nbytes == 0:
        raise ValueError("invalid node-gradient arguments")
    ws = _workspace(nbytes, dev, workspace)
    gn = torch.empty((P, Q, 2), dtype=torch.float64, device=dev)
    a = complex(alpha)
    geo = _lib.Geometry(P, Q, nodes.data_ptr())
    _lib.check(lib.qbx_solve_dirichlet_node_gradient(
        C.byref(geo), sigma.data_ptr(), lam.data_ptr(), float(k), int(p), float(r),
        int(oversample), int(side), a.real, a.imag, float(gamma), gn.data_ptr(), ws.data_ptr(),
        ws.numel(), _stream(dev)))
    return gn


def _require_converged(what: str, iterations: int, residual: float, tol: float) -> None:
    """Raise when a solve inside the differentiable wrapper stopped (max_iter) with a true
    relative residual above 100 tol: its value and gradients would not be those of A^-1."""
    if not residual <= 100.0 * tol:
        raise RuntimeError(f"{what}: GMRES stopped after {iterations} products at relative "
                           f"residual {residual:.3g} (tol {tol:.3g}); raise max_iter or restart")


class _DirichletSolve(torch.autograd.Function):
    """sigma = A(nodes)^-1 f with A of solve_dirichlet; backward: lambda = A^-H grad_sigma
    is the gradient for f, and -grad_nodes Re <lambda, A(nodes) sigma> (sigma held) the one
    for the nodes, from the layer potentials' node adjoint with the cotangents
    conj(alpha) lambda / 2 (S) and -lambda / 2 (D) on both sides."""

    @staticmethod
    def forward(ctx, nodes, f, k, p, r, oversample, side, alpha, gamma, tol, restart, max_iter):
        sigma, it, res = solve_dirichlet(nodes.detach(), f.detach(), k, p, r, oversample, side,
                                         alpha, gamma, tol, restart, max_iter)
        _require_converged("dirichlet_solve_apply", it, res, tol)
        ctx.save_for_backward(nodes, sigma)
        ctx.args = (k, p, r, oversample, side, alpha, gamma, tol, restart, max_iter)
        return sigma

    @staticmethod
    def backward(ctx, grad_sigma):
        nodes, sigma = ctx.saved_tensors
        k, p, r, oversample, side, alpha, gamma, tol, restart, max_iter = ctx.args
        lam, it, res = solve_dirichlet_adjoint(nodes.detach(),
                                               grad_sigma.contiguous().to(torch.complex128), k,
                                               p, r, oversample, side, alpha, gamma, tol, restart,
                                               max_iter)
        _require_converged("dirichlet_solve_apply backward", it, res, tol)
        gn = None
        if ctx.needs_input_grad[0]:
            gn = solve_dirichlet_node_gradient(nodes.detach(), sigma, lam, k, p, r, oversample,
                                               side, alpha, gamma)
        gf = lam if ctx.needs_input_grad[1] else None
        return gn, gf, None, None, None, None, None, None, None, None, None, None


def dirichlet_solve_apply(nodes: torch.Tensor, f: torch.Tensor, k: float, p: int,
                          r: float = 0.5, oversample: int = 4, side: int = EXTERIOR,
                          alpha: complex = 1j, gamma: float = 0.0, tol: float = 1e-14,
                          restart: int = 100, max_iter: int = 1000) -> torch.Tensor:
    """Differentiable solve_dirichlet: sigma with gradients for f (an adjoint solve) and
    for the nodes (the products' node adjoint, plain or split as gamma says).  Raises
    RuntimeError when either solve ends (max_iter) with a true relative residual above
    100 tol."""
    return _DirichletSolve.apply(nodes, f, float(k), int(p), float(r), int(oversample), int(side),
                                 complex(alpha), float(gamma), float(tol), int(restart),
                                 int(max_iter))


def layer_potential_gradient(nodes: torch.Tensor, density: torch.Tensor, k: float, p: int,
                             r: float = 0.5, oversample: int = 4, side: int = EXTERIOR,
                             kind: int = S, want_grad: bool = True, want_dn: bool = True,
                             workspace: Optional[torch.Tensor] = None):
    """One-sided limits of the target derivatives (qbx_layer_potential_gradient):
    (grad [n_sides, n_kinds, 16P, 2] complex128 or None, dn [n_sides, n_kinds, 16P]
    complex128 or None), dn = n . grad u (S', D'), exterior first."""
    lib = _lib.load()
    P = int(nodes.shape[0]) if nodes.dim() == 3 else -1
    _need(nodes, "nodes", torch.float64, (P, Q, 2))
    nk = n_kinds(kind)
    _need(density, "density", torch.complex128, (nk, P * Q))
    dev = nodes.device
    shape = (n_sides(side), nk, P * Q)
    grad = torch.empty(shape + (2,), dtype=torch.complex128, device=dev) if want_grad else None
    dn = torch.empty(shape, dtype=torch.complex128, device=dev) if want_dn else None
    ws = _workspace(workspace_bytes(P, p, oversample, side, kind), dev, workspace)
    geo = _lib.Geometry(P, Q, nodes.data_ptr())
    _lib.check(lib.qbx_layer_potential_gradient(
        C.byref(geo), density.data_ptr(), float(k), int(p), float(r), int(oversample), int(side),
        int(kind), grad.data_ptr() if grad is not None else None,
        dn.data_ptr() if dn is not None else None, ws.data_ptr(), ws.numel(), _stream(dev)))
    return grad, dn


def principal_value(out: torch.Tensor, density: Optional[torch.Tensor], side: int,
                    kind: int) -> torch.Tensor:
    """Principal value [n_kinds, 16P] from the one-sided limits ``out`` (Section 3.2):
    the average of both limits for side=BOTH, else the one limit with the D jump removed."""
    lib = _lib.load()
    nk = n_kinds(kind)
    T = int(out.shape[-1])
    _need(out, "out", torch.complex128, (n_sides(side), nk, T))
    if density is not None:
        _need(density, "density", torch.complex128, (nk, T))
    pv = torch.empty((nk, T), dtype=torch.complex128, device=out.device)
    _lib.check(lib.qbx_principal_value(out.data_ptr(),
                                       density.data_ptr() if density is not None else None,
                                       T // Q, int(side), int(kind), pv.data_ptr(),
                                       _stream(out.device)))
    return pv


def gradient_principal_value(nodes: torch.Tensor, density: Optional[torch.Tensor], side: int,
                             kind: int, grad: Optional[torch.Tensor] = None,
                             dn: Optional[torch.Tensor] = None):
    """On-surface target derivatives (qbx_gradient_principal_value, Section 3.2): from the
    one-sided limits of layer_potential_gradient, the principal value of grad S (and S')
    and the finite part of grad D (and D').  Returns (grad [n_kinds, T, 2],
    dn [n_kinds, T]); an output is None when its input is."""
    lib = _lib.load()
    P = int(nodes.shape[0]) if nodes.dim() == 3 else -1
    _need(nodes, "nodes", torch.float64, (P, Q, 2))
    nk, T = n_kinds(kind), P * Q
    if grad is not None:
        _need(grad, "grad", torch.complex128, (n_sides(side), nk, T, 2))
    if dn is not None:
        _need(dn, "dn", torch.complex128, (n_sides(side), nk, T))
    if density is not None:
        _need(density, "density", torch.complex128, (nk, T))
    gp = (torch.empty((nk, T, 2), dtype=torch.complex128, device=nodes.device)
          if grad is not None else None)
    dp = torch.empty((nk, T), dtype=torch.complex128, device=nodes.device) if dn is not None else None
    geo = _lib.Geometry(P, Q, nodes.data_ptr())
    ptr = lambda t: t.data_ptr() if t is not None else None
    _lib.check(lib.qbx_gradient_principal_value(C.byref(geo), ptr(density), int(side), int(kind),
                                                ptr(grad), ptr(dn), ptr(gp), ptr(dp),
                                                _stream(nodes.device)))
    return gp, dp


def check_geometry(nodes: torch.Tensor, p: int, r: float = 0.5, oversample: int = 4,
                   side: int = EXTERIOR) -> Tuple[int, float, float]:
    """Synchronous check: (status, signed area, min |x'-c|/R).  status is 0, QBX_EORIENT
    or QBX_EGRAF."""
    lib = _lib.load()
    P = int(nodes.shape[0])
    _need(nodes, "nodes", torch.float64, (P, Q, 2))
    ws = torch.empty(workspace_bytes(P, p, oversample, side, S), dtype=torch.uint8,
                     device=nodes.device)
    area, ratio = C.c_double(), C.c_double()
    geo = _lib.Geometry(P, Q, nodes.data_ptr())
    rc = lib.qbx_check_geometry(C.byref(geo), int(p), float(r), int(oversample), int(side),
                                C.byref(area), C.byref(ratio), ws.data_ptr(), ws.numel(),
                                _stream(nodes.device))
    if rc not in (_lib.QBX_OK, _lib.QBX_EORIENT, _lib.QBX_EGRAF):
        _lib.check(rc)
    return rc, area.value, ratio.value


def hankel01(z: torch.Tensor) -> Tuple[torch.Tensor, torch.Tensor]:
    """H_0^(1)(z), H_1^(1)(z) as the pair kernels compute them (test hook)."""
    lib = _lib.load()
    _need(z, "z", torch.float64, (z.numel(),))
    h0 = torch.empty(z.numel(), dtype=torch.complex128, device=z.device)
    h1 = torch.empty_like(h0)
    _lib.check(lib.qbx_debug_hankel01(z.data_ptr(), z.numel(), h0.data_ptr(), h1.data_ptr(),
                                      _stream(z.device)))
    return h0, h1


def besselj_table(x: torch.Tensor, L: int) -> torch.Tensor:
    """J_0..J_L(x) by the library's Miller recurrence (test hook): [n, L+1]."""
    lib = _lib.load()
    _need(x, "x", torch.float64, (x.numel(),))
    out = torch.empty((x.numel(), L + 1), dtype=torch.float64, device=x.device)
    _lib.check(lib.qbx_debug_besselj(x.data_ptr(), x.numel(), int(L), out.data_ptr(),
                                     _stream(x.device)))
    return out


def layer_potential_vjp(nodes: torch.Tensor, density: torch.Tensor, cotangent: torch.Tensor,
                        k: float, p: int, r: float = 0.5, oversample: int = 4,
                        side: int = EXTERIOR, kind: int = S, tape: Optional[torch.Tensor] = None,
                        want_density: bool = True, want_nodes: bool = True,
                        workspace: Optional[torch.Tensor] = None):
    """Vector-Jacobian product of layer_potential for L = Re sum conj(cotangent) * out.

    Returns (grad_density [n_kinds, 16P] complex128, grad_nodes [P, 16, 2] float64); an
    entry is None when not wanted.  ``tape``: the forward's tape (else recomputed)."""
    lib = _lib.load()
    P = int(nodes.shape[0]) if nodes.dim() == 3 else -1
    _need(nodes, "nodes", torch.float64, (P, Q, 2))
    nk = n_kinds(kind)
    _need(density, "density", torch.complex128, (nk, P * Q))
    _need(cotangent, "cotangent", torch.complex128, (n_sides(side), nk, P * Q))
    dev = nodes.device
    ws = _workspace(workspace_bytes(P, p, oversample, side, kind), dev, workspace)
    gd = torch.empty((nk, P * Q), dtype=torch.complex128, device=dev) if want_density else None
    gn = torch.empty((P, Q, 2), dtype=torch.float64, device=dev) if want_nodes else None
    tp = None
    if tape is not None:
        if tape.device != dev or tape.numel() * tape.element_size() < tape_bytes(P, p, side, kind):
            raise ValueError("tape too small or on the wrong device")
        tp = tape.data_ptr()
    geo = _lib.Geometry(P, Q, nodes.data_ptr())
    rc = lib.qbx_layer_potential_adjoint(
        C.byref(geo), density.data_ptr(), float(k), int(p), float(r), int(oversample), int(side),
        int(kind), cotangent.data_ptr(), tp, gd.data_ptr() if gd is not None else None,
        gn.data_ptr() if gn is not None else None, ws.data_ptr(), ws.numel(), _stream(dev))
    _lib.check(rc)
    return gd, gn


class _LayerPotential(torch.autograd.Function):
    """out = layer_potential(nodes, density, ...) with the library's adjoint as backward."""

    @staticmethod
    def forward(ctx, nodes, density, k, p, r, oversample, side, kind):
        # no tape: the backward runs the fused pass (each pair evaluated once for
        # both gradient sides), cheaper than a forward with tape plus a
        # source-major pass, and it keeps no per-center state between the calls
        out = layer_potential(nodes.detach(), density.detach(), k, p, r, oversample, side, kind)
        ctx.save_for_backward(nodes, density)
        ctx.tape = None
        ctx.args = (k, p, r, oversample, side, kind)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        nodes, density = ctx.saved_tensors
        k, p, r, oversample, side, kind = ctx.args
        gd, gn = layer_potential_vjp(nodes.detach(), density.detach(),
                                     grad_out.contiguous().to(torch.complex128), k, p, r,
                                     oversample, side, kind, tape=ctx.tape,
                                     want_density=ctx.needs_input_grad[1],
                                     want_nodes=ctx.needs_input_grad[0])
        return gn, gd, None, None, None, None, None, None


class _SplitLayerPotential(torch.autograd.Function):
    """out = layer_potential_split(nodes, density, ...) with its adjoint as backward
    (density and node gradients)."""

    @staticmethod
    def forward(ctx, nodes, density, k, p, r, oversample, side, kind, gamma):
        out = layer_potential_split(nodes.detach(), density.detach(), k, p, r, oversample, side,
                                    kind, gamma=gamma)
        ctx.save_for_backward(nodes, density)
        ctx.args = (k, p, r, oversample, side, kind, gamma)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        nodes, density = ctx.saved_tensors
        k, p, r, oversample, side, kind, gamma = ctx.args
        want_n, want_d = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        gd = gn = None
        if want_n or want_d:
            res = layer_potential_split_vjp(nodes.detach(), density.detach(),
                                            grad_out.contiguous().to(torch.complex128), k, p, r,
                                            oversample, side, kind, gamma=gamma,
                                            want_nodes=want_n, want_density=want_d)
            gd, gn = res if want_n else (res, None)
        return gn, gd, None, None, None, None, None, None, None


def qbx_apply(nodes: torch.Tensor, density: torch.Tensor, k: float, p: int, r: float = 0.5,
              oversample: int = 4, side: int = EXTERIOR, kind: int = S,
              gamma: Optional[float] = None) -> torch.Tensor:
    """Differentiable layer_potential (gradients for density and nodes via the HIP adjoint).
    With gamma: the near/far split (layer_potential_split) and its adjoint, also for both."""
    if gamma is not None:
        return _SplitLayerPotential.apply(nodes, density, float(k), int(p), float(r),
                                          int(oversample), int(side), int(kind), float(gamma))
    return _LayerPotential.apply(nodes, density, float(k), int(p), float(r), int(oversample),
                                 int(side), int(kind))


def explicit_workspace_bytes(n_src: int, n_ctr: int, p: int, kind: int = S) -> int:
    return int(_lib.load().qbx_explicit_workspace_bytes(int(n_src), int(n_ctr), int(p), int(kind)))


def explicit_tape_bytes(n_ctr: int, kind: int = S) -> int:
    return int(_lib.load().qbx_explicit_tape_bytes(int(n_ctr), int(kind)))


def _explicit_args(src_xy, src_nu, src_q, ctr_xy, ctr_r, ctr_dir, kind):
    n_src = int(src_xy.shape[0])
    n_ctr = int(ctr_xy.shape[0])
    _need(src_xy, "src_xy", torch.float64, (n_src, 2))
    if kind & D:
        _need(src_nu, "src_nu", torch.float64, (n_src, 2))
    _need(src_q, "src_q", torch.complex128, (n_kinds(kind), n_src))
    _need(ctr_xy, "ctr_xy", torch.float64, (n_ctr, 2))
    _need(ctr_r, "ctr_r", torch.float64, (n_ctr,))
    _need(ctr_dir, "ctr_dir", torch.complex128, (n_ctr,))
    nu = src_nu.data_ptr() if (kind & D) else None
    return n_src, n_ctr, (n_src, src_xy.data_ptr(), nu, src_q.data_ptr(), n_ctr,
                          ctr_xy.data_ptr(), ctr_r.data_ptr(), ctr_dir.data_ptr())


def apply_explicit(src_xy, src_nu, src_q, ctr_xy, ctr_r, ctr_dir, k: float, p: int,
                   kind: int = S, tape: Optional[torch.Tensor] = None,
                   workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """qbx_apply_explicit: out[n_kinds, n_ctr] complex128 for explicit sources
    (points, normals, weighted densities) and centers (point, radius, unit e^{i theta})."""
    lib = _lib.load()
    n_src, n_ctr, a = _explicit_args(src_xy, src_nu, src_q, ctr_xy, ctr_r, ctr_dir, kind)
    dev = src_xy.device
    out = torch.empty((n_kinds(kind), n_ctr), dtype=torch.complex128, device=dev)
    ws = _workspace(explicit_workspace_bytes(n_src, n_ctr, p, kind), dev, workspace)
    tp = None
    if tape is not None:
        if tape.device != dev or tape.numel() * tape.element_size() < explicit_tape_bytes(n_ctr, kind):
            raise ValueError("tape too small or on the wrong device")
        tp = tape.data_ptr()
    _lib.check(lib.qbx_apply_explicit(*a, float(k), int(p), int(kind), out.data_ptr(), tp,
                                      ws.data_ptr(), ws.numel(), _stream(dev)))
    return out


def apply_explicit_gradient(src_xy, src_nu, src_q, ctr_xy, ctr_r, ctr_dir, k: float, p: int,
                            kind: int = S, workspace: Optional[torch.Tensor] = None
                            ) -> torch.Tensor:
    """qbx_apply_explicit_gradient: the target gradient of each center's expansion,
    [n_kinds, n_ctr, 2] complex128 (d/dx, d/dy at x = c + R e^{i theta})."""
    lib = _lib.load()
    n_src, n_ctr, a = _explicit_args(src_xy, src_nu, src_q, ctr_xy, ctr_r, ctr_dir, kind)
    dev = src_xy.device
    grad = torch.empty((n_kinds(kind), n_ctr, 2), dtype=torch.complex128, device=dev)
    ws = _workspace(explicit_workspace_bytes(n_src, n_ctr, p, kind), dev, workspace)
    _lib.check(lib.qbx_apply_explicit_gradient(*a, float(k), int(p), int(kind), grad.data_ptr(),
                                               ws.data_ptr(), ws.numel(), _stream(dev)))
    return grad


def apply_explicit_vjp(src_xy, src_nu, src_q, ctr_xy, ctr_r, ctr_dir, cotangent, k: float, p: int,
                       kind: int = S, tape: Optional[torch.Tensor] = None,
                       workspace: Optional[torch.Tensor] = None) -> dict:
    """qbx_apply_explicit_adjoint: dict with q (complex [n_kinds, n_src]), src_xy, src_nu
    (D), ctr_xy, ctr_r, ctr_theta."""
    lib = _lib.load()
    n_src, n_ctr, a = _explicit_args(src_xy, src_nu, src_q, ctr_xy, ctr_r, ctr_dir, kind)
    dev = src_xy.device
    _need(cotangent, "cotangent", torch.complex128, (n_kinds(kind), n_ctr))
    g = {"q": torch.empty_like(src_q), "src_xy": torch.empty_like(src_xy),
         "ctr_xy": torch.empty_like(ctr_xy), "ctr_r": torch.empty_like(ctr_r),
         "ctr_theta": torch.empty_like(ctr_r)}
    if kind & D:
        g["src_nu"] = torch.empty_like(src_xy)
    ws = _workspace(explicit_workspace_bytes(n_src, n_ctr, p, kind), dev, workspace)
    _lib.check(lib.qbx_apply_explicit_adjoint(
        *a, float(k), int(p), int(kind), cotangent.data_ptr(),
        tape.data_ptr() if tape is not None else None, g["q"].data_ptr(), g["src_xy"].data_ptr(),
        g["src_nu"].data_ptr() if "src_nu" in g else None, g["ctr_xy"].data_ptr(),
        g["ctr_r"].data_ptr(), g["ctr_theta"].data_ptr(), ws.data_ptr(), ws.numel(),
        _stream(dev)))
    return g


def _tuning_dict(t) -> dict:
    return {f: getattr(t, f) for f, _ in _lib.Tuning._fields_}


def get_tuning() -> dict:
    """The process-wide launch tuning (qbx_get_tuning)."""
    lib = _lib.load()
    t = _lib.Tuning()
    _lib.check(lib.qbx_get_tuning(C.byref(t)))
    return _tuning_dict(t)


def set_tuning(**fields) -> dict:
    """Change fields of the launch tuning (qbx_set_tuning); returns the new tuning."""
    lib = _lib.load()
    t = _lib.Tuning()
    _lib.check(lib.qbx_get_tuning(C.byref(t)))
    for f, v in fields.items():
        if f not in dict(_lib.Tuning._fields_):
            raise KeyError(f)
        setattr(t, f, v)
    _lib.check(lib.qbx_set_tuning(C.byref(t)))
    return _tuning_dict(t)


TUNE_FORWARD, TUNE_TAPE, TUNE_ADJOINT, TUNE_FUSED, TUNE_ALL = (
    _lib.QBX_TUNE_FORWARD, _lib.QBX_TUNE_TAPE, _lib.QBX_TUNE_ADJOINT, _lib.QBX_TUNE_FUSED,
    _lib.QBX_TUNE_ALL)


def autotune(nodes: torch.Tensor, density: torch.Tensor, k: float, p: int, r: float = 0.5,
             oversample: int = 4, side: int = EXTERIOR, kind: int = S, passes: int = 2,
             fields: int = TUNE_ALL, cache_path: Optional[str] = None) -> dict:
    """Time the per-contour launch shapes of the passes in ``fields`` (TUNE_* bits)
    on this problem and install the fastest (qbx_autotune); returns the tuning.
    ``cache_path``: a text file of earlier results per device and problem; a hit is
    installed untimed, a miss is timed and written back."""
    lib = _lib.load()
    P = int(nodes.shape[0]) if nodes.dim() == 3 else -1
    _need(nodes, "nodes", torch.float64, (P, Q, 2))
    _need(density, "density", torch.complex128, (n_kinds(kind), P * Q))
    nbytes = lib.qbx_autotune_workspace_bytes(P, Q, int(p), int(oversample), int(side), int(kind))
    if nbytes == 0:
        raise ValueError("invalid autotune arguments")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=nodes.device)
    geo = _lib.Geometry(P, Q, nodes.data_ptr())
    t = _lib.Tuning()
    _lib.check(lib.qbx_autotune(C.byref(geo), density.data_ptr(), float(k), int(p), float(r),
                                int(oversample), int(side), int(kind), int(passes), int(fields),
                                cache_path.encode() if cache_path else None, C.byref(t),
                                ws.data_ptr(), ws.numel(), _stream(nodes.device)))
    return _tuning_dict(t)


class Batch:
    """Many contours packed for the batched C entry points (one persistent launch per pass).

    ``problems``: sequence of objects with attributes nodes [P,16,2] (numpy or tensor),
    density [n_kinds, 16P] complex, k, p, r, side, kind.  All share ``oversample``.
    Packing (host -> device copies, item table, workspace) happens once here."""

    def __init__(self, problems, oversample: int = 4, device="cuda"):
        lib = _lib.load()
        self.oversample = int(oversample)
        self.problems = list(problems)
        n = len(self.problems)
        self.items = (_lib.BatchItem * n)()
        node_off = dens_off = out_off = 0
        nodes, dens = [], []
        self.slices = []
        for i, pb in enumerate(self.problems):
            P = int(pb.nodes.shape[0])
            nk, ns = n_kinds(pb.kind), n_sides(pb.side)
            T = P * Q
            it = self.items[i]
            it.node_offset, it.density_offset, it.out_offset = node_off, dens_off, out_off
            it.n_panels, it.p, it.kind, it.side = P, int(pb.p), int(pb.kind), int(pb.side)
            it.k, it.r = float(pb.k), float(pb.r)
            self.slices.append(((node_off, P), (dens_off, nk, T), (out_off, ns, nk, T)))
            nodes.append(torch.as_tensor(pb.nodes, dtype=torch.float64).reshape(-1))
            dens.append(torch.as_tensor(pb.density, dtype=torch.complex128).reshape(-1))
            node_off += P
            dens_off += nk * T
            out_off += ns * nk * T
        dev = torch.device(device)
        self.nodes = torch.cat(nodes).to(dev).contiguous()
        self.density = torch.cat(dens).to(dev).contiguous()
        self.n_out = out_off
        self.device = dev
        self._lib = lib
        self.ws = torch.empty(0, dtype=torch.uint8, device=dev)
        self._ensure_workspace()
        self.tape = torch.empty(int(lib.qbx_batched_tape_bytes(self.items, n)), dtype=torch.uint8,
                                device=dev)

    def _ensure_workspace(self) -> None:
        # the workspace size depends on the launch tuning, which may change
        nb = int(self._lib.qbx_batched_workspace_bytes(self.items, len(self.problems),
                                                       self.oversample))
        if nb == 0:
            raise _lib.QBXError(_lib.QBX_EINVAL, "invalid batch")
        if self.ws.numel() < nb:
            self.ws = torch.empty(nb, dtype=torch.uint8, device=self.device)

    def autotune(self, passes: int = 2, fields: int = TUNE_ALL,
                 cache_path: Optional[str] = None) -> dict:
        """Time the batched launch shapes of the passes in ``fields`` (TUNE_* bits)
        on this batch and install the fastest (qbx_autotune_batched); returns the
        resulting tuning.  ``cache_path`` as for ``autotune``."""
        nbytes = self._lib.qbx_autotune_batched_workspace_bytes(self.items, len(self.problems),
                                                                self.oversample)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        t = _lib.Tuning()
        _lib.check(self._lib.qbx_autotune_batched(
            self.items, len(self.problems), C.c_void_p(self.nodes.data_ptr()),
            C.c_void_p(self.density.data_ptr()), self.oversample, int(passes), int(fields),
            cache_path.encode() if cache_path else None, C.byref(t),
            C.c_void_p(ws.data_ptr()), C.c_size_t(ws.numel()), C.c_void_p(_stream(self.device))))
        del ws
        self._ensure_workspace()
        return _tuning_dict(t)

    def forward(self, with_tape: bool = False) -> torch.Tensor:
        """Packed one-sided limits (concatenated per-contour out blocks)."""
        self._ensure_workspace()
        out = torch.empty(self.n_out, dtype=torch.complex128, device=self.device)
        _lib.check(self._lib.qbx_layer_potential_batched(
            self.items, len(self.problems), C.c_void_p(self.nodes.data_ptr()),
            C.c_void_p(self.density.data_ptr()), C.c_void_p(out.data_ptr()),
            C.c_void_p(self.tape.data_ptr()) if with_tape else None, self.oversample,
            C.c_void_p(self.ws.data_ptr()), C.c_size_t(self.ws.numel()),
            C.c_void_p(_stream(self.device))))
        return out

    def adjoint(self, cotangent: torch.Tensor, use_tape: bool = False):
        """(grad_density, grad_nodes) packed like density and nodes."""
        self._ensure_workspace()
        gd = torch.empty_like(self.density)
        gn = torch.empty_like(self.nodes)
        _lib.check(self._lib.qbx_layer_potential_batched_adjoint(
            self.items, len(self.problems), C.c_void_p(self.nodes.data_ptr()),
            C.c_void_p(self.density.data_ptr()), C.c_void_p(cotangent.data_ptr()),
            C.c_void_p(self.tape.data_ptr()) if use_tape else None, C.c_void_p(gd.data_ptr()),
            C.c_void_p(gn.data_ptr()), self.oversample, C.c_void_p(self.ws.data_ptr()),
            C.c_size_t(self.ws.numel()), C.c_void_p(_stream(self.device))))
        return gd, gn

    def split_out(self, out: torch.Tensor):
        res = []
        for (_, (o, ns, nk, T)) in ((s[0], s[2]) for s in self.slices):
            res.append(out[o:o + ns * nk * T].reshape(ns, nk, T))
        return res

    def split_density(self, d: torch.Tensor):
        return [d[o:o + nk * T].reshape(nk, T) for (_, (o, nk, T), _) in self.slices]

    def split_nodes(self, x: torch.Tensor):
        return [x[o * 32:(o + P) * 32].reshape(P, Q, 2) for ((o, P), _, _) in self.slices]

    def pack_out(self, per_contour):
        return torch.cat([torch.as_tensor(a, dtype=torch.complex128).reshape(-1)
                          for a in per_contour]).to(self.device).contiguous()
