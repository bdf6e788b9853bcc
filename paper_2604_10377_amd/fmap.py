"""Python binding of libfmap: the C-ABI entry points under the same names.

Each function only marshals arguments: it checks tensor placement and shape,
allocates outputs/workspaces with torch (device memory plumbing), and calls
the library on the current HIP stream of the tensors' device.  Every
arithmetic step runs in the library's HIP kernels; nothing here computes.

Layouts (row-major, contiguous, float32 unless stated):
  phi  [b, n, k]  float32 or bfloat16      mass [b, n]      feat [b, n, d] float32 or bfloat16
  A    [b, k, d]                           dF   [b, n, d]
  A [P, kx, d], B [P, ky, d], evals_x [P, kx], evals_y [P, ky], lam [P]
  C [P, ky, kx], factors [P, ky, kx(kx+1)/2], info [P, ky] int32
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib
from ._lib import FMAP_BF16, FMAP_F32, FMAP_MASK_LAPLACIAN, FMAP_MASK_RESOLVENT, FmapError  # noqa: F401


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(dev: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _need(t: torch.Tensor, name: str, dtype, shape, dev) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if t.device != dev:
        raise ValueError(f"{name} is on {t.device}, expected {dev}")
    if dtype is not None and t.dtype not in (dtype if isinstance(dtype, tuple) else (dtype,)):
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _dtype_code(t: torch.Tensor) -> int:
    return FMAP_BF16 if t.dtype == torch.bfloat16 else FMAP_F32


def _workspace(nbytes: int, dev, ws: Optional[torch.Tensor]) -> Optional[torch.Tensor]:
    if nbytes == 0:
        return ws
    if ws is None or ws.numel() * ws.element_size() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    return ws


def _wsbytes(ws: Optional[torch.Tensor]) -> int:
    return 0 if ws is None else ws.numel() * ws.element_size()


# ---------------------------------------------------------------------------- library facts

def fmap_abi_version() -> int:
    return int(_lib.lib().fmap_abi_version())


def fmap_max_k() -> int:
    return int(_lib.lib().fmap_max_k())


def fmap_status_str(status: int) -> str:
    return _lib.status_str(status)


def fmap_project_workspace_bytes(batch: int, n: int, k: int, d: int, in_dtype: int = FMAP_F32) -> int:
    return int(_lib.lib().fmap_project_workspace_bytes(batch, n, k, d, in_dtype))


def fmap_solve_workspace_bytes(pairs: int, kx: int, ky: int, d: int) -> int:
    return int(_lib.lib().fmap_solve_workspace_bytes(pairs, kx, ky, d))


def fmap_factor_floats(kx: int, ky: int) -> int:
    return int(_lib.lib().fmap_factor_floats(kx, ky))


# ---------------------------------------------------------------------------- projection

def fmap_project(phi: torch.Tensor, mass: torch.Tensor, feat: torch.Tensor, A: Optional[torch.Tensor] = None,
                 workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """A = Phi^T diag(mass) F per batch item (Eq. 1, mass-weighted pseudo-inverse)."""
    dev = phi.device
    b, n, k = phi.shape
    d = feat.shape[-1]
    _need(phi, "phi", (torch.float32, torch.bfloat16), (b, n, k), dev)
    _need(feat, "feat", phi.dtype, (b, n, d), dev)
    _need(mass, "mass", torch.float32, (b, n), dev)
    if A is None:
        A = torch.empty((b, k, d), dtype=torch.float32, device=dev)
    _need(A, "A", torch.float32, (b, k, d), dev)
    dt = _dtype_code(phi)
    workspace = _workspace(fmap_project_workspace_bytes(b, n, k, d, dt), dev, workspace)
    _lib.check("fmap_project", _lib.lib().fmap_project(_ptr(phi), _ptr(mass), _ptr(feat), dt, b, n, k, d, _ptr(A),
                                                       _ptr(workspace), _wsbytes(workspace), _stream(dev)))
    return A


def fmap_project_backward(phi: torch.Tensor, mass: torch.Tensor, dA: torch.Tensor,
                          dF: Optional[torch.Tensor] = None) -> torch.Tensor:
    """dF = diag(mass) Phi dA per batch item."""
    dev = phi.device
    b, n, k = phi.shape
    d = dA.shape[-1]
    _need(phi, "phi", (torch.float32, torch.bfloat16), (b, n, k), dev)
    _need(mass, "mass", torch.float32, (b, n), dev)
    _need(dA, "dA", torch.float32, (b, k, d), dev)
    if dF is None:
        dF = torch.empty((b, n, d), dtype=torch.float32, device=dev)
    _need(dF, "dF", torch.float32, (b, n, d), dev)
    _lib.check("fmap_project_backward",
               _lib.lib().fmap_project_backward(_ptr(phi), _ptr(mass), _dtype_code(phi), _ptr(dA), b, n, k, d,
                                                _ptr(dF), _stream(dev)))
    return dF


# ---------------------------------------------------------------------------- solve

def fmap_solve(A: torch.Tensor, B: torch.Tensor, evals_x: torch.Tensor, evals_y: torch.Tensor, lam: torch.Tensor,
               mask_kind: int = FMAP_MASK_LAPLACIAN, gamma: float = 0.5, *, refine_steps: int = 0,
               cond_fp64_threshold: float = 0.0, store_factors: bool = True, want_cond: bool = False,
               C: Optional[torch.Tensor] = None, factors: Optional[torch.Tensor] = None,
               info: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None):
    """Row-wise regularised solve (Eqs. 4-9).  Returns (C, factors or None, info, cond or None)."""
    dev = A.device
    P, kx, d = A.shape
    ky = B.shape[1]
    _need(A, "A", torch.float32, (P, kx, d), dev)
    _need(B, "B", torch.float32, (P, ky, d), dev)
    _need(evals_x, "evals_x", torch.float32, (P, kx), dev)
    _need(evals_y, "evals_y", torch.float32, (P, ky), dev)
    _need(lam, "lam", torch.float32, (P,), dev)
    if C is None:
        C = torch.empty((P, ky, kx), dtype=torch.float32, device=dev)
    if info is None:
        info = torch.empty((P, ky), dtype=torch.int32, device=dev)
    store_factors = store_factors or refine_steps > 0  # refinement reuses the float32 factors
    if store_factors and factors is None:
        factors = torch.empty((P, fmap_factor_floats(kx, ky)), dtype=torch.float32, device=dev)
    if not store_factors:
        factors = None
    cond = torch.empty((P,), dtype=torch.float32, device=dev) if want_cond else None
    workspace = _workspace(fmap_solve_workspace_bytes(P, kx, ky, d), dev, workspace)
    _lib.check("fmap_solve", _lib.lib().fmap_solve(
        _ptr(A), _ptr(B), _ptr(evals_x), _ptr(evals_y), _ptr(lam), int(mask_kind), float(gamma), P, kx, ky, d,
        int(refine_steps), float(cond_fp64_threshold), _ptr(C), _ptr(factors), _ptr(info), _ptr(cond),
        _ptr(workspace), _wsbytes(workspace), _stream(dev)))
    return C, factors, info, cond


def fmap_solve_backward(dC: torch.Tensor, A: torch.Tensor, B: torch.Tensor, C: torch.Tensor, evals_x: torch.Tensor,
                        evals_y: torch.Tensor, lam: torch.Tensor, mask_kind: int = FMAP_MASK_LAPLACIAN,
                        gamma: float = 0.5, factors: Optional[torch.Tensor] = None, *, want_dlam: bool = False,
                        dA: Optional[torch.Tensor] = None, dB: Optional[torch.Tensor] = None,
                        info: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None):
    """Reverse mode of fmap_solve.  Returns (dA, dB, dlam or None)."""
    dev = A.device
    P, kx, d = A.shape
    ky = B.shape[1]
    _need(dC, "dC", torch.float32, (P, ky, kx), dev)
    _need(C, "C", torch.float32, (P, ky, kx), dev)
    if factors is not None:
        _need(factors, "factors", torch.float32, (P, fmap_factor_floats(kx, ky)), dev)
    if dA is None:
        dA = torch.empty((P, kx, d), dtype=torch.float32, device=dev)
    if dB is None:
        dB = torch.empty((P, ky, d), dtype=torch.float32, device=dev)
    dlam = torch.empty((P,), dtype=torch.float32, device=dev) if want_dlam else None
    workspace = _workspace(fmap_solve_workspace_bytes(P, kx, ky, d), dev, workspace)
    _lib.check("fmap_solve_backward", _lib.lib().fmap_solve_backward(
        _ptr(dC), _ptr(A), _ptr(B), _ptr(C), _ptr(evals_x), _ptr(evals_y), _ptr(lam), int(mask_kind), float(gamma),
        P, kx, ky, d, _ptr(factors), _ptr(dA), _ptr(dB), _ptr(dlam), _ptr(info), _ptr(workspace),
        _wsbytes(workspace), _stream(dev)))
    return dA, dB, dlam


# ---------------------------------------------------------------------------- autograd

class FmapSolveFn(torch.autograd.Function):
    """C = solve(project(Phi_x, M_x, F_x), project(Phi_y, M_y, F_y)) with a hand-written backward.

    Inputs are stacked per shape: phi [2P, n, k], mass [2P, n], feat [2P, n, d],
    evals [2P, k] with the P source shapes first, lam [P].  Gradients flow to
    feat (and to lam when it requires grad); the spectral data are constants.
    backward reuses the forward's Cholesky factors (bwd="stored") or
    refactorises (bwd="recompute", no factor storage).
    """

    @staticmethod
    def forward(ctx, feat, phi, mass, evals, lam, mask_kind, gamma, bwd="stored"):
        P = lam.shape[0]
        AB = fmap_project(phi, mass, feat)
        A, B = AB[:P], AB[P:]
        C, factors, info, _ = fmap_solve(A, B, evals[:P].contiguous(), evals[P:].contiguous(), lam, mask_kind, gamma,
                                         store_factors=(bwd == "stored"))
        ctx.mask_kind, ctx.gamma, ctx.P = mask_kind, gamma, P
        ctx.save_for_backward(phi, mass, evals, lam, AB, C, factors if factors is not None else torch.empty(0))
        ctx.has_factors = factors is not None
        ctx.mark_non_differentiable(info)
        return C, info

    @staticmethod
    def backward(ctx, dC, _dinfo):
        phi, mass, evals, lam, AB, C, factors = ctx.saved_tensors
        P = ctx.P
        dAB = torch.empty_like(AB)
        _, _, dlam = fmap_solve_backward(dC.contiguous(), AB[:P], AB[P:], C, evals[:P].contiguous(),
                                         evals[P:].contiguous(), lam, ctx.mask_kind, ctx.gamma,
                                         factors if ctx.has_factors else None, want_dlam=ctx.needs_input_grad[4],
                                         dA=dAB[:P], dB=dAB[P:])
        dF = fmap_project_backward(phi, mass, dAB) if ctx.needs_input_grad[0] else None
        return dF, None, None, None, dlam, None, None, None


def functional_map(feat, phi, mass, evals, lam, mask_kind=FMAP_MASK_LAPLACIAN, gamma=0.5, bwd="stored"):
    """Differentiable batched functional map; returns (C [P,k,k], info [P,k])."""
    return FmapSolveFn.apply(feat, phi, mass, evals, lam, mask_kind, gamma, bwd)
