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


def fmap_solve_vectorized_workspace_bytes(pairs: int, kx: int, ky: int, d: int) -> int:
    return int(_lib.lib().fmap_solve_vectorized_workspace_bytes(pairs, kx, ky, d))


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


def fmap_project_noalloc(phi: torch.Tensor, mass: torch.Tensor, feat: torch.Tensor,
                         A: torch.Tensor) -> torch.Tensor:
    """fmap_project with the library's built-in scratch array instead of a workspace (no device allocation
    by the library; A is the caller's).  Calls overlapping in time on one device must not be issued."""
    dev = phi.device
    b, n, k = phi.shape
    d = feat.shape[-1]
    _need(phi, "phi", (torch.float32, torch.bfloat16), (b, n, k), dev)
    _need(feat, "feat", phi.dtype, (b, n, d), dev)
    _need(mass, "mass", torch.float32, (b, n), dev)
    _need(A, "A", torch.float32, (b, k, d), dev)
    _lib.check("fmap_project_noalloc", _lib.lib().fmap_project_noalloc(
        _ptr(phi), _ptr(mass), _ptr(feat), _dtype_code(phi), b, n, k, d, _ptr(A), _stream(dev)))
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


# ---------------------------------------------------------------------------- projector input, resolutions

def fmap_project_pinv(pinv_t: torch.Tensor, feat: torch.Tensor, A: Optional[torch.Tensor] = None,
                      workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """A = P^T F per batch item with the projector given directly: pinv_t [b, n, k] = (Phi^+)^T."""
    dev = pinv_t.device
    b, n, k = pinv_t.shape
    d = feat.shape[-1]
    _need(pinv_t, "pinv_t", (torch.float32, torch.bfloat16), (b, n, k), dev)
    _need(feat, "feat", pinv_t.dtype, (b, n, d), dev)
    if A is None:
        A = torch.empty((b, k, d), dtype=torch.float32, device=dev)
    _need(A, "A", torch.float32, (b, k, d), dev)
    dt = _dtype_code(pinv_t)
    workspace = _workspace(int(_lib.lib().fmap_project_pinv_workspace_bytes(b, n, k, d, dt)), dev, workspace)
    _lib.check("fmap_project_pinv", _lib.lib().fmap_project_pinv(
        _ptr(pinv_t), _ptr(feat), dt, b, n, k, d, _ptr(A), _ptr(workspace), _wsbytes(workspace), _stream(dev)))
    return A


def fmap_project_pinv_backward(pinv_t: torch.Tensor, dA: torch.Tensor, dF: Optional[torch.Tensor] = None,
                               workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """dF = P dA per batch item (reverse mode of fmap_project_pinv)."""
    dev = pinv_t.device
    b, n, k = pinv_t.shape
    d = dA.shape[-1]
    _need(pinv_t, "pinv_t", (torch.float32, torch.bfloat16), (b, n, k), dev)
    _need(dA, "dA", torch.float32, (b, k, d), dev)
    if dF is None:
        dF = torch.empty((b, n, d), dtype=torch.float32, device=dev)
    _need(dF, "dF", torch.float32, (b, n, d), dev)
    workspace = _workspace(b * n * 4, dev, workspace)
    _lib.check("fmap_project_pinv_backward", _lib.lib().fmap_project_pinv_backward(
        _ptr(pinv_t), _dtype_code(pinv_t), _ptr(dA), b, n, k, d, _ptr(dF), _ptr(workspace), _wsbytes(workspace),
        _stream(dev)))
    return dF


def fmap_solve_resolutions(A: torch.Tensor, B: torch.Tensor, evals_x: torch.Tensor, evals_y: torch.Tensor,
                           lam: torch.Tensor, mask_kind: int, gamma: float, resolutions, *,
                           workspace: Optional[torch.Tensor] = None):
    """Maps at several resolutions [(kx', ky'), ...] from one projection; returns [(C_r, info_r), ...]."""
    dev = A.device
    P, kx, d = A.shape
    ky = B.shape[1]
    _need(A, "A", torch.float32, (P, kx, d), dev)
    _need(B, "B", torch.float32, (P, ky, d), dev)
    _need(evals_x, "evals_x", torch.float32, (P, kx), dev)
    _need(evals_y, "evals_y", torch.float32, (P, ky), dev)
    _need(lam, "lam", torch.float32, (P,), dev)
    nres = len(resolutions)
    kxs = (ctypes.c_int32 * nres)(*[int(r[0]) for r in resolutions])
    kys = (ctypes.c_int32 * nres)(*[int(r[1]) for r in resolutions])
    Cs = [torch.empty((P, int(r[1]), int(r[0])), dtype=torch.float32, device=dev) for r in resolutions]
    infos = [torch.empty((P, int(r[1])), dtype=torch.int32, device=dev) for r in resolutions]
    cptr = (ctypes.c_void_p * nres)(*[c.data_ptr() for c in Cs])
    iptr = (ctypes.c_void_p * nres)(*[x.data_ptr() for x in infos])
    nbytes = int(_lib.lib().fmap_solve_resolutions_workspace_bytes(P, kx, ky, d, nres, kxs, kys))
    workspace = _workspace(nbytes, dev, workspace)
    _lib.check("fmap_solve_resolutions", _lib.lib().fmap_solve_resolutions(
        _ptr(A), _ptr(B), _ptr(evals_x), _ptr(evals_y), _ptr(lam), int(mask_kind), float(gamma), P, kx, ky, d, nres,
        kxs, kys, cptr, iptr, _ptr(workspace), _wsbytes(workspace), _stream(dev)))
    return list(zip(Cs, infos))


def fmap_solve_vectorized(A: torch.Tensor, B: torch.Tensor, op_x: torch.Tensor, op_y: torch.Tensor,
                          lam: torch.Tensor, *, workspace: Optional[torch.Tensor] = None):
    """Vectorized solve with general commutativity operators (op_x [P, kx, kx], op_y [P, ky, ky]):
    C = argmin ||C A - B||^2 + lam ||C op_x - op_y C||^2 per pair, kx * ky <= fmap_max_k().  Returns
    (C [P, ky, kx], info [P])."""
    dev = A.device
    P, kx, d = A.shape
    ky = B.shape[1]
    _need(A, "A", torch.float32, (P, kx, d), dev)
    _need(B, "B", torch.float32, (P, ky, d), dev)
    _need(op_x, "op_x", torch.float32, (P, kx, kx), dev)
    _need(op_y, "op_y", torch.float32, (P, ky, ky), dev)
    _need(lam, "lam", torch.float32, (P,), dev)
    C = torch.empty((P, ky, kx), dtype=torch.float32, device=dev)
    info = torch.empty((P,), dtype=torch.int32, device=dev)
    nbytes = fmap_solve_vectorized_workspace_bytes(P, kx, ky, d)
    workspace = _workspace(nbytes, dev, workspace)
    _lib.check("fmap_solve_vectorized", _lib.lib().fmap_solve_vectorized(
        _ptr(A), _ptr(B), _ptr(op_x), _ptr(op_y), _ptr(lam), P, kx, ky, d, _ptr(C), _ptr(info), _ptr(workspace),
        _wsbytes(workspace), _stream(dev)))
    return C, info


# ---------------------------------------------------------------------------- gradient features

def fmap_gradient_features(z: torch.Tensor, A_re: torch.Tensor, A_im: torch.Tensor, variant: str = "A",
                           g: Optional[torch.Tensor] = None) -> torch.Tensor:
    """DiffusionNet spatial-gradient features (Sec. 3.2): z [V, D, 2] float32 (x, y of each channel's tangent
    vector), A_re, A_im [D, D]; variant "A" (complex product) or "B"; returns g [V, D]."""
    dev = z.device
    V, D, _ = z.shape
    _need(z, "z", torch.float32, (V, D, 2), dev)
    _need(A_re, "A_re", torch.float32, (D, D), dev)
    _need(A_im, "A_im", torch.float32, (D, D), dev)
    if variant not in ("A", "B"):
        raise ValueError("variant must be 'A' or 'B'")
    if g is None:
        g = torch.empty((V, D), dtype=torch.float32, device=dev)
    _need(g, "g", torch.float32, (V, D), dev)
    _lib.check("fmap_gradient_features", _lib.lib().fmap_gradient_features(
        _ptr(z), _ptr(A_re), _ptr(A_im), 0 if variant == "A" else 1, V, D, _ptr(g), _stream(dev)))
    return g


# ---------------------------------------------------------------------------- overlap metrics

OVERLAP_METRICS = ("accuracy", "precision", "recall", "specificity", "iou", "f1", "balanced_accuracy")


def fmap_overlap_metrics(scores: torch.Tensor, truth: torch.Tensor, offsets: torch.Tensor, threshold: float = 0.5,
                         counts: Optional[torch.Tensor] = None, metrics: Optional[torch.Tensor] = None):
    """Per-shape confusion counts [S, 4] int64 (TP, FP, FN, TN) and metrics [S, 7] float32 (OVERLAP_METRICS
    order) of a thresholded score against the ground-truth overlap (Sec. 3.3).  scores [total] float32,
    truth [total] uint8, offsets [S + 1] int64 on the same device."""
    dev = offsets.device
    S = offsets.shape[0] - 1
    total = scores.shape[0]
    _need(scores, "scores", torch.float32, (total,), dev)
    _need(truth, "truth", torch.uint8, (total,), dev)
    _need(offsets, "offsets", torch.int64, (S + 1,), dev)
    if counts is None:
        counts = torch.empty((S, 4), dtype=torch.int64, device=dev)
    if metrics is None:
        metrics = torch.empty((S, 7), dtype=torch.float32, device=dev)
    _need(counts, "counts", torch.int64, (S, 4), dev)
    _need(metrics, "metrics", torch.float32, (S, 7), dev)
    _lib.check("fmap_overlap_metrics", _lib.lib().fmap_overlap_metrics(
        _ptr(scores), _ptr(truth), _ptr(offsets), S, total, float(threshold), _ptr(counts), _ptr(metrics),
        _stream(dev)))
    return counts, metrics


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


# ---------------------------------------------------------------------------- uneven batches

class FmapPlan:
    """Captured forward (and backward) pass over shape pairs of different n and k.

    `pairs` is a sequence of dicts with device tensors phi_x [n_x, k], phi_y [n_y, k],
    mass_x [n_x], mass_y [n_y], feat_x [n_x, d], feat_y [n_y, d], evals_x [k],
    evals_y [k] and lam [1] (all float32, one device).  The plan owns the outputs
    C[i] [k, k] and info[i] [k] (and, with backward=True, the upstream gradient
    slots dC[i] [k, k] and the results dF_x[i], dF_y[i]).  The input tensors are
    captured by address: update them in place between replays, never rebind.
    """

    def __init__(self, pairs, mask_kind: int = FMAP_MASK_LAPLACIAN, gamma: float = 0.5, *, backward: bool = True,
                 recompute: bool = False, tune_cache: Optional[str] = None, want_AB: bool = False):
        if len(pairs) == 0:
            raise ValueError("a plan needs at least one pair")
        dev = pairs[0]["phi_x"].device
        d = pairs[0]["feat_x"].shape[1]
        self.device, self.d = dev, d
        self.inputs = [dict(p) for p in pairs]
        self.C, self.info, self.A, self.B, self.dC, self.dF_x, self.dF_y = [], [], [], [], [], [], []
        arr = (_lib.FmapPair * len(pairs))()
        for i, p in enumerate(self.inputs):
            nx, k = p["phi_x"].shape
            ny = p["phi_y"].shape[0]
            _need(p["phi_x"], "phi_x", torch.float32, (nx, k), dev)
            _need(p["phi_y"], "phi_y", torch.float32, (ny, k), dev)
            _need(p["mass_x"], "mass_x", torch.float32, (nx,), dev)
            _need(p["mass_y"], "mass_y", torch.float32, (ny,), dev)
            _need(p["feat_x"], "feat_x", torch.float32, (nx, d), dev)
            _need(p["feat_y"], "feat_y", torch.float32, (ny, d), dev)
            _need(p["evals_x"], "evals_x", torch.float32, (k,), dev)
            _need(p["evals_y"], "evals_y", torch.float32, (k,), dev)
            _need(p["lam"], "lam", torch.float32, (1,), dev)
            self.C.append(torch.empty((k, k), dtype=torch.float32, device=dev))
            self.info.append(torch.empty((k,), dtype=torch.int32, device=dev))
            self.A.append(torch.empty((k, d), dtype=torch.float32, device=dev) if want_AB else None)
            self.B.append(torch.empty((k, d), dtype=torch.float32, device=dev) if want_AB else None)
            self.dC.append(torch.zeros((k, k), dtype=torch.float32, device=dev) if backward else None)
            self.dF_x.append(torch.empty((nx, d), dtype=torch.float32, device=dev) if backward else None)
            self.dF_y.append(torch.empty((ny, d), dtype=torch.float32, device=dev) if backward else None)
            e = arr[i]
            for name in ("phi_x", "phi_y", "mass_x", "mass_y", "feat_x", "feat_y", "evals_x", "evals_y"):
                setattr(e, name, p[name].data_ptr())
            e.lambda_ = p["lam"].data_ptr()
            e.C, e.info = self.C[i].data_ptr(), self.info[i].data_ptr()
            e.A = self.A[i].data_ptr() if want_AB else None
            e.B = self.B[i].data_ptr() if want_AB else None
            if backward:
                e.dC, e.dF_x, e.dF_y = self.dC[i].data_ptr(), self.dF_x[i].data_ptr(), self.dF_y[i].data_ptr()
            e.n_x, e.n_y, e.k = nx, ny, k
        handle = ctypes.c_void_p()
        cache = None if tune_cache is None else str(tune_cache).encode()
        _lib.check("fmap_plan_create", _lib.lib().fmap_plan_create(
            ctypes.cast(arr, ctypes.c_void_p), len(pairs), d, int(mask_kind), float(gamma), int(bool(recompute)),
            cache, _stream(dev), ctypes.byref(handle)))
        self._h = handle

    def forward(self):
        """Replays the captured forward on the current stream; returns the list of C."""
        _lib.check("fmap_plan_forward", _lib.lib().fmap_plan_forward(self._h, _stream(self.device)))
        return self.C

    def backward(self):
        """Replays the captured backward (reads dC[i], writes dF_x[i], dF_y[i])."""
        _lib.check("fmap_plan_backward", _lib.lib().fmap_plan_backward(self._h, _stream(self.device)))
        return self.dF_x, self.dF_y

    def tuning(self) -> dict:
        v = [ctypes.c_int32() for _ in range(4)]
        _lib.check("fmap_plan_tuning", _lib.lib().fmap_plan_tuning(self._h, *[ctypes.byref(x) for x in v]))
        return dict(chunk=v[0].value, grid=v[1].value, systems_per_wg=v[2].value, from_cache=bool(v[3].value))

    def groups(self) -> list:
        """Per k group (increasing k): dict(k, pairs, systems_per_wg) as tuned for this plan."""
        n = ctypes.c_int32()
        _lib.check("fmap_plan_groups", _lib.lib().fmap_plan_groups(self._h, ctypes.byref(n)))
        out = []
        for g in range(n.value):
            v = [ctypes.c_int32() for _ in range(3)]
            _lib.check("fmap_plan_group", _lib.lib().fmap_plan_group(self._h, g, *[ctypes.byref(x) for x in v]))
            out.append(dict(k=v[0].value, pairs=v[1].value, systems_per_wg=v[2].value))
        return out

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check("fmap_plan_destroy", _lib.lib().fmap_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
