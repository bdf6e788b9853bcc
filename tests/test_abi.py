"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and host-side validation rejects bad arguments before any
launch (so these calls never reach the HIP runtime)."""
import ctypes
import os
import re

import pytest

from paper_2604_10377_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmap.h")

FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first
NULL = None


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fmap_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    return _lib.lib()


def test_every_declared_symbol_is_exported_and_bound(L):
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), f"{name} not exported by libfmap.so"
        assert name in _lib.SIGNATURES, f"{name} has no ctypes signature"
    assert set(_lib.SIGNATURES) == set(names)


def test_library_facts(L):
    assert L.fmap_abi_version() >= 1
    assert L.fmap_max_k() >= 64
    for code in range(8):
        assert len(_lib.status_str(code)) > 0
    assert _lib.status_str(99) == "unknown status"


def test_workspace_and_factor_sizes(L):
    assert L.fmap_factor_floats(50, 50) == 50 * 50 * 51 // 2
    assert L.fmap_factor_floats(3, 7) == 7 * 6
    assert L.fmap_factor_floats(0, 5) == 0
    ws = L.fmap_solve_workspace_bytes(32, 50, 50, 256)
    assert ws >= 32 * 50 * 50 * 4 * 3 and ws % 256 == 0
    assert L.fmap_solve_workspace_bytes(0, 50, 50, 256) == 0
    # split-K partials: batch x chunks x k x d floats, or 0 when one chunk suffices
    w = L.fmap_project_workspace_bytes(64, 5000, 50, 256, 0)
    assert w % (64 * 50 * 256 * 4) == 0
    assert L.fmap_project_workspace_bytes(1, 100, 8, 8, 0) == 0


def _project(L, phi=FAKE, mass=FAKE, feat=FAKE, dt=0, b=2, n=100, k=8, d=16, A=FAKE, ws=FAKE, wsb=1 << 30):
    return L.fmap_project(phi, mass, feat, dt, b, n, k, d, A, ws, wsb, None)


def test_project_validation(L):
    assert _project(L, phi=NULL) == 1
    assert _project(L, A=NULL) == 1
    assert _project(L, dt=7) == 4
    assert _project(L, k=0) == 2
    assert _project(L, n=-3) == 2
    assert _project(L, b=0) == 2
    big = dict(b=64, n=5000, k=50, d=256)
    need = L.fmap_project_workspace_bytes(64, 5000, 50, 256, 0)
    assert need > 0
    assert _project(L, ws=NULL, **big) == 5
    assert _project(L, wsb=need - 1, **big) == 5
    assert L.fmap_project_backward(FAKE, FAKE, 0, NULL, 2, 10, 4, 4, FAKE, None) == 1
    assert L.fmap_project_backward(FAKE, FAKE, 3, FAKE, 2, 10, 4, 4, FAKE, None) == 4
    assert L.fmap_project_backward(FAKE, FAKE, 0, FAKE, 2, 10, 0, 4, FAKE, None) == 2


def _solve(L, A=FAKE, B=FAKE, ex=FAKE, ey=FAKE, lam=FAKE, mask=0, gamma=0.5, P=4, kx=10, ky=10, d=16, refine=0,
           thr=0.0, C=FAKE, fac=NULL, info=FAKE, cond=NULL, ws=FAKE, wsb=1 << 30):
    return L.fmap_solve(A, B, ex, ey, lam, mask, gamma, P, kx, ky, d, refine, thr, C, fac, info, cond, ws, wsb, None)


def test_solve_validation(L):
    assert _solve(L, A=NULL) == 1
    assert _solve(L, lam=NULL) == 1
    assert _solve(L, C=NULL) == 1
    assert _solve(L, info=NULL) == 1
    assert _solve(L, kx=0) == 2
    assert _solve(L, P=0) == 2
    assert _solve(L, d=0) == 2
    assert _solve(L, mask=2) == 3
    assert _solve(L, mask=1, gamma=0.0) == 3
    assert _solve(L, mask=1, gamma=float("nan")) == 3
    assert _solve(L, refine=-1) == 3
    assert _solve(L, refine=100) == 3
    assert _solve(L, thr=float("nan")) == 3
    mk = L.fmap_max_k()
    assert _solve(L, kx=mk + 1, ky=mk + 1) == 6
    need = L.fmap_solve_workspace_bytes(4, 10, 10, 16)
    assert _solve(L, ws=NULL) == 5
    assert _solve(L, wsb=need - 1) == 5


def test_solve_backward_validation(L):
    def sb(dC=FAKE, C=FAKE, dA=FAKE, dB=FAKE, ws=FAKE, wsb=1 << 30, kx=10, mask=0, gamma=0.5):
        return L.fmap_solve_backward(dC, FAKE, FAKE, C, FAKE, FAKE, FAKE, mask, gamma, 4, kx, 10, 16, NULL, dA, dB,
                                     NULL, NULL, ws, wsb, None)
    assert sb(dC=NULL) == 1
    assert sb(C=NULL) == 1
    assert sb(dA=NULL) == 1
    assert sb(kx=0) == 2
    assert sb(mask=9) == 3
    assert sb(ws=NULL) == 5
    assert sb(wsb=16) == 5


def _pairs(n=2, k=8, **over):
    arr = (_lib.FmapPair * n)()
    for e in arr:
        for name, _ in _lib.FmapPair._fields_[:16]:
            setattr(e, name, 0x1000)
        e.A = e.B = None
        e.dC = e.dF_x = e.dF_y = None
        e.n_x, e.n_y, e.k = 100, 120, k
    for key, val in over.items():
        setattr(arr[-1], key, val)
    return arr


def _create(L, arr, npairs=None, d=16, mask=0, gamma=0.5):
    h = ctypes.c_void_p()
    n = len(arr) if npairs is None else npairs
    st = L.fmap_plan_create(ctypes.cast(arr, ctypes.c_void_p), n, d, mask, gamma, 0, None, None, ctypes.byref(h))
    assert not h.value  # nothing is created on a validation error
    return st


def test_plan_validation(L):
    h = ctypes.c_void_p()
    assert L.fmap_plan_create(NULL, 2, 16, 0, 0.5, 0, None, None, ctypes.byref(h)) == 1
    assert L.fmap_plan_create(ctypes.cast(_pairs(), ctypes.c_void_p), 2, 16, 0, 0.5, 0, None, None, NULL) == 1
    assert _create(L, _pairs(), npairs=0) == 2
    assert _create(L, _pairs(), d=0) == 2
    assert _create(L, _pairs(), mask=4) == 3
    assert _create(L, _pairs(), mask=1, gamma=-1.0) == 3
    assert _create(L, _pairs(phi_y=None)) == 1
    assert _create(L, _pairs(info=None)) == 1
    assert _create(L, _pairs(k=0)) == 2
    assert _create(L, _pairs(n_x=0)) == 2
    assert _create(L, _pairs(k=L.fmap_max_k() + 1)) == 6
    # backward slots: all pairs or none, and dF with dC
    assert _create(L, _pairs(dC=0x1000, dF_x=0x1000, dF_y=0x1000)) == 1
    arr = _pairs()
    for e in arr:
        e.dC, e.dF_x = 0x1000, 0x1000
    assert _create(L, arr) == 1
    assert L.fmap_plan_forward(NULL, None) == 1
    assert L.fmap_plan_backward(NULL, None) == 1
    assert L.fmap_plan_tuning(NULL, NULL, NULL, NULL, NULL) == 1
    assert L.fmap_plan_groups(NULL, NULL) == 1
    # several resolutions and the projector input: host validation
    kx1 = (ctypes.c_int32 * 1)(5)
    kbad = (ctypes.c_int32 * 1)(9)
    assert L.fmap_solve_resolutions_workspace_bytes(2, 8, 8, 16, 1, kx1, kx1) > 0
    assert L.fmap_solve_resolutions_workspace_bytes(2, 8, 8, 16, 1, kbad, kx1) == 0
    assert L.fmap_solve_resolutions_workspace_bytes(2, 8, 8, 16, 0, kx1, kx1) == 0
    cp = (ctypes.c_void_p * 1)(0x1000)
    res = lambda **kw: L.fmap_solve_resolutions(*[kw.get(n, v) for n, v in (
        ("A", FAKE), ("B", FAKE), ("ex", FAKE), ("ey", FAKE), ("lam", FAKE), ("mask", 0), ("gamma", 0.5), ("P", 2),
        ("kx", 8), ("ky", 8), ("d", 16), ("nres", 1), ("kxs", kx1), ("kys", kx1), ("C", cp), ("info", None),
        ("ws", FAKE), ("wsb", 1 << 30), ("st", None))])
    assert res(A=NULL) == 1
    assert res(kxs=kbad) == 2
    assert res(nres=0) == 2
    assert res(mask=3) == 3
    assert res(wsb=0) == 5
    assert L.fmap_project_pinv(NULL, FAKE, 0, 1, 10, 4, 4, FAKE, FAKE, 1 << 20, None) == 1
    assert L.fmap_project_pinv(FAKE, FAKE, 7, 1, 10, 4, 4, FAKE, FAKE, 1 << 20, None) == 4
    assert L.fmap_project_pinv(FAKE, FAKE, 0, 1, 10, 4, 4, FAKE, FAKE, 0, None) == 5
    assert L.fmap_project_pinv_backward(FAKE, 0, FAKE, 1, 10, 4, 4, FAKE, FAKE, 0, None) == 5
    assert L.fmap_project_pinv_workspace_bytes(2, 100, 8, 16, 0) >= 2 * 100 * 4
    # gradient features: host validation
    assert L.fmap_gradient_features(NULL, FAKE, FAKE, 0, 10, 8, FAKE, None) == 1
    assert L.fmap_gradient_features(FAKE, FAKE, FAKE, 2, 10, 8, FAKE, None) == 3
    assert L.fmap_gradient_features(FAKE, FAKE, FAKE, 0, 0, 8, FAKE, None) == 2
    assert L.fmap_gradient_features(FAKE, FAKE, FAKE, 1, 10, 5000, FAKE, None) == 2
    # overlap metrics: host validation
    assert L.fmap_overlap_metrics(FAKE, FAKE, NULL, 2, 10, 0.5, FAKE, FAKE, None) == 1
    assert L.fmap_overlap_metrics(NULL, FAKE, FAKE, 2, 10, 0.5, FAKE, FAKE, None) == 1
    assert L.fmap_overlap_metrics(FAKE, FAKE, FAKE, 0, 10, 0.5, FAKE, FAKE, None) == 2
    assert L.fmap_overlap_metrics(FAKE, FAKE, FAKE, 2, -1, 0.5, FAKE, FAKE, None) == 2
    assert L.fmap_overlap_metrics(FAKE, FAKE, FAKE, 2, 10, float("nan"), FAKE, FAKE, None) == 3
    assert L.fmap_plan_group(NULL, 0, NULL, NULL, NULL) == 1
    assert L.fmap_plan_destroy(NULL) == 1


def test_vectorized_validation(L):
    """General-operator solve: sizes, pointers and the workspace are checked before any launch."""
    mk = L.fmap_max_k()
    assert L.fmap_solve_vectorized_workspace_bytes(4, 8, 8, 64) > 0
    assert L.fmap_solve_vectorized_workspace_bytes(0, 8, 8, 64) == 0
    assert L.fmap_solve_vectorized_workspace_bytes(4, 0, 8, 64) == 0
    assert L.fmap_solve_vectorized_workspace_bytes(4, mk, 2, 64) == 0  # kx ky above fmap_max_k()
    assert L.fmap_solve_vectorized_workspace_bytes((1 << 20) + 1, 2, 2, 8) == 0
    # the workspace grows with the batch
    assert L.fmap_solve_vectorized_workspace_bytes(8, 8, 8, 64) > L.fmap_solve_vectorized_workspace_bytes(4, 8, 8, 64)

    def sv(A=FAKE, B=FAKE, X=FAKE, Y=FAKE, lam=FAKE, P=4, kx=8, ky=8, d=64, C=FAKE, info=FAKE, ws=FAKE,
           wsb=1 << 30):
        return L.fmap_solve_vectorized(A, B, X, Y, lam, P, kx, ky, d, C, info, ws, wsb, None)
    assert sv(A=NULL) == 1
    assert sv(X=NULL) == 1
    assert sv(Y=NULL) == 1
    assert sv(lam=NULL) == 1
    assert sv(C=NULL) == 1
    assert sv(info=NULL) == 1
    assert sv(P=0) == 2
    assert sv(kx=0) == 2
    assert sv(ky=-1) == 2
    assert sv(d=0) == 2
    assert sv(P=(1 << 20) + 1) == 2
    assert sv(kx=18, ky=18) == 6  # n = 324 above fmap_max_k()
    assert sv(kx=mk + 1, ky=1) == 6
    need = L.fmap_solve_vectorized_workspace_bytes(4, 8, 8, 64)
    assert sv(ws=NULL) == 5
    assert sv(wsb=need - 1) == 5
