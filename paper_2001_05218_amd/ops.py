"""Torch-facing wrappers of the C ABI (include/wilson.h).

Tensors are passed as device pointers and the current HIP stream; every
step of the computation runs in the library's kernels. Shapes:
  U    complex128 (4, Lt, Lz, Ly, Lx, 3, 3)
  psi  complex128 (Lt, Lz, Ly, Lx, 4, 3)   (complex64 allowed for solver I/O)
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import WD_C64, WD_C128, WD_F64, WD_RHS_NORMAL, WD_RHS_SOURCE, WD_TWO_ROW_LINKS, PREC_NAMES


def _spinor_prec(prec: str) -> int:
    """Spinor storage of a precision name (the two-row flag concerns links only)."""
    return PREC_NAMES[prec] & ~WD_TWO_ROW_LINKS


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def dims_of_spinor(psi: torch.Tensor):
    if psi.dim() < 6 or tuple(psi.shape[-2:]) != (4, 3):
        raise ValueError(f"spinor shape {tuple(psi.shape)} is not (..., Lt, Lz, Ly, Lx, 4, 3)")
    lt, lz, ly, lx = psi.shape[-6:-2]
    return (int(lx), int(ly), int(lz), int(lt))


def _need(t: torch.Tensor, name: str, dtypes, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU device (got {t.device})")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def gauge_shape(dims):
    lx, ly, lz, lt = dims
    return (4, lt, lz, ly, lx, 3, 3)


def spinor_shape(dims):
    lx, ly, lz, lt = dims
    return (lt, lz, ly, lx, 4, 3)


def wilson_apply(U: torch.Tensor, psi: torch.Tensor, mass: float, dagger: bool = False,
                 out: torch.Tensor | None = None) -> torch.Tensor:
    """D psi (or D^+ psi) on canonical complex128 fields."""
    dims = dims_of_spinor(psi)
    _need(psi, "psi", (torch.complex128,), spinor_shape(dims))
    _need(U, "U", (torch.complex128,), gauge_shape(dims))
    if out is None:
        out = torch.empty_like(psi)
    _need(out, "out", (torch.complex128,), psi.shape)
    lib = _lib.load()
    fn = lib.wilson_apply_dagger if dagger else lib.wilson_apply
    rc = fn(ctypes.byref(_lib.lattice(dims)), float(mass), U.data_ptr(), psi.data_ptr(), out.data_ptr(),
            _stream(psi.device))
    _lib.check(rc, fn.__name__)
    return out


def wilson_force(a: torch.Tensor, b: torch.Tensor, coeff: float = 1.0, out: torch.Tensor | None = None,
                 accumulate: bool = False) -> torch.Tensor:
    """coeff * G(a, b) (gauge-shaped complex128), optionally added into out."""
    dims = dims_of_spinor(a)
    _need(a, "a", (torch.complex128,), spinor_shape(dims))
    _need(b, "b", (torch.complex128,), spinor_shape(dims))
    if out is None:
        if accumulate:
            raise ValueError("accumulate needs out")
        out = torch.empty(gauge_shape(dims), dtype=torch.complex128, device=a.device)
    _need(out, "out", (torch.complex128,), gauge_shape(dims))
    lib = _lib.load()
    rc = lib.wilson_force(ctypes.byref(_lib.lattice(dims)), a.data_ptr(), b.data_ptr(), float(coeff),
                          1 if accumulate else 0, out.data_ptr(), _stream(a.device))
    _lib.check(rc, "wilson_force")
    return out


def make_params(tol=1e-10, max_iter=10000, inner="f64", reliable_interval=50, rhs="source", io_dtype=WD_C128,
                zero_guess=True, history_len=0, profile=False, scheme="reliable", inner_tol=0.0, ring_len=0,
                schedule="auto"):
    p = _lib.WdCgParams()
    p.tol = float(tol)
    p.max_iter = int(max_iter)
    p.inner_prec = PREC_NAMES[inner] if isinstance(inner, str) else int(inner)
    p.reliable_interval = int(reliable_interval)
    p.rhs_mode = {"source": WD_RHS_SOURCE, "normal": WD_RHS_NORMAL}[rhs] if isinstance(rhs, str) else int(rhs)
    p.io_dtype = int(io_dtype)
    p.zero_guess = 1 if zero_guess else 0
    hist = None
    if history_len > 0:
        hist = (ctypes.c_double * int(history_len))()
        p.history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
    p.history_len = int(history_len)
    p.profile = 1 if profile else 0
    p.scheme = {"reliable": 0, "refinement": 1}[scheme] if isinstance(scheme, str) else int(scheme)
    p.inner_tol = float(inner_tol)
    p.ring_len = int(ring_len)
    p.batch_schedule = ({"auto": _lib.WD_BATCH_AUTO, "persistent": _lib.WD_BATCH_PERSISTENT,
                         "lockstep": _lib.WD_BATCH_LOCKSTEP}[schedule] if isinstance(schedule, str) else int(schedule))
    return p, hist


def workspace_bytes(dims, params, nrhs=1) -> int:
    lib = _lib.load()
    n = lib.wd_workspace_bytes(ctypes.byref(_lib.lattice(dims)), ctypes.byref(params), int(nrhs))
    if n == 0:
        raise _lib.WilsonError(_lib.WD_ERR_INVALID, "wd_workspace_bytes", _lib.last_error())
    return int(n)


def cg_solve(U: torch.Tensor, b: torch.Tensor, mass: float, tol: float = 1e-10, max_iter: int = 10000,
             inner: str = "f64", reliable_interval: int = 50, rhs: str = "source", x0: torch.Tensor | None = None,
             history: int = 0, workspace: torch.Tensor | None = None, raise_on_nonconvergence: bool = True,
             profile: bool = False, scheme: str = "reliable", inner_tol: float = 0.0, ring_len: int = 0):
    """Solve D^+ D x = D^+ b (rhs="source") or D^+ D x = b (rhs="normal").

    Returns (x, info); info holds the wd_cg_result fields (and "history" if
    asked). complex64 b gives complex64 x (inner arithmetic unchanged).
    profile=True fills info["kernel_seconds"] with the inner loop's average
    kernel times. scheme="refinement" selects iterative refinement (defect
    correction) instead of reliable updates for a mixed solve. ring_len sets
    how many search directions a mixed solve keeps before folding them into x
    (0: the library default)."""
    dims = dims_of_spinor(b)
    _need(b, "b", (torch.complex128, torch.complex64), spinor_shape(dims))
    _need(U, "U", (torch.complex128,), gauge_shape(dims))
    io = WD_C64 if b.dtype == torch.complex64 else WD_C128
    params, hist = make_params(tol, max_iter, inner, reliable_interval, rhs, io, x0 is None, history, profile,
                               scheme, inner_tol, ring_len)
    if x0 is None:
        x = torch.empty_like(b)
    else:
        _need(x0, "x0", (b.dtype,), b.shape)
        x = x0.clone()
    need = workspace_bytes(dims, params, 1)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=b.device)
    res = _lib.WdCgResult()
    lib = _lib.load()
    rc = lib.cg_solve(ctypes.byref(_lib.lattice(dims)), float(mass), U.data_ptr(), b.data_ptr(), x.data_ptr(),
                      ctypes.byref(params), ctypes.byref(res), workspace.data_ptr(), workspace.numel(),
                      _stream(b.device))
    ok = (_lib.WD_OK,) if raise_on_nonconvergence else (_lib.WD_OK, _lib.WD_NOT_CONVERGED)
    _lib.check(rc, "cg_solve", ok)
    info = res.as_dict()
    if hist is not None:
        info["history"] = list(hist)[: min(history, res.iterations)]
    return x, info


def cg_solve_batched(U: torch.Tensor, B: torch.Tensor, mass: float, tol: float = 1e-10, max_iter: int = 10000,
                     reliable_interval: int = 50, rhs: str = "source", X0: torch.Tensor | None = None,
                     workspace: torch.Tensor | None = None, raise_on_nonconvergence: bool = True,
                     inner: str = "f32", schedule: str = "auto"):
    """Solve nrhs systems sharing U. B: (nrhs, Lt, Lz, Ly, Lx, 4, 3).
    inner: storage of the inner vectors ("f32", "bf16", "f16" or "i8"; FP32 arithmetic).
    schedule: "persistent" (one cooperative launch for the whole solve), "lockstep" (each CG
    step one launch over all systems; "bf16", "f16" or "i8" storage, extents multiples of 4)
    or "auto" (lockstep where it applies)."""
    dims = dims_of_spinor(B)
    if B.dim() != 7:
        raise ValueError("B must be (nrhs, Lt, Lz, Ly, Lx, 4, 3)")
    nrhs = int(B.shape[0])
    _need(B, "B", (torch.complex128, torch.complex64))
    _need(U, "U", (torch.complex128,), gauge_shape(dims))
    io = WD_C64 if B.dtype == torch.complex64 else WD_C128
    params, _ = make_params(tol, max_iter, inner, reliable_interval, rhs, io, X0 is None, 0, schedule=schedule)
    X = torch.empty_like(B) if X0 is None else X0.clone()
    need = workspace_bytes(dims, params, nrhs)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=B.device)
    res = (_lib.WdCgResult * nrhs)()
    lib = _lib.load()
    rc = lib.cg_solve_batched(ctypes.byref(_lib.lattice(dims)), float(mass), U.data_ptr(), nrhs, B.data_ptr(),
                              X.data_ptr(), ctypes.byref(params), res, workspace.data_ptr(), workspace.numel(),
                              _stream(B.device))
    ok = (_lib.WD_OK,) if raise_on_nonconvergence else (_lib.WD_OK, _lib.WD_NOT_CONVERGED)
    _lib.check(rc, "cg_solve_batched", ok)
    return X, [r.as_dict() for r in res]


# ---- the gauge-covariant Laplacian (colour vectors) ------------------------

def colour_shape(dims):
    lx, ly, lz, lt = dims
    return (lt, lz, ly, lx, 3)


def dims_of_colour(v: torch.Tensor):
    if v.dim() != 5 or v.shape[-1] != 3:
        raise ValueError(f"colour-field shape {tuple(v.shape)} is not (Lt, Lz, Ly, Lx, 3)")
    lt, lz, ly, lx = v.shape[:4]
    return (int(lx), int(ly), int(lz), int(lt))


def laplace_apply(U: torch.Tensor, psi: torch.Tensor, m2: float, out: torch.Tensor | None = None) -> torch.Tensor:
    """L psi on canonical complex128 colour fields (Lt, Lz, Ly, Lx, 3)."""
    dims = dims_of_colour(psi)
    _need(psi, "psi", (torch.complex128,), colour_shape(dims))
    _need(U, "U", (torch.complex128,), gauge_shape(dims))
    if out is None:
        out = torch.empty_like(psi)
    _need(out, "out", (torch.complex128,), psi.shape)
    lib = _lib.load()
    rc = lib.laplace_apply(ctypes.byref(_lib.lattice(dims)), float(m2), U.data_ptr(), psi.data_ptr(),
                           out.data_ptr(), _stream(psi.device))
    _lib.check(rc, "laplace_apply")
    return out


def laplace_workspace_bytes(dims, params) -> int:
    lib = _lib.load()
    n = lib.laplace_workspace_bytes(ctypes.byref(_lib.lattice(dims)), ctypes.byref(params))
    if n == 0:
        raise _lib.WilsonError(_lib.WD_ERR_INVALID, "laplace_workspace_bytes", _lib.last_error())
    return int(n)


def laplace_cg_solve(U: torch.Tensor, b: torch.Tensor, m2: float, tol: float = 1e-10, max_iter: int = 10000,
                     x0: torch.Tensor | None = None, history: int = 0, workspace: torch.Tensor | None = None,
                     raise_on_nonconvergence: bool = True, profile: bool = False):
    """Solve L x = b (FP64 CG). b: complex128 or complex64 (Lt, Lz, Ly, Lx, 3).
    Returns (x, info) like cg_solve."""
    dims = dims_of_colour(b)
    _need(b, "b", (torch.complex128, torch.complex64), colour_shape(dims))
    _need(U, "U", (torch.complex128,), gauge_shape(dims))
    io = WD_C64 if b.dtype == torch.complex64 else WD_C128
    params, hist = make_params(tol, max_iter, "f64", 50, "source", io, x0 is None, history, profile)
    if x0 is None:
        x = torch.empty_like(b)
    else:
        _need(x0, "x0", (b.dtype,), b.shape)
        x = x0.clone()
    need = laplace_workspace_bytes(dims, params)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=b.device)
    res = _lib.WdCgResult()
    lib = _lib.load()
    rc = lib.laplace_cg_solve(ctypes.byref(_lib.lattice(dims)), float(m2), U.data_ptr(), b.data_ptr(),
                              x.data_ptr(), ctypes.byref(params), ctypes.byref(res), workspace.data_ptr(),
                              workspace.numel(), _stream(b.device))
    ok = (_lib.WD_OK,) if raise_on_nonconvergence else (_lib.WD_OK, _lib.WD_NOT_CONVERGED)
    _lib.check(rc, "laplace_cg_solve", ok)
    info = res.as_dict()
    if hist is not None:
        info["history"] = list(hist)[: min(history, res.iterations)]
    return x, info


# ---- packed fields -------------------------------------------------------

def _gauge_dims(U):
    if U.dim() != 7 or U.shape[0] != 4 or tuple(U.shape[-2:]) != (3, 3):
        raise ValueError(f"gauge shape {tuple(U.shape)} is not (4, Lt, Lz, Ly, Lx, 3, 3)")
    lt, lz, ly, lx = U.shape[1:5]
    return (int(lx), int(ly), int(lz), int(lt))


def pack_gauge(U: torch.Tensor, prec: str = "f64") -> torch.Tensor:
    """Packed (site-blocked) copy of U in precision prec, as a uint8 device tensor."""
    dims = _gauge_dims(U)
    _need(U, "U", (torch.complex128,))
    lib = _lib.load()
    lat = _lib.lattice(dims)
    p = PREC_NAMES[prec]
    n = int(lib.wd_gauge_bytes(ctypes.byref(lat), p))
    if n == 0:
        raise _lib.WilsonError(_lib.WD_ERR_INVALID, "wd_gauge_bytes", _lib.last_error())
    out = torch.empty(n, dtype=torch.uint8, device=U.device)
    _lib.check(lib.wd_pack_gauge(ctypes.byref(lat), U.data_ptr(), p, out.data_ptr(), _stream(U.device)),
               "wd_pack_gauge")
    return out


def pack_spinor(psi: torch.Tensor, prec: str = "f64") -> torch.Tensor:
    dims = dims_of_spinor(psi)
    _need(psi, "psi", (torch.complex128, torch.complex64), spinor_shape(dims))
    lib = _lib.load()
    lat = _lib.lattice(dims)
    p = _spinor_prec(prec)
    out = torch.empty(int(lib.wd_spinor_bytes(ctypes.byref(lat), p)), dtype=torch.uint8, device=psi.device)
    io = WD_C64 if psi.dtype == torch.complex64 else WD_C128
    _lib.check(lib.wd_pack_spinor(ctypes.byref(lat), psi.data_ptr(), io, p, out.data_ptr(), _stream(psi.device)),
               "wd_pack_spinor")
    return out


def unpack_spinor(packed: torch.Tensor, dims, prec: str = "f64", dtype=torch.complex128) -> torch.Tensor:
    lib = _lib.load()
    lat = _lib.lattice(dims)
    p = _spinor_prec(prec)
    out = torch.empty(spinor_shape(dims), dtype=dtype, device=packed.device)
    io = WD_C64 if dtype == torch.complex64 else WD_C128
    _lib.check(lib.wd_unpack_spinor(ctypes.byref(lat), packed.data_ptr(), p, out.data_ptr(), io,
                                    _stream(packed.device)), "wd_unpack_spinor")
    return out


def empty_packed_spinor(dims, prec: str, device) -> torch.Tensor:
    lib = _lib.load()
    n = int(lib.wd_spinor_bytes(ctypes.byref(_lib.lattice(dims)), _spinor_prec(prec)))
    return torch.empty(n, dtype=torch.uint8, device=device)


def wilson_apply_packed(U_packed: torch.Tensor, in_packed: torch.Tensor, out_packed: torch.Tensor, dims, mass: float,
                        prec: str = "f64", dagger: bool = False, stream=None) -> None:
    lib = _lib.load()
    s = ctypes.c_void_p(stream) if stream is not None else _stream(in_packed.device)
    rc = lib.wilson_apply_packed(ctypes.byref(_lib.lattice(dims)), float(mass), PREC_NAMES[prec],
                                 U_packed.data_ptr(), in_packed.data_ptr(), out_packed.data_ptr(),
                                 1 if dagger else 0, s)
    _lib.check(rc, "wilson_apply_packed")


# ---- out-of-core solve: host-resident fields streamed through the GPU in t-slabs

def _need_pinned(t: torch.Tensor, name: str, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if t.device.type != "cpu" or not t.is_pinned():
        raise ValueError(f"{name} must be a pinned host tensor (torch.empty(..., pin_memory=True) or .pin_memory())")
    if t.dtype != torch.complex128:
        raise TypeError(f"{name} has dtype {t.dtype}, expected torch.complex128")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def ooc_workspace_bytes(dims, slab_planes: int, history_len: int = 0):
    """(device bytes, pinned host bytes) of an out-of-core solve whose slabs hold
    `slab_planes` time planes."""
    lib = _lib.load()
    dev = ctypes.c_size_t(0)
    host = ctypes.c_size_t(0)
    rc = lib.wd_ooc_workspace_bytes(ctypes.byref(_lib.lattice(dims)), int(slab_planes), int(history_len),
                                    ctypes.byref(dev), ctypes.byref(host))
    _lib.check(rc, "wd_ooc_workspace_bytes")
    return int(dev.value), int(host.value)


def cg_solve_ooc(U: torch.Tensor, b: torch.Tensor, mass: float, tol: float = 1e-10, max_iter: int = 10000,
                 rhs: str = "source", x0: torch.Tensor | None = None, history: int = 0,
                 device_bytes: int | None = None, device_workspace: torch.Tensor | None = None,
                 host_workspace: torch.Tensor | None = None, device=None, raise_on_nonconvergence: bool = True):
    """FP64 CG on D^+D x = D^+b (or b) with U, b and x in pinned HOST memory, streamed
    through the GPU in t-slabs. The device holds at most `device_bytes` (or the
    given device_workspace); the CG vectors live in a pinned host workspace.
    Returns (x, info) with x a pinned host tensor."""
    dims = dims_of_spinor(b)
    _need_pinned(b, "b", spinor_shape(dims))
    _need_pinned(U, "U", gauge_shape(dims))
    dev = torch.device(device if device is not None else "cuda")
    params, hist = make_params(tol, max_iter, "f64", 50, rhs, WD_C128, x0 is None, history)
    if x0 is None:
        x = torch.empty(b.shape, dtype=torch.complex128, pin_memory=True)
    else:
        _need_pinned(x0, "x0", b.shape)
        x = torch.empty(b.shape, dtype=torch.complex128, pin_memory=True)
        x.copy_(x0)
    _, host_need = ooc_workspace_bytes(dims, 1, history)
    if host_workspace is None or host_workspace.numel() < host_need:
        host_workspace = torch.empty(host_need, dtype=torch.uint8, pin_memory=True)
    if device_workspace is None:
        if device_bytes is None:
            raise ValueError("give device_bytes (the device memory budget) or a device_workspace")
        device_workspace = torch.empty(int(device_bytes), dtype=torch.uint8, device=dev)
    res = _lib.WdCgResult()
    lib = _lib.load()
    with torch.cuda.device(device_workspace.device):
        rc = lib.cg_solve_ooc(ctypes.byref(_lib.lattice(dims)), float(mass), U.data_ptr(), b.data_ptr(),
                              x.data_ptr(), ctypes.byref(params), ctypes.byref(res), host_workspace.data_ptr(),
                              host_workspace.numel(), device_workspace.data_ptr(), device_workspace.numel(),
                              _stream(device_workspace.device))
    ok = (_lib.WD_OK,) if raise_on_nonconvergence else (_lib.WD_OK, _lib.WD_NOT_CONVERGED)
    _lib.check(rc, "cg_solve_ooc", ok)
    info = res.as_dict()
    if hist is not None:
        info["history"] = list(hist)[: min(history, res.iterations)]
    return x, info
