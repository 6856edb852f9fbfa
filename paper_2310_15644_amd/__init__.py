"""Python binding of libefie (gfx950 EFIE hot path).

Argument marshalling only: every step of the computation runs in the HIP
kernels of `libefie.so`; torch supplies device memory and the current stream.
Importing this package does not need a GPU; calling anything that launches
work does, and fails loudly if the library or the device is missing.

Layouts follow include/efie.h: complex tensors are interleaved (torch complex
dtypes), multi-vectors are (nrhs, N) row-major, Z is (N, N).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

__all__ = [
    "lib", "library_path", "EfieError", "Mesh", "assemble", "excite_planewave", "farfield", "zx", "solve",
    "SolveStats", "ktilde", "ETA0", "C128", "C64", "COCG", "CGS",
]

ETA0 = 376.730313668
C128, C64 = 0, 1
COCG, CGS = 0, 1
_STATUS = {
    0: "EFIE_OK", 1: "EFIE_NOT_CONVERGED", -1: "EFIE_ERR_ARG", -2: "EFIE_ERR_MESH_OPEN",
    -3: "EFIE_ERR_MESH_NONMANIFOLD", -4: "EFIE_ERR_MESH_ORIENT", -5: "EFIE_ERR_DEGENERATE", -6: "EFIE_ERR_HIP",
    -7: "EFIE_ERR_BREAKDOWN", -8: "EFIE_ERR_NAN", -9: "EFIE_ERR_STATE",
}

HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.environ.get("EFIE_LIBRARY") or os.path.join(HERE, "libefie.so")

# symbols declared in include/efie.h (checked by the CPU tests)
EXPORTED = [
    "efie_abi_version", "efie_last_error", "efie_mesh_create", "efie_mesh_destroy", "efie_mesh_sizes",
    "efie_mesh_rwg_table", "efie_mesh_upload", "efie_mesh_set_far_rule", "efie_assemble", "efie_excite_planewave",
    "efie_farfield_workspace_size", "efie_farfield", "efie_zx", "efie_solve_workspace_size", "efie_solve",
    "efie_prof_enable", "efie_prof_reset", "efie_prof_read",
    "efie_gemm_variants", "efie_gemm_variant_info", "efie_gemm_autotune", "efie_gemm_select",
    "efie_zx_flush64_workspace_size", "efie_zx_flush64",
    "efie_calderon_create", "efie_calderon_destroy", "efie_calderon_sizes", "efie_calderon_upload",
    "efie_calderon_host_matrices", "efie_calderon_assemble", "efie_calderon_set_far_rule", "efie_solve_precond_workspace_size", "efie_solve_precond",
    "efie_batch_create", "efie_batch_destroy", "efie_batch_sizes", "efie_batch_upload", "efie_batch_assemble",
    "efie_batch_solve", "efie_farfield_adjoint", "efie_vertex_grad_workspace_size", "efie_vertex_grad",
    "efie_assemble_workspace_size", "efie_assemble_ws", "efie_calderon_assemble_ex", "efie_solve_precond_ex",
    "efie_convert", "efie_ktilde", "efie_mesh_fp32_kmax", "efie_zx_flush64_noalloc_max", "efie_zx_flush64_noalloc",
    "efie_gemm_autotune_cached_workspace_size", "efie_gemm_autotune_cached",
    "efie_bie2d_create", "efie_bie2d_destroy", "efie_bie2d_sizes", "efie_bie2d_upload", "efie_bie2d_perimeter",
    "efie_bie2d_assemble", "efie_bie2d_setup", "efie_bie2d_apply", "efie_bie2d_rhs", "efie_bie2d_skeleton",
    "efie_bie2d_solve", "efie_bie2d_factors", "efie_bie2d_counterpart", "efie_bie2d_farfield",
    "efie_calderon_cfie_assemble", "efie_calderon_mfie_rhs_workspace_size", "efie_calderon_mfie_rhs",
    "efie_solve_cfie_workspace_size", "efie_solve_cfie", "efie_farfield_objective",
]
PROF_IDS = {"far": 0, "near": 1, "mfma": 2, "gemv": 3, "zgemm": 4, "krylov": 5, "excite": 6, "farfield": 7, "grad_far": 8,
            "grad_near": 9, "grad_tri": 10, "rows_near": 11, "mfma_small": 12}


class EfieError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class _SolveOpts(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_int32), ("maxit", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_refine", ctypes.c_int32), ("inner_tol", ctypes.c_double), ("fp32_acc", ctypes.c_int32)]


class _RhsStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("relres_recur", ctypes.c_double),
                ("relres_true", ctypes.c_double)]


_lib = None


def lib():
    """Load libefie.so (built in-tree by paper_2310_15644_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(library_path):
        raise RuntimeError(f"{library_path} is missing: run `python -m paper_2310_15644_amd.build`")
    L = ctypes.CDLL(library_path)
    P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    sig = {
        "efie_abi_version": ([], ctypes.c_int),
        "efie_last_error": ([], ctypes.c_char_p),
        "efie_mesh_create": ([P, I64, P, I64, D, ctypes.POINTER(P)], ctypes.c_int),
        "efie_mesh_destroy": ([P], None),
        "efie_mesh_sizes": ([P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I64),
                             ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "efie_mesh_rwg_table": ([P, P, P], ctypes.c_int),
        "efie_mesh_upload": ([P, P, ctypes.c_size_t, P], ctypes.c_int),
        "efie_mesh_set_far_rule": ([P, D], ctypes.c_int),
        "efie_assemble": ([P, D, D, D, ctypes.c_int, P, P, ctypes.c_int, P], ctypes.c_int),
        "efie_excite_planewave": ([P, D, P, P, I64, D, P, P], ctypes.c_int),
        "efie_farfield_workspace_size": ([P, I64, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "efie_farfield": ([P, D, D, P, I64, P, I64, P, P, ctypes.c_size_t, P], ctypes.c_int),
        "efie_zx": ([P, ctypes.c_int, I64, P, P, I64, P], ctypes.c_int),
        "efie_zx_flush64_workspace_size": ([I64, I64, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "efie_zx_flush64": ([P, I64, P, P, I64, P, ctypes.c_size_t, P], ctypes.c_int),
        "efie_solve_workspace_size": ([I64, I64, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "efie_solve": ([P, ctypes.c_int, I64, P, P, I64, ctypes.POINTER(_SolveOpts), ctypes.POINTER(_RhsStats),
                        P, ctypes.c_size_t, P], ctypes.c_int),
        "efie_prof_enable": ([ctypes.c_int], ctypes.c_int),
        "efie_prof_reset": ([], ctypes.c_int),
        "efie_prof_read": ([ctypes.c_int, ctypes.POINTER(I64), ctypes.POINTER(D), ctypes.POINTER(D)], ctypes.c_int),
        "efie_gemm_variants": ([ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "efie_gemm_variant_info": ([ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "efie_gemm_autotune": ([P, I64, P, I64, ctypes.c_int, P, ctypes.c_size_t, ctypes.c_int,
                                ctypes.POINTER(D), ctypes.POINTER(ctypes.c_int), P], ctypes.c_int),
        "efie_gemm_select": ([ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "efie_calderon_create": ([P, ctypes.POINTER(P)], ctypes.c_int),
        "efie_calderon_destroy": ([P], None),
        "efie_calderon_sizes": ([P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(ctypes.c_size_t),
                                 ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "efie_calderon_upload": ([P, P, ctypes.c_size_t, P], ctypes.c_int),
        "efie_calderon_host_matrices": ([P, P, P], ctypes.c_int),
        "efie_calderon_set_far_rule": ([P, D], ctypes.c_int),
        "efie_calderon_assemble": ([P, D, D, D, P, P, D, I32, ctypes.POINTER(D), P, ctypes.c_size_t, P], ctypes.c_int),
        "efie_calderon_assemble_ex": ([P, D, D, D, ctypes.c_int, P, P, D, I32, ctypes.POINTER(D), P, ctypes.c_size_t,
                                       P], ctypes.c_int),
        "efie_convert": ([P, ctypes.c_int, P, ctypes.c_int, I64, P], ctypes.c_int),
        "efie_ktilde": ([D, D, ctypes.POINTER(D), ctypes.POINTER(D)], ctypes.c_int),
        "efie_mesh_fp32_kmax": ([P, ctypes.POINTER(D)], ctypes.c_int),
        "efie_zx_flush64_noalloc_max": ([ctypes.POINTER(I64)], ctypes.c_int),
        "efie_bie2d_create": ([P, P, I64, ctypes.c_int, ctypes.POINTER(P)], ctypes.c_int),
        "efie_bie2d_destroy": ([P], None),
        "efie_bie2d_sizes": ([P, I64, I64, I64, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)],
                             ctypes.c_int),
        "efie_bie2d_upload": ([P, P, ctypes.c_size_t, P], ctypes.c_int),
        "efie_bie2d_perimeter": ([P, ctypes.c_int, ctypes.POINTER(D)], ctypes.c_int),
        "efie_bie2d_assemble": ([P, ctypes.c_int, D, D, P, P, P, I64, I64, I64, I64, I64, P], ctypes.c_int),
        "efie_bie2d_setup": ([P, ctypes.c_int, D, D, D, I64, I64, I64, P, ctypes.c_size_t, P], ctypes.c_int),
        "efie_bie2d_apply": ([P, ctypes.c_int, P, P, I64, P], ctypes.c_int),
        "efie_bie2d_rhs": ([P, P, I64, D, P, P, P, P], ctypes.c_int),
        "efie_bie2d_skeleton": ([P, P, I64, D, ctypes.POINTER(I64), ctypes.POINTER(D), ctypes.POINTER(D), P],
                                ctypes.c_int),
        "efie_bie2d_solve": ([P, P, P, I64, P], ctypes.c_int),
        "efie_bie2d_factors": ([P, P, P, P], ctypes.c_int),
        "efie_bie2d_counterpart": ([P, P, P, P], ctypes.c_int),
        "efie_bie2d_farfield": ([P, ctypes.c_int, D, P, I64, P, I64, P, P], ctypes.c_int),
        "efie_zx_flush64_noalloc": ([P, I64, P, P, I64, P], ctypes.c_int),
        "efie_gemm_autotune_cached_workspace_size": ([I64, I64, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "efie_gemm_autotune_cached": ([ctypes.c_char_p, P, I64, I64, ctypes.c_int, ctypes.c_int, P, ctypes.c_size_t,
                                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(D),
                                       ctypes.POINTER(D), ctypes.POINTER(ctypes.c_int), P], ctypes.c_int),
        "efie_solve_precond_ex": ([P, ctypes.c_int, P, ctypes.c_int, I64, P, P, I64, ctypes.POINTER(_SolveOpts),
                                   ctypes.POINTER(_RhsStats), P, ctypes.c_size_t, P], ctypes.c_int),
        "efie_solve_precond_workspace_size": ([I64, I64, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "efie_calderon_cfie_assemble": ([P, D, D, D, D, P, P, P, P, D, I32, ctypes.POINTER(D), P, ctypes.c_size_t, P],
                                        ctypes.c_int),
        "efie_calderon_mfie_rhs_workspace_size": ([P, I64, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "efie_calderon_mfie_rhs": ([P, D, P, P, I64, P, P, ctypes.c_size_t, P], ctypes.c_int),
        "efie_solve_cfie_workspace_size": ([I64, I64, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "efie_solve_cfie": ([P, P, P, P, I64, P, P, P, I64, ctypes.POINTER(_SolveOpts), ctypes.POINTER(_RhsStats), P,
                             ctypes.c_size_t, P], ctypes.c_int),
        "efie_solve_precond": ([P, P, I64, P, P, I64, ctypes.POINTER(_SolveOpts), ctypes.POINTER(_RhsStats), P,
                                ctypes.c_size_t, P], ctypes.c_int),
        "efie_batch_create": ([P, I32, ctypes.POINTER(P)], ctypes.c_int),
        "efie_batch_destroy": ([P], None),
        "efie_batch_sizes": ([P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                              ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I64)], ctypes.c_int),
        "efie_batch_upload": ([P, P, ctypes.c_size_t, P], ctypes.c_int),
        "efie_batch_assemble": ([P, P, D, ctypes.c_int, P, P, ctypes.c_size_t, P], ctypes.c_int),
        "efie_batch_solve": ([P, P, ctypes.c_int, P, P, ctypes.POINTER(_SolveOpts), ctypes.POINTER(_RhsStats), P,
                              ctypes.c_size_t, P], ctypes.c_int),
        "efie_farfield_adjoint": ([P, D, D, P, I64, P, I64, P, P, ctypes.c_size_t, P], ctypes.c_int),
        "efie_farfield_objective": ([P, I64, P, P, P], ctypes.c_int),
        "efie_assemble_workspace_size": ([P, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t),
                                          ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "efie_assemble_ws": ([P, D, D, D, ctypes.c_int, P, P, ctypes.c_size_t, P], ctypes.c_int),
        "efie_vertex_grad_workspace_size": ([P, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "efie_vertex_grad": ([P, D, D, P, P, P, P, I64, ctypes.POINTER(D), ctypes.POINTER(D), D, P, P,
                              ctypes.c_size_t, P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(code, allow_not_converged=False):
    if code == 0 or (allow_not_converged and code == 1):
        return code
    msg = lib().efie_last_error().decode()
    raise EfieError(code, msg)


# ------------------------------------------------------------------ torch glue
def _torch():
    import torch

    return torch


def _stream(device=None):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _require_cuda(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.is_complex() and (t.is_conj() or t.is_neg()):
        # a lazy conjugate/negative view: its memory holds the unconjugated values
        raise ValueError(f"{name} is a lazy conj/neg view: call .resolve_conj() / .resolve_neg() first")


def ktilde(k: float, a: float = 1.0) -> complex:
    """Complex wavenumber of the Calderon preconditioner (paper, Sec. III),
    k~ = k - 0.4 j k^(1/3) a^(-2/3) with a an average radius of curvature, as the
    library computes it (efie_ktilde)."""
    re, im = ctypes.c_double(), ctypes.c_double()
    _check(lib().efie_ktilde(float(k), float(a), ctypes.byref(re), ctypes.byref(im)))
    return complex(re.value, im.value)


class Mesh:
    """Closed triangle mesh with RWG topology (host) and device tables (torch-owned)."""

    def __init__(self, vertices, triangles, near_factor: float = 2.0, device=None):
        L = lib()
        v = np.ascontiguousarray(vertices, dtype=np.float64)
        t = np.ascontiguousarray(triangles, dtype=np.int32)
        h = ctypes.c_void_p()
        _check(L.efie_mesh_create(v.ctypes.data, len(v), t.ctypes.data, len(t), float(near_factor), ctypes.byref(h)))
        self._h = h
        n, nt, nn, tb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
        _check(L.efie_mesh_sizes(h, ctypes.byref(n), ctypes.byref(nt), ctypes.byref(nn), ctypes.byref(tb)))
        self.n, self.t, self.n_near, self.table_bytes = n.value, nt.value, nn.value, tb.value
        self.nv = len(v)
        self.vertices = v
        self.triangles = t
        self.near_factor = near_factor
        self.far3 = 0.0
        self._dev = None
        self._device = device

    def set_far_rule(self, ratio: float = 0.0):
        """Distance-adaptive far rule: pairs with centroid distance >= ratio times the
        larger longest edge take the 3x3 product of the interior 3-point rule
        (0: the 7x7 rule everywhere).  Applies to later assemblies of this mesh and
        to the barycentric operator of a Calderon built from it."""
        _check(lib().efie_mesh_set_far_rule(self._h, float(ratio)))
        self.far3 = float(ratio)
        return self

    def fp32_kmax(self) -> float:
        """Largest |Re k| that complex64 assembly of this mesh accepts (the FP32
        phase range of its far-pair kernels)."""
        v = ctypes.c_double()
        _check(lib().efie_mesh_fp32_kmax(self._h, ctypes.byref(v)))
        return v.value

    def rwg_table(self):
        ev = np.zeros((self.n, 2), dtype=np.int32)
        et = np.zeros((self.n, 2), dtype=np.int32)
        _check(lib().efie_mesh_rwg_table(self._h, ev.ctypes.data, et.ctypes.data))
        return ev, et

    def upload(self, device=None):
        """Copy the geometry tables to a torch-owned device buffer (kept by this object)."""
        torch = _torch()
        device = device or self._device or "cuda"
        buf = torch.empty(self.table_bytes + 256, dtype=torch.uint8, device=device)
        off = (-buf.data_ptr()) % 256
        view = buf[off:off + self.table_bytes]
        _check(lib().efie_mesh_upload(self._h, ctypes.c_void_p(view.data_ptr()), self.table_bytes,
                                      _stream(buf.device)))
        self._dev = buf
        self._device = buf.device
        return self

    @property
    def device(self):
        if self._dev is None:
            self.upload()
        return self._device

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.efie_mesh_destroy(h)
            self._h = None


def _cdtype(dtype):
    torch = _torch()
    if dtype in (C128, "c128", torch.complex128):
        return C128, torch.complex128
    if dtype in (C64, "c64", torch.complex64):
        return C64, torch.complex64
    raise ValueError(f"bad dtype {dtype}")




def assemble(mesh: Mesh, k, eta: float = ETA0, dtype=C128, parts: bool = False, out=None, out2=None,
             atomic: bool = False, workspace_bytes: int | None = None):
    """Dense Z (N, N) on the device; parts=True returns (T_A, T_Phi) instead.

    By default Z is built by the owner-computes tiles of efie_assemble_ws (written
    once, deterministic, exactly symmetric; the workspace holds the near-pair
    blocks, and `workspace_bytes` is accepted for compatibility and otherwise
    unused); atomic=True (and parts mode) use efie_assemble."""
    torch = _torch()
    dev = mesh.device
    code, tdt = _cdtype(dtype)
    k = complex(k)
    Z = out if out is not None else torch.empty((mesh.n, mesh.n), dtype=tdt, device=dev)
    Z2 = None
    if parts:
        Z2 = out2 if out2 is not None else torch.empty((mesh.n, mesh.n), dtype=tdt, device=dev)
    _require_cuda(Z, "Z")
    if not parts and not atomic:
        lo, full = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().efie_assemble_workspace_size(mesh._h, code, ctypes.byref(lo), ctypes.byref(full)))
        nb = full.value
        ws = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
        off = (-ws.data_ptr()) % 256
        _check(lib().efie_assemble_ws(mesh._h, k.real, k.imag, float(eta), code, _ptr(Z),
                                      ctypes.c_void_p(ws.data_ptr() + off), nb, _stream(dev)))
        return Z
    _check(lib().efie_assemble(mesh._h, k.real, k.imag, float(eta), code, _ptr(Z),
                               _ptr(Z2) if Z2 is not None else None, int(parts), _stream(dev)))
    return (Z, Z2) if parts else Z


def _dev_vectors(a, dev):
    """(n, 3) float64 device tensor from a numpy array or a torch tensor."""
    torch = _torch()
    if isinstance(a, torch.Tensor):
        t = a.to(device=dev, dtype=torch.float64)
    else:
        t = torch.as_tensor(np.atleast_2d(np.asarray(a, dtype=np.float64)), device=dev)
    return t.reshape(-1, 3).contiguous()


def excite_planewave(mesh: Mesh, k: float, khat, pol, e0: float = 1.0, out=None):
    """V (nrhs, N) complex128 for plane waves E0 pol exp(-j k khat . r)."""
    torch = _torch()
    dev = mesh.device
    kh = _dev_vectors(khat, dev)
    po = _dev_vectors(pol, dev)
    S = kh.shape[0]
    V = out if out is not None else torch.empty((S, mesh.n), dtype=torch.complex128, device=dev)
    _check(lib().efie_excite_planewave(mesh._h, float(k), _ptr(kh), _ptr(po), S, float(e0), _ptr(V), _stream(dev)))
    return V


def farfield(mesh: Mesh, k: float, J, dirs, eta: float = ETA0):
    """F (nrhs, ndir, 2) complex128: (theta, phi) components of the far-field pattern."""
    torch = _torch()
    dev = mesh.device
    J = J.reshape(-1, mesh.n)
    _require_cuda(J, "J")
    d = _dev_vectors(dirs, dev)
    nd = d.shape[0]
    nb = ctypes.c_size_t()
    _check(lib().efie_farfield_workspace_size(mesh._h, nd, ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    F = torch.empty((J.shape[0], nd, 2), dtype=torch.complex128, device=dev)
    _check(lib().efie_farfield(mesh._h, float(k), float(eta), _ptr(J), J.shape[0], _ptr(d), nd, _ptr(F), _ptr(ws),
                               nb.value, _stream(dev)))
    return F


def farfield_adjoint(mesh: Mesh, k: float, W, dirs, eta: float = ETA0):
    """G (nrhs, N) complex128 with G[s] = R^T W[s], R the far-field matrix (F = R J).

    W (nrhs, ndir, 2) complex128 on the device (W = conj(F) for J = sum |F|^2)."""
    torch = _torch()
    dev = mesh.device
    d = _dev_vectors(dirs, dev)
    nd = d.shape[0]
    W = W.reshape(-1, nd, 2)
    _require_cuda(W, "W")
    if W.dtype != torch.complex128:
        raise ValueError("W must be complex128")
    nb = ctypes.c_size_t()
    _check(lib().efie_farfield_workspace_size(mesh._h, nd, ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    G = torch.empty((W.shape[0], mesh.n), dtype=torch.complex128, device=dev)
    _check(lib().efie_farfield_adjoint(mesh._h, float(k), float(eta), _ptr(W), W.shape[0], _ptr(d), nd, _ptr(G),
                                       _ptr(ws), nb.value, _stream(dev)))
    return G


def farfield_objective(F, with_weight: bool = True):
    """(J, W): J = sum |F|^2 (a 0-d float64 tensor on F's device) and W = conj(F)
    (efie_farfield_objective; W is None unless with_weight).  F complex128 on the
    device, any shape."""
    torch = _torch()
    _require_cuda(F, "F")
    if F.dtype != torch.complex128:
        raise ValueError("F must be complex128")
    F = F.contiguous()
    J = torch.empty((), dtype=torch.float64, device=F.device)
    W = torch.empty_like(F) if with_weight else None
    _check(lib().efie_farfield_objective(_ptr(F), F.numel(), _ptr(J), _ptr(W) if W is not None else None,
                                         _stream(F.device)))
    return J, W


def vertex_grad(mesh: Mesh, k: float, J, lam, W, dirs, khat, pol, e0: float = 1.0, eta: float = ETA0):
    """(nv, 3) float64: 2 Re[W^T dR/dx J + lam^T dV/dx - lam^T dZ/dx J] for one right-hand side."""
    torch = _torch()
    dev = mesh.device
    d = _dev_vectors(dirs, dev)
    nd = d.shape[0]
    for t, name in ((J, "J"), (lam, "lambda"), (W, "W")):
        _require_cuda(t, name)
        if t.dtype != torch.complex128:
            raise ValueError(f"{name} must be complex128")
    if J.numel() != mesh.n or lam.numel() != mesh.n or W.numel() != 2 * nd:
        raise ValueError("J, lambda must hold N values and W 2 ndir values")
    kh = (ctypes.c_double * 3)(*np.asarray(khat, dtype=np.float64).reshape(3))
    po = (ctypes.c_double * 3)(*np.asarray(pol, dtype=np.float64).reshape(3))
    nb = ctypes.c_size_t()
    _check(lib().efie_vertex_grad_workspace_size(mesh._h, ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    out = torch.empty((mesh.nv, 3), dtype=torch.float64, device=dev)
    _check(lib().efie_vertex_grad(mesh._h, float(k), float(eta), _ptr(J), _ptr(lam), _ptr(W), _ptr(d), nd, kh, po,
                                  float(e0), _ptr(out), _ptr(ws), nb.value, _stream(dev)))
    return out


def convert(A, dtype):
    """A copy of the complex device tensor A in dtype (C128 or C64), made by the library."""
    torch = _torch()
    _require_cuda(A, "A")
    src, _ = _cdtype(A.dtype)
    dst, tdt = _cdtype(dtype)
    out = torch.empty(A.shape, dtype=tdt, device=A.device)
    _check(lib().efie_convert(_ptr(A), src, _ptr(out), dst, A.numel(), _stream(A.device)))
    return out


def zx(Z, X):
    """Y = Z X for X (nrhs, N) of Z's dtype (one right-hand side: GEMV; complex64: MFMA GEMM)."""
    torch = _torch()
    code, tdt = _cdtype(Z.dtype)
    _require_cuda(Z, "Z")
    X = X.reshape(-1, Z.shape[0])
    if X.dtype != tdt:
        raise ValueError("X must have the dtype of Z")
    _require_cuda(X, "X")
    Y = torch.empty_like(X)
    _check(lib().efie_zx(_ptr(Z), code, Z.shape[0], _ptr(X), _ptr(Y), X.shape[0], _stream(Z.device)))
    return Y


@dataclass
class SolveStats:
    iters: np.ndarray
    status: np.ndarray
    relres_recur: np.ndarray
    relres_true: np.ndarray
    code: int


def solve(Z, V, solver=COCG, tol=1e-8, maxit=1000, max_refine=4, inner_tol=1e-3, fp32_acc=False, out=None):
    """Solve Z J = V for V (nrhs, N) complex128; Z complex128 (FP64) or complex64 (mixed:
    FP32 matrix-core products with their partial sums flushed into FP64 every K chunk,
    or with fp32_acc accumulated in FP32)."""
    torch = _torch()
    code_dt, _ = _cdtype(Z.dtype)
    _require_cuda(Z, "Z")
    n = Z.shape[0]
    V = V.reshape(-1, n)
    _require_cuda(V, "V")
    if V.dtype != torch.complex128:
        raise ValueError("V must be complex128")
    S = V.shape[0]
    J = out if out is not None else torch.empty_like(V)
    nb = ctypes.c_size_t()
    _check(lib().efie_solve_workspace_size(n, S, code_dt, ctypes.byref(nb)))
    ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=Z.device)
    off = (-ws.data_ptr()) % 256
    opts = _SolveOpts(int(solver), int(maxit), float(tol), int(max_refine), float(inner_tol), int(bool(fp32_acc)))
    st = (_RhsStats * S)()
    code = lib().efie_solve(_ptr(Z), code_dt, n, _ptr(V), _ptr(J), S, ctypes.byref(opts), st,
                            ctypes.c_void_p(ws.data_ptr() + off), nb.value, _stream(Z.device))
    _check(code, allow_not_converged=True)
    stats = SolveStats(
        iters=np.array([s.iters for s in st]), status=np.array([s.status for s in st]),
        relres_recur=np.array([s.relres_recur for s in st]), relres_true=np.array([s.relres_true for s in st]),
        code=code,
    )
    return J, stats


def prof_enable(on: bool = True):
    """Turn the library's HIP-event launch timing on or off."""
    _check(lib().efie_prof_enable(int(on)))


def prof_reset():
    _check(lib().efie_prof_reset())


def prof_read(with_work: bool = False):
    """{kernel: (launches, total_ms[, total_work])} since the last prof_reset (waits for the events)."""
    out = {}
    for name, i in PROF_IDS.items():
        n, ms, wk = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        _check(lib().efie_prof_read(i, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(wk)))
        out[name] = (n.value, ms.value, wk.value) if with_work else (n.value, ms.value)
    return out


# ------------------------------------------------------------- GEMM tile autotuner
def gemm_variants():
    """[(bm, bn, kc)] of the complex64 matrix-core GEMM: block tile of bm right-hand
    sides x bn unknowns, K chunk of kc complex elements."""
    L = lib()
    c = ctypes.c_int()
    _check(L.efie_gemm_variants(ctypes.byref(c)))
    out = []
    for v in range(c.value):
        bm, bn, kc = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(L.efie_gemm_variant_info(v, ctypes.byref(bm), ctypes.byref(bn), ctypes.byref(kc)))
        out.append((bm.value, bn.value, kc.value))
    return out


def gemm_kernel_name(variant, acc64: bool) -> str:
    """The kernel's name as profilers print it (template arguments included)."""
    bm, bn, kc = variant[:3]
    return f"cgemm_planar_kernel<{bm}, {bn}, {kc}, {'true' if acc64 else 'false'}>"


def zx_flush64(Z, X):
    """Y = Z X with Z complex64 and X complex128 (nrhs, N): the mixed solves' product
    (FP32 matrix cores, partial sums flushed into FP64 every K chunk), Y complex128."""
    torch = _torch()
    _require_cuda(Z, "Z")
    if Z.dtype != torch.complex64:
        raise ValueError("Z must be complex64")
    n = Z.shape[0]
    X = X.reshape(-1, n)
    _require_cuda(X, "X")
    if X.dtype != torch.complex128:
        raise ValueError("X must be complex128")
    S = X.shape[0]
    Y = torch.empty_like(X)
    nb = ctypes.c_size_t()
    _check(lib().efie_zx_flush64_workspace_size(n, S, ctypes.byref(nb)))
    ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=Z.device)
    off = (-ws.data_ptr()) % 256
    _check(lib().efie_zx_flush64(_ptr(Z), n, _ptr(X), _ptr(Y), S, ctypes.c_void_p(ws.data_ptr() + off), nb.value,
                                 _stream(Z.device)))
    return Y


def gemm_select(acc64: bool, variant: int) -> int:
    prev = ctypes.c_int()
    _check(lib().efie_gemm_select(int(acc64), int(variant), ctypes.byref(prev)))
    return prev.value


def default_tuning_cache():
    return os.path.join(os.path.expanduser("~"), ".cache", "efie", "gemm_tiles.txt")


def gemm_autotune(Z, M: int, reps: int = 3, cache: str | None = None, force: bool = False):
    """Pick and select the matrix-core tile shape of both GEMM paths for Z (n x n
    complex64) times M right-hand sides (efie_gemm_autotune_cached: the library
    times the tiles and keeps its choice in the cache file, reused unless force).
    Returns {"acc32": variant, "acc64": variant, "ms": {...}, "tiles": [...],
    "from_cache": bool}."""
    torch = _torch()
    if Z.dtype != torch.complex64:
        raise ValueError("autotuning is for the complex64 matrix-core GEMM")
    _require_cuda(Z, "Z")
    n = Z.shape[0]
    cache = cache or default_tuning_cache()
    try:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
    except OSError:
        pass
    nb = ctypes.c_size_t()
    _check(lib().efie_gemm_autotune_cached_workspace_size(n, int(M), ctypes.byref(nb)))
    ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=Z.device)
    off = (-ws.data_ptr()) % 256
    tiles = gemm_variants()
    v32, v64, hit = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    ms32, ms64 = (ctypes.c_double * len(tiles))(), (ctypes.c_double * len(tiles))()
    _check(lib().efie_gemm_autotune_cached(cache.encode(), _ptr(Z), n, int(M), int(reps), int(bool(force)),
                                           ctypes.c_void_p(ws.data_ptr() + off), nb.value, ctypes.byref(v32),
                                           ctypes.byref(v64), ms32, ms64, ctypes.byref(hit), _stream(Z.device)))
    del ws
    return {"acc32": v32.value, "acc64": v64.value, "tiles": tiles, "from_cache": bool(hit.value),
            "ms": {"acc32": [round(x, 4) for x in ms32], "acc64": [round(x, 4) for x in ms64]}}


# ------------------------------------------------------------------ Calderon
class Calderon:
    """Calderon preconditioner of a mesh (paper, Sec. III, eq. 16 structure):
    P = T_BC(k~) G_mix^-1 with Buffa-Christiansen functions on the barycentric
    refinement; solves P Z J = P V."""

    def __init__(self, mesh: Mesh):
        L = lib()
        h = ctypes.c_void_p()
        _check(L.efie_calderon_create(mesh._h, ctypes.byref(h)))
        self._h = h
        self.mesh = mesh          # keeps the primal handle alive
        nb, tb, tbytes, wbytes = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t(), ctypes.c_size_t()
        _check(L.efie_calderon_sizes(h, ctypes.byref(nb), ctypes.byref(tb), ctypes.byref(tbytes), ctypes.byref(wbytes)))
        self.n_bary, self.t_bary, self.table_bytes, self.ws_bytes = nb.value, tb.value, tbytes.value, wbytes.value
        self._dev = None

    def set_far_rule(self, ratio: float = -1.0):
        """Far rule of the barycentric operator alone (ratio >= 0; see Mesh.set_far_rule);
        ratio < 0: follow the primal mesh's rule (the default)."""
        _check(lib().efie_calderon_set_far_rule(self._h, float(ratio)))
        return self

    def host_matrices(self):
        """Dense (R: N_bary x N, G_mix: N x N) host copies (small meshes)."""
        R = np.zeros((self.n_bary, self.mesh.n))
        G = np.zeros((self.mesh.n, self.mesh.n))
        _check(lib().efie_calderon_host_matrices(self._h, R.ctypes.data, G.ctypes.data))
        return R, G

    def upload(self, device=None):
        torch = _torch()
        device = device or self.mesh.device
        buf = torch.empty(self.table_bytes + 256, dtype=torch.uint8, device=device)
        off = (-buf.data_ptr()) % 256
        _check(lib().efie_calderon_upload(self._h, ctypes.c_void_p(buf.data_ptr() + off), self.table_bytes,
                                          _stream(buf.device)))
        self._dev = buf
        return self

    def assemble(self, ktilde_value, eta: float = ETA0, tol: float = 1e-13, maxit: int = 500, with_tbc=False,
                 bary_dtype=C128):
        """P (N x N complex128) on the device; with_tbc also returns T_BC.  bary_dtype
        C64 computes the barycentric far pairs in FP32 (the contractions, T_BC and P
        stay FP64)."""
        torch = _torch()
        if self._dev is None:
            self.upload()
        dev = self.mesh.device
        n = self.mesh.n
        kt = complex(ktilde_value)
        Pm = torch.empty((n, n), dtype=torch.complex128, device=dev)
        T = torch.empty((n, n), dtype=torch.complex128, device=dev) if with_tbc else None
        ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=dev)
        off = (-ws.data_ptr()) % 256
        rel = ctypes.c_double()
        code = lib().efie_calderon_assemble_ex(self._h, kt.real, kt.imag, float(eta), _cdtype(bary_dtype)[0],
                                               _ptr(Pm), _ptr(T) if T is not None else None, float(tol), int(maxit),
                                               ctypes.byref(rel), ctypes.c_void_p(ws.data_ptr() + off),
                                               self.ws_bytes, _stream(dev))
        _check(code, allow_not_converged=True)
        del ws
        self.gram_relres = rel.value
        return (Pm, T) if with_tbc else Pm

    def cfie(self, k: float, kt=None, eta: float = ETA0, tol: float = 1e-13, maxit: int = 500, with_k=False,
             a: float = 1.0):
        """The MFIE factors of the Calderon-stabilized CFIE on the device: M =
        eta (-G_mix^T/2 - K_BC(k)) and Q = eta (-G_mix^T/2 + K_BC(k~)) G_mix^-T (N x N
        complex128 each), with eta^2 C_p = P Z + Q M; k~ the paper's complex
        wavenumber of radius a unless given.  with_k also returns K_BC(k), K_BC(k~)."""
        torch = _torch()
        if self._dev is None:
            self.upload()
        dev = self.mesh.device
        n = self.mesh.n
        kt = ktilde(k, a) if kt is None else complex(kt)
        M = torch.empty((n, n), dtype=torch.complex128, device=dev)
        Q = torch.empty((n, n), dtype=torch.complex128, device=dev)
        K1 = torch.empty((n, n), dtype=torch.complex128, device=dev) if with_k else None
        K2 = torch.empty((n, n), dtype=torch.complex128, device=dev) if with_k else None
        ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=dev)
        off = (-ws.data_ptr()) % 256
        rel = ctypes.c_double()
        code = lib().efie_calderon_cfie_assemble(self._h, float(k), kt.real, kt.imag, float(eta), _ptr(M), _ptr(Q),
                                                 _ptr(K1) if with_k else None, _ptr(K2) if with_k else None,
                                                 float(tol), int(maxit), ctypes.byref(rel),
                                                 ctypes.c_void_p(ws.data_ptr() + off), self.ws_bytes, _stream(dev))
        _check(code, allow_not_converged=True)
        del ws
        self.cfie_gram_relres = rel.value
        return (M, Q, K1, K2) if with_k else (M, Q)

    def mfie_rhs(self, k: float, khat, pol):
        """H (nrhs, N) complex128: H[s][m] = (g_m, (khat_s x pol_s) exp(-j k khat_s . r)),
        eta times the BC-tested incident magnetic field of E = pol exp(-j k khat . r)."""
        torch = _torch()
        if self._dev is None:
            self.upload()
        dev = self.mesh.device
        kh = _dev_vectors(khat, dev)
        po = _dev_vectors(pol, dev)
        S = kh.shape[0]
        nb = ctypes.c_size_t()
        _check(lib().efie_calderon_mfie_rhs_workspace_size(self._h, S, ctypes.byref(nb)))
        ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=dev)
        off = (-ws.data_ptr()) % 256
        H = torch.empty((S, self.mesh.n), dtype=torch.complex128, device=dev)
        _check(lib().efie_calderon_mfie_rhs(self._h, float(k), _ptr(kh), _ptr(po), S, _ptr(H),
                                            ctypes.c_void_p(ws.data_ptr() + off), nb.value, _stream(dev)))
        return H

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.efie_calderon_destroy(h)
            self._h = None


def solve_precond(Z, Pm, V, tol=1e-8, maxit=1000, max_refine=6, inner_tol=1e-4, fp32_acc=False, out=None):
    """CGS on P Z J = P V with outer refinement on the unpreconditioned FP64 true
    residual (up to max_refine passes); Z and P complex128 (FP64 throughout) or
    complex64 (FP32 matrix-core products inside CGS, flushed into FP64 per K chunk
    or with fp32_acc accumulated in FP32; each pass to at least inner_tol).  Stats report the
    true residual and the iterations summed over the passes."""
    torch = _torch()
    _require_cuda(Z, "Z")
    _require_cuda(Pm, "P")
    zdt, _ = _cdtype(Z.dtype)
    pdt, _ = _cdtype(Pm.dtype)
    n = Z.shape[0]
    V = V.reshape(-1, n)
    _require_cuda(V, "V")
    S = V.shape[0]
    J = out if out is not None else torch.empty_like(V)
    nb = ctypes.c_size_t()
    _check(lib().efie_solve_precond_workspace_size(n, S, ctypes.byref(nb)))
    ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=Z.device)
    off = (-ws.data_ptr()) % 256
    opts = _SolveOpts(CGS, int(maxit), float(tol), int(max_refine), float(inner_tol), int(bool(fp32_acc)))
    st = (_RhsStats * S)()
    code = lib().efie_solve_precond_ex(_ptr(Z), zdt, _ptr(Pm), pdt, n, _ptr(V), _ptr(J), S, ctypes.byref(opts), st,
                                       ctypes.c_void_p(ws.data_ptr() + off), nb.value, _stream(Z.device))
    _check(code, allow_not_converged=True)
    return J, SolveStats(
        iters=np.array([s.iters for s in st]), status=np.array([s.status for s in st]),
        relres_recur=np.array([s.relres_recur for s in st]), relres_true=np.array([s.relres_true for s in st]),
        code=code,
    )


def solve_cfie(Z, Pm, M, Q, V, H, tol=1e-8, maxit=1000, out=None):
    """CGS on the Calderon-stabilized CFIE (P Z + Q M) J = P V + Q H (every matrix
    complex128, FP64 products); stats report the FP64 true residual of that system."""
    torch = _torch()
    for t, nm in ((Z, "Z"), (Pm, "P"), (M, "M"), (Q, "Q")):
        _require_cuda(t, nm)
        if t.dtype != torch.complex128:
            raise ValueError(f"{nm} must be complex128")
    n = Z.shape[0]
    V = V.reshape(-1, n)
    H = H.reshape(-1, n)
    _require_cuda(V, "V")
    _require_cuda(H, "H")
    if V.shape != H.shape:
        raise ValueError("V and H must have the same shape")
    S = V.shape[0]
    J = out if out is not None else torch.empty_like(V)
    nb = ctypes.c_size_t()
    _check(lib().efie_solve_cfie_workspace_size(n, S, ctypes.byref(nb)))
    ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=Z.device)
    off = (-ws.data_ptr()) % 256
    opts = _SolveOpts(CGS, int(maxit), float(tol), 1, 1e-4, 0)
    st = (_RhsStats * S)()
    code = lib().efie_solve_cfie(_ptr(Z), _ptr(Pm), _ptr(M), _ptr(Q), n, _ptr(V), _ptr(H), _ptr(J), S,
                                 ctypes.byref(opts), st, ctypes.c_void_p(ws.data_ptr() + off), nb.value,
                                 _stream(Z.device))
    _check(code, allow_not_converged=True)
    return J, SolveStats(
        iters=np.array([s.iters for s in st]), status=np.array([s.status for s in st]),
        relres_recur=np.array([s.relres_recur for s in st]), relres_true=np.array([s.relres_true for s in st]),
        code=code,
    )


# --------------------------------------------------------------- many meshes
class Batch:
    """Uneven meshes assembled in one persistent launch and solved together
    (one right-hand side per mesh).  Z of mesh i is Zcat[zoff[i] : zoff[i] + N_i^2]
    viewed as (N_i, N_i); vectors are Vcat[voff[i] : voff[i+1]]."""

    def __init__(self, meshes):
        L = lib()
        for m in meshes:
            m.device   # uploads if needed
        arr = (ctypes.c_void_p * len(meshes))(*[m._h.value for m in meshes])
        h = ctypes.c_void_p()
        _check(L.efie_batch_create(arr, len(meshes), ctypes.byref(h)))
        self._h = h
        self.meshes = list(meshes)
        tb, wb, ze, ve, it = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(L.efie_batch_sizes(h, ctypes.byref(tb), ctypes.byref(wb), ctypes.byref(ze), ctypes.byref(ve),
                                  ctypes.byref(it)))
        self.table_bytes, self.ws_bytes, self.z_elems, self.v_elems, self.items = (
            tb.value, wb.value, ze.value, ve.value, it.value)
        ns = [m.n for m in meshes]
        self.zoff = np.concatenate([[0], np.cumsum([n * n for n in ns])[:-1]]).astype(np.int64)
        self.voff = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
        torch = _torch()
        dev = meshes[0].device
        self._dev = torch.empty(self.table_bytes + 256, dtype=torch.uint8, device=dev)
        off = (-self._dev.data_ptr()) % 256
        _check(L.efie_batch_upload(h, ctypes.c_void_p(self._dev.data_ptr() + off), self.table_bytes, _stream(dev)))
        self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=dev)
        self._ws_ptr = ctypes.c_void_p(self._ws.data_ptr() + (-self._ws.data_ptr()) % 256)
        self.device = dev

    def assemble(self, k, eta: float = ETA0, dtype=C64, out=None):
        """Concatenated Z of every mesh (flat complex tensor of z_elems)."""
        torch = _torch()
        code, tdt = _cdtype(dtype)
        ks = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.float64), (len(self.meshes),)))
        Z = out if out is not None else torch.empty(self.z_elems, dtype=tdt, device=self.device)
        _check(lib().efie_batch_assemble(self._h, ks.ctypes.data, float(eta), code, _ptr(Z), self._ws_ptr,
                                         self.ws_bytes, _stream(self.device)))
        return Z

    def z_of(self, Zcat, i):
        n = self.meshes[i].n
        return Zcat[self.zoff[i]:self.zoff[i] + n * n].view(n, n)

    def solve(self, Zcat, Vcat, tol=1e-6, maxit=2000, out=None):
        torch = _torch()
        code, _ = _cdtype(Zcat.dtype)
        J = out if out is not None else torch.empty(self.v_elems, dtype=torch.complex128, device=self.device)
        opts = _SolveOpts(COCG, int(maxit), float(tol), 1, 1e-3, 0)
        st = (_RhsStats * len(self.meshes))()
        rc = lib().efie_batch_solve(self._h, _ptr(Zcat), code, _ptr(Vcat), _ptr(J), ctypes.byref(opts), st,
                                    self._ws_ptr, self.ws_bytes, _stream(self.device))
        _check(rc, allow_not_converged=True)
        return J, SolveStats(
            iters=np.array([s.iters for s in st]), status=np.array([s.status for s in st]),
            relres_recur=np.array([s.relres_recur for s in st]), relres_true=np.array([s.relres_true for s in st]),
            code=rc,
        )

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.efie_batch_destroy(h)
            self._h = None


# ------------------------------------------------------ the paper's 2-D method
class Bie2d:
    """The paper's 2-D fast direct solver on a closed curve (Sec. II-III): TM CFIE
    of a PEC cylinder, its Calderon-stabilized operator C_p (eq. 16), the circular
    counterpart C_p,c, a randomized skeleton of C_p - C_p,c and the Woodbury
    inverse (eqs. 17-18).  Vectors are rows: (count, n) complex128 device tensors.

    nodes, circle_nodes: (n, 2) counter-clockwise; q: Gauss points per segment."""

    APPLY = {"cp": 0, "cpt": 1, "cc": 2, "ccinv": 3, "ginv": 4, "a": 5}

    def __init__(self, nodes, circle_nodes, q: int = 4, device=None):
        torch = _torch()
        L = lib()
        v = np.ascontiguousarray(nodes, dtype=np.float64)
        c = np.ascontiguousarray(circle_nodes, dtype=np.float64)
        if v.shape != c.shape or v.ndim != 2 or v.shape[1] != 2:
            raise ValueError("nodes and circle_nodes must both be (n, 2)")
        h = ctypes.c_void_p()
        _check(L.efie_bie2d_create(v.ctypes.data, c.ctypes.data, len(v), int(q), ctypes.byref(h)))
        self._h = h
        self.n = len(v)
        self.q = q
        tb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        _check(L.efie_bie2d_sizes(h, 0, 1, 1, ctypes.byref(tb), ctypes.byref(wb)))
        self.device = torch.device(device or "cuda")
        self._tab = torch.empty(tb.value + 256, dtype=torch.uint8, device=self.device)
        off = (-self._tab.data_ptr()) % 256
        _check(L.efie_bie2d_upload(h, ctypes.c_void_p(self._tab.data_ptr() + off), tb.value, _stream(self.device)))
        self._ws = None
        self.nvec = 0

    def perimeter(self, which: int = 0) -> float:
        p = ctypes.c_double()
        _check(lib().efie_bie2d_perimeter(self._h, int(which), ctypes.byref(p)))
        return p.value

    def assemble(self, k, which: int = 0, rows=None, cols=None):
        """(S, D*, N) at complex k on the curve (which = 0) or the circle (1), for the
        window rows x cols (slices; default the whole matrix)."""
        torch = _torch()
        r0, r1 = (0, self.n) if rows is None else (rows.start or 0, rows.stop)
        c0, c1 = (0, self.n) if cols is None else (cols.start or 0, cols.stop)
        k = complex(k)
        out = [torch.empty((r1 - r0, c1 - c0), dtype=torch.complex128, device=self.device) for _ in range(3)]
        _check(lib().efie_bie2d_assemble(self._h, int(which), k.real, k.imag, *[_ptr(t) for t in out], r0, r1 - r0,
                                          c0, c1 - c0, c1 - c0, _stream(self.device)))
        return tuple(out)

    def setup(self, k: float, kt=None, rmax: int | None = None, block: int = 64, nvec: int = 64, a: float = 1.0,
              pol: str = "TM"):
        """Assemble the four operators of C_p for polarization pol ("TM": S_k, D*_k,
        N_k~, D*_k~; "TE": N_k, D*_k, S_k~, D*_k~) and the counterpart (k~ = the
        paper's complex wavenumber with radius a unless given); workspace for a
        skeleton of rank <= rmax (default n) in blocks of `block` and calls of <=
        nvec vectors."""
        torch = _torch()
        kt = ktilde(k, a) if kt is None else complex(kt)
        rmax = self.n if rmax is None else int(rmax)
        nvec = max(int(nvec), int(block))
        tb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().efie_bie2d_sizes(self._h, rmax, int(block), nvec, ctypes.byref(tb), ctypes.byref(wb)))
        self._ws = None
        self._ws = torch.empty(wb.value + 256, dtype=torch.uint8, device=self.device)
        off = (-self._ws.data_ptr()) % 256
        if pol not in ("TM", "TE"):
            raise ValueError("pol must be TM or TE")
        _check(lib().efie_bie2d_setup(self._h, 0 if pol == "TM" else 1, float(k), kt.real, kt.imag, rmax, int(block),
                                      nvec,
                                      ctypes.c_void_p(self._ws.data_ptr() + off), wb.value, _stream(self.device)))
        self.k, self.kt, self.rmax, self.block, self.nvec, self.pol = float(k), kt, rmax, int(block), nvec, pol
        return self

    def _vec(self, X, name):
        torch = _torch()
        X = X.reshape(-1, self.n)
        _require_cuda(X, name)
        if X.dtype != torch.complex128:
            raise ValueError(f"{name} must be complex128")
        return X

    def apply(self, op: str, X):
        """op X for rows X: "cp" C_p, "cpt" C_p^T, "cc" C_c, "ccinv" C_c^-1, "ginv" G^-1,
        "a" C_p - C_c."""
        torch = _torch()
        X = self._vec(X, "X")
        Y = torch.empty_like(X)
        _check(lib().efie_bie2d_apply(self._h, self.APPLY[op], _ptr(X), _ptr(Y), X.shape[0], _stream(self.device)))
        return Y

    def rhs(self, phis, eta: float = ETA0, stabilized: bool = True):
        """(e, h, b_p) for plane waves of incidence angles phis (b_p None unless
        stabilized); TM: e = (lambda, E_z), h = (lambda, H_t); TE: e = (lambda, E_t),
        h = (lambda, H_z)."""
        torch = _torch()
        ph = np.ascontiguousarray(np.atleast_1d(phis), dtype=np.float64)
        e = torch.empty((len(ph), self.n), dtype=torch.complex128, device=self.device)
        hv = torch.empty_like(e)
        bp = torch.empty_like(e) if stabilized else None
        _check(lib().efie_bie2d_rhs(self._h, ph.ctypes.data, len(ph), float(eta), _ptr(e), _ptr(hv),
                                    _ptr(bp) if bp is not None else None, _stream(self.device)))
        return e, hv, bp

    def skeleton(self, omega, tol: float = 1e-4):
        """Randomized skeleton of C_p - C_p,c with the test matrix omega (rows:
        (ncols, n) complex128 device tensor); returns (rank, est, ref)."""
        omega = self._vec(omega, "omega")
        r, est, ref = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        _check(lib().efie_bie2d_skeleton(self._h, _ptr(omega), omega.shape[0], float(tol), ctypes.byref(r),
                                         ctypes.byref(est), ctypes.byref(ref), _stream(self.device)))
        self.rank = r.value
        return r.value, est.value, ref.value

    def solve(self, B):
        """X = C_p^-1 B (rows) by the Woodbury formula around the counterpart."""
        torch = _torch()
        B = self._vec(B, "B")
        X = torch.empty_like(B)
        _check(lib().efie_bie2d_solve(self._h, _ptr(B), _ptr(X), B.shape[0], _stream(self.device)))
        return X

    def factors(self):
        """(U, V^T): rank x n rows each."""
        torch = _torch()
        U = torch.empty((self.rank, self.n), dtype=torch.complex128, device=self.device)
        Vt = torch.empty_like(U)
        _check(lib().efie_bie2d_factors(self._h, _ptr(U), _ptr(Vt), _stream(self.device)))
        return U, Vt

    def counterpart(self):
        """First columns of C_p,c and of its inverse."""
        torch = _torch()
        c = torch.empty(self.n, dtype=torch.complex128, device=self.device)
        ci = torch.empty_like(c)
        _check(lib().efie_bie2d_counterpart(self._h, _ptr(c), _ptr(ci), _stream(self.device)))
        return c, ci

    def farfield(self, k: float, J, phis, pol: str | None = None):
        """F (nrhs, nphi) at observation angles phis: TM int J exp(j k rhat . r) dS,
        TE int (rhat . n) J exp(j k rhat . r) dS (pol defaults to the setup's, else TM)."""
        torch = _torch()
        pol = pol or getattr(self, "pol", "TM")
        if pol not in ("TM", "TE"):
            raise ValueError("pol must be TM or TE")
        J = self._vec(J, "J")
        ph = torch.as_tensor(np.atleast_1d(phis), dtype=torch.float64, device=self.device).contiguous()
        F = torch.empty((J.shape[0], ph.numel()), dtype=torch.complex128, device=self.device)
        _check(lib().efie_bie2d_farfield(self._h, 0 if pol == "TM" else 1, float(k), _ptr(J), J.shape[0], _ptr(ph),
                                         ph.numel(), _ptr(F), _stream(self.device)))
        return F

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.efie_bie2d_destroy(h)
            self._h = None
