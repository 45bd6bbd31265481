"""Thin ctypes binding of the C ABI declared in include/lmdg.h.

Argument marshalling only: every step of the transport path runs in the HIP
library.  Functions keep the ABI's names; tensors are passed as device pointers
(torch CUDA float64 tensors in the moment-major layouts the header documents) and
the stream is torch's current stream.  Importing this module fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblmdg.so")

LMDG_OK = 0
LMDG_INVALID_ARG = 1
LMDG_NOT_CONVERGED = 2
LMDG_NONFINITE = 3
LMDG_HIP_ERROR = 4
LMDG_UNSUPPORTED = 5

SCHEMES = {"std": 0, "lmdg": 1, "rlmdg": 2}
PRECS = {"fp64": 0, "fp32": 1}
MODES = {"fp64": 0, "mixed": 1}
PRECONDS = {"none": 0, "cell": 1, "two-level": 2}

EXPORTED = ["lmdg_status_string", "lmdg_last_error", "lmdg_quadrature_level_symmetric", "lmdg_create",
            "lmdg_destroy", "lmdg_set_materials", "lmdg_set_sources", "lmdg_sweep", "lmdg_apply", "lmdg_rhs",
            "lmdg_recover", "lmdg_solve", "lmdg_set_augment", "lmdg_adjoint_solve", "lmdg_profile",
            "lmdg_sweep_kernel_time", "lmdg_synchronize", "lmdg_set_wait_limit", "lmdg_set_source_moments",
            "lmdg_workspace_bytes", "lmdg_apply_noalloc", "lmdg_set_reconstruction", "lmdg_set_preconditioner",
            "lmdg_precond_apply", "lmdg_set_refinement"]


class LmdgInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("restarts", ctypes.c_int), ("ir_passes", ctypes.c_int),
                ("converged", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("time_total_ms", ctypes.c_double), ("time_apply_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LmdgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_1907_01027_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "lmdg_status_string": (ctypes.c_char_p, [I]),
        "lmdg_last_error": (ctypes.c_char_p, [P]),
        "lmdg_quadrature_level_symmetric": (I, [I, I, I, ctypes.POINTER(I), P, P]),
        "lmdg_create": (I, [I, P, P, I, P, P, ctypes.POINTER(P)]),
        "lmdg_destroy": (None, [P]),
        "lmdg_set_materials": (I, [P, P, P, P, P, P, P]),
        "lmdg_set_sources": (I, [P, I, P, P]),
        "lmdg_sweep": (I, [P, I, I, P, I, P, P, P]),
        "lmdg_apply": (I, [P, I, I, P, P, P]),
        "lmdg_rhs": (I, [P, I, I, P, P]),
        "lmdg_recover": (I, [P, I, I, P, P, P, P]),
        "lmdg_solve": (I, [P, I, I, D, I, I, P, P, P, ctypes.POINTER(LmdgInfo), P]),
        "lmdg_adjoint_solve": (I, [P, I, I, P, D, I, I, P, P, P, ctypes.POINTER(D), ctypes.POINTER(LmdgInfo), P]),
        "lmdg_set_augment": (I, [P, I]),
        "lmdg_set_refinement": (I, [P, D]),
        "lmdg_profile": (I, [P, I]),
        "lmdg_sweep_kernel_time": (I, [P, ctypes.POINTER(D), ctypes.POINTER(I)]),
        "lmdg_synchronize": (I, [P, P]),
        "lmdg_set_wait_limit": (I, [P, ctypes.c_longlong, I]),
        "lmdg_set_source_moments": (I, [P, I, P, P]),
        "lmdg_workspace_bytes": (I, [P, I, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
        "lmdg_apply_noalloc": (I, [P, I, I, P, P, P]),
        "lmdg_set_reconstruction": (I, [P, I, I]),
        "lmdg_set_preconditioner": (I, [P, I, I]),
        "lmdg_precond_apply": (I, [P, I, P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def library():
    return _lib


def _ptr(t):
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        if not t.is_cuda or t.dtype.itemsize != 8 or not t.is_contiguous():
            raise ValueError("expected a contiguous CUDA float64 tensor")
        return ctypes.c_void_p(t.data_ptr())
    return ctypes.c_void_p(int(t))


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(status, handle=None):
    if status != LMDG_OK:
        msg = _lib.lmdg_status_string(status).decode()
        if handle is not None:
            msg += ": " + _lib.lmdg_last_error(handle).decode()
        raise LmdgError(status, msg)


def lmdg_quadrature_level_symmetric(dim: int, order: int):
    """(omega (n_dir, dim), w (n_dir,)) from the library's host generator."""
    cap = order * (order + 2)
    om = np.zeros(cap * dim)
    w = np.zeros(cap)
    n = ctypes.c_int(0)
    st = _lib.lmdg_quadrature_level_symmetric(dim, order, cap, ctypes.byref(n),
                                              om.ctypes.data_as(ctypes.c_void_p), w.ctypes.data_as(ctypes.c_void_p))
    _check(st)
    return om[: n.value * dim].reshape(n.value, dim).copy(), w[: n.value].copy()


def _init_torch_device():
    """Let torch bring up the HIP runtime first: the library shares torch's runtime
    (same soname), and torch's lazy device initialisation must run before any other
    HIP call in the process."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def lmdg_create(n, length, omega, w):
    _init_torch_device()
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    dim = len(n)
    nn = (ctypes.c_int64 * 3)(*([int(v) for v in n] + [1] * (3 - dim)))
    ll = (ctypes.c_double * 3)(*([float(v) for v in length] + [1.0] * (3 - dim)))
    h = ctypes.c_void_p()
    st = _lib.lmdg_create(dim, nn, ll, int(w.size), omega.ctypes.data_as(ctypes.c_void_p),
                          w.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h))
    _check(st)
    return h


def lmdg_destroy(h):
    _lib.lmdg_destroy(h)


def lmdg_set_materials(h, sigma_s, sigma_a, eps, q, alpha=None, stream=None):
    _check(_lib.lmdg_set_materials(h, _ptr(sigma_s), _ptr(sigma_a), _ptr(eps), _ptr(q), _ptr(alpha),
                                   _stream(stream)), h)


def lmdg_set_source_moments(h, qm, per_direction=False, stream=None):
    """qm: CUDA float64 tensor of cell moments, (4, n_cells) isotropic or (n_dir, 4, n_cells)."""
    _check(_lib.lmdg_set_source_moments(h, int(bool(per_direction)), _ptr(qm), _stream(stream)), h)


def lmdg_workspace_bytes(h, restart):
    """(bytes held by the handle, bytes a solve with this restart would add)."""
    held = ctypes.c_int64(0)
    solve = ctypes.c_int64(0)
    _check(_lib.lmdg_workspace_bytes(h, int(restart), ctypes.byref(held), ctypes.byref(solve)), h)
    return held.value, solve.value


def lmdg_set_sources(h, q, stream=None):
    """q: CUDA float64 tensor (n_rhs, n_cells) or (n_cells,); sets the handle's right-hand sides."""
    n_rhs = 1 if q.dim() == 1 else int(q.shape[0])
    _check(_lib.lmdg_set_sources(h, n_rhs, _ptr(q), _stream(stream)), h)


def lmdg_sweep(h, scheme, prec, x, use_q, out, psi=None, stream=None):
    _check(_lib.lmdg_sweep(h, SCHEMES[scheme], PRECS[prec], _ptr(x), int(bool(use_q)), _ptr(out), _ptr(psi),
                           _stream(stream)), h)


def lmdg_apply(h, scheme, prec, x, y, stream=None):
    _check(_lib.lmdg_apply(h, SCHEMES[scheme], PRECS[prec], _ptr(x), _ptr(y), _stream(stream)), h)


def lmdg_apply_noalloc(h, scheme, prec, x, y, stream=None):
    """K x with the library's fixed per-GPU workspace (no allocation)."""
    _check(_lib.lmdg_apply_noalloc(h, SCHEMES[scheme], PRECS[prec], _ptr(x), _ptr(y), _stream(stream)), h)


def lmdg_rhs(h, scheme, prec, b, stream=None):
    _check(_lib.lmdg_rhs(h, SCHEMES[scheme], PRECS[prec], _ptr(b), _stream(stream)), h)


def lmdg_recover(h, scheme, prec, x, phi, psi=None, stream=None):
    _check(_lib.lmdg_recover(h, SCHEMES[scheme], PRECS[prec], _ptr(x), _ptr(phi), _ptr(psi), _stream(stream)), h)


def lmdg_solve(h, scheme, mode, tol, restart, max_iter, x_out, phi_out=None, x0=None, stream=None,
               raise_on_nonconvergence=True):
    info = LmdgInfo()
    st = _lib.lmdg_solve(h, SCHEMES[scheme], MODES[mode], float(tol), int(restart), int(max_iter), _ptr(x0),
                         _ptr(x_out), _ptr(phi_out), ctypes.byref(info), _stream(stream))
    if st == LMDG_NOT_CONVERGED and not raise_on_nonconvergence:
        return info.as_dict()
    _check(st, h)
    return info.as_dict()


def lmdg_adjoint_solve(h, scheme, mode, det, tol, restart, max_iter, g_sigma_s, g_sigma_a, g_q, stream=None):
    """J and the gradients (written into g_*) for detector moments det; returns (J, info)."""
    info = LmdgInfo()
    J = ctypes.c_double(0)
    _check(_lib.lmdg_adjoint_solve(h, SCHEMES[scheme], MODES[mode], _ptr(det), float(tol), int(restart),
                                   int(max_iter), _ptr(g_sigma_s), _ptr(g_sigma_a), _ptr(g_q), ctypes.byref(J),
                                   ctypes.byref(info), _stream(stream)), h)
    return J.value, info.as_dict()


def lmdg_set_reconstruction(h, stencil=2, suppress=False):
    """RLMDG reconstruction variant: stencil 2 (default) or 3 (RLMDG*), suppression at jumps."""
    _check(_lib.lmdg_set_reconstruction(h, int(stencil), int(bool(suppress))), h)


def lmdg_set_preconditioner(h, kind="two-level", cycles=1):
    _check(_lib.lmdg_set_preconditioner(h, PRECONDS[kind], int(cycles)), h)


def lmdg_precond_apply(h, scheme, r, z, stream=None):
    _check(_lib.lmdg_precond_apply(h, SCHEMES[scheme], _ptr(r), _ptr(z), _stream(stream)), h)


def lmdg_set_augment(h, k):
    """Number of earlier restart corrections each GMRES cycle also searches (LGMRES); 0 = plain GMRES."""
    _check(_lib.lmdg_set_augment(h, int(k)), h)


def lmdg_set_refinement(h, inner_tol):
    """Residual reduction each inner FP32 solve of mode "mixed" aims for (default 1e-3)."""
    _check(_lib.lmdg_set_refinement(h, float(inner_tol)), h)


def lmdg_profile(h, enable):
    _check(_lib.lmdg_profile(h, int(bool(enable))), h)


def lmdg_sweep_kernel_time(h):
    """(summed sweep-kernel milliseconds, launches) since the last query."""
    ms = ctypes.c_double(0)
    n = ctypes.c_int(0)
    _check(_lib.lmdg_sweep_kernel_time(h, ctypes.byref(ms), ctypes.byref(n)), h)
    return ms.value, n.value


def lmdg_synchronize(h, stream=None):
    """Wait for the handle's work; raises LmdgError if a sweep wait gave up."""
    _check(_lib.lmdg_synchronize(h, _stream(stream)), h)


def lmdg_set_wait_limit(h, spins, unreachable=False):
    """Bounded-wait policy of the sweeps (failure-handling tests)."""
    _check(_lib.lmdg_set_wait_limit(h, int(spins), int(bool(unreachable))), h)


class Solver:
    """Owning wrapper of one handle (mesh + quadrature + materials)."""

    def __init__(self, n, length, omega, w):
        self.n = tuple(int(v) for v in n)
        self.ncell = int(np.prod(self.n))
        self.ndir = len(w)
        self.h = lmdg_create(n, length, omega, w)

    def close(self):
        if self.h is not None:
            lmdg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
