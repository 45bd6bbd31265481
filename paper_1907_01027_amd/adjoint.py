"""Detector response J(sigma_s, sigma_a, q) as a differentiable torch function.

The forward pass runs ``lmdg_adjoint_solve`` (forward solve, adjoint solve and the
gradient reduction all happen in the HIP library); the backward pass scales the
stored gradients by the incoming gradient.  Also provides the detector moments of
an axis-aligned box, the input that defines J = int_box phi_h dx.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lmdg


def box_detector_moments(n, length, lo, hi) -> np.ndarray:
    """det[r, p] = int_{K_p cap box} b_r dx for the Legendre basis b = (1, xi, eta, xi*eta).

    On one axis, with xi = 2 (x - x_c) / h mapping the cell to [-1, 1] and [a, b] the
    part of the cell inside the box (in xi), int 1 dx = (h/2)(b - a) and
    int xi dx = (h/4)(b^2 - a^2); the 2D integrals are products of these.
    Returned moment-major, shape (4, n_x * n_y), x fastest.
    """
    fac = []
    for a in range(2):
        h = length[a] / n[a]
        c = (np.arange(n[a]) + 0.5) * h
        lo_x = np.clip((lo[a] - c) / (h / 2), -1.0, 1.0)
        hi_x = np.clip((hi[a] - c) / (h / 2), -1.0, 1.0)
        hi_x = np.maximum(hi_x, lo_x)
        i0 = (h / 2) * (hi_x - lo_x)
        i1 = (h / 4) * (hi_x ** 2 - lo_x ** 2)
        fac.append((i0, i1))
    (x0, x1), (y0, y1) = fac
    out = np.empty((4, n[1], n[0]))
    out[0] = y0[:, None] * x0[None, :]
    out[1] = y0[:, None] * x1[None, :]
    out[2] = y1[:, None] * x0[None, :]
    out[3] = y1[:, None] * x1[None, :]
    return out.reshape(4, -1)


class DetectorResponse(torch.autograd.Function):
    """J = int phi_h d for per-cell sigma_s, sigma_a, q (CUDA float64 tensors)."""

    @staticmethod
    def forward(ctx, sigma_s, sigma_a, q, solver, eps, det, scheme="lmdg", mode="fp64", tol=1e-12,
                restart=60, max_iter=100000):
        sigma_s, sigma_a, q = (t.detach().contiguous() for t in (sigma_s, sigma_a, q))
        lmdg.lmdg_set_materials(solver.h, sigma_s, sigma_a, eps, q)
        g = [torch.empty_like(sigma_s) for _ in range(3)]
        J, info = lmdg.lmdg_adjoint_solve(solver.h, scheme, mode, det, tol, restart, max_iter, g[0], g[1], g[2])
        ctx.save_for_backward(*g)
        ctx.info = info
        return torch.tensor(J, dtype=torch.float64, device=sigma_s.device)

    @staticmethod
    def backward(ctx, grad_out):
        gs, ga, gq = ctx.saved_tensors
        return (grad_out * gs, grad_out * ga, grad_out * gq) + (None,) * 8


def detector_response(solver, sigma_s, sigma_a, q, eps, det, **kw):
    """Differentiable J; keyword arguments as DetectorResponse.forward."""
    return DetectorResponse.apply(sigma_s, sigma_a, q, solver, eps, det, kw.get("scheme", "lmdg"),
                                  kw.get("mode", "fp64"), kw.get("tol", 1e-12), kw.get("restart", 60),
                                  kw.get("max_iter", 100000))
