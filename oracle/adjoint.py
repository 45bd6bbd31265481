"""Adjoint solves and gradients of a detector functional (oracle; test infrastructure).

The paper does not treat sensitivities; the quantities here are defined from its
variational forms.  For a scheme  B(psi_h, v) = Q_alpha(v)  (eq-sndg-scheme,
eq-gene-scheme) on trial = test space W_h, and the functional
    J(psi_h) = int_D phi_h d(x) dx  (phi_h = scalar flux, d = detector weight),
the adjoint lambda_h in W_h solves  B(u, lambda_h) = J(u) for all u in W_h, and
    dJ/dtheta = Q_theta(lambda_h) - B_theta(psi_h, lambda_h).
Algebraically, with A y = b the assembled system and j = dJ/dy,
    A^T lambda = j,    dJ/dtheta = lambda . (db/dtheta - dA/dtheta y).
The derivative matrices are assembled by the same Gauss assembly with unit
per-cell coefficients, so no closed forms enter.

RLMDG is Petrov-Galerkin (eq-rlmdg-vari): trial functions Psi = T_R y + t_alpha carry
the upwind reconstruction, test functions T z do not, A = T^T (L - M P) T_R.  Its
adjoint is the transpose of that system, A^T lambda = j, whose solution lives in the
test space: the adjoint field is T lambda (per-direction cell constants plus isotropic
slopes), and dJ/dtheta = (T lambda) . (dQ/dtheta - dB/dtheta Psi) with the forward
field Psi including its reconstructed slopes.  The reconstruction itself does not depend
on the cross sections (the variant that suppresses it at cross-section jumps is only
piecewise differentiable and is not covered).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .dg import Mesh, assemble_mass, assemble_source, assemble_transport, eval_basis, tensor_rule
from .schemes import Problem, lm_trial_map, rlm_trial_map


def detector_moments(mesh: Mesh, lo, hi, nq=4):
    """d[K, r] = int_{K cap box} b_r dx for the box [lo, hi] (exact Gauss on the overlap)."""
    d = mesh.dim
    out = np.zeros((mesh.n_cells, mesh.n_p))
    pts, wts = tensor_rule(d, nq)
    for p in range(mesh.n_cells):
        a = np.maximum(mesh.centers[p] - mesh.h / 2, lo)
        b = np.minimum(mesh.centers[p] + mesh.h / 2, hi)
        if np.any(b <= a):
            continue
        x = 0.5 * (a + b) + 0.5 * (b - a) * pts           # points of the overlap box
        xi = (x - mesh.centers[p]) / (mesh.h / 2)          # reference coordinates
        val, _ = eval_basis(d, xi)
        out[p] = np.prod((b - a) / 2) * wts @ val
    return out


def _system(prob: Problem, scheme: str):
    """(A, b, T) with A y = b and Psi = T y for 'std' or 'lmdg'; for 'rlmdg' T is the
    test map and the trial field is given by _trial_field."""
    B = prob.L() - prob.M() @ prob.P()
    if scheme == "std":
        T = sp.identity(B.shape[0], format="csr")
    elif scheme in ("lmdg", "rlmdg"):
        T = lm_trial_map(prob)
    else:
        raise ValueError(scheme)
    if scheme == "rlmdg":
        TR, t_alpha = rlm_trial_map(prob)
        return (T.T @ B @ TR).tocsc(), T.T @ (prob.Q() - B @ t_alpha), T
    return (T.T @ B @ T).tocsc(), T.T @ prob.Q(), T


def _trial_field(prob: Problem, scheme: str, y, T):
    """Forward angular field (all moments) of the solution y."""
    if scheme == "rlmdg":
        TR, t_alpha = rlm_trial_map(prob)
        return TR @ y + t_alpha
    return T @ y


def functional_vector(prob: Problem, scheme: str, det):
    """j with J = j . y (scalar flux moments against detector moments det (n_x, n_P))."""
    nd = prob.n_dir
    if scheme == "std":
        return np.concatenate([prob.w[l] * det.ravel() for l in range(nd)])
    j0 = np.concatenate([prob.w[l] * det[:, 0] for l in range(nd)])
    return np.concatenate([j0, det[:, 1:].ravel()])


def forward_adjoint(prob: Problem, scheme: str, det):
    A, b, T = _system(prob, scheme)
    y = spla.spsolve(A, b)
    j = functional_vector(prob, scheme, det)
    lam = spla.spsolve(A.T.tocsc(), j)
    return y, lam, float(j @ y), T


def _weighted_blocks(prob: Problem, coef_t, coef_scat):
    """Weighted (L - M P) for given per-cell sigma_t and scattering coefficients."""
    nd = prob.n_dir
    Lw = sp.block_diag([prob.w[l] * assemble_transport(prob.mesh, prob.omega[l], coef_t, prob.ref)
                        for l in range(nd)], format="csr")
    Mu = assemble_mass(prob.mesh, coef_scat, prob.ref)
    M = sp.vstack([prob.w[l] * Mu for l in range(nd)], format="csr")
    return Lw - M @ prob.P()


def gradients(prob: Problem, scheme: str, det):
    """(J, dJ/dsigma_s, dJ/dsigma_a, dJ/dq) for per-cell constant q (prob.q array).

    Derivative of the operator with respect to the cross section of cell K is the
    operator assembled with sigma_t and scattering coefficients nonzero on K only:
    d sigma_t / d sigma_s = 1/eps, d sigma_t / d sigma_a = eps, d(sigma_s/eps)/d sigma_s = 1/eps.
    The streaming part does not depend on them, so it is removed by differencing
    against the operator with zero coefficients.
    """
    y, lam, J, T = forward_adjoint(prob, scheme, det)
    nx = prob.mesh.n_cells
    zero = _weighted_blocks(prob, np.zeros(nx), np.zeros(nx))
    g_s, g_a, g_q = np.zeros(nx), np.zeros(nx), np.zeros(nx)
    lam_full = T @ lam
    psi_full = _trial_field(prob, scheme, y, T)
    for K in range(nx):
        e = np.zeros(nx)
        e[K] = 1.0
        dA_a = _weighted_blocks(prob, prob.eps * e, np.zeros(nx)) - zero
        dA_s = _weighted_blocks(prob, e / prob.eps, e / prob.eps) - zero
        g_a[K] = -lam_full @ (dA_a @ psi_full)
        g_s[K] = -lam_full @ (dA_s @ psi_full)
        dq = np.concatenate([prob.w[l] * assemble_source(prob.mesh, prob.omega[l], prob.eps, e)
                             for l in range(prob.n_dir)])
        g_q[K] = lam_full @ dq
    return J, g_s, g_a, g_q


def adjoint_flux(prob: Problem, scheme: str, det):
    """Adjoint angular field lambda_h as moments (n_dir, n_x, n_P) and forward Psi."""
    y, lam, J, T = forward_adjoint(prob, scheme, det)
    shape = (prob.n_dir, prob.mesh.n_cells, prob.n_p)
    return _trial_field(prob, scheme, y, T).reshape(shape), (T @ lam).reshape(shape), J
