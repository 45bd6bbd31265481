"""Diffusion-limit reference schemes of Sec. 3.1 (oracle; test infrastructure).

As eps -> 0 the S_N-DG solution tends to the solution of a discrete diffusion
problem posed on continuous, piecewise Q^1 functions vanishing on the boundary
(the space C_{h,zero}):

* standard Q^1 S_N-DG (Thm "Asymptotic scheme", and case 2 of Sec. 3.1 with
  piecewise constant cross sections): the classical continuous Galerkin problem
  eq-lmdg-cg,  sum_K int (1/(3 sigma_s)) grad psi . grad phi + sigma_a psi phi = int q phi;
* the low-memory space V_{h,0} + D_{h,1} (case 3 of Sec. 3.1): the same with each
  gradient replaced by its cell average, eq-difflimPF.

Both are assembled here with bilinear Lagrange (nodal) functions and Gauss
quadrature, independently of the transport assembly, and returned as Legendre
moments per cell so they can be compared with transport scalar fluxes.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .dg import Mesh, eval_basis, tensor_rule


def _nodal(dim, xi):
    """Bilinear Lagrange functions of the 2^d corners and their reference gradients."""
    corners = list(itertools.product((-1.0, 1.0), repeat=dim))
    corners = [tuple(reversed(c)) for c in corners]  # x varies fastest
    val = np.ones((xi.shape[0], len(corners)))
    grad = np.ones((xi.shape[0], len(corners), dim))
    for c, cs in enumerate(corners):
        for k in range(dim):
            f = 0.5 * (1.0 + cs[k] * xi[:, k])
            df = 0.5 * cs[k] * np.ones(xi.shape[0])
            val[:, c] *= f
            for m in range(dim):
                grad[:, c, m] *= df if m == k else f
    return np.array(corners), val, grad


def _node_index(mesh: Mesh):
    """Global node numbers of the 2^d corners of every cell (x fastest)."""
    nn = [v + 1 for v in mesh.n]
    corners, _, _ = _nodal(mesh.dim, np.zeros((1, mesh.dim)))
    idx = np.zeros((mesh.n_cells, len(corners)), dtype=np.int64)
    for c, cs in enumerate(corners):
        node = mesh.idx + (np.array(cs) > 0).astype(int)
        flat = np.zeros(mesh.n_cells, dtype=np.int64)
        stride = 1
        for k in range(mesh.dim):
            flat += node[:, k] * stride
            stride *= nn[k]
        idx[:, c] = flat
    return idx, int(np.prod(nn))


def solve_limit(mesh: Mesh, sigma_s, sigma_a, q_fn, projected: bool, nq=4):
    """Nodal Q^1 solution of eq-lmdg-cg (projected=False) or eq-difflimPF (True).

    sigma_s, sigma_a: per-cell constants.  q_fn(x) -> source values.
    Returns (nodal values, Legendre moments per cell (n_x, n_P)).
    """
    d = mesh.dim
    pts, wts = tensor_rule(d, nq)
    _, val, grad_ref = _nodal(d, pts)
    grad = grad_ref * (2.0 / mesh.h)[None, None, :]
    jac = mesh.volume / 2 ** d
    if projected:
        # Pi_0 of the gradient: its cell average, int_K grad N_c / |K|
        gbar = jac * np.einsum("q,qcm->cm", wts, grad) / mesh.volume
        stiff_ref = mesh.volume * gbar @ gbar.T
    else:
        stiff_ref = jac * np.einsum("q,qam,qbm->ab", wts, grad, grad)
    mass_ref = jac * np.einsum("q,qa,qb->ab", wts, val, val)
    idx, n_nodes = _node_index(mesh)
    rows, cols, vals = [], [], []
    rhs = np.zeros(n_nodes)
    ss = np.broadcast_to(np.asarray(sigma_s, float), (mesh.n_cells,))
    sa = np.broadcast_to(np.asarray(sigma_a, float), (mesh.n_cells,))
    for p in range(mesh.n_cells):
        blk = stiff_ref / (3.0 * ss[p]) + sa[p] * mass_ref
        rows.append(np.repeat(idx[p], idx.shape[1]))
        cols.append(np.tile(idx[p], idx.shape[1]))
        vals.append(blk.ravel())
        x = mesh.to_physical(p, pts)
        rhs[idx[p]] += jac * (wts * q_fn(x)) @ val
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n_nodes, n_nodes))
    # zero Dirichlet data: keep interior nodes only
    nn = [v + 1 for v in mesh.n]
    node_multi = np.stack(np.unravel_index(np.arange(n_nodes), tuple(reversed(nn))), axis=1)[:, ::-1]
    interior = np.all((node_multi > 0) & (node_multi < np.array(nn) - 1), axis=1)
    u = np.zeros(n_nodes)
    ii = np.nonzero(interior)[0]
    u[ii] = spla.spsolve(A[ii][:, ii].tocsc(), rhs[ii])
    return u, nodal_to_legendre(mesh, u, idx)


def nodal_to_legendre(mesh: Mesh, u, idx=None):
    """L^2 projection of a nodal Q^1 field onto the cell Legendre basis (exact)."""
    if idx is None:
        idx, _ = _node_index(mesh)
    d = mesh.dim
    pts, wts = tensor_rule(d, 3)
    _, val, _ = _nodal(d, pts)
    leg, _ = eval_basis(d, pts)
    norm = wts @ (leg * leg)
    proj = np.einsum("q,qr,qc->rc", wts, leg, val) / norm[:, None]
    return u[idx] @ proj.T


def assembled_matrix(mesh: Mesh, sigma_s, sigma_a, projected: bool, nq=4):
    """Full nodal matrix (no boundary elimination), for stencil checks."""
    d = mesh.dim
    pts, wts = tensor_rule(d, nq)
    _, val, grad_ref = _nodal(d, pts)
    grad = grad_ref * (2.0 / mesh.h)[None, None, :]
    jac = mesh.volume / 2 ** d
    if projected:
        gbar = jac * np.einsum("q,qcm->cm", wts, grad) / mesh.volume
        stiff_ref = mesh.volume * gbar @ gbar.T
    else:
        stiff_ref = jac * np.einsum("q,qam,qbm->ab", wts, grad, grad)
    mass_ref = jac * np.einsum("q,qa,qb->ab", wts, val, val)
    idx, n_nodes = _node_index(mesh)
    A = sp.lil_matrix((n_nodes, n_nodes))
    for p in range(mesh.n_cells):
        blk = stiff_ref / (3.0 * sigma_s) + sigma_a * mass_ref
        for a in range(idx.shape[1]):
            for b in range(idx.shape[1]):
                A[idx[p, a], idx[p, b]] += blk[a, b]
    return A.tocsr()
