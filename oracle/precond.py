"""Two-level preconditioner of the reduced low-memory systems (oracle; test infrastructure).

The paper leaves preconditioning of the dimension-reduced system open (Sec. 5, future
work (ii)) and gives the eps -> 0 limit of the low-memory scheme in Sec. 3.1: continuous
Q^1 functions with cell-averaged gradients, eq-difflimPF (case 3 of the limit analysis).
This module defines, plainly, the preconditioner the GPU library applies, for the 2D
LMDG and RLMDG reduced systems K X = b of eq-nonrec-block (X = [X_0 ; X_1], X_1 cell-major
(xi, eta, xi eta) here):

    M^{-1} r = K_loc^{-1} r + Z B^{-1} W r      (used on the right: K M^{-1} u = b, X = M^{-1} u)

Why this form.  K e = r is the reduced system of the full scheme whose source is the
residual: the isotropic source M_0 r_0 in the cell-average rows and -r_1 in the slope rows
(Steps 1-3 of Sec. 3.2 read backwards).  Its solution is e = [r_0 + phi_0 ; -phi_1]
(LMDG) or [r_0 + phi_0 ; -phi_1 + P_1 R Psi_0] (RLMDG), phi the scalar flux of that
problem.  In diffusive regimes phi is close to the eq-difflimPF solution with the same
source, which Z B^{-1} W returns; the cell blocks K_loc^{-1} take the part that no
continuous field carries.

Parts (each one a plain definition):

* K_loc: for every cell, the 4 x 4 diagonal block of K, rows and columns (X_0, X_1) of that
  cell.  It is formed from the cell-diagonal entries of the assembled blocks,
      K_loc = diag(1, B_11|_KK) - sum_l [P_0 ; G]_{K,(l,K)} [L~_00]_{(l,K),(l,K)}^{-1} [M_0, L_01 Sigma^T]_{(l,K),K},
  which is the exact diagonal block of K: L~_00 is triangular in the upwind order (its
  inverse has the reciprocal diagonal), and neither P_0 nor G reads angular fluxes
  downwind of a cell.
* W: the residual as a source: cell-wise Legendre moments
      s_0 = (sigma_s/eps) r_0,  s_m = -r_m / (|K| n_m)  (n = 1/3, 1/3, 1/9 for xi, eta, xi eta),
  loaded onto the nodal Q^1 functions, f_c = sum_K int_K s N_c dx (Gauss quadrature).
* B: the eq-difflimPF form on nodal Q^1 functions, with the coefficient 1/(3 sigma_t)
  (sigma_t = sigma_s/eps + eps sigma_a, the total cross section of the scaled equation,
  which tends to sigma_s/eps as eps -> 0) and absorption eps sigma_a, plus a vacuum
  (Marshak) term 1/2 int_{dD} u v on the boundary of D.  Reading (not in the paper): the
  absorption and boundary matrices are lumped (row sums on the diagonal).  With
  a = u_NE - u_SW and b = u_SE - u_NW the cell-averaged gradient energy of a cell is
  D |K| [(a^2 + b^2)(1/(4 h_x^2) + 1/(4 h_y^2)) + 2 a b (1/(4 h_x^2) - 1/(4 h_y^2))];
  the second term (zero on square cells) couples nodes of unlike parity of i + j and is
  left out of B (reading, not in the paper), so B is two independent systems, one per
  parity class.
* Z: nodal u -> its cell Legendre moments (exact L^2 projection), mapped to reduced
  unknowns [m_0 ; -m_slopes]; for RLMDG the angular average of the reconstructed slopes of
  the isotropic cell averages, P_1 R (1 (x) m_0), is added to the slope part (the reduced
  unknown is -Phi_1 + P_1 R Psi_0 there, Step 4 of Sec. 3.3.2 as corrected).

B is solved directly here.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .dg import Mesh, eval_basis, tensor_rule
from .diffusion import _nodal, _node_index, nodal_to_legendre
from .schemes import LowMemoryReduced, Problem

SLOPE_NORMS = np.array([1.0 / 3.0, 1.0 / 3.0, 1.0 / 9.0])   # int_K b_m^2 / |K| for xi, eta, xi eta


def cell_blocks(red: LowMemoryReduced):
    """K_loc: (n_x, 4, 4), rows/cols (X_0, X_1 xi, eta, xi eta) of each cell."""
    prob = red.prob
    nx, nd = prob.mesh.n_cells, prob.n_dir
    if prob.mesh.dim != 2:
        raise ValueError("2D only")
    Lt = red.Lt00.tocsr()
    L01St = (red.L01 @ red.St).tocsr()
    G = red.G.tocsc()
    B11 = red.B11.tocsr()
    P0 = red.P0.tocsc()
    M0 = red.M0.tocsr()
    cells = np.arange(nx)
    blocks = np.zeros((nx, 4, 4))
    blocks[:, 0, 0] = 1.0
    for m in range(3):
        for k in range(3):
            blocks[:, 1 + m, 1 + k] = np.asarray(B11[cells * 3 + m, cells * 3 + k]).ravel()
    for l in range(nd):
        rows = l * nx + cells
        a = np.asarray(Lt[rows, rows]).ravel()
        left = np.stack([np.asarray(P0[cells, rows]).ravel()]
                        + [np.asarray(G[cells * 3 + m, rows]).ravel() for m in range(3)], axis=1)
        right = np.stack([np.asarray(M0[rows, cells]).ravel()]
                         + [np.asarray(L01St[rows, cells * 3 + k]).ravel() for k in range(3)], axis=1)
        blocks -= (left / a[:, None])[:, :, None] * right[:, None, :]
    return blocks


def diffusion_matrix(mesh: Mesh, d_coef, absorb, lumped=True):
    """B on all (n_x+1)(n_y+1) nodes: int D Pi_0 grad u . Pi_0 grad v (eq-difflimPF with the
    per-cell coefficient D) without its couplings between nodes of unlike i + j parity,
    int absorb u v and 1/2 int_{dD} u v, the last two lumped.
    Returns (B, node index of the 4 corners of every cell)."""
    d = mesh.dim
    pts, wts = tensor_rule(d, 3)
    _, val, grad_ref = _nodal(d, pts)
    grad = grad_ref * (2.0 / mesh.h)[None, None, :]
    jac = mesh.volume / 2 ** d
    gbar = jac * np.einsum("q,qcm->cm", wts, grad) / mesh.volume     # Pi_0 grad N_c
    stiff = mesh.volume * gbar @ gbar.T
    mass = jac * np.einsum("q,qa,qb->ab", wts, val, val)
    idx, nn = _node_index(mesh)
    d_coef = np.broadcast_to(np.asarray(d_coef, float), (mesh.n_cells,))
    absorb = np.broadcast_to(np.asarray(absorb, float), (mesh.n_cells,))
    rows = np.repeat(idx, 4, axis=1).ravel()
    cols = np.tile(idx, (1, 4)).ravel()
    S = sp.csr_matrix(((d_coef[:, None, None] * stiff[None]).ravel(), (rows, cols)), shape=(nn, nn)).tocoo()
    nnx = mesh.n[0] + 1
    parity = (np.arange(nn) % nnx + np.arange(nn) // nnx) % 2
    keep = parity[S.row] == parity[S.col]
    S = sp.csr_matrix((S.data[keep], (S.row[keep], S.col[keep])), shape=(nn, nn))
    Mm = sp.csr_matrix(((absorb[:, None, None] * mass[None]).ravel(), (rows, cols)), shape=(nn, nn))
    # boundary term: 1/2 int over boundary edges of u v (two-point Gauss on each edge)
    ge, gw = np.polynomial.legendre.leggauss(2)
    phi = np.stack([(1 - ge) / 2, (1 + ge) / 2], axis=1)             # end-point hat functions
    edge = np.einsum("q,qa,qb->ab", gw / 2, phi, phi)                  # on a unit-length edge
    brow, bcol, bval = [], [], []
    for axis in range(2):
        other = 1 - axis
        for side in (0, mesh.n[axis]):
            k = np.arange(mesh.n[other])
            if axis == 0:
                a, b = side + nnx * k, side + nnx * (k + 1)
            else:
                a, b = k + nnx * side, k + 1 + nnx * side
            hlen = mesh.h[other]
            for (p, q_), e in np.ndenumerate(edge):
                ends = (a, b)
                brow.append(ends[p]); bcol.append(ends[q_]); bval.append(np.full(k.size, 0.5 * hlen * e))
    Bd = sp.csr_matrix((np.concatenate(bval), (np.concatenate(brow), np.concatenate(bcol))), shape=(nn, nn))
    if lumped:
        extra = sp.diags(np.asarray((Mm + Bd).sum(axis=1)).ravel())
    else:
        extra = Mm + Bd
    return (S + extra).tocsr(), idx


def load(mesh: Mesh, s, idx, nn):
    """f_c = sum_K int_K s_K N_c (s: (n_x, 4) Legendre moments per cell), Gauss quadrature."""
    pts, wts = tensor_rule(2, 3)
    _, val, _ = _nodal(2, pts)
    leg, _ = eval_basis(2, pts)
    jac = mesh.volume / 4
    cell_load = jac * np.einsum("q,pr,qr,qc->pc", wts, s, leg, val)   # (n_x, 4 corners)
    f = np.zeros(nn)
    np.add.at(f, idx.ravel(), cell_load.ravel())
    return f


class TwoLevel:
    """M^{-1} of the module docstring for one reduced system (LowMemoryReduced)."""

    def __init__(self, red: LowMemoryReduced):
        prob = red.prob
        mesh = prob.mesh
        if mesh.dim != 2:
            raise ValueError("2D only")
        self.red, self.prob, self.mesh = red, prob, mesh
        self.nx = mesh.n_cells
        self.blocks = cell_blocks(red)
        self.blocks_inv = np.linalg.inv(self.blocks)
        d_coef = 1.0 / (3.0 * prob.sigma_t)
        self.B, self.idx = diffusion_matrix(mesh, d_coef, prob.eps * prob.sigma_a)
        self.nn = self.B.shape[0]
        self.B_lu = spla.splu(self.B.tocsc())
        self.P1R = (red.P1 @ red.R).tocsr() if red.rec else None

    def smooth(self, r):
        """K_loc^{-1} r."""
        nx = self.nx
        rc = np.concatenate([r[:nx, None], r[nx:].reshape(nx, 3)], axis=1)
        out = np.einsum("pab,pb->pa", self.blocks_inv, rc)
        return np.concatenate([out[:, 0], out[:, 1:].ravel()])

    def source(self, r):
        """W r as cell Legendre moments of the source (before loading)."""
        nx = self.nx
        s = np.zeros((nx, 4))
        s[:, 0] = self.prob.scat * r[:nx]
        s[:, 1:] = -r[nx:].reshape(nx, 3) / (self.mesh.volume * SLOPE_NORMS)[None, :]
        return s

    def W(self, r):
        return load(self.mesh, self.source(r), self.idx, self.nn)

    def Z(self, u):
        mom = nodal_to_legendre(self.mesh, u, self.idx)
        slopes = -mom[:, 1:]
        if self.P1R is not None:
            slopes = slopes + (self.P1R @ np.tile(mom[:, 0], self.prob.n_dir)).reshape(self.nx, 3)
        return np.concatenate([mom[:, 0], slopes.ravel()])

    def coarse(self, r):
        return self.Z(self.B_lu.solve(self.W(r)))

    def apply(self, r):
        return self.smooth(r) + self.coarse(r)


def solve(red: LowMemoryReduced, tol=1e-12, restart=60, maxiter=2000):
    """Right-preconditioned GMRES from X = 0 on the reduced system; returns (X, iterations)."""
    pc = TwoLevel(red)
    b = red.rhs()
    n = b.size
    op = spla.LinearOperator((n, n), matvec=lambda u: red.apply(pc.apply(u)), dtype=float)
    it = [0]

    def cb(_):
        it[0] += 1
    u, info = spla.gmres(op, b, rtol=tol, atol=0.0, restart=restart, maxiter=maxiter,
                         callback=cb, callback_type="pr_norm")
    if info != 0:
        raise RuntimeError(f"oracle preconditioned GMRES did not converge (info={info})")
    return pc.apply(u), it[0]
