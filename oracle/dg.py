"""Upwind S_N-DG assembly on uniform Cartesian meshes (oracle; test infrastructure).

Follows Sec. 2.1 (Formulation) and Appendix A (Assembly of the matrices):

* Z_1(K) = Q^1(K) on a Cartesian mesh (eq-cV); the basis on each cell is the
  tensor Legendre set b = prod_k P_{a_k}(xi_k), a_k in {0, 1}, ordered
  r = a_x + 2 a_y + 4 a_z (2D: 1, xi, eta, xi*eta).  It is orthogonal and its
  first member is constant, as Sec. 3.2 requires for the low-memory split.
* For direction Omega_l the local form L_{j,K}(u, v) (eq-Ljk) is
      -int_K u Omega.grad v  +  int_dK u_hat Omega.nu v_int  +  int_K sigma_t u v,
  with the upwind trace u_hat taken from the cell the flow comes from and zero
  outside the domain.  Test index = row, trial index = column.
* S_{j,K} (eq-Sjk) factors as M P with M the sigma_s/eps mass (Appendix A) and P
  the weighted angular sum.
* Q_{j,K,alpha}(v) = int_K eps q v_j - int_{dK on boundary} alpha Omega.nu v_j.
  Reading: alpha is data on the inflow part of the boundary only (it is defined on
  Gamma^- in eq-main), so the boundary integral runs over faces with Omega.nu < 0.
* Per-cell eps: eq-main has one constant eps; cells may carry their own eps_K so
  that a multiscale medium can be described (sigma_t = sigma_s/eps + eps sigma_a,
  scattering sigma_s/eps and source eps q are all formed per cell).

Everything is evaluated by tensor Gauss quadrature on the reference cell (three
points per axis integrate the Q^1 x Q^1 products exactly), with no closed forms.
Unknowns are ordered (direction l, cell p, moment r) -> (l * n_x + p) * n_P + r,
cells x-fastest: p = i + n_x (j + n_y k).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from .quadrature import gauss_legendre


class Mesh:
    """Uniform Cartesian mesh of [0, length_0] x ... with n_k cells per axis."""

    def __init__(self, n, length=None):
        self.n = tuple(int(v) for v in n)
        self.dim = len(self.n)
        self.length = tuple(float(v) for v in (length or (1.0,) * self.dim))
        self.h = np.array(self.length) / np.array(self.n)
        self.n_cells = int(np.prod(self.n))
        self.n_p = 2 ** self.dim
        self.volume = float(np.prod(self.h))
        grids = np.meshgrid(*[np.arange(v) for v in self.n], indexing="ij")
        # multi-index of every cell, x fastest in the flat numbering
        self.idx = np.stack([g.transpose(*reversed(range(self.dim))).ravel()
                             for g in grids], axis=1)
        self.centers = (self.idx + 0.5) * self.h

    def flat(self, idx):
        idx = np.asarray(idx)
        p = np.zeros(idx.shape[:-1], dtype=np.int64)
        stride = 1
        for k in range(self.dim):
            p = p + idx[..., k] * stride
            stride *= self.n[k]
        return p

    def neighbor(self, axis, side):
        """Flat index of the neighbour across face (axis, side), -1 outside."""
        nb = self.idx.copy()
        nb[:, axis] += side
        inside = (nb[:, axis] >= 0) & (nb[:, axis] < self.n[axis])
        out = np.full(self.n_cells, -1, dtype=np.int64)
        out[inside] = self.flat(nb[inside])
        return out

    def to_physical(self, p, xi):
        """Map reference points xi (npts, dim) of cell p to physical points."""
        return self.centers[p] + 0.5 * self.h * xi


def basis_exponents(dim):
    return [tuple((r >> k) & 1 for k in range(dim)) for r in range(2 ** dim)]


def eval_basis(dim, xi):
    """Values (npts, n_P) and reference gradients (npts, n_P, dim) at xi."""
    xi = np.atleast_2d(xi)
    exps = basis_exponents(dim)
    val = np.ones((xi.shape[0], len(exps)))
    grad = np.ones((xi.shape[0], len(exps), dim))
    for r, a in enumerate(exps):
        for k in range(dim):
            f = xi[:, k] if a[k] else np.ones(xi.shape[0])
            df = np.ones(xi.shape[0]) if a[k] else np.zeros(xi.shape[0])
            val[:, r] *= f
            for m in range(dim):
                grad[:, r, m] *= df if m == k else f
    return val, grad


def tensor_rule(dim, npts):
    x, w = gauss_legendre(npts)
    pts = np.array(list(itertools.product(x, repeat=dim)))
    wts = np.array([np.prod(c) for c in itertools.product(w, repeat=dim)])
    return pts, wts


def face_rule(dim, axis, side, npts):
    """Gauss points on the reference face xi_axis = side and their weights."""
    pts, wts = tensor_rule(dim - 1, npts) if dim > 1 else (np.zeros((1, 0)), np.ones(1))
    full = np.insert(pts, axis, side, axis=1)
    return full, wts


class ReferenceIntegrals:
    """Cell and face integrals of basis products for one mesh spacing."""

    def __init__(self, mesh, nq=3):
        d = mesh.dim
        h = mesh.h
        jac = np.prod(h / 2.0)
        pts, wts = tensor_rule(d, nq)
        val, grad = eval_basis(d, pts)
        self.mass = jac * np.einsum("q,qr,qs->rs", wts, val, val)
        # int_K b_s d/dx_m b_r  for each axis m (rows r = test, cols s = trial)
        self.deriv = np.stack([jac * (2.0 / h[m]) * np.einsum("q,qr,qs->rs", wts, grad[:, :, m], val)
                               for m in range(d)])
        self.face_own = {}
        self.face_nb = {}
        for axis in range(d):
            fjac = np.prod(np.delete(h, axis) / 2.0) if d > 1 else 1.0
            for side in (-1.0, 1.0):
                fp, fw = face_rule(d, axis, side, nq)
                v_in, _ = eval_basis(d, fp)
                fp_nb = fp.copy()
                fp_nb[:, axis] = -side  # the same physical point seen from the neighbour
                v_nb, _ = eval_basis(d, fp_nb)
                self.face_own[(axis, side)] = fjac * np.einsum("q,qr,qs->rs", fw, v_in, v_in)
                self.face_nb[(axis, side)] = fjac * np.einsum("q,qr,qs->rs", fw, v_in, v_nb)


def assemble_transport(mesh, omega_l, sigma_t, ref=None):
    """Unweighted L_l for one direction (eq-Ljk summed over cells), CSR.

    Rows are test functions (cell p, moment r), columns trial functions.
    """
    ref = ref or ReferenceIntegrals(mesh)
    d, n_p, nx = mesh.dim, mesh.n_p, mesh.n_cells
    stream = -np.einsum("m,mrs->rs", omega_l, ref.deriv)
    local = sigma_t[:, None, None] * ref.mass[None] + stream[None]
    rows, cols, vals = [], [], []
    for axis in range(d):
        for side in (-1.0, 1.0):
            on = omega_l[axis] * side  # Omega . nu on this face of every cell
            if on > 0:  # outflow face: the trace is the cell's own
                local = local + on * ref.face_own[(axis, side)][None]
            elif on < 0:  # inflow face: the trace comes from the neighbour
                nb = mesh.neighbor(axis, int(side))
                has = nb >= 0
                p = np.nonzero(has)[0]
                q = nb[has]
                blk = on * ref.face_nb[(axis, side)]
                rr, ss = np.meshgrid(np.arange(n_p), np.arange(n_p), indexing="ij")
                rows.append((p[:, None, None] * n_p + rr[None]).ravel())
                cols.append((q[:, None, None] * n_p + ss[None]).ravel())
                vals.append(np.broadcast_to(blk, (p.size, n_p, n_p)).ravel())
    rr, ss = np.meshgrid(np.arange(n_p), np.arange(n_p), indexing="ij")
    pp = np.arange(nx)
    rows.append((pp[:, None, None] * n_p + rr[None]).ravel())
    cols.append((pp[:, None, None] * n_p + ss[None]).ravel())
    vals.append(local.ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(nx * n_p, nx * n_p))


def assemble_mass(mesh, coef, ref=None):
    """Block-diagonal int_K coef_K b_r b_s (CSR), coef per cell."""
    ref = ref or ReferenceIntegrals(mesh)
    n_p = mesh.n_p
    blocks = coef[:, None, None] * ref.mass[None]
    return sp.block_diag(list(blocks), format="csr")


def assemble_source(mesh, omega_l, eps, q=None, alpha=None, nq=5):
    """Unweighted Q_{l,K,alpha} moments (n_x * n_P,) for direction Omega_l.

    q: None, per-cell constants (n_x,), or callable q(x, omega) -> values at the
       physical points x (npts, dim) for this direction (manufactured sources
       may depend on Omega).  alpha: None (vacuum) or callable alpha(x, omega).
    """
    d, n_p, nx = mesh.dim, mesh.n_p, mesh.n_cells
    out = np.zeros((nx, n_p))
    pts, wts = tensor_rule(d, nq)
    val, _ = eval_basis(d, pts)
    jac = mesh.volume / 2 ** d
    if q is not None:
        if callable(q):
            for p in range(nx):
                x = mesh.to_physical(p, pts)
                qv = q(x, omega_l)
                out[p] += eps[p] * jac * (wts * qv) @ val
        else:
            q = np.asarray(q, dtype=float)
            out += (eps * q)[:, None] * (jac * (wts @ val))[None]
    if alpha is not None:
        for axis in range(d):
            fjac = np.prod(np.delete(mesh.h, axis) / 2.0) if d > 1 else 1.0
            for side in (-1.0, 1.0):
                on = omega_l[axis] * side
                if on >= 0:
                    continue  # alpha is prescribed on inflow faces only
                fp, fw = face_rule(d, axis, side, nq)
                v_in, _ = eval_basis(d, fp)
                boundary = mesh.neighbor(axis, int(side)) < 0
                for p in np.nonzero(boundary)[0]:
                    x = mesh.to_physical(p, fp)
                    out[p] -= on * fjac * (fw * alpha(x, omega_l)) @ v_in
    return out.ravel()


def cell_average_integral(mesh, coef_fn, nq=5):
    """int_K f for a callable f(x) on every cell (used for error norms)."""
    pts, wts = tensor_rule(mesh.dim, nq)
    jac = mesh.volume / 2 ** mesh.dim
    return np.array([jac * wts @ coef_fn(mesh.to_physical(p, pts)) for p in range(mesh.n_cells)])


def l1_error(mesh, phi_moments, exact_fn, nq=5):
    """int_D |phi_h - phi| dx of a Q^1 field given by Legendre moments (n_x, n_P).

    Reading: the error norm of Sec. 4 is the absolute L^1 norm of the scalar flux.
    """
    pts, wts = tensor_rule(mesh.dim, nq)
    val, _ = eval_basis(mesh.dim, pts)
    jac = mesh.volume / 2 ** mesh.dim
    total = 0.0
    for p in range(mesh.n_cells):
        x = mesh.to_physical(p, pts)
        total += jac * wts @ np.abs(val @ phi_moments[p] - exact_fn(x))
    return total
