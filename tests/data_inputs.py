"""Input preparation for the tests with source and inflow data (no transport arithmetic).

The library takes a source through its cell moments and inflow data through face
moments (include/lmdg.h); the oracle takes the same data as functions and integrates
them itself.  These helpers project analytic data onto what the library takes, with
tensor Gauss rules: cell moments (1/|K|) int_K f b_r (b = 1, xi, eta, xi eta), and per
inflow face the average, the linear Legendre coefficient along the face and the
midpoint value.
"""
from __future__ import annotations

import numpy as np

_X, _W = np.polynomial.legendre.leggauss(6)


def cell_moments_2d(n, length, f):
    """(4, n_x n_y) cell moments of f(points (m, 2)) on the uniform mesh, cells x fastest."""
    nx, ny = n
    hx, hy = length[0] / nx, length[1] / ny
    xi, eta = np.meshgrid(_X, _X, indexing="ij")
    wq = np.outer(_W, _W).ravel() / 4.0          # reference-cell average
    xi, eta = xi.ravel(), eta.ravel()
    basis = np.stack([np.ones_like(xi), xi, eta, xi * eta])      # (4, q)
    ic, jc = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    xc = ((ic.ravel() + 0.5) * hx)[:, None] + 0.5 * hx * xi[None]
    yc = ((jc.ravel() + 0.5) * hy)[:, None] + 0.5 * hy * eta[None]
    vals = f(np.stack([xc.ravel(), yc.ravel()], axis=1)).reshape(nx * ny, -1)
    return np.einsum("pq,rq,q->rp", vals, basis, wq)


def cell_moments_1d(n, length, f):
    """(4, n) moments for a slab handle: rows 0, 1 the 1D Legendre moments, rows 2, 3 zero."""
    h = length / n
    xs = ((np.arange(n) + 0.5) * h)[:, None] + 0.5 * h * _X[None]
    vals = f(xs.reshape(-1, 1)).reshape(n, -1)
    out = np.zeros((4, n))
    out[0] = vals @ (_W / 2.0)
    out[1] = vals @ (_W * _X / 2.0)
    return out


def direction_moments_2d(n, length, omega, q):
    """(n_dir, 4, n_cells) cell moments of q(points, omega_l) for every direction."""
    return np.stack([cell_moments_2d(n, length, lambda x, o=o: q(x, o)) for o in omega])


def direction_moments_1d(n, length, mu, q):
    return np.stack([cell_moments_1d(n, length, lambda x, o=np.array([m]): q(x, o)) for m in mu])


def inflow_faces_2d(n, length, omega, alpha):
    """(n_dir, n_y + n_x, 3): per direction the x-inflow faces of the rows, then the
    y-inflow faces of the columns, each (average, linear coefficient, midpoint value)."""
    nx, ny = n
    hx, hy = length[0] / nx, length[1] / ny
    out = np.zeros((len(omega), ny + nx, 3))
    for l, o in enumerate(omega):
        xb = 0.0 if o[0] > 0 else length[0]
        yb = 0.0 if o[1] > 0 else length[1]
        # x faces: points along y
        yc = (np.arange(ny) + 0.5) * hy
        pts = np.stack([np.full(ny * _X.size, xb), (yc[:, None] + 0.5 * hy * _X[None]).ravel()], axis=1)
        v = alpha(pts, o).reshape(ny, -1)
        out[l, :ny, 0] = v @ (_W / 2.0)
        out[l, :ny, 1] = 3.0 * (v @ (_W * _X / 2.0))
        out[l, :ny, 2] = alpha(np.stack([np.full(ny, xb), yc], axis=1), o)
        xc = (np.arange(nx) + 0.5) * hx
        pts = np.stack([(xc[:, None] + 0.5 * hx * _X[None]).ravel(), np.full(nx * _X.size, yb)], axis=1)
        v = alpha(pts, o).reshape(nx, -1)
        out[l, ny:, 0] = v @ (_W / 2.0)
        out[l, ny:, 1] = 3.0 * (v @ (_W * _X / 2.0))
        out[l, ny:, 2] = alpha(np.stack([xc, np.full(nx, yb)], axis=1), o)
    return out


def inflow_points_1d(length, mu, alpha):
    """(n_dir,) alpha at the inflow end of each slab direction."""
    return np.array([alpha(np.array([[0.0 if m > 0 else length]]), np.array([m]))[0] for m in mu])
