"""Seeded synthetic inputs for the benchmark workloads (no transport arithmetic).

The paper's experiments are analytic and use no dataset; the workloads below are
synthetic media of the shapes the benchmark names, drawn with numpy's PCG64 from
the seed 20190701 + k (k = workload number).  Draw order: sigma_s block values,
sigma_a block values (row-major, x fastest), then the per-cell sources (one field
per right-hand side).  Arrays are float64, cells x fastest.  The same arrays are
handed to the GPU library and to the CPU oracle.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 20190701


@dataclass(frozen=True)
class Workload:
    key: int
    name: str
    dim: int
    n: tuple
    order: int            # level-symmetric S_N order
    scheme: str           # "std", "lmdg" or "rlmdg"
    eps: object           # float, or ("split", left, right) at x = 0.5
    sigma: object         # float (constant) or (lo, hi) uniform on an 8 x 8 block grid
    q_range: tuple = (0.0, 1.0)
    q_const: float = None
    n_rhs: int = 1
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    1: Workload(1, "unit square 20x20, S4, eps=1, sigma_s=sigma_a=q=1", 2, (20, 20), 4, "lmdg", 1.0, 1.0,
                q_const=1.0, extra={"schemes": ("std", "lmdg"), "tol": 1e-10}),
    2: Workload(2, "256x256, S8, eps=1e-3, 8x8 block cross sections U[0.5,2], q U[0,1], RLMDG", 2, (256, 256),
                8, "rlmdg", 1e-3, (0.5, 2.0)),
    3: Workload(3, "1024x1024, S16, eps 1 | 1e-4 at x = 0.5, 8x8 blocks U[0.1,10], q U[0,1], RLMDG mixed", 2,
                (1024, 1024), 16, "rlmdg", ("split", 1.0, 1e-4), (0.1, 10.0)),
    4: Workload(4, "512x512, S12, eps=1e-2, 8x8 blocks U[0.5,2], q U[0,1], LMDG adjoint", 2, (512, 512), 12,
                "lmdg", 1e-2, (0.5, 2.0), extra={"detector": ((0.7, 0.7), (0.9, 0.9))}),
    5: Workload(5, "128^3, 3D S8, eps=1, sigma=1, 8 sources U[0,1], RLMDG", 3, (128, 128, 128), 8, "rlmdg",
                1.0, 1.0, n_rhs=8),
}


def _blocks(rng, n, nb, lo, hi):
    """Values on an nb x nb (x nb) block grid expanded to cells (x fastest)."""
    dim = len(n)
    vals = rng.uniform(lo, hi, size=nb ** dim)
    idx = [np.minimum((np.arange(n[k]) * nb) // n[k], nb - 1) for k in range(dim)]
    if dim == 2:
        bi = idx[0][None, :] + nb * idx[1][:, None]
    else:
        bi = idx[0][None, None, :] + nb * (idx[1][None, :, None] + nb * idx[2][:, None, None])
    return vals[bi].ravel()


def materials(key: int, n=None, seed=None):
    """(sigma_s, sigma_a, eps, q) for workload `key`; n overrides the mesh (same recipe).

    q has shape (n_rhs, n_cells).
    """
    wl = WORKLOADS[key]
    n = tuple(n or wl.n)
    rng = np.random.default_rng(SEED_BASE + key if seed is None else seed)
    ncell = int(np.prod(n))
    if isinstance(wl.sigma, tuple):
        ss = _blocks(rng, n, 8, *wl.sigma)
        sa = _blocks(rng, n, 8, *wl.sigma)
    else:
        ss = np.full(ncell, float(wl.sigma))
        sa = np.full(ncell, float(wl.sigma))
    if isinstance(wl.eps, tuple):
        _, left, right = wl.eps
        xc = (np.arange(n[0]) + 0.5) / n[0]
        row = np.where(xc < 0.5, left, right)
        eps = np.tile(row, ncell // n[0])
    else:
        eps = np.full(ncell, float(wl.eps))
    if wl.q_const is not None:
        q = np.full((wl.n_rhs, ncell), float(wl.q_const))
    else:
        q = rng.uniform(*wl.q_range, size=(wl.n_rhs, ncell))
    return ss, sa, eps, q
