"""Shared set-up for the GPU parity tests: identical inputs for oracle and library.

Quadrature arrays come from the oracle's generator and are handed to both sides;
materials come from the seeded workload generator.  Layout helpers convert the
oracle's cell-major moment vectors to the ABI's moment-major layout.
"""
from __future__ import annotations

import numpy as np

from oracle import schemes as S
from oracle.dg import Mesh
from oracle.quadrature import level_symmetric
from paper_1907_01027_amd.workloads import materials


class Case:
    def __init__(self, n, order, key=2, eps=None, length=(1.0, 1.0), seed=None):
        self.n = tuple(n)
        self.length = tuple(length)
        self.order = order
        self.omega, self.w = level_symmetric(order, 2)
        ss, sa, ep, q = materials(key, n=self.n, seed=seed)
        if eps is not None:
            ep = np.full_like(ep, eps)
        self.sigma_s, self.sigma_a, self.eps, self.q = ss, sa, ep, q[0]
        self.ncell = self.n[0] * self.n[1]
        self._prob = None

    @property
    def prob(self):
        if self._prob is None:
            self._prob = S.Problem(Mesh(self.n, self.length), self.omega, self.w, self.sigma_s, self.sigma_a,
                                   self.eps, q=self.q)
        return self._prob

    def solver(self):
        import torch
        from paper_1907_01027_amd import lmdg
        s = lmdg.Solver(self.n, self.length, self.omega, self.w)
        dev = torch.device("cuda")
        t = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)
        lmdg.lmdg_set_materials(s.h, t(self.sigma_s), t(self.sigma_a), t(self.eps), t(self.q))
        torch.cuda.synchronize()
        return s


def lm_to_abi(x, ncell):
    """[X0 (n); X1 (n, 3) cell-major] -> moment-major (4 n)."""
    x0 = x[:ncell]
    x1 = x[ncell:].reshape(ncell, 3)
    return np.concatenate([x0, x1[:, 0], x1[:, 1], x1[:, 2]])


def abi_to_lm(v, ncell):
    v = v.reshape(4, ncell)
    return np.concatenate([v[0], v[1:].T.ravel()])


def std_to_abi(phi, ncell):
    return phi.reshape(ncell, 4).T.ravel().copy()


def abi_to_std(v, ncell):
    return v.reshape(4, ncell).T.ravel().copy()


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
