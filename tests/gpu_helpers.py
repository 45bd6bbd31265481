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
        self._red = {}

    def reduced(self, scheme):
        """The oracle's reduced operator for scheme ("std", "lmdg", "rlmdg"), built once."""
        if scheme not in self._red:
            if scheme == "std":
                self._red[scheme] = S.StdReduced(self.prob)
            else:
                self._red[scheme] = S.LowMemoryReduced(self.prob, scheme == "rlmdg")
        return self._red[scheme]

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


def oracle_sweep(case, scheme, x_abi, use_q):
    """Per-cell reductions of one sweep in the ABI layout, from the oracle's matrices."""
    prob = case.prob
    nc = case.ncell
    if scheme == "std":
        red = case.reduced("std")
        phi = abi_to_std(x_abi, nc)
        src = prob.Mu @ phi
        rhs = np.broadcast_to(src, (prob.n_dir, src.size)) + (prob.Qu if use_q else 0.0)
        psi = red.Linv(rhs)                       # (n_dir, nc*4) cell-major
        out = std_to_abi(prob.w @ psi, nc)
        psi_abi = psi.reshape(prob.n_dir, nc, 4).transpose(0, 2, 1).ravel()
        return out, psi_abi
    red = case.reduced(scheme)
    x = abi_to_lm(x_abi, nc)
    rhs = red.M0 @ x[:nc] + red.L01 @ (red.St @ x[nc:])
    if use_q:
        rhs = rhs + red.Qt0
    psi = red.Lt00_lu.solve(rhs)
    p0 = red.P0 @ psi
    if scheme == "rlmdg":
        # second block row G = Sigma (L_10 + L_11 R) - Sigma M_1 P_1 R of Sec. 3.3.2 (corrected)
        g = red.G @ psi
        pr = (red.P1 @ (red.R @ psi)).reshape(nc, 3)
    else:
        g = red.S @ (red.L10 @ psi)
    g = g.reshape(nc, 3)
    rows = [p0, g[:, 0], g[:, 1], g[:, 2]]
    if scheme == "rlmdg":
        rows += [pr[:, 0], pr[:, 1]]
    return np.concatenate(rows), psi
