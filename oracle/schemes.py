"""Standard, low-memory and reconstructed S_N-DG systems (oracle; test infrastructure).

What is computed (all FP64, CPU):

STD   (Sec. 2.1, eq-sndg-scheme / eq-sndg-mat): find Psi with (L - M P) Psi = Q,
      L, M, P, Q assembled as in Appendix A, rows weighted by w_l.
LMDG  (Sec. 3.2, eq-gene-scheme / eq-lmdg-block): the same bilinear form with trial
      and test space V^lm = V_{h,0} + D_{h,1}, i.e. Psi = T y with
      y = [Psi_0 ; Phi_1], T = [[I, 0], [0, Sigma^T]], solve T^T (L - M P) T y = T^T Q.
RLMDG (Sec. 3.3, eq-rlmdg-vari / eq-rlmdg-block): trial functions carry the upwind
      reconstruction, Psi_1 = Sigma^T Phi_1 + (I - Sigma^T P_1)(R Psi_0 + r_alpha),
      test space V^lm; solve T^T (L - M P)(T_R y + t_alpha) = T^T Q.

These direct solves are the definition of each scheme.  The module also holds the
paper's own reduced Krylov route (eq-sndg-phi / eq-sndg-final-sweep; Steps 1-4 of
Sec. 3.2 with eq-nonrec-block; Steps 1-4 of Sec. 3.3.2) built from the same
assembled blocks, with L^{-1} applied by a sparse direct factorisation of each
direction's block and GMRES as the Krylov method.

Readings (also listed in the design notes):
* The printed RLMDG reduced operator of Sec. 3.3.2 (Step 3) and its recovery formula
  (Step 4) do not follow from eq-rlmdg-block-tilde.  Multiplying the definition of
  X_1 by B_11 gives the second block row  G = Sigma L~_10 + B_11 P_1 R  (used here in
  both the operator and the right-hand side), and Step 2 gives the recovery
  Phi_1 = c - X_1 + P_1 R Psi_0 with c = B_11^{-1} Sigma Q~_1.  The direct solve above
  is the arbiter; the tests check the reduced route against it.
* Reconstruction (Sec. 3.3.1): the slope along axis k in direction Omega uses the
  one-sided difference from the upwind side (s = -sign(Omega_k)); at the inflow
  boundary cell it uses the value of alpha at the midpoint of the inflow face.
  Only the single-axis linear Legendre modes are reconstructed ("only P^1
  slopes"); cross terms get zero.  The slope delta*(x - x_i) has Legendre
  coefficient delta*h/2 on the basis function xi = 2 (x - x_i)/h.
* The Krylov method (unnamed in the paper) is restarted GMRES from x_0 = 0 with a
  relative residual stopping rule.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .dg import (Mesh, ReferenceIntegrals, assemble_mass, assemble_source,
                 assemble_transport, basis_exponents)


class Problem:
    """Discrete S_N-DG data for one mesh, quadrature and set of cross sections.

    sigma_s, sigma_a, eps: per-cell arrays (scalars are broadcast).
    q: None, per-cell constants, or callable q(x, omega) (may depend on omega).
    alpha: None (vacuum inflow) or callable alpha(x, omega).
    """

    def __init__(self, mesh: Mesh, omega, w, sigma_s, sigma_a, eps=1.0, q=None, alpha=None,
                 reconstruction="two-cell", suppress=False):
        if reconstruction not in ("two-cell", "three-cell"):
            raise ValueError("reconstruction must be 'two-cell' or 'three-cell'")
        self.recon_kind = reconstruction
        self.suppress = bool(suppress)
        self.mesh = mesh
        self.omega = np.asarray(omega, dtype=float)
        self.w = np.asarray(w, dtype=float)
        nx = mesh.n_cells
        self.sigma_s = np.broadcast_to(np.asarray(sigma_s, float), (nx,)).copy()
        self.sigma_a = np.broadcast_to(np.asarray(sigma_a, float), (nx,)).copy()
        self.eps = np.broadcast_to(np.asarray(eps, float), (nx,)).copy()
        self.q = q
        self.alpha = alpha
        self.n_dir = self.omega.shape[0]
        self.n_p = mesh.n_p
        # eq-main: total cross section, scattering coefficient and source scaling
        self.sigma_t = self.sigma_s / self.eps + self.eps * self.sigma_a
        self.scat = self.sigma_s / self.eps
        self.ref = ReferenceIntegrals(mesh)
        self._lu = None
        self._mu = None
        self._qu = None

    # ----- unweighted per-direction blocks (rows divided by w_l) -----
    @property
    def Lu(self):
        if self._lu is None:
            self._lu = [assemble_transport(self.mesh, self.omega[l], self.sigma_t, self.ref)
                        for l in range(self.n_dir)]
        return self._lu

    @property
    def Mu(self):
        if self._mu is None:
            self._mu = assemble_mass(self.mesh, self.scat, self.ref)
        return self._mu

    @property
    def Qu(self):
        if self._qu is None:
            self._qu = np.stack([assemble_source(self.mesh, self.omega[l], self.eps, self.q, self.alpha)
                                 for l in range(self.n_dir)])
        return self._qu

    # ----- weighted global matrices of Appendix A -----
    def L(self):
        return sp.block_diag([self.w[l] * self.Lu[l] for l in range(self.n_dir)], format="csr")

    def M(self):
        return sp.vstack([self.w[l] * self.Mu for l in range(self.n_dir)], format="csr")

    def P(self):
        eye = sp.identity(self.mesh.n_cells * self.n_p, format="csr")
        return sp.hstack([self.w[l] * eye for l in range(self.n_dir)], format="csr")

    def Q(self):
        return (self.w[:, None] * self.Qu).ravel()

    # ----- index sets of the low-memory split (Sec. 3.2) -----
    def split_indices(self):
        nd, nx, n_p = self.n_dir, self.mesh.n_cells, self.n_p
        full = np.arange(nd * nx * n_p).reshape(nd, nx, n_p)
        return full[:, :, 0].ravel(), full[:, :, 1:].ravel()

    def sigma_t_matrix(self):
        """Sigma^T: copy per-cell slope moments (n_x*(n_P-1)) to every direction."""
        nd, nx, n_p = self.n_dir, self.mesh.n_cells, self.n_p
        n1 = nx * (n_p - 1)
        return sp.vstack([sp.identity(n1, format="csr")] * nd, format="csr")

    def reconstruction(self):
        """R (maps Psi_0 to per-direction slope moments on I_1) and r_alpha.

        Sec. 3.3.1: along axis k the slope is delta^{s_k} u^0 with s_k = -sign(Omega_k);
        interior one-sided difference over h, boundary difference with alpha over h/2.
        Legendre coefficient of the slope = delta * h_k / 2 (basis xi_k = 2(x-x_c)/h_k).

        Variants (readings of passages that name them without a formula):
        * three-cell (RLMDG*, the wider upwind stencil of the discussion of
          fig-efficiency): where a cell has two upwind neighbours along k, the slope is
          the derivative at the cell centre of the quadratic with the three cell averages
          u_i, u_{i-1}, u_{i-2}, (3 u_i - 4 u_{i-1} + u_{i-2}) / (2h), Legendre
          coefficient (3 u_i - 4 u_{i-1} + u_{i-2}) / 4; with one upwind neighbour the
          two-cell difference, in the inflow cell the boundary difference as above.
        * suppress (examp-disccross1): no slope along k in a cell whose upwind
          neighbour along k has other cross sections (sigma_s/eps or eps sigma_a), and a
          three-cell stencil falls back to two cells when its far cell differs from the
          near one.  The inflow cell keeps its boundary difference.
        """
        mesh = self.mesh
        nd, nx, n_p, d = self.n_dir, mesh.n_cells, self.n_p, mesh.dim
        exps = basis_exponents(d)
        # moment index of the single-axis linear mode along axis k
        lin = {k: exps.index(tuple(1 if m == k else 0 for m in range(d))) for k in range(d)}
        rows, cols, vals = [], [], []
        r_alpha = np.zeros((nd, nx, n_p - 1))
        cells = np.arange(nx)
        for l in range(nd):
            om = self.omega[l]
            for k in range(d):
                hk = mesh.h[k]
                upwind_side = -1 if om[k] > 0 else 1          # s_k = -sign(Omega_k)
                sgn = 1.0 if upwind_side == -1 else -1.0      # delta^- = (u_i - u_up)/h, delta^+ = (u_up - u_i)/h
                nb = mesh.neighbor(k, upwind_side)
                row = (l * nx + cells) * (n_p - 1) + (lin[k] - 1)
                inner = nb >= 0
                nb2 = np.full(nx, -1)
                nb2[inner] = mesh.neighbor(k, upwind_side)[nb[inner]]
                if self.suppress:
                    same = np.zeros(nx, dtype=bool)
                    same[inner] = self._same_material(cells[inner], nb[inner])
                    has2 = nb2 >= 0
                    same2 = np.zeros(nx, dtype=bool)
                    same2[has2] = self._same_material(nb[has2], nb2[has2])
                    inner = inner & same
                    nb2 = np.where(same2, nb2, -1)
                three = inner & (nb2 >= 0) if self.recon_kind == "three-cell" else np.zeros(nx, dtype=bool)
                two = inner & ~three
                coef = (hk / 2.0) / hk                         # interior: difference over h
                rows += [row[two], row[two]]
                cols += [l * nx + cells[two], l * nx + nb[two]]
                vals += [np.full(two.sum(), sgn * coef), np.full(two.sum(), -sgn * coef)]
                # quadratic through three upwind cell averages: (3 u - 4 u_up + u_upup) / 4
                rows += [row[three]] * 3
                cols += [l * nx + cells[three], l * nx + nb[three], l * nx + nb2[three]]
                vals += [np.full(three.sum(), sgn * 0.75), np.full(three.sum(), -sgn * 1.0),
                         np.full(three.sum(), sgn * 0.25)]
                inner = nb >= 0                                # boundary rule below: inflow cells only
                bnd = ~inner
                coef_b = (hk / 2.0) / (hk / 2.0)               # inflow cell: difference over h/2
                rows.append(row[bnd])
                cols.append(l * nx + cells[bnd])
                vals.append(np.full(bnd.sum(), sgn * coef_b))
                if self.alpha is not None and bnd.any():
                    # alpha at the midpoint of the inflow face of each boundary cell
                    x = mesh.centers[bnd].copy()
                    x[:, k] = 0.0 if upwind_side == -1 else mesh.length[k]
                    a = np.asarray(self.alpha(x, om), dtype=float)
                    r_alpha[l, cells[bnd], lin[k] - 1] += -sgn * coef_b * a
        R1 = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                           shape=(nd * nx * (n_p - 1), nd * nx))
        return R1, r_alpha.ravel()

    def _same_material(self, a, b):
        """Cells a and b have the same cross sections (sigma_s/eps and eps sigma_a)."""
        return (self.scat[a] == self.scat[b]) & (self.eps[a] * self.sigma_a[a] == self.eps[b] * self.sigma_a[b])


# ---------------------------------------------------------------------------
# direct solves (the definition of each scheme)
# ---------------------------------------------------------------------------

def solve_std_direct(prob: Problem):
    """Psi (n_dir, n_x, n_P) with (L - M P) Psi = Q  (eq-sndg-mat)."""
    A = (prob.L() - prob.M() @ prob.P()).tocsc()
    psi = spla.spsolve(A, prob.Q())
    return psi.reshape(prob.n_dir, prob.mesh.n_cells, prob.n_p)


def lm_trial_map(prob: Problem):
    """T of eq-gene-scheme: y = [Psi_0 (n_dir*n_x) ; Phi_1 (n_x*(n_P-1))] -> Psi."""
    nd, nx, n_p = prob.n_dir, prob.mesh.n_cells, prob.n_p
    i0, i1 = prob.split_indices()
    n0 = nd * nx
    rows = np.concatenate([i0, i1])
    cols = np.concatenate([np.arange(n0), n0 + np.tile(np.arange(nx * (n_p - 1)), nd)])
    return sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(nd * nx * n_p, n0 + nx * (n_p - 1)))


def solve_lmdg_direct(prob: Problem):
    """(Psi_0 (n_dir, n_x), Phi_1 (n_x, n_P-1)) of eq-gene-scheme."""
    T = lm_trial_map(prob)
    A = (T.T @ (prob.L() - prob.M() @ prob.P()) @ T).tocsc()
    y = spla.spsolve(A, T.T @ prob.Q())
    n0 = prob.n_dir * prob.mesh.n_cells
    return y[:n0].reshape(prob.n_dir, -1), y[n0:].reshape(prob.mesh.n_cells, -1)


def rlm_trial_map(prob: Problem):
    """T_R and t_alpha of eq-rlmdg-vari: Psi = T_R y + t_alpha."""
    nd, nx, n_p = prob.n_dir, prob.mesh.n_cells, prob.n_p
    i0, i1 = prob.split_indices()
    R1, r_alpha = prob.reconstruction()
    St = prob.sigma_t_matrix()
    P1 = sp.hstack([prob.w[l] * sp.identity(nx * (n_p - 1)) for l in range(nd)], format="csr")
    aniso = sp.identity(nd * nx * (n_p - 1), format="csr") - St @ P1  # I - Sigma^T P_1
    n0 = nd * nx
    top = sp.csr_matrix((np.ones(n0), (i0, np.arange(n0))), shape=(nd * nx * n_p, n0))
    embed1 = sp.csr_matrix((np.ones(i1.size), (i1, np.arange(i1.size))), shape=(nd * nx * n_p, i1.size))
    TR = sp.hstack([top + embed1 @ (aniso @ R1), embed1 @ St], format="csr")
    t_alpha = embed1 @ (aniso @ r_alpha)
    return TR, t_alpha


def solve_rlmdg_direct(prob: Problem):
    """(Psi_0, Phi_1) of the Petrov-Galerkin scheme eq-rlmdg-vari."""
    T = lm_trial_map(prob)
    TR, t_alpha = rlm_trial_map(prob)
    B = prob.L() - prob.M() @ prob.P()
    A = (T.T @ B @ TR).tocsc()
    y = spla.spsolve(A, T.T @ (prob.Q() - B @ t_alpha))
    n0 = prob.n_dir * prob.mesh.n_cells
    return y[:n0].reshape(prob.n_dir, -1), y[n0:].reshape(prob.mesh.n_cells, -1)


def rlmdg_angular_flux(prob: Problem, psi0, phi1):
    """Full Psi = T_R y + t_alpha of a RLMDG solution (n_dir, n_x, n_P)."""
    TR, t_alpha = rlm_trial_map(prob)
    y = np.concatenate([np.ravel(psi0), np.ravel(phi1)])
    return (TR @ y + t_alpha).reshape(prob.n_dir, prob.mesh.n_cells, prob.n_p)


def lmdg_angular_flux(prob: Problem, psi0, phi1):
    T = lm_trial_map(prob)
    y = np.concatenate([np.ravel(psi0), np.ravel(phi1)])
    return (T @ y).reshape(prob.n_dir, prob.mesh.n_cells, prob.n_p)


def scalar_flux_std(prob: Problem, psi):
    """P Psi as Legendre moments (n_x, n_P)."""
    return np.einsum("l,lpr->pr", prob.w, psi)


def scalar_flux_lm(prob: Problem, psi0, phi1):
    """[P_0 Psi_0 ; Phi_1] as Legendre moments (n_x, n_P)."""
    return np.concatenate([(prob.w @ psi0)[:, None], phi1], axis=1)


# ---------------------------------------------------------------------------
# the paper's reduced Krylov route
# ---------------------------------------------------------------------------

def gmres(apply, b, tol=1e-13, restart=200, maxiter=100000):
    """Restarted GMRES from x_0 = 0 (scipy), relative residual tol."""
    n = b.size
    op = spla.LinearOperator((n, n), matvec=apply, dtype=float)
    if np.linalg.norm(b) == 0:
        return np.zeros(n), 0
    it = [0]

    def cb(_):
        it[0] += 1
    x, info = spla.gmres(op, b, rtol=tol, atol=0.0, restart=restart, maxiter=maxiter,
                         callback=cb, callback_type="pr_norm")
    if info != 0:
        raise RuntimeError(f"oracle GMRES did not converge (info={info})")
    return x, it[0]


class StdReduced:
    """Reduced system Phi - P L^{-1} M Phi = P L^{-1} Q (eq-sndg-phi) and the final
    sweep Psi = L^{-1} M Phi + L^{-1} Q (eq-sndg-final-sweep)."""

    def __init__(self, prob: Problem):
        self.prob = prob
        self.lu = [spla.splu(prob.Lu[l].tocsc()) for l in range(prob.n_dir)]

    def Linv(self, rhs):  # rhs (n_dir, n_x*n_P) unweighted rows
        return np.stack([self.lu[l].solve(rhs[l]) for l in range(self.prob.n_dir)])

    def PLinv(self, rhs):
        return self.prob.w @ self.Linv(rhs)

    def apply(self, phi):
        """K Phi = Phi - P L^{-1} M Phi (rows of L and M carry the same w_l)."""
        mphi = self.prob.Mu @ phi
        return phi - self.PLinv(np.broadcast_to(mphi, (self.prob.n_dir, mphi.size)))

    def rhs(self):
        return self.PLinv(self.prob.Qu)

    def recover(self, phi):
        mphi = self.prob.Mu @ phi
        return self.Linv(self.prob.Qu + mphi[None, :]).reshape(self.prob.n_dir, self.prob.mesh.n_cells, -1)

    def solve(self, tol=1e-13, restart=200):
        phi, its = gmres(self.apply, self.rhs(), tol, restart)
        return self.recover(phi), its


class LowMemoryReduced:
    """Steps 1-4 of Sec. 3.2 (LMDG) and of Sec. 3.3.2 (RLMDG, with the corrected
    second block row described in the module docstring).

    X = [X_0 (n_x) ; X_1 (n_x*(n_P-1))].  The operator is applied in the form of
    eq-nonrec-block:  K X = diag(I, B_11) X - [P_0 ; G] L~_00^{-1}(M_0 X_0 + L_01 Sigma^T X_1)
    with G = Sigma L_10 (LMDG) or Sigma L~_10 + B_11 P_1 R (RLMDG).
    """

    def __init__(self, prob: Problem, reconstructed: bool):
        self.prob = prob
        self.rec = reconstructed
        nd, nx, n_p = prob.n_dir, prob.mesh.n_cells, prob.n_p
        L = prob.L()
        M = prob.M()
        Q = prob.Q()
        i0, i1 = prob.split_indices()
        self.L00 = L[i0][:, i0]
        self.L01 = L[i0][:, i1]
        self.L10 = L[i1][:, i0]
        self.L11 = L[i1][:, i1]
        # M = [M_0 ; M_1] restricted to the constant / slope columns (orthogonal basis)
        cols0 = np.arange(nx) * n_p
        cols1 = (np.arange(nx)[:, None] * n_p + np.arange(1, n_p)[None]).ravel()
        self.M0 = M[i0][:, cols0]
        self.M1 = M[i1][:, cols1]
        self.Q0 = Q[i0]
        self.Q1 = Q[i1]
        n1 = nx * (n_p - 1)
        self.St = prob.sigma_t_matrix()          # Sigma^T
        self.S = self.St.T.tocsr()               # Sigma (sums over directions)
        self.P0 = sp.hstack([prob.w[l] * sp.identity(nx) for l in range(nd)], format="csr")
        self.P1 = sp.hstack([prob.w[l] * sp.identity(n1) for l in range(nd)], format="csr")
        # eq-lmdg-psi1: B_11 = Sigma L_11 Sigma^T - Sigma M_1
        self.B11 = (self.S @ self.L11 @ self.St - self.S @ self.M1).tocsc()
        self.B11_lu = spla.splu(self.B11)
        if reconstructed:
            R1, r_alpha = prob.reconstruction()
            self.R = R1
            # (I - Sigma^T P_1) is dense in angle; it is applied by distributing the
            # products so that no n_dir^2 operator is formed:
            #   L_11 (I - Sigma^T P_1) R = L_11 R - (L_11 Sigma^T)(P_1 R)
            P1R = (self.P1 @ R1).tocsr()
            P1r = self.P1 @ r_alpha
            L11St = (self.L11 @ self.St).tocsr()
            self.Lt00 = (self.L00 + self.L01 @ R1).tocsc()                       # L~_00
            self.Qt0 = self.Q0 - self.L01 @ r_alpha + self.L01 @ (self.St @ P1r)  # Q~_0
            self.Qt1 = self.Q1 - self.L11 @ r_alpha + L11St @ P1r                 # Q~_1
            # Step 3 second block row: G = Sigma L~_10 + B_11 P_1 R with
            # L~_10 = L_10 + L_11 (I - Sigma^T P_1) R
            S_Lt10 = self.S @ self.L10 + self.S @ (self.L11 @ R1) - (self.S @ L11St) @ P1R
            self.G = (S_Lt10 + self.B11 @ P1R).tocsr()
        else:
            self.R = None
            self.Lt00 = self.L00.tocsc()
            self.Qt0, self.Qt1 = self.Q0, self.Q1
            self.G = (self.S @ self.L10).tocsr()
        self.Lt00_lu = spla.splu(self.Lt00)
        # Step 1 with Psi_0-independent part: c = B_11^{-1} Sigma Q~_1
        self.c = self.B11_lu.solve(self.S @ self.Qt1)
        self.g = self.Lt00_lu.solve(self.Qt0 - self.L01 @ (self.St @ self.c))
        self.nx = nx

    def sweep(self, x):
        """Psi = L~_00^{-1}(M_0 X_0 + L_01 Sigma^T X_1)."""
        x0, x1 = x[: self.nx], x[self.nx:]
        return self.Lt00_lu.solve(self.M0 @ x0 + self.L01 @ (self.St @ x1))

    def apply(self, x):
        psi = self.sweep(x)
        x0, x1 = x[: self.nx], x[self.nx:]
        return np.concatenate([x0 - self.P0 @ psi, self.B11 @ x1 - self.G @ psi])

    def rhs(self):
        return np.concatenate([self.P0 @ self.g, self.G @ self.g])

    def recover(self, x):
        """Step 4: Psi_0 and Phi_1 from X (Step 2 and Step 1 rearranged)."""
        psi0 = self.sweep(x) + self.g
        x1 = x[self.nx:]
        if self.rec:
            phi1 = self.c - x1 + self.P1 @ (self.R @ psi0)
        else:
            phi1 = self.c - x1
        nd = self.prob.n_dir
        return psi0.reshape(nd, -1), phi1.reshape(self.nx, -1)

    def solve(self, tol=1e-13, restart=200):
        x, its = gmres(self.apply, self.rhs(), tol, restart)
        return self.recover(x), its
