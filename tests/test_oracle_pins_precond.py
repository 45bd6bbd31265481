"""Pins of the oracle's two-level preconditioner (oracle/precond.py).

Each part is checked against something other than itself: the cell blocks against the
diagonal blocks of the dense reduced operator, the residual-problem identity that
motivates the coarse correction against the direct solve of the full scheme, the
diffusion matrix against the eq-difflimPF assembly of the diffusion module and its
invariants, the transfer maps against exact polynomial moments, and the preconditioned
solve against the direct solve.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import diffusion as DIF
from oracle import precond as PC
from oracle import schemes as S
from oracle.dg import Mesh
from oracle.quadrature import level_symmetric
from paper_1907_01027_amd.workloads import materials


def _problem(n, order, key=3, rec=True, eps=None):
    ss, sa, ep, q = materials(key, n=n)
    if eps is not None:
        ep = np.full_like(ep, eps)
    om, w = level_symmetric(order, 2)
    prob = S.Problem(Mesh(n), om, w, ss, sa, ep, q=q[0])
    return prob, S.LowMemoryReduced(prob, reconstructed=rec)


def _dense(red, N):
    return np.stack([red.apply(e) for e in np.eye(N)], axis=1)


@pytest.mark.parametrize("rec", [False, True])
def test_cell_blocks_are_the_diagonal_blocks_of_K(rec):
    """K_loc equals the 4 x 4 cell-diagonal blocks of K probed column by column."""
    n = (5, 4)
    prob, red = _problem(n, 4, rec=rec)
    nx = prob.mesh.n_cells
    K = _dense(red, 4 * nx)
    blocks = PC.cell_blocks(red)
    for p in range(nx):
        ii = [p] + [nx + 3 * p + m for m in range(3)]
        ref = K[np.ix_(ii, ii)]
        assert np.abs(blocks[p] - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("rec", [False, True])
def test_residual_problem_identity(rec):
    """K^{-1} r is [r_0 + phi_0 ; -phi_1 (+ P_1 R Psi_0)] with (Psi_0, Phi_1) the full scheme's
    solution for the source (M_0 r_0 in the cell-average rows, -r_1 in the slope rows)."""
    n = (4, 3)
    prob, red = _problem(n, 4, rec=rec, eps=0.05)
    nx, nd = prob.mesh.n_cells, prob.n_dir
    N = 4 * nx
    r = np.random.default_rng(7).normal(size=N)
    e = np.linalg.solve(_dense(red, N), r)
    T = S.lm_trial_map(prob)
    A = T.T @ (prob.L() - prob.M() @ prob.P()) @ (S.rlm_trial_map(prob)[0] if rec else T)
    rhs = np.concatenate([red.M0 @ r[:nx], -r[nx:]])
    y = spla.spsolve(A.tocsc(), rhs)
    psi0, phi1 = y[: nd * nx], y[nd * nx:]
    e0 = red.P0 @ psi0 + r[:nx]
    e1 = -phi1 + (red.P1 @ (red.R @ psi0) if rec else 0.0)
    assert np.abs(np.concatenate([e0, e1]) - e).max() <= 1e-11 * np.abs(e).max()


def test_diffusion_matrix_stiffness_is_the_pi0_form():
    """Without absorption and boundary term, B is eq-difflimPF as assembled by the diffusion
    module (itself pinned to the printed stencil); nodes of unlike i + j parity decouple."""
    n = (6, 5)
    mesh = Mesh(n, (6 / 8, 5 / 8))                      # square cells
    sig = 1.7
    B, _ = PC.diffusion_matrix(mesh, 1.0 / (3.0 * sig), 0.0, lumped=True)
    ref = DIF.assembled_matrix(mesh, sig, 0.0, projected=True)
    nnx = n[0] + 1
    nn = B.shape[0]
    # remove the lumped boundary term (diagonal) before comparing the couplings
    off = (B - sp.diags(B.diagonal())).toarray()
    off_ref = (ref - sp.diags(ref.diagonal())).toarray()
    assert np.abs(off - off_ref).max() < 1e-14
    par = (np.arange(nn) % nnx + np.arange(nn) // nnx) % 2
    cross = par[:, None] != par[None, :]
    assert np.abs(B.toarray()[cross]).max() < 1e-15


def test_diffusion_matrix_drops_only_the_cross_parity_term():
    """On rectangular cells B's couplings are those of eq-difflimPF between nodes of equal
    parity of i + j; what is dropped is the 2 a b term of the cell energy (it vanishes for
    a field constant on one parity class)."""
    n = (5, 4)
    mesh = Mesh(n)                                      # h_x = 1/5, h_y = 1/4
    sig = 0.8
    B, _ = PC.diffusion_matrix(mesh, 1.0 / (3.0 * sig), 0.0)
    ref = DIF.assembled_matrix(mesh, sig, 0.0, projected=True).toarray()
    nnx, nn = n[0] + 1, B.shape[0]
    par = (np.arange(nn) % nnx + np.arange(nn) // nnx) % 2
    same = par[:, None] == par[None, :]
    Bd = B.toarray() - np.diag(B.diagonal())
    refd = ref - np.diag(ref.diagonal())
    assert np.abs(Bd[same] - refd[same]).max() < 1e-14
    assert np.abs(Bd[~same]).max() == 0.0 and np.abs(refd[~same]).max() > 0.01
    assert np.abs(B.diagonal() - ref.diagonal()).max() > 0       # boundary term present
    u = np.where(par == 0, np.random.default_rng(4).normal(size=nn), 0.0)   # b = 0 or a = 0 in every cell
    lump = B.diagonal() - ref.diagonal()
    e = u @ ref @ u
    assert e > 1.0 and abs(u @ (B.toarray() - np.diag(lump)) @ u - e) < 1e-13 * e


def test_diffusion_matrix_lumping_invariants():
    """1^T B 1 = int absorb + (1/2) |dD| (lumping keeps row sums; Pi_0 grad of a constant is 0),
    and B is symmetric positive definite."""
    n = (7, 7)
    mesh = Mesh(n)
    rng = np.random.default_rng(3)
    d = rng.uniform(0.1, 2.0, mesh.n_cells)
    a = rng.uniform(0.0, 1.0, mesh.n_cells)
    B, _ = PC.diffusion_matrix(mesh, d, a)
    one = np.ones(B.shape[0])
    assert abs(one @ B @ one - (a.sum() * mesh.volume + 0.5 * 4.0)) < 1e-12
    Bd = B.toarray()
    assert np.abs(Bd - Bd.T).max() < 1e-15
    assert np.linalg.eigvalsh(Bd).min() > 0


def test_transfer_maps():
    """Z of a bilinear field gives its exact Legendre moments (sign-flipped slopes); for RLMDG
    a linear field's reconstructed slopes are exact inside, so its slope unknowns vanish
    there; W is the load of the source moments (sum over nodes = integral of the source)."""
    n = (6, 6)
    prob, red = _problem(n, 4, rec=False, eps=0.1)
    pcl = PC.TwoLevel(red)
    nnx = n[0] + 1
    X = (np.arange(pcl.nn) % nnx) / n[0]
    Y = (np.arange(pcl.nn) // nnx) / n[1]
    u = 1.0 + 2.0 * X - 3.0 * Y + 5.0 * X * Y
    z = pcl.Z(u)
    c = prob.mesh.centers
    h = prob.mesh.h
    avg = 1 + 2 * c[:, 0] - 3 * c[:, 1] + 5 * c[:, 0] * c[:, 1]
    sx = (2 + 5 * c[:, 1]) * h[0] / 2
    sy = (-3 + 5 * c[:, 0]) * h[1] / 2
    sxy = 5 * h[0] * h[1] / 4
    nx = prob.mesh.n_cells
    assert np.abs(z[:nx] - avg).max() < 1e-13
    ref1 = -np.stack([sx, sy, np.full(nx, sxy)], axis=1)
    assert np.abs(z[nx:].reshape(nx, 3) - ref1).max() < 1e-13
    r = np.random.default_rng(2).normal(size=4 * nx)
    f = pcl.W(r)
    assert abs(f.sum() - (prob.scat * r[:nx]).sum() * prob.mesh.volume) < 1e-12 * np.abs(f).sum()
    prob2, red2 = _problem(n, 4, rec=True, eps=0.1)
    z2 = PC.TwoLevel(red2).Z(1.0 + 2.0 * X)
    inner = (prob.mesh.idx[:, 0] > 0) & (prob.mesh.idx[:, 0] < n[0] - 1)
    assert np.abs(z2[nx:].reshape(nx, 3)[inner, 0]).max() < 1e-13


@pytest.mark.parametrize("rec", [False, True])
def test_preconditioned_solve_matches_direct_and_cuts_iterations(rec):
    """Right preconditioning does not change the solution (direct solve of the scheme), and
    in a diffusive multiscale medium it cuts GMRES iterations by more than 10x."""
    n = (12, 12)
    prob, red = _problem(n, 4, rec=rec)
    x, its = PC.solve(red, tol=1e-11)
    psi0, phi1 = red.recover(x)
    d0, d1 = (S.solve_rlmdg_direct if rec else S.solve_lmdg_direct)(prob)
    ref = S.scalar_flux_lm(prob, d0, d1)
    got = S.scalar_flux_lm(prob, psi0, phi1)
    assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max()
    b = red.rhs()
    it = [0]
    op = spla.LinearOperator((b.size, b.size), matvec=red.apply, dtype=float)
    spla.gmres(op, b, rtol=1e-8, atol=0.0, restart=30, maxiter=200,
               callback=lambda _: it.__setitem__(0, it[0] + 1), callback_type="pr_norm")
    _, its8 = PC.solve(red, tol=1e-8, restart=30)
    assert its8 * 10 < it[0], (its8, it[0])
