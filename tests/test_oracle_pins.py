"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: exactness of
the quadrature, closed-form integrals, exact solutions that lie in the discrete
space, theorems of the paper, and printed convergence orders.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import adjoint as ADJ
from oracle import diffusion as DIF
from oracle import schemes as S
from oracle.dg import Mesh, ReferenceIntegrals, eval_basis, face_rule, l1_error, tensor_rule
from oracle.quadrature import level_symmetric, level_symmetric_mu1, quadrant_of

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------- quadrature
@pytest.mark.parametrize("order,count2,count3", [(4, 12, 24), (8, 40, 80), (12, 84, 168), (16, 144, 288)])
def test_quadrature_conditions_and_counts(order, count2, count3):
    """Conditions (i)-(iii) of Sec. 2.1, positivity, central symmetry, set sizes."""
    for dim, count in ((2, count2), (3, count3)):
        om, w = level_symmetric(order, dim)
        assert om.shape == (count, dim)
        assert np.all(w > 0)
        assert abs(w.sum() - 1) < 1e-14
        assert np.abs(w @ om).max() < 1e-14
        assert np.abs(np.einsum("j,ja,jb->ab", w, om, om) - np.eye(dim) / 3).max() < 1e-14
        if dim == 3:
            assert np.allclose(np.linalg.norm(om, axis=1), 1.0, atol=1e-14)
        # central symmetry (needed for B_11 symmetric positive definite, Thm lem-B11)
        for j in range(count):
            k = np.argmin(np.abs(om + om[j]).sum(axis=1))
            assert np.abs(om[k] + om[j]).max() < 1e-14 and abs(w[k] - w[j]) < 1e-15
        assert np.bincount(quadrant_of(om)).tolist() == [count // 2 ** dim] * 2 ** dim


def test_quadrature_s4_mu1_closed_form():
    """S4: one weight class; exactness for mu^4 gives 6 mu^4 - 4 mu^2 + 2/5 = 0."""
    mu1 = level_symmetric_mu1(4)
    root = np.sqrt((4 - np.sqrt(16 - 4 * 6 * 0.4)) / 12)
    assert abs(mu1 - root) < 1e-15


@pytest.mark.parametrize("order,exact_to", [(4, 2), (8, 4), (12, 6), (16, 8)])
def test_quadrature_even_moments(order, exact_to):
    """The sphere averages of mu^(2m) = 1/(2m+1) are integrated exactly up to the design degree."""
    om, w = level_symmetric(order, 3)
    for m in range(exact_to + 1):
        for ax in range(3):
            assert abs(w @ om[:, ax] ** (2 * m) - 1 / (2 * m + 1)) < 1e-12


# --------------------------------------------------------------------------- assembly
@pytest.mark.parametrize("dim", [1, 2, 3])
def test_mass_is_legendre_diagonal(dim):
    """Orthogonal Legendre basis: int_K b_r b_s = |K| prod_k (1 or 1/3) delta_rs."""
    mesh = Mesh((3,) * dim, (1.0, 0.7, 1.3)[:dim])
    ref = ReferenceIntegrals(mesh)
    diag = [np.prod([1 / 3 if (r >> k) & 1 else 1.0 for k in range(dim)]) for r in range(2 ** dim)]
    assert np.abs(ref.mass - mesh.volume * np.diag(diag)).max() < 1e-15


def _project(mesh, fn, nq=4):
    """Legendre moments (n_x, n_P) of a callable on every cell (L2 projection)."""
    pts, wts = tensor_rule(mesh.dim, nq)
    val, _ = eval_basis(mesh.dim, pts)
    norm = wts @ (val * val)
    return np.stack([(wts * fn(mesh.to_physical(p, pts))) @ val / norm for p in range(mesh.n_cells)])


def _exact_problem(mesh, om, w, coeffs, eps, rng):
    """Manufactured psi_l = a_l + b_l x + c_l y + d_l x y with the consistent source.

    q_l = [Omega_l . grad psi_l + sigma_t psi_l - (sigma_s/eps) sum_j w_j psi_j] / eps,
    cross sections piecewise constant, alpha = psi_l on the inflow boundary.
    """
    ss = rng.uniform(0.5, 2.0, mesh.n_cells)
    sa = rng.uniform(0.5, 2.0, mesh.n_cells)
    a, b, c, d = coeffs

    def cell_of(x):
        i = np.minimum((x / mesh.h).astype(int), np.array(mesh.n) - 1)
        return mesh.flat(i)

    def lidx(o):
        return int(np.argmin(np.abs(om - o).sum(axis=1)))

    def psi(x, o):
        l = lidx(o)
        return a[l] + b[l] * x[:, 0] + c[l] * x[:, 1] + d[l] * x[:, 0] * x[:, 1]

    def psibar(x):
        return (w @ a) + (w @ b) * x[:, 0] + (w @ c) * x[:, 1] + (w @ d) * x[:, 0] * x[:, 1]

    def q(x, o):
        l = lidx(o)
        k = cell_of(x)
        grad = np.stack([b[l] + d[l] * x[:, 1], c[l] + d[l] * x[:, 0]], axis=1)
        st = ss[k] / eps + eps * sa[k]
        return (grad @ o + st * psi(x, o) - ss[k] / eps * psibar(x)) / eps

    prob = S.Problem(mesh, om, w, ss, sa, eps, q=q, alpha=psi)
    return prob, psi, psibar


@pytest.mark.parametrize("eps", [1.0, 0.05])
def test_exact_solution_in_discrete_space(eps):
    """Consistency + unisolvency: a solution lying in the trial space is reproduced.

    STD (Q^1 per direction) any bilinear psi_l; LMDG needs isotropic slopes;
    RLMDG reproduces per-direction linear fields plus an isotropic xy term, since
    the upwind differences of Sec. 3.3.1 are exact for linear data (with alpha).
    """
    rng = np.random.default_rng(7)
    mesh = Mesh((5, 4), (1.0, 0.8))
    om, w = level_symmetric(4, 2)
    nd = len(w)
    # STD: fully anisotropic bilinear
    co = [rng.normal(size=nd) for _ in range(4)]
    prob, psi, _ = _exact_problem(mesh, om, w, co, eps, rng)
    ps = S.solve_std_direct(prob)
    ex = np.stack([_project(mesh, lambda x, o=om[l]: psi(x, o)) for l in range(nd)])
    assert np.abs(ps - ex).max() < 1e-11
    # LMDG: anisotropic cell constants, isotropic slopes
    co = [rng.normal(size=nd)] + [np.full(nd, rng.normal()) for _ in range(3)]
    prob, psi, psibar = _exact_problem(mesh, om, w, co, eps, rng)
    p0, p1 = S.solve_lmdg_direct(prob)
    ex0 = np.stack([_project(mesh, lambda x, o=om[l]: psi(x, o))[:, 0] for l in range(nd)])
    assert np.abs(p0 - ex0).max() < 1e-11
    assert np.abs(p1 - _project(mesh, psibar)[:, 1:]).max() < 1e-11
    # RLMDG: anisotropic linear part, isotropic xy
    co = [rng.normal(size=nd), rng.normal(size=nd), rng.normal(size=nd), np.full(nd, rng.normal())]
    prob, psi, psibar = _exact_problem(mesh, om, w, co, eps, rng)
    p0, p1 = S.solve_rlmdg_direct(prob)
    full = S.rlmdg_angular_flux(prob, p0, p1)
    ex = np.stack([_project(mesh, lambda x, o=om[l]: psi(x, o)) for l in range(nd)])
    assert np.abs(full - ex).max() < 1e-10
    assert np.abs(S.scalar_flux_lm(prob, p0, p1) - _project(mesh, psibar)).max() < 1e-10


def _upwind_order(mesh, omega):
    """Cell permutation in which every upwind neighbour comes first."""
    key = np.zeros(mesh.n_cells)
    for k in range(mesh.dim):
        key += mesh.idx[:, k] if omega[k] > 0 else (mesh.n[k] - 1 - mesh.idx[:, k])
    return np.argsort(key, kind="stable")


@pytest.mark.parametrize("dim", [2, 3])
def test_transport_blocks_are_sweepable(dim):
    """Sec. 2.1.1: with upwind traces each L_l is block lower triangular in upwind order."""
    mesh = Mesh((4, 3, 3)[:dim])
    om, w = level_symmetric(4, dim)
    prob = S.Problem(mesh, om, w, 1.0, 1.0, 1.0)
    n_p = mesh.n_p
    for l in range(len(w)):
        perm = _upwind_order(mesh, om[l])
        idx = (perm[:, None] * n_p + np.arange(n_p)[None]).ravel()
        Lp = prob.Lu[l][idx][:, idx].toarray()
        blocks = Lp.reshape(mesh.n_cells, n_p, mesh.n_cells, n_p)
        upper = np.triu(np.ones((mesh.n_cells, mesh.n_cells)), 1).astype(bool)
        assert np.abs(blocks.transpose(0, 2, 1, 3)[upper]).max() == 0.0


def test_rlmdg_sweep_block_is_lower_triangular():
    """Sec. 3.3.2: L~_00 = L_00 + L_01 R uses only upwind information."""
    mesh = Mesh((4, 3))
    om, w = level_symmetric(4, 2)
    prob = S.Problem(mesh, om, w, 1.0, 1.0, 0.5)
    red = S.LowMemoryReduced(prob, reconstructed=True)
    nx = mesh.n_cells
    for l in range(len(w)):
        blk = red.Lt00[l * nx:(l + 1) * nx][:, l * nx:(l + 1) * nx].toarray()
        perm = _upwind_order(mesh, om[l])
        assert np.abs(np.triu(blk[perm][:, perm], 1)).max() == 0.0


# --------------------------------------------------------------------------- schemes
@pytest.mark.parametrize("eps", [1.0, 0.1, 1e-3])
def test_uniform_infinite_medium(eps):
    """eq-main with constant data and alpha = q/sigma_a has psi = q/sigma_a; constants
    lie in every space and the reconstruction of a constant with matching alpha is 0."""
    mesh = Mesh((5, 4), (1.0, 0.8))
    om, w = level_symmetric(4, 2)
    sa, ss, q = 0.7, 1.3, 2.0
    prob = S.Problem(mesh, om, w, ss, sa, eps, q=np.full(mesh.n_cells, q),
                     alpha=lambda x, o: np.full(len(x), q / sa))
    tol = 1e-12 / min(eps, 1.0)
    phi = S.scalar_flux_std(prob, S.solve_std_direct(prob))
    assert np.abs(phi[:, 0] - q / sa).max() < tol and np.abs(phi[:, 1:]).max() < tol
    for fn in (S.solve_lmdg_direct, S.solve_rlmdg_direct):
        p0, p1 = fn(prob)
        assert np.abs(p0 - q / sa).max() < tol and np.abs(p1).max() < tol


def _random_problem(mesh, order=4, eps=0.3, seed=0, alpha=True):
    rng = np.random.default_rng(seed)
    om, w = level_symmetric(order, mesh.dim)
    q = lambda x, o: 1 + x[:, 0] * o[0] + x[:, -1] ** 2
    al = (lambda x, o: 0.5 + x[:, 0] + o[-1] ** 2) if alpha else None
    return S.Problem(mesh, om, w, rng.uniform(0.5, 2, mesh.n_cells), rng.uniform(0.5, 2, mesh.n_cells),
                     eps, q=q, alpha=al)


@pytest.mark.parametrize("n", [(6, 5), (2, 3, 2)])
def test_sherman_morrison_reduced_route_std(n):
    """eq-sndg-phi + eq-sndg-final-sweep reproduce the direct solve (Remark, Sec. 2.1.1),
    in 2D and 3D."""
    prob = _random_problem(Mesh(n, (1.0,) * len(n)))
    psi = S.solve_std_direct(prob)
    psir, _ = S.StdReduced(prob).solve(tol=1e-14)
    assert np.abs(psi - psir).max() < 1e-11


@pytest.mark.parametrize("rec", [False, True])
@pytest.mark.parametrize("alpha", [False, True])
def test_low_memory_reduction_matches_direct(rec, alpha):
    """Steps 1-4 of Sec. 3.2 (and of Sec. 3.3.2 with the corrected second row) give
    the solution of the un-reduced system, including c = B_11^{-1} Sigma Q~_1 != 0."""
    prob = _random_problem(Mesh((6, 5)), alpha=alpha)
    p0, p1 = (S.solve_rlmdg_direct if rec else S.solve_lmdg_direct)(prob)
    (q0, q1), _ = S.LowMemoryReduced(prob, rec).solve(tol=1e-14)
    scale = np.abs(p0).max()
    assert np.abs(p0 - q0).max() < 1e-11 * scale and np.abs(p1 - q1).max() < 1e-11 * scale


def test_low_memory_reduction_3d():
    prob = _random_problem(Mesh((3, 3, 2)), order=4, alpha=True)
    for rec, fn in ((False, S.solve_lmdg_direct), (True, S.solve_rlmdg_direct)):
        p0, p1 = fn(prob)
        (q0, q1), _ = S.LowMemoryReduced(prob, rec).solve(tol=1e-14)
        assert np.abs(p0 - q0).max() < 1e-10 and np.abs(p1 - q1).max() < 1e-10


def _b11_jump_form(prob):
    """Appendix C form of B_11 on D_{h,1}: eps sigma_a mass + sum_F c_F int_F [u][v],
    c_F = sum over directions with Omega . nu_F > 0 of w Omega . nu_F, exterior trace 0."""
    mesh = prob.mesh
    n_p, d = mesh.n_p, mesh.dim
    ref = ReferenceIntegrals(mesh)
    n1 = mesh.n_cells * (n_p - 1)
    B = sp.lil_matrix((n1, n1))
    idx = lambda p, r: p * (n_p - 1) + r - 1
    for p in range(mesh.n_cells):
        for r in range(1, n_p):
            for s in range(1, n_p):
                B[idx(p, r), idx(p, s)] += prob.eps[p] * prob.sigma_a[p] * ref.mass[r, s]
    for k in range(d):
        cF = sum(prob.w[j] * prob.omega[j, k] for j in range(len(prob.w)) if prob.omega[j, k] > 0)
        own_hi = ref.face_own[(k, 1.0)]   # trace of the cell on its +k face
        own_lo = ref.face_own[(k, -1.0)]
        cross = ref.face_nb[(k, 1.0)]     # (+k face of K) x (-k face of its neighbour)
        nb = mesh.neighbor(k, 1)
        for p in range(mesh.n_cells):
            for r in range(1, n_p):
                for s in range(1, n_p):
                    B[idx(p, r), idx(p, s)] += cF * own_hi[r, s]
                    if nb[p] >= 0:
                        B[idx(nb[p], r), idx(nb[p], s)] += cF * own_lo[r, s]
                        B[idx(p, r), idx(nb[p], s)] -= cF * cross[r, s]
                        B[idx(nb[p], r), idx(p, s)] -= cF * cross[s, r]
            # boundary face on the low side of the first cell of each line
        low = mesh.neighbor(k, -1) < 0
        for p in np.nonzero(low)[0]:
            for r in range(1, n_p):
                for s in range(1, n_p):
                    B[idx(p, r), idx(p, s)] += cF * own_lo[r, s]
    return B.tocsr()


@pytest.mark.parametrize("dim", [2, 3])
def test_b11_spd_and_jump_form(dim):
    """Thm lem-B11: B_11 = Sigma L_11 Sigma^T - Sigma M_1 is symmetric positive definite
    for a centrally symmetric quadrature and equals the face-jump form of Appendix C."""
    mesh = Mesh((4, 3, 2)[:dim])
    prob = _random_problem(mesh, eps=0.2)
    red = S.LowMemoryReduced(prob, reconstructed=False)
    B = red.B11.toarray()
    assert np.abs(B - B.T).max() < 1e-14 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0
    assert np.abs(B - _b11_jump_form(prob).toarray()).max() < 1e-14 * np.abs(B).max()


def test_reduced_operators_invertible():
    """Thm thm-sndg-mat-psi (I - P L^{-1} M) and Thm thm-K (K) are nonsingular."""
    prob = _random_problem(Mesh((3, 3)), alpha=False)
    n = prob.mesh.n_cells * prob.n_p
    std = S.StdReduced(prob)
    Kstd = np.stack([std.apply(e) for e in np.eye(n)], axis=1)
    lm = S.LowMemoryReduced(prob, False)
    Klm = np.stack([lm.apply(e) for e in np.eye(n)], axis=1)
    for K in (Kstd, Klm):
        assert np.linalg.svd(K, compute_uv=False).min() > 1e-6


def _energy_terms(prob, psi):
    """Left side of eq-stab for a full angular field psi (n_dir, n_x, n_P), alpha = 0."""
    mesh = prob.mesh
    ref = ReferenceIntegrals(mesh)
    w = prob.w
    psibar = np.einsum("l,lpr->pr", w, psi)
    dev = psi - psibar[None]
    norm2 = lambda v, c: float(np.einsum("l,p,lpr,rs,lps->", w, c, v, ref.mass, v))
    t1 = norm2(dev, prob.sigma_s) / prob.eps[0]
    t2 = 0.5 * prob.eps[0] * norm2(psi, prob.sigma_a)
    jump = 0.0
    for k in range(mesh.dim):
        nb = mesh.neighbor(k, 1)
        for l in range(len(w)):
            a = abs(prob.omega[l, k])
            for p in range(mesh.n_cells):
                up = psi[l, p]
                # -k boundary face of a first cell: exterior zero
                if mesh.neighbor(k, -1)[p] < 0:
                    jump += w[l] * a * up @ ref.face_own[(k, -1.0)] @ up
                if nb[p] >= 0:
                    vn = psi[l, nb[p]]
                    jump += w[l] * a * (up @ ref.face_own[(k, 1.0)] @ up - 2 * up @ ref.face_nb[(k, 1.0)] @ vn
                                        + vn @ ref.face_own[(k, -1.0)] @ vn)
                else:
                    jump += w[l] * a * up @ ref.face_own[(k, 1.0)] @ up
    return t1 + t2 + 0.5 * jump


def test_energy_estimate():
    """eq-stab of Thm thm-gene-uni-solvency (alpha = 0) for STD and LMDG."""
    rng = np.random.default_rng(3)
    mesh = Mesh((5, 4))
    om, w = level_symmetric(4, 2)
    eps = 0.3
    q = rng.uniform(0, 1, mesh.n_cells)
    prob = S.Problem(mesh, om, w, rng.uniform(0.5, 2, mesh.n_cells), rng.uniform(0.5, 2, mesh.n_cells), eps, q=q)
    qnorm2 = float(np.sum(q * q) * mesh.volume)
    bound = eps / (2 * prob.sigma_a.min()) * qnorm2
    psi = S.solve_std_direct(prob)
    assert _energy_terms(prob, psi) <= bound
    p0, p1 = S.solve_lmdg_direct(prob)
    assert _energy_terms(prob, S.lmdg_angular_flux(prob, p0, p1)) <= bound


def test_mirror_symmetry():
    """Data symmetric under x <-> 1 - x gives a mirror-symmetric scalar flux."""
    mesh = Mesh((6, 4))
    om, w = level_symmetric(4, 2)
    rng = np.random.default_rng(5)
    half = rng.uniform(0.5, 2, (4, 3))
    field = np.concatenate([half, half[:, ::-1]], axis=1).ravel()
    prob = S.Problem(mesh, om, w, field, field[::-1].reshape(4, 6)[::-1].ravel(), 0.5, q=field)
    for scheme in ("std", "lm", "rlm"):
        if scheme == "std":
            phi = S.scalar_flux_std(prob, S.solve_std_direct(prob))
        else:
            fn = S.solve_lmdg_direct if scheme == "lm" else S.solve_rlmdg_direct
            phi = S.scalar_flux_lm(prob, *fn(prob))
        grid = phi.reshape(4, 6, 4)
        mirrored = grid[:, ::-1].copy()
        mirrored[..., 1] *= -1  # the xi moment changes sign under x -> 1 - x
        mirrored[..., 3] *= -1
        assert np.abs(grid - mirrored).max() < 1e-12


def test_dimension_counts():
    """Table tab-compare: Krylov dimension n_P n_x, solution dimension n_dir n_x + (n_P-1) n_x."""
    for dim in (2, 3):
        mesh = Mesh((3, 2, 2)[:dim])
        prob = _random_problem(mesh, alpha=False)
        T = S.lm_trial_map(prob)
        assert T.shape[1] == prob.n_dir * mesh.n_cells + (2 ** dim - 1) * mesh.n_cells
        lm = S.LowMemoryReduced(prob, False)
        assert lm.rhs().size == 2 ** dim * mesh.n_cells


# --------------------------------------------------------------------------- convergence
def _mms(case):
    if case == "iso":
        psi = lambda x, o: np.sin(x[:, 0] + x[:, 1])
        q = lambda x, o: (o[0] + o[1]) * np.cos(x[:, 0] + x[:, 1]) + np.sin(x[:, 0] + x[:, 1])
        ex = lambda x: np.sin(x[:, 0] + x[:, 1])
    else:
        s = lambda x: np.sin(2 * x[:, 0] + x[:, 1])
        psi = lambda x, o: (o[0] - 2 * o[1]) ** 2 * s(x)
        # sigma_t = 2, sigma_s/eps = 1, psibar = (1/3 + 4/3) sin(2x + y) (exact for degree 2)
        q = lambda x, o: ((o[0] - 2 * o[1]) ** 2 * (2 * o[0] + o[1]) * np.cos(2 * x[:, 0] + x[:, 1])
                          + (2 * (o[0] - 2 * o[1]) ** 2 - 5 / 3) * s(x))
        ex = lambda x: 5 / 3 * s(x)
    return psi, q, ex


@pytest.mark.slow
@pytest.mark.parametrize("case,key", [("iso", "isotropic_sin(x+y)"), ("aniso", "anisotropic_(Ox-2Oy)^2 sin(2x+y)")])
def test_convergence_orders_match_table(case, key):
    """Orders of Table tab-2d-aniso (Sec. 4.2): Q^1 2, LMDG 2 (iso) / 1 (aniso), RLMDG 2."""
    printed = json.load(open(os.path.join(GOLDEN, "tab_2d_orders.json")))[key]
    om, w = level_symmetric(4, 2)
    psi, q, ex = _mms(case)
    errs = {"Q1-DG": [], "LMDG": [], "RLMDG": []}
    for n in (12, 24):
        mesh = Mesh((n, n))
        prob = S.Problem(mesh, om, w, 1.0, 1.0, 1.0, q=q, alpha=psi)
        errs["Q1-DG"].append(l1_error(mesh, S.scalar_flux_std(prob, S.solve_std_direct(prob)), ex))
        errs["LMDG"].append(l1_error(mesh, S.scalar_flux_lm(prob, *S.solve_lmdg_direct(prob)), ex))
        errs["RLMDG"].append(l1_error(mesh, S.scalar_flux_lm(prob, *S.solve_rlmdg_direct(prob)), ex))
    for name, e in errs.items():
        order = np.log2(e[0] / e[1])
        assert abs(order - printed[name]) < 0.15, (name, order)


def test_pi0_form_matches_printed_stencil():
    """Sec. 3.1, case 3: on a uniform grid with constant cross sections eq-difflimPF is
    the printed finite-difference scheme: stiffness couples diagonal neighbours only,
    -(sum of 4 diagonal values - 4 psi_ij)/(3 sigma_s 2 h^2), mass = h^2 A[.]."""
    h = 0.25
    mesh = Mesh((4, 4), (1.0, 1.0))
    node = 2 + 5 * 2  # interior node (2, 2) of the 5 x 5 node grid
    st = DIF.assembled_matrix(mesh, 1.0, 0.0, projected=True).toarray()[node].reshape(5, 5)
    expect = np.zeros((5, 5))
    expect[2, 2] = 4.0
    for dj in (-1, 1):
        for di in (-1, 1):
            expect[2 + dj, 2 + di] = -1.0
    assert np.abs(st - expect / (3.0 * 2.0 * h * h) * h * h).max() < 1e-14
    ms = DIF.assembled_matrix(mesh, 1e300, 1.0, projected=True).toarray()[node].reshape(5, 5)
    mass = np.array([[1 / 36, 1 / 9, 1 / 36], [1 / 9, 4 / 9, 1 / 9], [1 / 36, 1 / 9, 1 / 36]])
    assert np.abs(ms[1:4, 1:4] - h * h * mass).max() < 1e-15


@pytest.mark.parametrize("scheme", ["std", "lmdg"])
def test_diffusion_limit(scheme):
    """Thm thm-sndg-asympscheme / thm-lmdg-asympscheme: as eps -> 0 the scalar flux tends
    to the Q^1 CG solution (std, eq-lmdg-cg) or the Pi_0 form (LMDG, eq-difflimPF)."""
    mesh = Mesh((6, 6))
    om, w = level_symmetric(4, 2)
    qf = lambda x: 1.0 + x[:, 0] * (1 - x[:, 1])
    _, ref = DIF.solve_limit(mesh, 1.0, 1.0, qf, projected=(scheme == "lmdg"))
    errs = []
    for eps in (1e-2, 1e-3, 1e-4):
        prob = S.Problem(mesh, om, w, 1.0, 1.0, eps, q=lambda x, o: qf(x))
        if scheme == "std":
            phi = S.scalar_flux_std(prob, S.solve_std_direct(prob))
        else:
            phi = S.scalar_flux_lm(prob, *S.solve_lmdg_direct(prob))
        errs.append(np.abs(phi - ref).max() / np.abs(ref).max())
    assert errs[2] < 2e-3
    assert errs[1] < 0.2 * errs[0] and errs[2] < 0.2 * errs[1]


# --------------------------------------------------------------------------- adjoint
@pytest.mark.parametrize("scheme", ["std", "lmdg", "rlmdg"])
def test_adjoint_duality_and_finite_differences(scheme):
    mesh = Mesh((4, 3))
    om, w = level_symmetric(4, 2)
    rng = np.random.default_rng(11)
    eps = 0.5
    ss, sa, q = rng.uniform(0.5, 2, 12), rng.uniform(0.5, 2, 12), rng.uniform(0, 1, 12)
    det = ADJ.detector_moments(mesh, np.array([0.3, 0.2]), np.array([0.8, 0.9]))

    def J(ss_, sa_, q_):
        prob = S.Problem(mesh, om, w, ss_, sa_, eps, q=q_)
        return ADJ.forward_adjoint(prob, scheme, det)[2]

    prob = S.Problem(mesh, om, w, ss, sa, eps, q=q)
    A, b, T = ADJ._system(prob, scheme)
    y, lam, J0, _ = ADJ.forward_adjoint(prob, scheme, det)
    assert abs(lam @ b - J0) < 1e-13 * abs(J0)
    J1, gs, ga, gq = ADJ.gradients(prob, scheme, det)
    for K in (0, 5, 11):
        for g, which in ((gs, 0), (ga, 1), (gq, 2)):
            step = 1e-5
            args_p = [ss.copy(), sa.copy(), q.copy()]
            args_m = [ss.copy(), sa.copy(), q.copy()]
            args_p[which][K] += step
            args_m[which][K] -= step
            fd = (J(*args_p) - J(*args_m)) / (2 * step)
            assert abs(fd - g[K]) < 1e-6 * max(1.0, abs(g[K]))


def test_adjoint_gradient_bilinear_forms():
    """dJ/dsigma_a = -eps sum_j w_j int_K psi_j lambda_j,
    dJ/dsigma_s = -(1/eps) int_K (sum_j w_j psi_j lambda_j - psibar lambdabar),
    dJ/dq = eps int_K lambdabar  (derivatives of eq-Ljk, eq-Sjk and Q_alpha)."""
    mesh = Mesh((4, 3))
    om, w = level_symmetric(4, 2)
    rng = np.random.default_rng(2)
    eps = 0.3
    prob = S.Problem(mesh, om, w, rng.uniform(0.5, 2, 12), rng.uniform(0.5, 2, 12), eps,
                     q=rng.uniform(0, 1, 12))
    det = ADJ.detector_moments(mesh, np.array([0.3, 0.2]), np.array([0.8, 0.9]))
    ref = ReferenceIntegrals(mesh)
    for scheme in ("std", "lmdg", "rlmdg"):
        psi, lam, _ = ADJ.adjoint_flux(prob, scheme, det)
        _, gs, ga, gq = ADJ.gradients(prob, scheme, det)
        wpl = np.einsum("l,lpr,rs,lps->p", w, psi, ref.mass, lam)
        pb, lb = np.einsum("l,lpr->pr", w, psi), np.einsum("l,lpr->pr", w, lam)
        bb = np.einsum("pr,rs,ps->p", pb, ref.mass, lb)
        assert np.abs(ga - (-eps * wpl)).max() < 1e-12
        assert np.abs(gs - (-(wpl - bb) / eps)).max() < 1e-12
        assert np.abs(gq - eps * mesh.volume * lb[:, 0]).max() < 1e-12
