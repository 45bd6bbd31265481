"""Pins of the oracle's reconstruction variants (RLMDG*, suppressed reconstruction).

The paper names both variants without formulas; the oracle takes these readings:
* RLMDG* (discussion of fig-efficiency, Sec. 4.1): in cells with two upwind
  neighbours the slope is the derivative at the cell centre of the quadratic with the
  three upwind-inclusive cell averages.  The paper states that RLMDG* stays second
  order, that its error is comparable to P^1-DG, and that it is markedly smaller than
  that of RLMDG; checked on the fabricated slab solutions of Table tab-1d-aniso.
* suppressed reconstruction (examp-disccross1, fig-disccross1-2): no slope across a
  cross-section discontinuity.  The paper states that this alleviates the kinks RLMDG
  shows at the discontinuity; checked on that example's data (uniform mesh h = 0.1,
  the example's finest spacing) against a refined P^1-DG solution near the interface.
Both variants keep what every scheme must satisfy: constants are exact (uniform
infinite medium) and the reduced route equals the direct solve.
"""
import numpy as np
import pytest

from oracle import schemes as S
from oracle.dg import Mesh, l1_error, tensor_rule
from oracle.quadrature import level_symmetric

MU, GW = np.polynomial.legendre.leggauss(32)


def _fab(case):
    if case == "cos x":
        psi = lambda x, o: np.cos(x[:, 0])
        q = lambda x, o: -o[0] * np.sin(x[:, 0]) + np.cos(x[:, 0])
        phi = lambda x: np.cos(x[:, 0])
    else:
        psi = lambda x, o: np.cos(x[:, 0] + o[0])
        q = lambda x, o: -o[0] * np.sin(x[:, 0] + o[0]) + 2 * np.cos(x[:, 0] + o[0]) - np.sin(1.0) * np.cos(x[:, 0])
        phi = lambda x: np.sin(1.0) * np.cos(x[:, 0])
    return psi, q, phi


@pytest.mark.parametrize("case", ["cos x", "cos(x+mu)"])
def test_three_cell_reconstruction_is_second_order_and_close_to_p1(case):
    psi, q, phi = _fab(case)
    err = {"P1": [], "RLMDG": [], "RLMDG*": []}
    for n in (40, 80):
        mesh = Mesh((n,), (1.0,))
        for name in err:
            kw = {"reconstruction": "three-cell"} if name == "RLMDG*" else {}
            prob = S.Problem(mesh, MU[:, None], GW / 2, 1.0, 1.0, 1.0, q=q, alpha=psi, **kw)
            f = (S.scalar_flux_std(prob, S.solve_std_direct(prob)) if name == "P1"
                 else S.scalar_flux_lm(prob, *S.solve_rlmdg_direct(prob)))
            err[name].append(l1_error(mesh, f, phi))
    e = {k: np.array(v) for k, v in err.items()}
    assert abs(np.log2(e["RLMDG*"][0] / e["RLMDG*"][1]) - 2.0) < 0.1
    assert np.all(e["RLMDG*"] < 2.0 * e["P1"])       # comparable to P^1-DG
    assert np.all(e["RLMDG*"] < 0.5 * e["RLMDG"])    # markedly smaller than RLMDG


def _disccross(n, kind, suppress=False):
    """examp-disccross1 on [0, 11]: sigma_s/eps = 0 | 100, eps sigma_a = 2 | 0 at x = 1,
    inflow 1 at x = 0 and 0 at x = 11, 16-point Gauss."""
    mu, gw = np.polynomial.legendre.leggauss(16)
    xc = (np.arange(n) + 0.5) * 11.0 / n
    left = xc < 1.0
    ss, sa = np.where(left, 0.0, 100.0), np.where(left, 2.0, 0.0)
    alpha = lambda x, o: np.full(x.shape[0], 1.0 if o[0] > 0 else 0.0)
    prob = S.Problem(Mesh((n,), (11.0,)), mu[:, None], gw / 2, ss, sa, 1.0, alpha=alpha, suppress=suppress)
    if kind == "std":
        return S.scalar_flux_std(prob, S.solve_std_direct(prob))
    return S.scalar_flux_lm(prob, *S.solve_rlmdg_direct(prob))


def _l1_window(n, f, ref, nref, lo, hi):
    pts, wts = tensor_rule(1, 6)
    h, href = 11.0 / n, 11.0 / nref
    tot = 0.0
    for p in range(n):
        x = (p + 0.5) * h + 0.5 * h * pts[:, 0]
        m = (x >= lo) & (x <= hi)
        if m.any():
            k = np.minimum((x / href).astype(int), nref - 1)
            ex = ref[k, 0] + ref[k, 1] * 2 * (x - (k + 0.5) * href) / href
            tot += 0.5 * h * (wts * m) @ np.abs(f[p, 0] + f[p, 1] * pts[:, 0] - ex)
    return tot


@pytest.mark.slow
def test_suppressed_reconstruction_reduces_the_error_at_the_discontinuity():
    nref = 1100
    ref = _disccross(nref, "std")
    f = _disccross(110, "rlmdg")
    fs = _disccross(110, "rlmdg", suppress=True)
    e, es = _l1_window(110, f, ref, nref, 0.5, 3.0), _l1_window(110, fs, ref, nref, 0.5, 3.0)
    assert es < 0.85 * e, (e, es)


@pytest.mark.parametrize("kw", [{"reconstruction": "three-cell"}, {"suppress": True},
                                {"reconstruction": "three-cell", "suppress": True}])
def test_variants_keep_constants_and_reduce_exactly(kw):
    om, w = level_symmetric(4, 2)
    n = (7, 6)
    rng = np.random.default_rng(3)
    # uniform infinite medium with matching inflow: psi = q / sigma_a exactly
    prob = S.Problem(Mesh(n), om, w, 0.8, 1.6, 0.3, q=2.0, alpha=lambda x, o: np.full(x.shape[0], 1.25), **kw)
    p0, p1 = S.solve_rlmdg_direct(prob)
    assert np.abs(p0 - 1.25).max() < 1e-12 and np.abs(p1).max() < 1e-12
    # blocky media (so that suppression acts): reduced route = direct solve
    ss = np.repeat(rng.uniform(0.5, 2.0, 3), 14)
    sa = np.repeat(rng.uniform(0.5, 2.0, 3), 14)
    prob = S.Problem(Mesh(n), om, w, ss, sa, 0.2, q=rng.uniform(0, 1, 42),
                     alpha=lambda x, o: 1.0 + x[:, 0] * o[1], **kw)
    d0, d1 = S.solve_rlmdg_direct(prob)
    (r0, r1), _ = S.LowMemoryReduced(prob, True).solve(tol=1e-14)
    ref = S.scalar_flux_lm(prob, d0, d1)
    assert np.abs(S.scalar_flux_lm(prob, r0, r1) - ref).max() < 1e-10 * np.abs(ref).max()


def test_suppression_changes_nothing_in_a_uniform_medium():
    om, w = level_symmetric(4, 2)
    prob = S.Problem(Mesh((5, 4)), om, w, 1.0, 1.0, 0.5, q=1.0)
    sup = S.Problem(Mesh((5, 4)), om, w, 1.0, 1.0, 0.5, q=1.0, suppress=True)
    assert (prob.reconstruction()[0] != sup.reconstruction()[0]).nnz == 0
