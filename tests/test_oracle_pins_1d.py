"""Pins of the CPU oracle against the paper's slab-geometry tables (Sec. 4.1).

The oracle is dimension-generic: on a 1D mesh with the 32-point Gauss rule in mu it is
the slab form eq-1d of the three schemes (P^1 = Q^1 in 1D).  Checked against the
printed values of Table tab-1d-aniso (fabricated solutions, orders) and Table
tab-1d-eps10-5 (diffusive and transport regimes against a 1280-cell P^1-DG
reference: orders, and the P^1-DG and LMDG errors at eps = 1e-5, which the oracle
reproduces to within 8% at every refinement).  Not pinned: the other absolute 1D
errors, which the oracle matches only up to a factor of 1.4-2.8 (RLMDG at eps = 1e-5
by a constant 1.8, more accurate than printed); the paper does not state the error
norm precisely enough to tell why.
"""
import json
import os

import numpy as np
import pytest

from oracle import schemes as S
from oracle.dg import Mesh, l1_error, tensor_rule

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tab_1d.json")))
MU, GW = np.polynomial.legendre.leggauss(32)
OMEGA = MU[:, None]
W = GW / 2.0  # weights normalised to sum 1: (1/2) int_{-1}^{1} d mu


def scalar_fluxes(prob):
    return {"P1-DG": S.scalar_flux_std(prob, S.solve_std_direct(prob)),
            "LMDG": S.scalar_flux_lm(prob, *S.solve_lmdg_direct(prob)),
            "RLMDG": S.scalar_flux_lm(prob, *S.solve_rlmdg_direct(prob))}


def fabricated(case):
    """psi, source q(x, mu) with eps = sigma_s = sigma_a = 1 (sigma_t = 2), exact phi."""
    if case == "cos x":
        psi = lambda x, o: np.cos(x[:, 0])
        q = lambda x, o: -o[0] * np.sin(x[:, 0]) + 2.0 * np.cos(x[:, 0]) - np.cos(x[:, 0])
        phi = lambda x: np.cos(x[:, 0])
    else:
        # (1/2) int cos(x + mu) d mu = sin(1) cos x
        psi = lambda x, o: np.cos(x[:, 0] + o[0])
        q = lambda x, o: -o[0] * np.sin(x[:, 0] + o[0]) + 2.0 * np.cos(x[:, 0] + o[0]) - np.sin(1.0) * np.cos(x[:, 0])
        phi = lambda x: np.sin(1.0) * np.cos(x[:, 0])
    return psi, q, phi


@pytest.mark.parametrize("case", ["cos x", "cos(x+mu)"])
def test_fabricated_orders_match_tab_1d_aniso(case):
    """Example examp-1dfab: P1-DG and RLMDG second order; LMDG second order for the
    isotropic solution, first order for the anisotropic one."""
    psi, q, phi = fabricated(case)
    errs = {}
    for n in (80, 160):
        mesh = Mesh((n,), (1.0,))
        prob = S.Problem(mesh, OMEGA, W, 1.0, 1.0, 1.0, q=q, alpha=psi)
        for name, f in scalar_fluxes(prob).items():
            errs.setdefault(name, []).append(l1_error(mesh, f, phi))
    for name, e in errs.items():
        printed = GOLDEN["tab-1d-aniso"][case][name]["order"][-1]
        assert abs(np.log2(e[0] / e[1]) - printed) < 0.1, (name, e)


def l1_against_field(n, length, coarse, ref, nref, nq=6):
    """int_D |phi_h - phi_ref| for two 1D Q^1 Legendre fields on uniform meshes."""
    pts, wts = tensor_rule(1, nq)
    h, href = length / n, length / nref
    total = 0.0
    for p in range(n):
        x = (p + 0.5) * h + 0.5 * h * pts[:, 0]
        k = np.minimum((x / href).astype(int), nref - 1)
        xi = 2.0 * (x - (k + 0.5) * href) / href
        exact = ref[k, 0] + ref[k, 1] * xi
        total += 0.5 * h * wts @ np.abs(coarse[p, 0] + coarse[p, 1] * pts[:, 0] - exact)
    return total


@pytest.mark.parametrize("eps_key,eps", [("1e-05", 1e-5), ("1", 1.0)])
def test_diffusive_and_transport_regimes_match_tab_1d_eps(eps_key, eps):
    """Example examp-1ddifflim on [0, pi], q = (4/3) sin x, vacuum inflow: orders of all
    three schemes; at eps = 1e-5 (asymptotic preserving) the P1-DG and LMDG errors."""
    length = np.pi
    q = lambda x, o: 4.0 / 3.0 * np.sin(x[:, 0])
    nref = 1280
    pref = S.Problem(Mesh((nref,), (length,)), OMEGA, W, 1.0, 1.0, eps, q=q)
    ref = S.scalar_flux_std(pref, S.solve_std_direct(pref))
    printed = GOLDEN["tab-1d-eps10-5"][eps_key]
    errs = {}
    for n in (20, 40, 80, 160):
        prob = S.Problem(Mesh((n,), (length,)), OMEGA, W, 1.0, 1.0, eps, q=q)
        for name, f in scalar_fluxes(prob).items():
            errs.setdefault(name, []).append(l1_against_field(n, length, f, ref, nref))
    for name, e in errs.items():
        assert abs(np.log2(e[-2] / e[-1]) - printed[name]["order"][-1]) < 0.1, (name, e)
        if eps < 1e-3 and name in ("P1-DG", "LMDG"):
            rel = np.abs(np.array(e) / np.array(printed[name]["error"]) - 1.0)
            assert rel.max() < 0.08, (name, e)
