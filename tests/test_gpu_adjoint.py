"""Adjoint solve and gradients through the C ABI, against the oracle and finite differences.

Bars: J and the three gradients within 1e-9 relative (max-norm) of the oracle's
direct sparse solves on small meshes with both solves at tol 1e-13 (the GMRES
tolerance times the conditioning of these small systems); central finite
differences of the library's own J (relative step 1e-5, solves at tol 1e-13) within
1e-6 relative of the adjoint gradient, the truncation error of the difference
quotient being O(1e-10) relative and the solver error / step O(1e-8).
"""
import numpy as np
import pytest

from gpu_helpers import Case
from oracle import adjoint as OA
from oracle.dg import Mesh

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1907_01027_amd import lmdg  # noqa: E402
from paper_1907_01027_amd.adjoint import box_detector_moments, detector_response  # noqa: E402

DEV = torch.device("cuda")
LO, HI = (0.7, 0.7), (0.9, 0.9)


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def run_adjoint(case, scheme, mode="fp64", tol=1e-13, det=None):
    s = case.solver()
    if det is None:
        det = box_detector_moments(case.n, case.length, LO, HI)
    g = [torch.zeros(case.ncell, dtype=torch.float64, device=DEV) for _ in range(3)]
    J, info = lmdg.lmdg_adjoint_solve(s.h, scheme, mode, T(det), tol, 80, 200000, *g)
    torch.cuda.synchronize()
    s.close()
    return J, [t.cpu().numpy() for t in g], info


@pytest.mark.parametrize("scheme", ["std", "lmdg", "rlmdg"])
@pytest.mark.parametrize("n,order,eps", [((8, 8), 4, 0.5), ((7, 5), 8, 0.05), ((6, 9), 4, 1.0), ((13, 11), 8, 0.2)])
def test_adjoint_matches_oracle(scheme, n, order, eps):
    print(f"adjoint parity {scheme} n={n} S{order} eps={eps}", flush=True)
    case = Case(n, order, key=4, eps=eps, seed=11)
    J, (gs, ga, gq), info = run_adjoint(case, scheme)
    prob = case.prob
    det = OA.detector_moments(Mesh(case.n, case.length), np.array(LO), np.array(HI))
    Jo, gso, gao, gqo = OA.gradients(prob, scheme, det)
    assert info["converged"] == 1
    assert abs(J - Jo) <= 1e-9 * abs(Jo)
    for name, a, b in (("sigma_s", gs, gso), ("sigma_a", ga, gao), ("q", gq, gqo)):
        err = np.abs(a - b).max() / np.abs(b).max()
        assert err < 1e-9, (name, err)


def test_adjoint_full_detector_slopes():
    """A detector with nonzero slope moments in every cell exercises the B_11 solve
    of the LMDG adjoint source (c = B_11^{-1} d_1) and the reconstruction terms of the
    RLMDG adjoint source (R'^T d_1)."""
    case = Case((9, 7), 4, key=4, eps=0.3, seed=5)
    rng = np.random.default_rng(3)
    det = rng.uniform(-1, 1, size=(4, case.ncell)) * 1e-2
    for scheme in ("std", "lmdg", "rlmdg"):
        J, (gs, ga, gq), _ = run_adjoint(case, scheme, det=det)
        Jo, gso, gao, gqo = OA.gradients(case.prob, scheme, det.T.copy())
        assert abs(J - Jo) <= 1e-9 * abs(Jo)
        for a, b in ((gs, gso), (ga, gao), (gq, gqo)):
            assert np.abs(a - b).max() / np.abs(b).max() < 1e-9


def test_rlmdg_adjoint_of_a_reconstruction_variant_unsupported():
    case = Case((4, 4), 4, key=4, eps=1.0, seed=1)
    s = case.solver()
    g = [torch.zeros(case.ncell, dtype=torch.float64, device=DEV) for _ in range(3)]
    det = T(box_detector_moments(case.n, case.length, LO, HI))
    lmdg.lmdg_set_reconstruction(s.h, 3, False)
    with pytest.raises(lmdg.LmdgError) as e:
        lmdg.lmdg_adjoint_solve(s.h, "rlmdg", "fp64", det, 1e-10, 20, 100, *g)
    assert e.value.status == lmdg.LMDG_UNSUPPORTED
    lmdg.lmdg_set_reconstruction(s.h, 2, False)
    J, info = lmdg.lmdg_adjoint_solve(s.h, "rlmdg", "fp64", det, 1e-12, 20, 2000, *g)
    assert info["converged"] == 1
    s.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("scheme", ["lmdg", "rlmdg"])
def test_finite_differences_64(scheme):
    """64^2, S12, eps = 1e-2: seeded (cell, parameter) pairs against central
    differences of J computed by forward solves of the library."""
    print(f"case finite differences 64^2 S12 {scheme}", flush=True)
    case = Case((64, 64), 12, key=4, eps=1e-2, seed=20190704)
    s = case.solver()
    lmdg.lmdg_set_augment(s.h, 20)
    det = T(box_detector_moments(case.n, case.length, LO, HI))
    g = [torch.zeros(case.ncell, dtype=torch.float64, device=DEV) for _ in range(3)]
    J0, info = lmdg.lmdg_adjoint_solve(s.h, scheme, "fp64", det, 1e-13, 80, 400000, *g)
    grads = [t.cpu().numpy() for t in g]
    x = torch.zeros(4 * case.ncell, dtype=torch.float64, device=DEV)
    phi = torch.zeros_like(x)
    base = [case.sigma_s.copy(), case.sigma_a.copy(), case.q.copy()]
    # cells near and inside the detector, where the response is not negligible
    rng = np.random.default_rng(20190704)
    ii = rng.integers(36, 64, size=8)
    jj = rng.integers(36, 64, size=8)
    pars = rng.integers(0, 3, size=8)
    for i, j, par in zip(ii, jj, pars):
        cell = int(j) * 64 + int(i)
        vals = []
        for sgn in (1, -1):
            arrs = [a.copy() for a in base]
            hstep = 1e-5 * arrs[par][cell]
            arrs[par][cell] += sgn * hstep
            lmdg.lmdg_set_materials(s.h, T(arrs[0]), T(arrs[1]), T(case.eps), T(arrs[2]))
            lmdg.lmdg_solve(s.h, scheme, "fp64", 1e-13, 80, 400000, x, phi)
            vals.append(float(torch.dot(det.reshape(-1), phi)))
        fd = (vals[0] - vals[1]) / (2 * hstep)
        gv = grads[par][cell]
        print(f"cell {cell} par {par}: adjoint {gv:.10e} fd {fd:.10e}", flush=True)
        assert abs(fd - gv) <= 1e-6 * max(abs(gv), 1e-3 * np.abs(grads[par]).max())
    s.close()


def test_autograd_function_and_mixed():
    case = Case((24, 20), 8, key=4, eps=0.1, seed=9)
    s = case.solver()
    det = T(box_detector_moments(case.n, case.length, LO, HI))
    ss = T(case.sigma_s).requires_grad_()
    sa = T(case.sigma_a).requires_grad_()
    q = T(case.q).requires_grad_()
    J = detector_response(s, ss, sa, q, T(case.eps), det, scheme="lmdg", tol=1e-13)
    (J * 2.0).backward()
    g = [torch.zeros(case.ncell, dtype=torch.float64, device=DEV) for _ in range(3)]
    J2, _ = lmdg.lmdg_adjoint_solve(s.h, "lmdg", "fp64", det, 1e-13, 60, 100000, *g)
    assert abs(float(J.detach()) - J2) <= 1e-12 * abs(J2)
    for a, b in ((ss.grad, g[0]), (sa.grad, g[1]), (q.grad, g[2])):
        assert torch.allclose(a, 2.0 * b, rtol=1e-12, atol=0)
    # mixed precision (FP32 sweeps inside FP64 refinement) to the same FP64 tolerance
    gm = [torch.zeros_like(t) for t in g]
    Jm, info = lmdg.lmdg_adjoint_solve(s.h, "lmdg", "mixed", det, 1e-11, 60, 100000, *gm)
    assert info["converged"] == 1
    assert abs(Jm - J2) <= 1e-9 * abs(J2)
    for a, b in zip(gm, g):
        assert float((a - b).abs().max() / b.abs().max()) < 1e-8
    s.close()


def test_autograd_rlmdg_and_mixed():
    """The autograd wrapper with the reconstructed scheme, and its mixed-precision adjoint."""
    case = Case((20, 17), 8, key=4, eps=0.1, seed=13)
    s = case.solver()
    det = T(box_detector_moments(case.n, case.length, LO, HI))
    ss = T(case.sigma_s).requires_grad_()
    sa = T(case.sigma_a).requires_grad_()
    q = T(case.q).requires_grad_()
    J = detector_response(s, ss, sa, q, T(case.eps), det, scheme="rlmdg", tol=1e-13)
    J.backward()
    Jo, gso, gao, gqo = OA.gradients(case.prob, "rlmdg",
                                     OA.detector_moments(Mesh(case.n, case.length), np.array(LO), np.array(HI)))
    assert abs(float(J.detach()) - Jo) <= 1e-9 * abs(Jo)
    for a, b in ((ss.grad, gso), (sa.grad, gao), (q.grad, gqo)):
        assert np.abs(a.cpu().numpy() - b).max() / np.abs(b).max() < 1e-9
    g = [torch.zeros(case.ncell, dtype=torch.float64, device=DEV) for _ in range(3)]
    Jm, info = lmdg.lmdg_adjoint_solve(s.h, "rlmdg", "mixed", det, 1e-11, 60, 100000, *g)
    assert info["converged"] == 1
    assert abs(Jm - Jo) <= 1e-8 * abs(Jo)
    for a, b in zip(g, (gso, gao, gqo)):
        err = np.abs(a.cpu().numpy() - b).max() / np.abs(b).max()
        print(f"mixed RLMDG gradient vs oracle: {err:.2e}", flush=True)
        assert err < 1e-7
    s.close()
