"""GMRES with augmented restarts (LGMRES) through the C ABI.

Restarted GMRES stalls on the reduced systems of small eps, whose spectra reach close
to zero; augmenting each cycle with the corrections of earlier cycles keeps what those
cycles learned.  The augmented solves must reach the same solution: the scalar flux
against the oracle's direct solve, at a bar from the conditioning (the reduced RLMDG
operator of a 32 x 28 mesh at eps = 1e-3 has a 2-norm condition number of about 3e4,
so tol 1e-12 leaves at most ~3e-8; bar 1e-7), for one and several sources, FP64 and
mixed precision.
"""
import numpy as np
import pytest

from gpu_helpers import Case, abi_to_std, rel_err
from oracle import schemes as S
from oracle.dg import Mesh

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1907_01027_amd import lmdg  # noqa: E402

DEV = torch.device("cuda")
M, K = 20, 5


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def direct(case, q, scheme):
    prob = S.Problem(Mesh(case.n, case.length), case.omega, case.w, case.sigma_s, case.sigma_a, case.eps, q=q)
    if scheme == "lmdg":
        return S.scalar_flux_lm(prob, *S.solve_lmdg_direct(prob)).ravel()
    return S.scalar_flux_lm(prob, *S.solve_rlmdg_direct(prob)).ravel()


def solve(s, scheme, mode, nr, nc, augment):
    lmdg.lmdg_set_augment(s.h, augment)
    x = torch.zeros(nr * 4 * nc, dtype=torch.float64, device=DEV)
    phi = torch.zeros_like(x)
    info = lmdg.lmdg_solve(s.h, scheme, mode, 1e-12, M, 20000, x, phi)
    torch.cuda.synchronize()
    return info, phi.cpu().numpy().reshape(nr, 4 * nc)


@pytest.mark.parametrize("scheme", ["lmdg", "rlmdg"])
@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_augmented_solve_against_direct(scheme, mode):
    print(f"case lgmres {scheme} {mode}", flush=True)
    case = Case((32, 28), 8, eps=1e-3, seed=3)
    nc = case.ncell
    s = case.solver()
    info_p, _ = solve(s, scheme, mode, 1, nc, 0)
    info, phi = solve(s, scheme, mode, 1, nc, K)
    s.close()
    print(f"  GMRES({M}) {info_p['iterations']} applications, LGMRES({M}+{K}) {info['iterations']}", flush=True)
    assert info["converged"] == 1
    assert rel_err(abi_to_std(phi[0], nc), direct(case, case.q, scheme)) < 1e-7
    if mode == "fp64":
        # the point of the augmentation: fewer operator applications at the same restart
        assert info["iterations"] < info_p["iterations"]


def test_augmented_stacked_sources():
    print("case lgmres three sources", flush=True)
    case = Case((32, 28), 8, eps=1e-3, seed=5)
    nc = case.ncell
    q = np.random.default_rng(9).uniform(0.0, 1.0, size=(3, nc))
    s = case.solver()
    lmdg.lmdg_set_sources(s.h, T(q))
    info, phi = solve(s, "rlmdg", "fp64", 3, nc, K)
    s.close()
    assert info["converged"] == 1
    for k in range(3):
        assert rel_err(abi_to_std(phi[k], nc), direct(case, q[k], "rlmdg")) < 1e-7, k


def test_augment_clamped_and_validated():
    """k beyond 250 - restart is clamped inside the solve; k outside [0, 249] is rejected."""
    case = Case((9, 7), 4, eps=0.1)
    nc = case.ncell
    s = case.solver()
    for bad in (-1, 250):
        with pytest.raises(lmdg.LmdgError):
            lmdg.lmdg_set_augment(s.h, bad)
    lmdg.lmdg_set_augment(s.h, 249)
    x = torch.zeros(4 * nc, dtype=torch.float64, device=DEV)
    phi = torch.zeros_like(x)
    info = lmdg.lmdg_solve(s.h, "rlmdg", "fp64", 1e-12, 240, 2000, x, phi)
    torch.cuda.synchronize()
    assert info["converged"] == 1
    assert rel_err(abi_to_std(phi.cpu().numpy(), nc), direct(case, case.q, "rlmdg")) < 1e-9
    s.close()
