"""Failure handling of the sweeps' bounded waits, forced from the host.

Every wait of a sweep for a progress word is bounded; lmdg_set_wait_limit makes every
wait target a value no producer writes and caps the polls, so every wait that is
reached gives up quickly while every kernel still runs to completion.  The
asynchronous calls return at once; the next synchronising call must report the
failure (LMDG_HIP_ERROR), and after the normal policy is restored the same calls give
the oracle's numbers again.
"""
import numpy as np
import pytest

from gpu_helpers import Case, abi_to_lm, lm_to_abi, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1907_01027_amd import lmdg  # noqa: E402

DEV = torch.device("cuda")


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_failed_wait_is_reported_2d(prec):
    print(f"case failed wait 2D {prec}", flush=True)
    case = Case((48, 40), 8, eps=0.1)   # three strips per quadrant: every item past the first waits
    nc = case.ncell
    s = case.solver()
    x = np.random.default_rng(7).normal(size=4 * nc)
    y = torch.zeros(4 * nc, dtype=torch.float64, device=DEV)
    lmdg.lmdg_set_wait_limit(s.h, 64, unreachable=True)
    lmdg.lmdg_apply(s.h, "rlmdg", prec, T(x), y)     # enqueues and returns
    with pytest.raises(lmdg.LmdgError) as exc:
        lmdg.lmdg_synchronize(s.h)
    assert exc.value.status == lmdg.LMDG_HIP_ERROR
    # the flag was cleared by the report
    lmdg.lmdg_set_wait_limit(s.h, 1 << 25, unreachable=False)
    lmdg.lmdg_synchronize(s.h)
    lmdg.lmdg_apply(s.h, "rlmdg", prec, T(x), y)
    lmdg.lmdg_synchronize(s.h)
    ref = lm_to_abi(case.reduced("rlmdg").apply(abi_to_lm(x, nc)), nc)
    assert rel_err(y.cpu().numpy(), ref) < (1e-12 if prec == "fp64" else 2e-5)
    # a solve reports a failed wait itself
    lmdg.lmdg_set_wait_limit(s.h, 64, unreachable=True)
    xs = torch.zeros(4 * nc, dtype=torch.float64, device=DEV)
    with pytest.raises(lmdg.LmdgError) as exc:
        lmdg.lmdg_solve(s.h, "rlmdg", "fp64", 1e-8, 10, 10, xs)
    assert exc.value.status == lmdg.LMDG_HIP_ERROR
    lmdg.lmdg_set_wait_limit(s.h, 1 << 25, unreachable=False)
    lmdg.lmdg_synchronize(s.h)
    s.close()


def test_failed_wait_is_reported_3d():
    print("case failed wait 3D", flush=True)
    from oracle.quadrature import level_symmetric
    from paper_1907_01027_amd.workloads import materials
    n = (6, 20, 3)   # two strips and three planes: both kinds of wait occur
    nc = int(np.prod(n))
    ss, sa, ep, q = materials(5, n=n)
    om, w = level_symmetric(4, 3)
    s = lmdg.Solver(n, (1.0, 1.0, 1.0), om, w)
    lmdg.lmdg_set_materials(s.h, T(ss), T(sa), T(ep), T(q[0]))
    x = T(np.random.default_rng(8).normal(size=8 * nc))
    y = torch.zeros(8 * nc, dtype=torch.float64, device=DEV)
    lmdg.lmdg_set_wait_limit(s.h, 64, unreachable=True)
    lmdg.lmdg_apply(s.h, "rlmdg", "fp64", x, y)
    with pytest.raises(lmdg.LmdgError) as exc:
        lmdg.lmdg_synchronize(s.h)
    assert exc.value.status == lmdg.LMDG_HIP_ERROR
    lmdg.lmdg_set_wait_limit(s.h, 1 << 25, unreachable=False)
    lmdg.lmdg_apply(s.h, "rlmdg", "fp64", x, y)
    lmdg.lmdg_synchronize(s.h)
    s.close()


def test_wait_limit_arguments():
    case = Case((8, 8), 4, eps=0.1)
    s = case.solver()
    for spins, unreachable in ((0, 0), (-5, 0)):
        with pytest.raises(lmdg.LmdgError):
            lmdg.lmdg_set_wait_limit(s.h, spins, unreachable)
    assert lmdg.library().lmdg_set_wait_limit(s.h, 10, 2) == lmdg.LMDG_INVALID_ARG
    s.close()
