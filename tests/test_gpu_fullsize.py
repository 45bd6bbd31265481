"""Full-size parity: the 256 x 256, S8, eps = 1e-3 RLMDG workload in the launch
configuration the benchmark times (one handle, FP64 operator applications).

The oracle assembles the whole operator (about a minute and 13 GB of host memory)
and applies it once; every output element is compared at the FP64 bar (1e-12)."""
import numpy as np
import pytest

from gpu_helpers import Case, abi_to_lm, lm_to_abi, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import schemes as S  # noqa: E402
from paper_1907_01027_amd import lmdg  # noqa: E402


@pytest.mark.timeout(900)
def test_workload2_operator_and_rhs_full_size():
    print("case full-size 256x256 S8 RLMDG apply/rhs", flush=True)
    case = Case((256, 256), 8, key=2)
    nc = case.ncell
    dev = torch.device("cuda")
    s = case.solver()
    x = np.random.default_rng(11).normal(size=4 * nc)
    y = torch.zeros(4 * nc, dtype=torch.float64, device=dev)
    b = torch.zeros(4 * nc, dtype=torch.float64, device=dev)
    lmdg.lmdg_apply(s.h, "rlmdg", "fp64", torch.tensor(x, device=dev), y)
    lmdg.lmdg_rhs(s.h, "rlmdg", "fp64", b)
    torch.cuda.synchronize()
    y, b = y.cpu().numpy(), b.cpu().numpy()
    s.close()
    print("oracle assembly", flush=True)
    red = S.LowMemoryReduced(case.prob, reconstructed=True)
    print("oracle apply", flush=True)
    assert rel_err(y, lm_to_abi(red.apply(abi_to_lm(x, nc)), nc)) < 1e-12
    assert rel_err(b, lm_to_abi(red.rhs(), nc)) < 1e-12
