"""The allocation-free spatial-solve entry point (pmgrit_phi_noalloc, for callers that cannot allocate)
against pmgrit_phi through the C ABI: the same kernels on the same inputs, so results and V-cycle
counts are bitwise equal, on two calls in a row (the second with fewer right-hand sides), for a plan
with every work vector in LDS, one with the work vectors in the scratch (FP32, h = 2^-7), and the
h-multigrid p = 1 solve (whose levels live in the scratch); sizes beyond the fixed scratch are
refused."""
import sys

import numpy as np
import pytest

try:  # imported at collection time so a slow first import is not charged to a test's timeout
    import torch as _torch  # noqa: F401
except Exception:  # pragma: no cover
    _torch = None

import paper_2107_05337_amd as pm
from paper_2107_05337_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a visible MI355X"
    return T


@pytest.mark.parametrize("p,n,precision,coarse", [(3, 16, 0, 0), (4, 128, 1, 0), (2, 32, 0, 1)])
def test_noalloc_matches_phi(torch, p, n, precision, coarse):
    say(f"case phi_noalloc p={p} n={n} precision={precision} coarse={coarse}")
    cfg = W.small("x", p, n, 16)
    d = cfg["instances"][0]
    S = pm.Solver([pm.problem(p, n, 16, d["kappa"], d["T"], 0)], pm.default_mgrit_opts(cfactor=4, coarsest_max=4),
                  pm.default_solver_opts(precision=precision, coarse=coarse), device=0)
    nd = S.dims()[0]
    say(f"  n_dof {nd}, LDS placement {S.group_info(0)['lds_mask']}")
    rng = np.random.default_rng(p + n)
    for level, nrhs in ((0, 9), (1, 4)):
        B = torch.tensor(rng.standard_normal((nrhs, nd)), device="cuda")
        X0 = torch.tensor(rng.standard_normal((nrhs, nd)) * 0.1, device="cuda")
        xa, xb = X0.clone(), X0.clone()
        va = torch.zeros(nrhs, dtype=torch.int32, device="cuda")
        vb = torch.zeros(nrhs, dtype=torch.int32, device="cuda")
        S.phi(0, level, B, xa, va)
        S.phi_noalloc(0, level, B, xb, vb)
        torch.cuda.synchronize()
        assert torch.equal(xa, xb), (level, nrhs)
        assert torch.equal(va, vb) and int(va.min()) >= 1
    S.close()


def test_noalloc_refuses_oversize(torch):
    # h = 2^-8, p = 4: about 400 000 scratch doubles per right-hand side, so 64 exceed 2^23
    S = pm.Solver([pm.problem(4, 256, 16)], pm.default_mgrit_opts(cfactor=4, coarsest_max=4),
                  pm.default_solver_opts(precision=1), device=0)
    nd = S.dims()[0]
    B = torch.zeros((64, nd), dtype=torch.float64, device="cuda")
    X = torch.zeros_like(B)
    with pytest.raises(pm.PmgritError) as e:
        S.phi_noalloc(0, 0, B, X)
    assert e.value.code == -1 and "scratch" in str(e.value)
    # a size within the limit works and matches pmgrit_phi
    B = torch.tensor(np.random.default_rng(3).standard_normal((4, nd)), device="cuda")
    xa, xb = torch.zeros_like(B), torch.zeros_like(B)
    S.phi(0, 0, B, xa)
    S.phi_noalloc(0, 0, B, xb)
    torch.cuda.synchronize()
    assert torch.equal(xa, xb)
    S.close()
