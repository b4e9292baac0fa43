"""admm_kkt_noalloc (static device scratch) against admm_kkt (workspace
scratch): the same kernels, so the same FP64 result, on two calls in a row,
the second on a smaller plan; and the size limit."""
import numpy as np
import pytest

import workloads as W
from tests._gpu import to_device


def _plan_and_image(torch, prob, iters=30):
    import paper_1811_05571_amd as A
    H = to_device(torch, prob.H)
    g = to_device(torch, prob.g)
    plan = A.Plan(H, prob.Q, prob.P, prob.rho, prob.lam, prob.row_off, prob.col_off)
    v = plan.solve(g, iters)
    return plan, g, v


@pytest.mark.gpu
def test_kkt_noalloc_matches_kkt_on_two_calls(torch_gpu):
    torch = torch_gpu
    big = W.iid_problem(m=300, n=2000, nnz=12, Q=3, P=5, rho=10.0, seed=41)
    small = W.iid_problem(m=128, n=600, nnz=6, Q=2, P=2, rho=10.0, seed=42)
    for prob in (big, small):
        plan, g, v = _plan_and_image(torch, prob)
        want = plan.kkt(g, v)
        got = plan.kkt_noalloc(g, v)
        print(f"kkt {prob.m}x{prob.n} Q={prob.Q} P={prob.P}: workspace {want!r} static {got!r}", flush=True)
        assert np.isfinite(want) and want > 0
        assert got == want
    # the first plan again, after the smaller one used the array
    plan, g, v = _plan_and_image(torch, big)
    assert plan.kkt_noalloc(g, v) == plan.kkt(g, v)


@pytest.mark.gpu
def test_kkt_noalloc_rejects_a_plan_beyond_the_scratch(torch_gpu):
    import paper_1811_05571_amd as A
    torch = torch_gpu
    # 64 x 1.2 M: the FP64 adjoint partials alone take 19 MB > 16 MiB
    m, n = 64, 1_200_000
    gen = torch.Generator(device="cuda").manual_seed(5)
    H = torch.randn((m, n), dtype=torch.complex64, device="cuda", generator=gen) / 8.0
    g = torch.randn(m, dtype=torch.complex64, device="cuda", generator=gen)
    plan = A.Plan(H, 1, 1, 1.0, 0.5)
    v = torch.zeros(n, dtype=torch.complex64, device="cuda")
    with pytest.raises(A.ADMMError) as e:
        plan.kkt_noalloc(g, v)
    assert e.value.status == "ADMM_EWORKSPACE"
    assert np.isfinite(plan.kkt(g, v))
