"""The device side of the split chooser: coefficients calibrated from timed
probe plans, and the measuring chooser that times the model's shortlist."""
import numpy as np
import pytest

import workloads as W
from tests._gpu import to_device

pytestmark = pytest.mark.gpu


def test_calibrate_and_measure(torch_gpu):
    import paper_1811_05571_amd as A
    p = W.iid_problem(m=512, n=4096, nnz=10, Q=4, P=1, rho=1.0, seed=51)
    H, g = to_device(torch_gpu, p.H), to_device(torch_gpu, p.g)
    coef = A.calibrate(H, g)
    print("calibrated:", coef, flush=True)
    assert coef.shape == (10,) and np.all(np.isfinite(coef)) and np.all(coef >= 0)
    assert coef[:5].sum() > 0 and coef[5:].sum() > 0
    K = 50
    short, _ = A.shortlist(p.m, p.n, K, 4, coef=coef)
    q, pp, t = A.choose_split_measure(H, g, K, coef=coef, shortlist_len=4)
    assert (q, pp) in [(a, b) for a, b, _ in short] and t > 0
    # a shortlist of one is the model's own pick
    q1, p1, _ = A.choose_split_measure(H, g, K, coef=coef, shortlist_len=1)
    assert (q1, p1) == A.choose_split(p.m, p.n, K, coef=coef)[:2]
    # the chosen split solves like any other (the plan is built from scratch)
    plan = A.Plan(H, q, pp, p.rho, p.lam)
    v = plan.solve(g, 5)
    assert bool(torch_gpu.isfinite(torch_gpu.view_as_real(v)).all())


def test_measure_rejects_a_too_small_workspace(torch_gpu):
    import paper_1811_05571_amd as A
    p = W.iid_problem(m=256, n=1024, nnz=5, Q=1, P=1, rho=1.0, seed=52)
    H, g = to_device(torch_gpu, p.H), to_device(torch_gpu, p.g)
    tiny = torch_gpu.empty(1 << 12, dtype=torch_gpu.uint8, device="cuda")
    with pytest.raises(A.ADMMError) as ei:
        A.choose_split_measure(H, g, 10, shortlist_len=3, workspace=tiny)
    assert ei.value.status == "ADMM_EWORKSPACE"
    with pytest.raises(A.ADMMError) as ei:
        A.calibrate(H, g, workspace=tiny)
    assert ei.value.status == "ADMM_EWORKSPACE"
