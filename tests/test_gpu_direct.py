"""The direct x-update (Sec. III-B, the remark on tall blocks after eq.
inversion_lemma2): u = (H_ij^H H_ij + rho I)^{-1}(H_ij^H g'_ij + rho c) with the
n_j x n_j inverse formed in FP64, ghat_ij = H_ij u, evaluated as a correction
of the previous iteration's u (from u = 0 after a reset or a state import).
Besides the parity runs of test_gpu_parity (every case in this form), its
state handling, stop rule, reduced-precision stores and bf16 inverse copy
against the FP64 oracle, whose own direct branch serves blocks with
m_b >= n_b."""
import numpy as np
import pytest

import workloads as W
from oracle import admm as O
from oracle import quant as QZ
from tests._gpu import check_image, gpu_solve, rel, to_device

pytestmark = pytest.mark.gpu

TOL = 1e-5
TOTAL_BOUND = {"bf16": 5e-3, "fp8": 5e-2}


def _tall(name):
    if name == "tall_combined_uneven":
        return W.iid_problem(m=900, n=600, nnz=10, Q=3, P=6, rho=10.0, seed=43, row_off=[0, 200, 500, 900],
                             col_off=[0, 90, 200, 300, 410, 500, 600]), 120
    if name == "tall_auto":
        return W.iid_problem(m=600, n=800, nnz=10, Q=1, P=8, rho=10.0, seed=41), 120
    raise KeyError(name)


def _oracle(p, iters, H=None, **kw):
    return O.solve(p.H if H is None else H, p.g, p.Q, p.P, p.rho, p.lam, iters, p.row_off, p.col_off, **kw)


def test_direct_warm_start_and_state_import(torch_gpu):
    """A warm continuation equals an uninterrupted run bit for bit; the
    oracle's state at iteration 40 imported and run 30 more equals 70 oracle
    iterations (g' of the first continued iteration comes from the imported
    estimates)."""
    torch = torch_gpu
    p, _ = _tall("tall_combined_uneven")
    plan, g, v_full = gpu_solve(torch, p, 70)
    assert plan.info()["direct"] == 1
    plan.solve(g, 40)
    v_warm = plan.solve(g, 30, warm=True)
    assert torch.equal(v_full, v_warm)
    _, _, st40 = _oracle(p, 40)
    v70, _, st70 = _oracle(p, 30, state=st40)
    plan.set_state(40, to_device(torch, st40.v.astype(np.complex64)), to_device(torch, st40.s.astype(np.complex64)),
                   to_device(torch, st40.ghat.astype(np.complex64)))
    v = plan.solve(g, 30, warm=True).cpu().numpy()
    check_image(v, v70, st70.s, p.lam / (p.Q * p.rho))
    k, _, s, gh = plan.get_state()
    assert k == 70
    assert rel(s.cpu().numpy(), st70.s) <= 10 * TOL and rel(gh.cpu().numpy(), st70.ghat) <= 10 * TOL


def test_direct_tolerance_stop_matches_oracle(torch_gpu):
    p, _ = _tall("tall_auto")
    v_ref, hist_ref, _ = _oracle(p, 600, tol=1e-3, check_every=10)
    plan, g, v = gpu_solve(torch_gpu, p, 600, tol=1e-3, check_every=10)
    assert plan.info()["direct"] == 1
    assert plan.iters_done == len(hist_ref) < 600, (plan.iters_done, len(hist_ref))
    assert rel(v.cpu().numpy(), v_ref) <= TOL


def test_direct_lambda_above_max_gives_zero(torch_gpu):
    p, _ = _tall("tall_auto")
    lam = 1.01 * O.lambda_max(p.H, p.g)
    plan, g, v = gpu_solve(torch_gpu, p, 300, lam=lam)
    v_ref, _, _ = O.solve(p.H, p.g, p.Q, p.P, p.rho, lam, 300)
    assert np.max(np.abs(v_ref)) == 0.0
    assert torch_gpu.count_nonzero(v).item() == 0


@pytest.mark.parametrize("name", ["tall_combined_uneven", "tall_auto"])
def test_direct_kkt_matches_oracle(torch_gpu, name):
    p, K = _tall(name)
    plan, g, v = gpu_solve(torch_gpu, p, K)
    got = plan.kkt(g, v)
    want = O.kkt_violation(p.H, p.g, v.cpu().numpy().astype(np.complex128), p.lam)
    assert abs(got - want) <= 1e-9 + 1e-7 * abs(want), (got, want)


@pytest.mark.parametrize("storage", ["bf16", "fp8"])
@pytest.mark.parametrize("name", ["tall_combined_uneven", "tall_auto"])
def test_direct_storage_two_way_error(torch_gpu, storage, name):
    """bf16 / fp8 H in the direct form: the FP64 Gram matrices H^H H are built
    from the dequantised values (row scales inside the column sums); against
    the oracle on the dequantised H the arithmetic bar 1e-5, against the
    oracle on the complex64 H the format's total bound."""
    import paper_1811_05571_amd as A
    p, K = _tall(name)
    Hd = QZ.dequantise(p.H, storage)
    v_deq, _, _ = _oracle(p, K, H=Hd)
    v_c64, _, _ = _oracle(p, K)
    plan = A.Plan(to_device(torch_gpu, p.H), p.Q, p.P, p.rho, p.lam, p.row_off, p.col_off, storage=storage)
    assert plan.info()["direct"] == 1
    v = plan.solve(to_device(torch_gpu, p.g), K).cpu().numpy()
    e_arith, e_total = rel(v, v_deq), rel(v, v_c64)
    print(f"{name} {storage} direct: vs oracle on stored H {e_arith:.2e}, on complex64 H {e_total:.2e}", flush=True)
    assert e_arith <= TOL
    assert e_total <= TOTAL_BOUND[storage]


def test_direct_inverse_bf16(torch_gpu):
    """The bfloat16 copy of the n_j x n_j inverses (pieces added per single
    tile by the z-update): within 2^-8 of the FP32-inverse image and of the
    oracle's."""
    import paper_1811_05571_amd as A
    p, K = _tall("tall_combined_uneven")
    H, g = to_device(torch_gpu, p.H), to_device(torch_gpu, p.g)
    v32 = A.Plan(H, p.Q, p.P, p.rho, p.lam, p.row_off, p.col_off, xupdate="direct").solve(g, K).cpu().numpy()
    plan16 = A.Plan(H, p.Q, p.P, p.rho, p.lam, p.row_off, p.col_off, inverse="bf16", xupdate="direct")
    assert plan16.info()["direct"] == 1
    v16 = plan16.solve(g, K).cpu().numpy()
    ref, _, _ = _oracle(p, K)
    print(f"direct bf16 inverse: vs FP32 inverse {rel(v16, v32):.2e}, vs oracle {rel(v16, ref):.2e}", flush=True)
    assert rel(v16, v32) <= 2.0 ** -8 and rel(v16, ref) <= 2.0 ** -8


def test_direct_has_no_reverse_sweep(torch_gpu):
    import paper_1811_05571_amd as A
    p, _ = _tall("tall_auto")
    plan, g, _ = gpu_solve(torch_gpu, p, 1)
    with pytest.raises(A.ADMMError) as ei:
        plan.solve_record(g, 4, 2)
    assert ei.value.status == "ADMM_EUNSUPPORTED"
