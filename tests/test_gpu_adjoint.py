"""Adjoint form: hand-written reverse mode of K unrolled iterations, checked
against (i) the FP64 oracle's autograd gradient (torch-CPU twin of the
oracle) and (ii) central finite differences of the GPU forward with a
relative step of 1e-3, for dL/dg (directional), dL/dlambda and dL/drho with
L = |v^K - u_true|^2.  Complex64 forward, FP32 adjoint."""
import numpy as np
import pytest

import workloads as W
from oracle import admm as O
from oracle import admm_torch as OT
from tests._gpu import rel, to_device

pytestmark = pytest.mark.gpu

# FP32 adjoint vs FP64 autograd (normalised error on dL/dg, relative on scalars)
TOL_AUTOGRAD = 2e-4
# central differences (step 1e-3 relative) of the FP32 forward vs the adjoint
TOL_FD = 2e-2


def _cases():
    return {
        "consensus": (W.iid_problem(m=128, n=1000, nnz=8, Q=4, P=1, rho=1.0, seed=21), 60),
        "combined_uneven": (W.iid_problem(m=300, n=2000, nnz=15, Q=3, P=5, rho=10.0, seed=3,
                                          row_off=[0, 90, 200, 300],
                                          col_off=[0, 333, 800, 1201, 1600, 2000]), 40),
        "cra_small": (W.cra_problem(n_tx=6, n_rx=6, n_f=8, nx=12, ny=12, nz=6, Q=2, P=2, rho=10.0,
                                    patch=(5, 2), iters=50, seed=22), 50),
        # 150 x 125 blocks, taller than wide: the twin differentiates the direct solve
        "tall_sectioning": (W.iid_problem(m=150, n=500, nnz=8, Q=1, P=4, rho=10.0, seed=23), 40),
        # lambda = 0: no threshold, the unrolled map is smooth in g and rho
        "lambda_zero": (W.iid_problem(m=128, n=600, nnz=8, Q=2, P=2, rho=10.0, lam_ratio=0.0, seed=24), 40),
    }


def _plan(torch, p, rho=None, storage="c64", inverse="c64"):
    import paper_1811_05571_amd as A
    return A.Plan(to_device(torch, p.H), p.Q, p.P, p.rho if rho is None else rho, p.lam, p.row_off, p.col_off,
                  storage=storage, inverse=inverse)


def _loss_and_grad_v(v, u_true):
    return float(np.sum(np.abs(v - u_true) ** 2)), 2 * (v - u_true)


@pytest.mark.parametrize("name", ["consensus", "combined_uneven", "cra_small", "tall_sectioning", "lambda_zero"])
def test_adjoint_matches_oracle_autograd(torch_gpu, name):
    torch = torch_gpu
    p, K = _cases()[name]
    plan = _plan(torch, p)
    g = to_device(torch, p.g)
    v, tape = plan.solve_record(g, K, interval=7)
    v = v.cpu().numpy()
    _, gv = _loss_and_grad_v(v.astype(np.complex128), p.u_true)
    gg, dl, dr = plan.backward(g, to_device(torch, gv.astype(np.complex64)), tape)
    tg, tl, tr, tv = OT.gradients(p.H.astype(np.complex128), p.g.astype(np.complex128), p.Q, p.P, p.rho, p.lam, K,
                                  gv, p.row_off, p.col_off)
    assert rel(v, tv) <= 1e-5
    eg, el, er = rel(gg.cpu().numpy(), tg), abs(dl - tl) / abs(tl), abs(dr - tr) / abs(tr)
    print(f"{name}: dL/dg {eg:.2e}  dL/dlam {el:.2e} ({dl:.6g} vs {tl:.6g})  dL/drho {er:.2e} ({dr:.6g} vs {tr:.6g})")
    assert eg <= TOL_AUTOGRAD and el <= TOL_AUTOGRAD and er <= TOL_AUTOGRAD


@pytest.mark.parametrize("storage", ["bf16", "fp8"])
def test_adjoint_reduced_storage_vs_oracle(torch_gpu, storage):
    """With H stored in bf16 or fp8 the forward and the reverse sweep both use
    the stored values: the gradients match the oracle's autograd on the
    dequantised H."""
    from oracle import quant as QZ
    torch = torch_gpu
    p, K = _cases()["cra_small"]
    plan = _plan(torch, p, storage=storage)
    g = to_device(torch, p.g)
    v, tape = plan.solve_record(g, K, interval=7)
    v = v.cpu().numpy()
    _, gv = _loss_and_grad_v(v.astype(np.complex128), p.u_true)
    gg, dl, dr = plan.backward(g, to_device(torch, gv.astype(np.complex64)), tape)
    Hd = QZ.dequantise(p.H, storage)
    tg, tl, tr, tv = OT.gradients(Hd.astype(np.complex128), p.g.astype(np.complex128), p.Q, p.P, p.rho, p.lam, K,
                                  gv, p.row_off, p.col_off)
    assert rel(v, tv) <= 1e-5
    eg, el, er = rel(gg.cpu().numpy(), tg), abs(dl - tl) / abs(tl), abs(dr - tr) / abs(tr)
    print(f"{storage}: dL/dg {eg:.2e}  dL/dlam {el:.2e}  dL/drho {er:.2e}")
    assert eg <= TOL_AUTOGRAD and el <= TOL_AUTOGRAD and er <= TOL_AUTOGRAD


def _trace(plan, g, K):
    """(v^K, zero pattern of v after each of the K iterations from zero): one
    warm single-iteration solve at a time, the same iterates as one solve."""
    plan.solve(g, 0)
    pats = []
    for _ in range(K):
        v = plan.solve(g, 1, warm=True)
        pats.append((v == 0).cpu().numpy())
    return v.cpu().numpy(), np.stack(pats)


def _fd_check(E, x0, h, ad, scale):
    """Central difference of the loss at x0 (step h) against the adjoint value
    ad.  E(x) -> (loss, zero patterns of v over the iterations).  A soft-
    threshold kink is crossed inside [x0 - h, x0 + h] exactly when some
    iteration's zero pattern differs between x0 - h, x0 and x0 + h; without
    one the map is smooth there and the central difference must match
    (TOL_FD); with one the derivative at x0 of the piecewise-smooth map,
    which the adjoint computes, lies between the two one-sided quotients.
    Returns True when a kink was crossed."""
    (fp, sp), (f0, s0), (fm, sm) = E(x0 + h), E(x0), E(x0 - h)
    c = (fp - fm) / (2 * h)
    tol = TOL_FD * (abs(c) + scale)
    if np.array_equal(sp, s0) and np.array_equal(sm, s0):
        assert abs(c - ad) <= tol, ("no kink crossed, yet the central difference misses", c, ad)
        return False
    fwd, bwd = (fp - f0) / h, (f0 - fm) / h
    assert min(fwd, bwd) - tol <= ad <= max(fwd, bwd) + tol, ("adjoint outside the one-sided slopes", fwd, bwd, ad)
    return True


def _fd_all(torch, p, K, interval, inverse="c64", directions=4, seed=5, check_lambda=True, g_step=1e-3,
            rho_step=1e-3):
    """The adjoint of K recorded iterations against central differences in
    `directions` random unit directions of g (step g_step |g|), in lambda
    (step 1e-3 lambda) and (FP32 inverses) in rho (step rho_step rho).
    Returns (kinks crossed, checks)."""
    g = to_device(torch, p.g)
    u_true = p.u_true.astype(np.complex128)

    def E(gg=None, lam=None, rho=None):
        plan = _plan(torch, p, rho=rho, inverse=inverse)
        if lam is not None:
            plan.set_lambda(lam)
        v, pats = _trace(plan, to_device(torch, gg) if gg is not None else g, K)
        plan.close()
        return float(np.sum(np.abs(v.astype(np.complex128) - u_true) ** 2)), pats

    plan = _plan(torch, p, inverse=inverse)
    v, tape = plan.solve_record(g, K, interval=interval)
    _, gv = _loss_and_grad_v(v.cpu().numpy().astype(np.complex128), u_true)
    gg, dl, dr = plan.backward(g, to_device(torch, gv.astype(np.complex64)), tape)
    gg = gg.cpu().numpy().astype(np.complex128)
    plan.close()
    rng = np.random.default_rng(seed)
    kinks = checks = 0
    for _ in range(directions):
        d = rng.standard_normal(p.m) + 1j * rng.standard_normal(p.m)
        d /= np.linalg.norm(d)
        h = g_step * np.linalg.norm(p.g)
        kinks += _fd_check(lambda t: E(gg=(p.g + t * d).astype(np.complex64)), 0.0, h,
                           float(np.real(np.vdot(gg, d))), 1e-2 * np.linalg.norm(gg))
        checks += 1
    if check_lambda:
        kinks += _fd_check(lambda x: E(lam=x), p.lam, 1e-3 * p.lam, dl, 0.0)
        checks += 1
    if inverse == "c64":
        kinks += _fd_check(lambda x: E(rho=x), p.rho, rho_step * p.rho, dr, 1e-6)
        checks += 1
    return kinks, checks


@pytest.mark.parametrize("name,inverse", [("consensus", "c64"), ("cra_small", "c64"), ("cra_small", "bf16")])
def test_adjoint_matches_central_differences(torch_gpu, name, inverse):
    """With the bfloat16 inverse copy the reverse sweep applies the same
    rounded inverse, so for g and lambda it is the adjoint of the map the
    forward computes.  The rounded inverse is a step function of rho (a step of
    1e-3 rho moves its entries by about one bf16 step), so the rho derivative,
    taken through the unrounded inverse, is checked with the FP32 inverse only."""
    p, K = _cases()[name]
    kinks, checks = _fd_all(torch_gpu, p, K, 10, inverse)
    print(f"{name} ({inverse} inverse): {kinks} of {checks} differences crossed a soft-threshold kink")


def test_adjoint_smooth_map_central_differences(torch_gpu):
    """lambda = 0 leaves the unrolled map without soft-threshold kinks: every
    central difference in g and in rho must match the adjoint (TOL_FD), and
    the zero patterns confirm that no kink was crossed.  (With lambda > 0 a
    step of 1e-3 crosses some kink among the thousands of entries and tens of
    iterations almost always, so there only the one-sided bracket applies.)
    Without the threshold v^K is affine in g and the loss quadratic, so the
    central difference in g is exact for any step: a step of half of |g|
    keeps the FP32 rounding of the forward (about 1e-6 in the loss) far below
    the difference; in rho, where the map is curved, a step of 1e-2 rho."""
    p, K = _cases()["lambda_zero"]
    kinks, checks = _fd_all(torch_gpu, p, K, 10, check_lambda=False, g_step=0.5, rho_step=1e-2)
    assert kinks == 0 and checks == 5


def test_autograd_function(torch_gpu):
    import paper_1811_05571_amd as A
    torch = torch_gpu
    p, K = _cases()["combined_uneven"]
    plan = _plan(torch, p)
    g = to_device(torch, p.g).requires_grad_(True)
    lam = torch.tensor(p.lam, dtype=torch.float64, requires_grad=True)
    rho = torch.tensor(p.rho, dtype=torch.float64, requires_grad=True)
    v = A.unrolled(g, lam, rho, plan, K, 10)
    ut = to_device(torch, p.u_true.astype(np.complex64))
    loss = ((v - ut).abs() ** 2).sum()
    loss.backward()
    plan2 = _plan(torch, p)
    v2, tape = plan2.solve_record(to_device(torch, p.g), K, 10)
    gg, dl, dr = plan2.backward(to_device(torch, p.g), 2 * (v2 - ut), tape)
    assert rel(g.grad.cpu().numpy(), gg.cpu().numpy()) <= 1e-6
    assert abs(lam.grad.item() - dl) <= 1e-6 * abs(dl) and abs(rho.grad.item() - dr) <= 1e-6 * abs(dr)


def test_state_after_backward(torch_gpu):
    """The reverse sweep leaves the plan at the end of the first checkpoint
    interval: get_state reports that iteration and its image."""
    torch = torch_gpu
    p, K = _cases()["consensus"]
    plan = _plan(torch, p)
    g = to_device(torch, p.g)
    v, tape = plan.solve_record(g, K, 7)
    plan.backward(g, torch.zeros_like(v), tape)
    k, vs, _, _ = plan.get_state()
    assert k == 7
    v7, _, _ = O.solve(p.H, p.g, p.Q, p.P, p.rho, p.lam, 7, p.row_off, p.col_off)
    assert rel(vs.cpu().numpy(), v7) <= 1e-5
    # a tape serves more than one backward call
    gg1 = plan.backward(g, v, tape)[0]
    gg2 = plan.backward(g, v, tape)[0]
    assert torch.equal(gg1, gg2)


def test_tape_errors(torch_gpu):
    import paper_1811_05571_amd as A
    torch = torch_gpu
    p, K = _cases()["consensus"]
    g = to_device(torch, p.g)
    plan, other = _plan(torch, p), _plan(torch, p)
    v, tape = plan.solve_record(g, 10, 5)
    gv = torch.zeros(p.n, dtype=torch.complex64, device="cuda")
    with pytest.raises(A.ADMMError) as ei:
        other.backward(g, gv, tape)
    assert ei.value.status == "ADMM_ESTATE"
    plan.set_lambda(2 * p.lam)
    with pytest.raises(A.ADMMError) as ei:
        plan.backward(g, gv, tape)
    assert ei.value.status == "ADMM_ESTATE"
    with pytest.raises(A.ADMMError) as ei:
        A.lib().admm_solve_record(plan.handle, g.data_ptr(), 10, 5, tape.data_ptr(), 16, v.data_ptr(), None) and None
        raise A.ADMMError(A.lib().admm_solve_record(plan.handle, g.data_ptr(), 10, 5, tape.data_ptr(), 16,
                                                    v.data_ptr(), None), "record")
    assert ei.value.status == "ADMM_EWORKSPACE"


def test_eight_scene_batch_gradients(torch_gpu):
    """Eight scenes of a small CRA geometry (seeds 2000..2007, consensus,
    sectioning and combined splits, uneven where Q or P is 3), K = 100 with a
    checkpoint every 10 iterations: every scene's v^K and adjoint match the
    oracle and its autograd gradient."""
    torch = torch_gpu
    splits = [(2, 2), (2, 4), (4, 2), (1, 2), (2, 1), (4, 4), (2, 3), (3, 2)]
    worst_v = worst = 0.0
    for seed, (Q, P) in zip(range(2000, 2008), splits):
        p = W.cra_problem(n_tx=4, n_rx=4, n_f=8, nx=10, ny=10, nz=5, Q=Q, P=P, rho=10.0, patch=(4, 2),
                          iters=100, seed=seed)
        plan = _plan(torch, p)
        g = to_device(torch, p.g)
        v, tape = plan.solve_record(g, 100, 10)
        v = v.cpu().numpy()
        _, gv = _loss_and_grad_v(v.astype(np.complex128), p.u_true)
        gg, dl, dr = plan.backward(g, to_device(torch, gv.astype(np.complex64)), tape)
        tg, tl, tr, tv = OT.gradients(p.H.astype(np.complex128), p.g.astype(np.complex128), p.Q, p.P, p.rho, p.lam,
                                      100, gv, p.row_off, p.col_off)
        e = max(rel(gg.cpu().numpy(), tg), abs(dl - tl) / abs(tl), abs(dr - tr) / abs(tr))
        print(f"scene {seed} (Q={Q}, P={P}): v {rel(v, tv):.2e}, max gradient rel err {e:.2e}")
        worst_v, worst = max(worst_v, rel(v, tv)), max(worst, e)
        plan.close()
    assert worst_v <= 1e-5
    assert worst <= TOL_AUTOGRAD
