"""Helpers shared by the GPU tests: move a generated problem to the device,
run the HIP solver through the C ABI binding, and compare images."""
import numpy as np


def to_device(torch, arr):
    return torch.from_numpy(np.ascontiguousarray(arr)).to("cuda")


def gpu_solve(torch, prob, iters, rho=None, lam=None, Q=None, P=None, row_off=None, col_off=None,
              history=False, two_pass=False, xupdate="auto", **kw):
    import paper_1811_05571_amd as A
    H = to_device(torch, prob.H)
    g = to_device(torch, prob.g)
    plan = A.Plan(H, Q or prob.Q, P or prob.P, rho if rho is not None else prob.rho,
                  lam if lam is not None else prob.lam,
                  row_off if row_off is not None else prob.row_off,
                  col_off if col_off is not None else prob.col_off, two_pass=two_pass, xupdate=xupdate)
    out = plan.solve(g, iters, history=history, **kw)
    return plan, g, out


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def check_image(v, v_ref, s_ref, kappa, tol=1e-5, margin=1e-4):
    """The image against the oracle's: normalised L2 error <= tol, largest
    element error <= tol * max|v_ref|, and the same zero pattern away from
    the threshold.  The oracle's last pre-threshold mean is a = v + mean_i s^i
    (its dual update s^K = s^{K-1} + u - v gives mean s^K + v = mean u +
    mean s^{K-1}); entries with ||a| - kappa| <= margin * max|a| are too close
    to the kink to decide and are left out of the pattern check.
    Returns (L2 error, max element error, entries compared)."""
    v = np.asarray(v, dtype=np.complex128)
    v_ref = np.asarray(v_ref, dtype=np.complex128)
    err = rel(v, v_ref)
    scale = float(np.max(np.abs(v_ref)))
    emax = float(np.max(np.abs(v - v_ref))) / (scale if scale > 0 else 1.0)
    assert err <= tol, f"normalised error {err:.3e} > {tol}"
    assert emax <= tol, f"largest element error {emax:.3e} of max|v| > {tol}"
    a = v_ref + np.asarray(s_ref, dtype=np.complex128).mean(axis=0)
    decided = np.abs(np.abs(a) - kappa) > margin * max(float(np.max(np.abs(a))), 1e-30)
    zg, zr = (v == 0)[decided], (v_ref == 0)[decided]
    bad = int(np.count_nonzero(zg != zr))
    assert bad == 0, f"{bad} of {int(decided.sum())} decided entries differ in being zero"
    return err, emax, int(decided.sum())
