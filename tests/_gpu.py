"""Helpers shared by the GPU tests: move a generated problem to the device and
run the HIP solver through the C ABI binding."""
import numpy as np


def to_device(torch, arr):
    return torch.from_numpy(np.ascontiguousarray(arr)).to("cuda")


def gpu_solve(torch, prob, iters, rho=None, lam=None, Q=None, P=None, row_off=None, col_off=None,
              history=False, **kw):
    import paper_1811_05571_amd as A
    H = to_device(torch, prob.H)
    g = to_device(torch, prob.g)
    plan = A.Plan(H, Q or prob.Q, P or prob.P, rho if rho is not None else prob.rho,
                  lam if lam is not None else prob.lam,
                  row_off if row_off is not None else prob.row_off,
                  col_off if col_off is not None else prob.col_off)
    out = plan.solve(g, iters, history=history, **kw)
    return plan, g, out


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))
