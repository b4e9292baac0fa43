"""Pins of the torch twin used for reference gradients: its forward equals the
numpy oracle, torch's complex-gradient convention is dL/dRe + j dL/dIm, and
its autograd gradients match central differences of the numpy oracle in FP64."""
import numpy as np
import pytest
import torch

from oracle import admm as O
from oracle import admm_torch as OT


def _problem(seed=0, m=40, n=120, Q=2, P=2, rho=6.0):
    rng = np.random.default_rng(seed)
    H = (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))) / np.sqrt(2 * m)
    u = np.zeros(n, complex)
    u[rng.choice(n, 6, replace=False)] = np.exp(2j * np.pi * rng.random(6))
    g = H @ u + 0.01 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    lam = 0.05 * O.lambda_max(H, g)
    return H, g, u, Q, P, rho, lam


def test_torch_gradient_convention():
    z = torch.tensor([1.0 + 2.0j], dtype=torch.complex128, requires_grad=True)
    (z.conj() * z).real.sum().backward()
    assert torch.allclose(z.grad, torch.tensor([2.0 + 4.0j], dtype=torch.complex128))


@pytest.mark.parametrize("Q,P", [(1, 1), (2, 1), (2, 2), (1, 2), (1, 4)])   # (1, 4): 40 x 30, direct
def test_twin_forward_equals_oracle(Q, P):
    H, g, u, _, _, rho, lam = _problem(Q=Q, P=P)
    v_ref, _, _ = O.solve(H, g, Q, P, rho, lam, 30)
    v = OT.unrolled(torch.from_numpy(H), torch.from_numpy(g), Q, P, torch.tensor(rho, dtype=torch.float64),
                    torch.tensor(lam, dtype=torch.float64), 30).numpy()
    assert np.linalg.norm(v - v_ref) <= 1e-12 * np.linalg.norm(v_ref)


@pytest.mark.parametrize("Q,P", [(2, 1), (2, 2), (1, 4)])
def test_twin_gradients_match_central_differences(Q, P):
    H, g, u_true, _, _, rho, lam = _problem(seed=1, Q=Q, P=P)
    K = 20
    v0, _, _ = O.solve(H, g, Q, P, rho, lam, K)
    grad_v = 2 * (v0 - u_true)                 # L = |v^K - u_true|^2

    def L(gg, ll, rr):
        v, _, _ = O.solve(H, gg, Q, P, rr, ll, K)
        return float(np.sum(np.abs(v - u_true) ** 2))

    dg, dlam, drho, _ = OT.gradients(H, g, Q, P, rho, lam, K, grad_v)
    rng = np.random.default_rng(2)
    for _ in range(3):
        d = rng.standard_normal(len(g)) + 1j * rng.standard_normal(len(g))
        d /= np.linalg.norm(d)
        h = 1e-6 * np.linalg.norm(g)
        fd = (L(g + h * d, lam, rho) - L(g - h * d, lam, rho)) / (2 * h)
        assert abs(fd - np.real(np.vdot(dg, d))) <= 1e-5 * (abs(fd) + 1e-3)
    h = 1e-6 * lam
    fd = (L(g, lam + h, rho) - L(g, lam - h, rho)) / (2 * h)
    assert abs(fd - dlam) <= 1e-5 * (abs(fd) + 1e-3)
    h = 1e-6 * rho
    fd = (L(g, lam, rho + h) - L(g, lam, rho - h)) / (2 * h)
    assert abs(fd - drho) <= 1e-5 * (abs(fd) + 1e-3)
