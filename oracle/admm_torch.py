"""FP64 torch-CPU twin of the oracle, for reference gradients.

TEST INFRASTRUCTURE ONLY (same rule as oracle/admm.py).

The same iteration as oracle/admm.py (paper Sec. III-C, combined scheme, in
the paper's order with the literal inversion lemma of eq. inversion_lemma3 for
blocks with fewer rows than columns and, as the paper remarks for the others,
a direct factor of H_ij^* H_ij + rho I),
written with torch complex128 CPU operations so that torch's autograd gives
d v^K / d(g, lambda, rho) for K unrolled iterations from the zero state.

Gradient convention of the results: for a real loss L and complex z the
reported gradient is dL/dRe z + j dL/dIm z (what central differences on the
real and imaginary parts measure).  torch's .grad for a real loss follows the
same convention (checked in tests/test_oracle_adjoint.py with L = |z|^2).

The soft threshold thresholds |a|^2 against kappa^2 and takes the square root
only where it is positive, so |a| = 0 contributes a zero gradient, not NaN.
"""

from __future__ import annotations

import torch

from oracle.admm import split_offsets


def soft_threshold(a: torch.Tensor, kappa: torch.Tensor) -> torch.Tensor:
    mag2 = a.real * a.real + a.imag * a.imag
    big = mag2 > kappa * kappa
    mag = torch.sqrt(torch.where(big, mag2, torch.ones_like(mag2)))
    scale = torch.where(big, 1.0 - kappa / mag, torch.zeros_like(mag))
    return a * scale


def unrolled(H: torch.Tensor, g: torch.Tensor, Q: int, P: int, rho: torch.Tensor, lam: torch.Tensor,
             iters: int, row_off=None, col_off=None) -> torch.Tensor:
    """v^K of K iterations from zero; differentiable in g, rho, lam."""
    m, n = H.shape
    ro = [int(x) for x in split_offsets(m, Q, row_off)]
    co = [int(x) for x in split_offsets(n, P, col_off)]
    blocks = {}
    for i in range(Q):
        for j in range(P):
            Hij = H[ro[i]:ro[i + 1], co[j]:co[j + 1]]
            mb, nb = Hij.shape
            if mb < nb:
                A = torch.eye(mb, dtype=H.dtype) + (Hij @ Hij.conj().T) / rho
                blocks[i, j] = (Hij, True, torch.linalg.cholesky(A))
            else:
                B = Hij.conj().T @ Hij + rho * torch.eye(nb, dtype=H.dtype)
                blocks[i, j] = (Hij, False, torch.linalg.cholesky(B))
    zc = lambda k: torch.zeros(k, dtype=H.dtype)
    v = zc(n)
    s = [zc(n) for _ in range(Q)]
    ghat = [[zc(ro[i + 1] - ro[i]) for _ in range(P)] for i in range(Q)]
    kappa = lam / (Q * rho)
    for _ in range(iters):
        u = [[None] * P for _ in range(Q)]
        ghat_new = [[None] * P for _ in range(Q)]
        for i in range(Q):
            gi = g[ro[i]:ro[i + 1]]
            for j in range(P):
                c0, c1 = co[j], co[j + 1]
                Hij, lemma, L = blocks[i, j]
                g_ij = gi
                for q in range(P):
                    if q != j:
                        g_ij = g_ij - ghat[i][q]
                b = Hij.conj().T @ g_ij + rho * (v[c0:c1] - s[i][c0:c1])
                if lemma:
                    t = torch.cholesky_solve((Hij @ b).unsqueeze(1), L).squeeze(1)
                    u[i][j] = b / rho - (Hij.conj().T @ t) / rho ** 2
                else:
                    u[i][j] = torch.cholesky_solve(b.unsqueeze(1), L).squeeze(1)
                ghat_new[i][j] = Hij @ u[i][j]
        ghat = ghat_new
        ui = [torch.cat(u[i]) for i in range(Q)]
        a = sum(ui) / Q + sum(s) / Q
        v = soft_threshold(a, kappa)
        s = [s[i] + ui[i] - v for i in range(Q)]
    return v


def gradients(H, g, Q, P, rho, lam, iters, grad_v, row_off=None, col_off=None):
    """Return (dL/dg, dL/dlam, dL/drho) for L = Re <grad_v, v^K>, i.e. the
    vector-Jacobian product of the unrolled map with the image adjoint grad_v
    (numpy complex128 arrays in, numpy / float out)."""
    import numpy as np
    Ht = torch.from_numpy(np.asarray(H, dtype=np.complex128))
    gt = torch.from_numpy(np.asarray(g, dtype=np.complex128)).clone().requires_grad_(True)
    rt = torch.tensor(float(rho), dtype=torch.float64, requires_grad=True)
    lt = torch.tensor(float(lam), dtype=torch.float64, requires_grad=True)
    v = unrolled(Ht, gt, Q, P, rt, lt, iters, row_off, col_off)
    w = torch.from_numpy(np.asarray(grad_v, dtype=np.complex128))
    L = (w.conj() * v).real.sum()
    L.backward()
    return gt.grad.numpy().copy(), float(lt.grad), float(rt.grad), v.detach().numpy()
