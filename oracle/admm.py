"""FP64 CPU oracle of the split-lasso ADMM (consensus / sectioning / both).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this module; only the test suite, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code with the HIP library.

Problem (paper Sec. III, lasso form):  minimise 1/2 |H u - g|^2 + lam |u|_1
over complex u.  H is split into Q row blocks i and P column blocks j
(H_ij, g_i, u_j); each block keeps a replica u_j^i, the consensus variable is
v_j and the scaled dual s_j^i.  One iteration, in the paper's order
(Sec. III-C, combined scheme; Q=1 is sectioning, Sec. III-B; P=1 is
consensus, Sec. III-A):

  1. local data      g_ij = g_i - sum_{q != j} ghat_iq            (eq. g_rows_columns)
  2. x-update        u_j^i = (H_ij^* H_ij + rho I)^{-1}
                             (H_ij^* g_ij + rho (v_j - s_j^i))   (eq. x_solution_rows_columns)
                     evaluated with the matrix inversion lemma when the
                     block is wide (eq. inversion_lemma3), directly otherwise
  3. estimated data  ghat_ij = H_ij u_j^i                          (Sec. III-C text)
  4. z-update        v_j = S_{lam/(Q rho)}(mean_i u_j^i + mean_i s_j^i)
                     with the previous duals                      (eq. v_variable_rows_columns)
  5. dual update     s_j^i += u_j^i - v_j                          (eq. s_variable_rows_columns)
  6. residuals       |r_p|^2 = sum_ij |u_j^i - v_j|^2,
                     |r_d|^2 = rho^2 Q sum_j |v_j - v_j^prev|^2     (Sec. III-C residual norms)

Readings where the paper is silent (all zero start; complex sign(a) = a/|a|;
Jacobi use of the previous iteration's estimated data by every block; the
output image is v = [v_1; ...; v_P]; uneven blocks by offsets with the
first (total mod parts) blocks one larger; stop rule only when tol > 0)
are listed with the design notes.

Pins (tests/test_oracle_*.py): prox characterisation of S by brute force,
inversion lemma vs direct solve, unitary-H closed form, lasso KKT at the
fixed point, equality of the limits of all splittings and an independent
FISTA minimiser, the lambda >= max|H^H g| zero solution, textbook lasso ADMM
for Q=P=1, the real special case against scikit-learn's Lasso, the block
shapes of the paper's timing table, the stop rule on states with hand-computed
norms, and the push-through form against the literal one.
"""

from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla


# --------------------------------------------------------------------------
# Partition (Sec. III: H_ij of size N_m/M x N_p/N; uneven blocks by offsets)
# --------------------------------------------------------------------------
def split_offsets(total: int, parts: int, offsets=None) -> np.ndarray:
    """Block boundaries 0 = o_0 < o_1 < ... < o_parts = total.

    Without explicit offsets the first (total mod parts) blocks get one extra
    element, so equal division is recovered when parts divides total.
    """
    if offsets is not None:
        o = np.asarray(offsets, dtype=np.int64)
        if o.shape != (parts + 1,) or o[0] != 0 or o[-1] != total or np.any(np.diff(o) <= 0):
            raise ValueError("offsets must increase strictly from 0 to total")
        return o
    if parts < 1 or parts > total:
        raise ValueError("parts must lie in [1, total]")
    base, extra = divmod(total, parts)
    sizes = np.full(parts, base, dtype=np.int64)
    sizes[:extra] += 1
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


# --------------------------------------------------------------------------
# Soft threshold (eq. softhresholding), complex sign(a) = a/|a|
# --------------------------------------------------------------------------
def soft_threshold(a: np.ndarray, kappa: float) -> np.ndarray:
    """S_kappa(a) = a - kappa a/|a| where |a| > kappa, else 0 (element-wise)."""
    a = np.asarray(a)
    mag = np.abs(a)
    out = np.zeros_like(a)
    big = mag > kappa
    out[big] = a[big] - kappa * a[big] / mag[big]
    return out


# --------------------------------------------------------------------------
# Per-block x-update operator
# --------------------------------------------------------------------------
@dataclasses.dataclass
class BlockSolver:
    """Solves (H^* H + rho I) x = b for one block H (m_b x n_b).

    Wide blocks (m_b < n_b) use the matrix inversion lemma
      (H^*H + rho I)^{-1} = I/rho - H^*/rho^2 (I + H H^*/rho)^{-1} H
    with a Cholesky factor of the small m_b x m_b matrix (eq. inversion_lemma3);
    other blocks factor H^*H + rho I directly (the paper's remark that the
    original inversion is cheaper when the block is tall).
    """
    H: np.ndarray
    rho: float
    woodbury: bool
    factor: tuple

    @classmethod
    def build(cls, H: np.ndarray, rho: float) -> "BlockSolver":
        mb, nb = H.shape
        if mb < nb:
            A = np.eye(mb, dtype=np.complex128) + (H @ H.conj().T) / rho
            return cls(H, rho, True, sla.cho_factor(A, lower=True))
        B = H.conj().T @ H + rho * np.eye(nb, dtype=np.complex128)
        return cls(H, rho, False, sla.cho_factor(B, lower=True))

    def solve(self, b: np.ndarray) -> np.ndarray:
        if self.woodbury:
            H, rho = self.H, self.rho
            t = sla.cho_solve(self.factor, H @ b)
            return b / rho - (H.conj().T @ t) / rho ** 2
        return sla.cho_solve(self.factor, b)


def setup(H: np.ndarray, row_off: np.ndarray, col_off: np.ndarray, rho: float):
    """Factor every block once (the paper's 'inversion time')."""
    H = np.asarray(H, dtype=np.complex128)
    Q, P = len(row_off) - 1, len(col_off) - 1
    return [[BlockSolver.build(H[row_off[i]:row_off[i + 1], col_off[j]:col_off[j + 1]].copy(), rho)
             for j in range(P)] for i in range(Q)]


# --------------------------------------------------------------------------
# Iteration state and one ADMM step
# --------------------------------------------------------------------------
@dataclasses.dataclass
class State:
    k: int                 # iterations done
    u: np.ndarray          # (Q, n) replicas u^i (each holds all P segments)
    v: np.ndarray          # (n,)  consensus image
    s: np.ndarray          # (Q, n) scaled duals
    ghat: np.ndarray       # (P, m) estimated data; rows of block i hold ghat_ij

    @classmethod
    def zeros(cls, m: int, n: int, Q: int, P: int) -> "State":
        z = lambda *sh: np.zeros(sh, dtype=np.complex128)
        return cls(0, z(Q, n), z(n), z(Q, n), z(P, m))

    def copy(self) -> "State":
        return State(self.k, self.u.copy(), self.v.copy(), self.s.copy(), self.ghat.copy())


def step(H, g, row_off, col_off, rho, lam, blocks, st: State):
    """One iteration k -> k+1 in the paper's order.  Returns (new state, rp2, rd2)."""
    H = np.asarray(H)
    g = np.asarray(g, dtype=np.complex128)
    Q, P = len(row_off) - 1, len(col_off) - 1
    u_new = np.empty_like(st.u)
    ghat_new = np.empty_like(st.ghat)
    for i in range(Q):
        r0, r1 = row_off[i], row_off[i + 1]
        for j in range(P):
            c0, c1 = col_off[j], col_off[j + 1]
            # eq. g_rows_columns: data left for block (i, j) by the other
            # sections of replica i, from the previous iteration (Jacobi)
            g_ij = g[r0:r1].copy()
            for q in range(P):
                if q != j:
                    g_ij -= st.ghat[q, r0:r1]
            Hij = blocks[i][j].H
            # eq. x_solution_rows_columns
            b = Hij.conj().T @ g_ij + rho * (st.v[c0:c1] - st.s[i, c0:c1])
            u_new[i, c0:c1] = blocks[i][j].solve(b)
            # estimated data handed to the other sections of replica i
            ghat_new[j, r0:r1] = Hij @ u_new[i, c0:c1]
    # eq. v_variable_rows_columns: threshold the mean over replicas, old duals
    kappa = lam / (Q * rho)
    v_new = soft_threshold(u_new.mean(axis=0) + st.s.mean(axis=0), kappa)
    # eq. s_variable_rows_columns
    s_new = st.s + u_new - v_new[None, :]
    rp2 = float(np.sum(np.abs(u_new - v_new[None, :]) ** 2))
    rd2 = float(rho ** 2 * Q * np.sum(np.abs(v_new - st.v) ** 2))
    return State(st.k + 1, u_new, v_new, s_new, ghat_new), rp2, rd2


# --------------------------------------------------------------------------
# The same iteration in push-through form (for timing on the host)
# --------------------------------------------------------------------------
@dataclasses.dataclass
class PushBlock:
    """x-update of one block with two products per iteration.

    With G = rho I + H H^* the inversion lemma (eq. inversion_lemma3) turns
    the x-update of eq. x_solution_rows_columns, for c = v_j - s_j^i, into
        y = G^{-1} (g' - H c),    u = c + H^* y,
    and since H H^* = G - rho I the estimated data is H u = g' - rho y.  One
    product with H, one Cholesky solve with G and one product with H^* per
    iteration, against three products and a solve in the literal form.
    Blocks with m_b >= n_b keep the direct factor of H^*H + rho I and form
    H u explicitly, as the literal form does.
    """
    H: np.ndarray
    rho: float
    wide: bool
    factor: tuple

    @classmethod
    def build(cls, H: np.ndarray, rho: float) -> "PushBlock":
        mb, nb = H.shape
        if mb < nb:
            G = H @ H.conj().T + rho * np.eye(mb, dtype=np.complex128)
            return cls(H, rho, True, sla.cho_factor(G, lower=True))
        B = H.conj().T @ H + rho * np.eye(nb, dtype=np.complex128)
        return cls(H, rho, False, sla.cho_factor(B, lower=True))

    def adjoint(self, y: np.ndarray) -> np.ndarray:
        """H^* y, as the conjugate of y^* H (no conjugated copy of H is formed)."""
        return np.conj(np.conj(y) @ self.H)

    def update(self, gp: np.ndarray, c: np.ndarray):
        """(u, H u) for local data gp and c = v_j - s_j^i."""
        H = self.H
        if self.wide:
            y = sla.cho_solve(self.factor, gp - H @ c)
            return c + self.adjoint(y), gp - self.rho * y
        u = sla.cho_solve(self.factor, self.adjoint(gp) + self.rho * c)
        return u, H @ u


def setup_push_through(H: np.ndarray, row_off: np.ndarray, col_off: np.ndarray, rho: float):
    H = np.asarray(H, dtype=np.complex128)
    Q, P = len(row_off) - 1, len(col_off) - 1
    return [[PushBlock.build(H[row_off[i]:row_off[i + 1], col_off[j]:col_off[j + 1]].copy(), rho)
             for j in range(P)] for i in range(Q)]


def step_push_through(g, row_off, col_off, rho, lam, pblocks, st: State):
    """The iteration of step() with the x-update of PushBlock (same order,
    same Jacobi local data, same z- and dual updates)."""
    g = np.asarray(g, dtype=np.complex128)
    Q, P = len(row_off) - 1, len(col_off) - 1
    u_new = np.empty_like(st.u)
    ghat_new = np.empty_like(st.ghat)
    for i in range(Q):
        r0, r1 = row_off[i], row_off[i + 1]
        total = st.ghat[:, r0:r1].sum(axis=0)
        for j in range(P):
            c0, c1 = col_off[j], col_off[j + 1]
            gp = g[r0:r1] - (total - st.ghat[j, r0:r1]) if P > 1 else g[r0:r1]
            u, hu = pblocks[i][j].update(gp, st.v[c0:c1] - st.s[i, c0:c1])
            u_new[i, c0:c1] = u
            ghat_new[j, r0:r1] = hu
    kappa = lam / (Q * rho)
    v_new = soft_threshold(u_new.mean(axis=0) + st.s.mean(axis=0), kappa)
    s_new = st.s + u_new - v_new[None, :]
    rp2 = float(np.sum(np.abs(u_new - v_new[None, :]) ** 2))
    rd2 = float(rho ** 2 * Q * np.sum(np.abs(v_new - st.v) ** 2))
    return State(st.k + 1, u_new, v_new, s_new, ghat_new), rp2, rd2


def converged(st: State, rp2: float, rd2: float, rho: float, tol: float) -> bool:
    """Relative stopping rule (absolute tolerance zero):
    |r_p| <= tol max(|(u^i)|, sqrt(Q)|v|) and |r_d| <= tol rho |(s^i)|."""
    Q = st.u.shape[0]
    pri = tol * max(np.linalg.norm(st.u), np.sqrt(Q) * np.linalg.norm(st.v))
    dual = tol * rho * np.linalg.norm(st.s)
    return bool(np.sqrt(rp2) <= pri and np.sqrt(rd2) <= dual)


def solve(H, g, Q: int, P: int, rho: float, lam: float, iters: int, row_off=None, col_off=None,
          tol: float = 0.0, check_every: int = 10, state: State | None = None, blocks=None,
          form: str = "literal"):
    """Run up to `iters` iterations from `state` (zeros by default).

    Returns (v, history (k, 2) of [|r_p|^2, |r_d|^2], final state).
    With tol <= 0 exactly `iters` iterations run; otherwise the stop rule is
    tested after every `check_every`-th iteration.  form="push_through" runs
    step_push_through (two products per block and iteration) instead of the
    literal step; `blocks` must then come from setup_push_through.
    """
    if form not in ("literal", "push_through"):
        raise ValueError("form must be 'literal' or 'push_through'")
    H = np.asarray(H, dtype=np.complex128)
    m, n = H.shape
    ro = split_offsets(m, Q, row_off)
    co = split_offsets(n, P, col_off)
    if blocks is None:
        blocks = (setup if form == "literal" else setup_push_through)(H, ro, co, rho)
    st = state.copy() if state is not None else State.zeros(m, n, Q, P)
    hist = []
    for it in range(iters):
        if form == "literal":
            st, rp2, rd2 = step(H, g, ro, co, rho, lam, blocks, st)
        else:
            st, rp2, rd2 = step_push_through(g, ro, co, rho, lam, blocks, st)
        hist.append((rp2, rd2))
        if tol > 0 and (it + 1) % check_every == 0 and converged(st, rp2, rd2, rho, tol):
            break
    return st.v.copy(), np.asarray(hist, dtype=np.float64).reshape(-1, 2), st


# --------------------------------------------------------------------------
# Lasso optimality (subgradient) check of an image v
# --------------------------------------------------------------------------
def kkt_violation(H, g, v, lam: float) -> float:
    """max_n of the distance of z_n = (H^H (g - H v))_n to lam * d|v_n|, over lam.

    On the support the subgradient is lam v_n/|v_n|; off it the set is the
    disc of radius lam.  Zero exactly at the lasso minimiser.
    """
    H = np.asarray(H, dtype=np.complex128)
    v = np.asarray(v, dtype=np.complex128)
    z = H.conj().T @ (np.asarray(g, dtype=np.complex128) - H @ v)
    mag = np.abs(v)
    on = mag > 0
    viol = np.maximum(np.abs(z) - lam, 0.0)
    viol[on] = np.abs(z[on] - lam * v[on] / mag[on])
    return float(np.max(viol) / lam)


def lambda_max(H, g) -> float:
    """Smallest lam for which u = 0 is the lasso minimiser: max|H^H g|."""
    H = np.asarray(H, dtype=np.complex128)
    return float(np.max(np.abs(H.conj().T @ np.asarray(g, dtype=np.complex128))))
