"""Pins of the FP64 oracle to facts that do not come from the oracle itself.

Each test pins one part of the method (arXiv 1811.05571 Sec. III) to the
mathematics or to the paper's printed numbers:
  * soft threshold  -> proximal characterisation by brute force on a grid
  * inversion lemma -> direct solve of (H^H H + rho I) x = b
  * whole solver    -> closed form S_lam(H^H g) for unitary H (every splitting)
                    -> lasso KKT conditions at convergence
                    -> an independent FISTA minimiser (every splitting)
                    -> lam >= max|H^H g| gives the zero image
                    -> iterate-by-iterate textbook lasso ADMM (Q=P=1) and the
                       textbook consensus form (P=1), written with dense solves
                    -> scikit-learn's Lasso in the real special case
  * residual norms  -> recomputed from consecutive states
  * estimated data  -> the identity H_ij u = g'_ij - rho G^{-1}(g'_ij - H_ij c)
  * block shapes    -> the paper's timing table (tests/golden/tab_timing.json)
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import admm as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def crandn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def fista(H, g, lam, iters=20000):
    """Accelerated proximal gradient for 1/2|Hu-g|^2 + lam|u|_1 (complex)."""
    L = np.linalg.norm(H, 2) ** 2
    x = np.zeros(H.shape[1], complex)
    y = x.copy()
    t = 1.0
    for _ in range(iters):
        grad = H.conj().T @ (H @ y - g)
        a = y - grad / L
        mag = np.abs(a)
        xn = np.where(mag > lam / L, a * (1 - (lam / L) / np.maximum(mag, 1e-300)), 0)
        tn = (1 + np.sqrt(1 + 4 * t * t)) / 2
        y = xn + (t - 1) / tn * (xn - x)
        x, t = xn, tn
    return x


# --------------------------------------------------------------------------
# soft threshold
# --------------------------------------------------------------------------
@pytest.mark.parametrize("a,kappa", [(0.7 + 0.4j, 0.3), (-1.2 + 0.1j, 0.5), (0.2 - 0.1j, 0.5),
                                     (2.0 + 0.0j, 0.5), (0.0 + 0.9j, 0.25)])
def test_soft_threshold_is_the_prox(a, kappa):
    # argmin_x kappa|x| + 1/2|x - a|^2 over a 2-D grid of spacing h
    h = 2e-3
    xs = np.arange(-2.0, 2.0 + h, h)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    Z = X + 1j * Y
    F = kappa * np.abs(Z) + 0.5 * np.abs(Z - a) ** 2
    k = np.unravel_index(np.argmin(F), F.shape)
    brute = Z[k]
    got = O.soft_threshold(np.array([a]), kappa)[0]
    assert abs(got - brute) <= 2 * h


def test_soft_threshold_special_cases():
    a = np.array([0.0, 0.3, -0.3, 0.3j, 2.0, 0.1 + 0.1j, 1e-30, 1e30 + 1e30j])
    k = 0.3
    s = O.soft_threshold(a, k)
    assert np.all(s[:4] == 0)                  # |a| <= kappa, tie included
    assert s[4] == 2.0 - k                       # real positive: a - kappa
    assert s[5] == 0 and s[6] == 0
    assert np.isclose(s[7], (1e30 + 1e30j) * (1 - k / (np.sqrt(2) * 1e30)))
    np.testing.assert_array_equal(O.soft_threshold(a, 0.0), a)   # kappa = 0: identity
    # modulus shrinks by exactly kappa and the phase is kept
    rng = np.random.default_rng(0)
    z = crandn(rng, 100) * 3
    out = O.soft_threshold(z, 0.5)
    big = np.abs(z) > 0.5
    np.testing.assert_allclose(np.abs(out[big]), np.abs(z[big]) - 0.5, rtol=1e-13)
    np.testing.assert_allclose(np.angle(out[big]), np.angle(z[big]), atol=1e-13)


# --------------------------------------------------------------------------
# inversion lemma
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(5, 17), (16, 40), (12, 12), (30, 7)])
@pytest.mark.parametrize("rho", [0.1, 1.0, 1e5])
def test_block_solver_equals_direct_solve(shape, rho):
    rng = np.random.default_rng(1)
    H = crandn(rng, *shape)
    b = crandn(rng, shape[1])
    x = O.BlockSolver.build(H, rho).solve(b)
    ref = np.linalg.solve(H.conj().T @ H + rho * np.eye(shape[1]), b)
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


# --------------------------------------------------------------------------
# closed form for unitary H
# --------------------------------------------------------------------------
@pytest.mark.parametrize("Q,P", [(1, 1), (2, 1), (4, 1), (1, 2), (1, 4)])
def test_unitary_closed_form(Q, P):
    rng = np.random.default_rng(2)
    n = 16
    U, _ = np.linalg.qr(crandn(rng, n, n))
    g = crandn(rng, n)
    lam = 0.4
    want = O.soft_threshold(U.conj().T @ g, lam)   # argmin 1/2|g-Uu|^2 + lam|u|_1
    v, hist, _ = O.solve(U, g, Q, P, 1.0, lam, 3000)
    assert np.linalg.norm(v - want) <= 1e-8 * max(1.0, np.linalg.norm(want))


# --------------------------------------------------------------------------
# lasso KKT at the fixed point; equality of all splittings' limits and FISTA
# --------------------------------------------------------------------------
def _random_problem(seed, m=48, n=160, k=6, ratio=0.1):
    rng = np.random.default_rng(seed)
    H = crandn(rng, m, n) / np.sqrt(m)
    u = np.zeros(n, complex)
    u[rng.choice(n, k, replace=False)] = np.exp(2j * np.pi * rng.random(k))
    g = H @ u + 0.01 * crandn(rng, m)
    lam = ratio * O.lambda_max(H, g)
    return H, g, lam


@pytest.mark.parametrize("Q,P,rho", [(1, 1, 1.0), (4, 1, 1.0), (1, 2, 2.0), (3, 2, 4.0), (2, 4, 12.0)])
def test_fixed_point_is_the_lasso_minimiser(Q, P, rho):
    H, g, lam = _random_problem(3)
    ref = fista(H, g, lam)
    assert O.kkt_violation(H, g, ref, lam) < 1e-8
    v, hist, st = O.solve(H, g, Q, P, rho, lam, 6000)
    assert O.kkt_violation(H, g, v, lam) < 1e-6, (Q, P, O.kkt_violation(H, g, v, lam))
    assert np.linalg.norm(v - ref) <= 1e-6 * np.linalg.norm(ref)
    # at the fixed point the replicas agree with the consensus variable
    assert hist[-1, 0] < 1e-16 and hist[-1, 1] < 1e-16


def test_lambda_above_max_gives_zero():
    H, g, _ = _random_problem(4)
    lam = 1.001 * O.lambda_max(H, g)
    assert O.kkt_violation(H, g, np.zeros(H.shape[1]), lam) == 0.0
    for Q, P, rho in [(1, 1, 1.0), (4, 1, 1.0), (2, 2, 4.0)]:
        v, _, _ = O.solve(H, g, Q, P, rho, lam, 3000)
        assert np.max(np.abs(v)) < 1e-9


# --------------------------------------------------------------------------
# textbook iterations (Boyd et al. 2011, lasso and consensus lasso)
# --------------------------------------------------------------------------
def test_unsplit_matches_textbook_lasso_admm():
    H, g, lam = _random_problem(5)
    rho = 1.3
    n = H.shape[1]
    A = H.conj().T @ H + rho * np.eye(n)
    x = np.zeros(n, complex)
    z = np.zeros(n, complex)
    u = np.zeros(n, complex)
    st = O.State.zeros(H.shape[0], n, 1, 1)
    ro, co = O.split_offsets(H.shape[0], 1), O.split_offsets(n, 1)
    blocks = O.setup(H, ro, co, rho)
    for _ in range(60):
        x = np.linalg.solve(A, H.conj().T @ g + rho * (z - u))
        a = x + u
        z = np.where(np.abs(a) > lam / rho, a * (1 - lam / rho / np.maximum(np.abs(a), 1e-300)), 0)
        u = u + x - z
        st, _, _ = O.step(H, g, ro, co, rho, lam, blocks, st)
        assert np.linalg.norm(st.v - z) <= 1e-11 * max(1.0, np.linalg.norm(z))
        assert np.linalg.norm(st.s[0] - u) <= 1e-11 * max(1.0, np.linalg.norm(u))


def test_consensus_matches_textbook_split_across_examples():
    H, g, lam = _random_problem(6, m=60)
    rho, Q = 0.7, 3
    m, n = H.shape
    ro = O.split_offsets(m, Q)
    co = O.split_offsets(n, 1)
    xs = np.zeros((Q, n), complex)
    us = np.zeros((Q, n), complex)
    z = np.zeros(n, complex)
    mats = [np.linalg.inv(H[ro[i]:ro[i + 1]].conj().T @ H[ro[i]:ro[i + 1]] + rho * np.eye(n)) for i in range(Q)]
    st = O.State.zeros(m, n, Q, 1)
    blocks = O.setup(H, ro, co, rho)
    for _ in range(40):
        for i in range(Q):
            Hi, gi = H[ro[i]:ro[i + 1]], g[ro[i]:ro[i + 1]]
            xs[i] = mats[i] @ (Hi.conj().T @ gi + rho * (z - us[i]))
        a = xs.mean(0) + us.mean(0)
        k = lam / (rho * Q)
        z = np.where(np.abs(a) > k, a * (1 - k / np.maximum(np.abs(a), 1e-300)), 0)
        us = us + xs - z
        st, _, _ = O.step(H, g, ro, co, rho, lam, blocks, st)
        assert np.linalg.norm(st.v - z) <= 1e-10 * max(1.0, np.linalg.norm(z))


# --------------------------------------------------------------------------
# real special case vs scikit-learn
# --------------------------------------------------------------------------
def test_real_case_matches_sklearn_lasso():
    sklearn = pytest.importorskip("sklearn.linear_model")
    rng = np.random.default_rng(7)
    m, n = 40, 120
    H = rng.standard_normal((m, n)) / np.sqrt(m)
    u = np.zeros(n)
    u[rng.choice(n, 5, replace=False)] = rng.standard_normal(5)
    g = H @ u + 0.01 * rng.standard_normal(m)
    lam = 0.1 * np.max(np.abs(H.T @ g))
    # sklearn: 1/(2m)|g - Hw|^2 + alpha|w|_1  ->  alpha = lam/m
    ref = sklearn.Lasso(alpha=lam / m, fit_intercept=False, tol=1e-14, max_iter=200000).fit(H, g).coef_
    for Q, P, rho in [(1, 1, 1.0), (2, 1, 1.0), (2, 2, 4.0)]:
        v, _, st = O.solve(H.astype(complex), g.astype(complex), Q, P, rho, lam, 5000)
        assert np.max(np.abs(v.imag)) == 0.0 and np.max(np.abs(st.s.imag)) == 0.0
        assert np.linalg.norm(v.real - ref) <= 1e-6 * np.linalg.norm(ref)


# --------------------------------------------------------------------------
# residual norms and the estimated-data identity
# --------------------------------------------------------------------------
def test_residual_norms_from_states():
    H, g, lam = _random_problem(8)
    Q, P, rho = 3, 2, 4.0
    m, n = H.shape
    ro, co = O.split_offsets(m, Q), O.split_offsets(n, P)
    blocks = O.setup(H, ro, co, rho)
    st = O.State.zeros(m, n, Q, P)
    for _ in range(5):
        prev = st
        st, rp2, rd2 = O.step(H, g, ro, co, rho, lam, blocks, st)
        # stacked vectors of the combined scheme: r_p = (u_j^i - v_j), r_d = -rho (v_j - v_j^prev) per replica
        r_p = np.concatenate([st.u[i] - st.v for i in range(Q)])
        r_d = np.concatenate([-rho * (st.v - prev.v) for _ in range(Q)])
        assert np.isclose(rp2, np.vdot(r_p, r_p).real, rtol=1e-12)
        assert np.isclose(rd2, np.vdot(r_d, r_d).real, rtol=1e-12)


def test_estimated_data_identity():
    """H_ij u = g' - rho y with y = (rho I + H H^H)^{-1}(g' - H c), c = v - s."""
    H, g, lam = _random_problem(9)
    Q, P, rho = 2, 2, 3.0
    m, n = H.shape
    ro, co = O.split_offsets(m, Q), O.split_offsets(n, P)
    blocks = O.setup(H, ro, co, rho)
    st = O.State.zeros(m, n, Q, P)
    for _ in range(3):
        st, _, _ = O.step(H, g, ro, co, rho, lam, blocks, st)
    nxt, _, _ = O.step(H, g, ro, co, rho, lam, blocks, st)
    for i in range(Q):
        for j in range(P):
            r0, r1, c0, c1 = ro[i], ro[i + 1], co[j], co[j + 1]
            Hij = H[r0:r1, c0:c1]
            gp = g[r0:r1] - sum(st.ghat[q, r0:r1] for q in range(P) if q != j)
            c = st.v[c0:c1] - st.s[i, c0:c1]
            y = np.linalg.solve(rho * np.eye(r1 - r0) + Hij @ Hij.conj().T, gp - Hij @ c)
            np.testing.assert_allclose(nxt.ghat[j, r0:r1], gp - rho * y, rtol=0, atol=1e-10)
            np.testing.assert_allclose(nxt.u[i, c0:c1], c + Hij.conj().T @ y, rtol=0, atol=1e-10)


# --------------------------------------------------------------------------
# block shapes of the paper's timing table
# --------------------------------------------------------------------------
def test_partition_matches_paper_timing_table():
    gold = json.load(open(os.path.join(GOLDEN, "tab_timing.json")))
    assert gold["N_Tx"] * gold["N_Rx"] * gold["N_f"] == gold["N_m"]
    tx, rx, freqs, vox = W.cra_geometry(gold["N_Tx"], gold["N_Rx"], gold["N_f"], nx=2, ny=2, nz=2)
    assert len(tx) * len(rx) * len(freqs) == gold["N_m"]
    for sp in gold["splits"]:
        ro = O.split_offsets(gold["N_m"], sp["M"])
        co = O.split_offsets(gold["N_p"], sp["N"])
        assert set(np.diff(ro)) == {sp["block"][0]}
        assert set(np.diff(co)) == {sp["block"][1]}
        # the small matrix of the inversion lemma is (rows of a block)^2
        assert sp["woodbury"] == [sp["block"][0]] * 2


def test_paper_table_workload_shapes():
    """The timing-table workload has the table's measurement and pixel counts,
    its splits, unit rows and the two-patch target."""
    gold = json.load(open(os.path.join(GOLDEN, "tab_timing.json")))
    p = W.paper_table_imaging()
    assert p.H.shape == (gold["N_m"], gold["N_p"])
    assert [(sp["M"], sp["N"]) for sp in gold["splits"]] == list(W.PAPER_TABLE_SPLITS)
    np.testing.assert_allclose(np.linalg.norm(p.H.astype(np.complex128), axis=1), 1.0, rtol=1e-5)
    assert np.count_nonzero(p.u_true) == 150 and p.lam > 0
    # same seed, same matrix for every split
    assert np.array_equal(W.paper_table_imaging(Q=1, P=3).H, p.H)


def test_uneven_split_offsets():
    np.testing.assert_array_equal(O.split_offsets(10, 3), [0, 4, 7, 10])
    np.testing.assert_array_equal(O.split_offsets(9, 3), [0, 3, 6, 9])
    with pytest.raises(ValueError):
        O.split_offsets(10, 3, [0, 5, 5, 10])
    with pytest.raises(ValueError):
        O.split_offsets(3, 4)


# --------------------------------------------------------------------------
# stop rule (relative tolerance) on states whose norms are known by hand
# --------------------------------------------------------------------------
def _uniform_state(Q, n, u, v, s):
    """Every replica entry u, every image entry v, every dual entry s."""
    st = O.State.zeros(1, n, Q, 1)
    st.u[:] = u
    st.v[:] = v
    st.s[:] = s
    return st


def test_stop_rule_on_hand_computed_norms():
    # Q = 2 replicas of n = 4 entries.  u = 3, v = 4, s = 1 (rho = 2):
    #   |(u^i)| = sqrt(2*4*9) = 6 sqrt 2,  sqrt(Q)|v| = sqrt 2 * sqrt(4*16) = 8 sqrt 2
    #   primal scale = tol * 8 sqrt 2,  |(s^i)| = sqrt 8 = 2 sqrt 2,  dual scale = tol * 2 * 2 sqrt 2
    # With |r_p|^2 = 8 (|r_p| = 2 sqrt 2) the primal test holds iff tol >= 1/4;
    # with |r_d|^2 = 8 the dual test holds iff tol >= 1/2.
    st = _uniform_state(2, 4, 3.0, 4.0, 1.0)
    for tol, want in [(0.2, False), (0.3, False), (0.49, False), (0.51, True), (2.0, True)]:
        assert O.converged(st, 8.0, 8.0, 2.0, tol) is want, tol
    # the dual test alone decides when the primal residual is zero
    assert O.converged(st, 0.0, 8.0, 2.0, 0.49) is False
    assert O.converged(st, 0.0, 8.0, 2.0, 0.51) is True
    # and the primal test alone when the dual residual is zero: tol >= 1/4
    assert O.converged(st, 8.0, 0.0, 2.0, 0.24) is False
    assert O.converged(st, 8.0, 0.0, 2.0, 0.26) is True


def test_stop_rule_takes_the_larger_primal_scale():
    # u = 5, v = 1 (Q = 3, n = 2): |(u^i)| = sqrt(3*2*25) = 5 sqrt 6 beats
    # sqrt(3)|v| = sqrt 3 * sqrt 2 = sqrt 6.  |r_p|^2 = 6 (|r_p| = sqrt 6):
    # primal holds iff tol >= 1/5 (with the smaller scale it would need tol >= 1).
    st = _uniform_state(3, 2, 5.0, 1.0, 1.0)
    assert O.converged(st, 6.0, 0.0, 1.0, 0.19) is False
    assert O.converged(st, 6.0, 0.0, 1.0, 0.21) is True
    # the complex modulus counts, not the real part: u = 3 + 4j has |u| = 5
    st2 = _uniform_state(3, 2, 3.0 + 4.0j, 1.0, 1.0)
    assert O.converged(st2, 6.0, 0.0, 1.0, 0.21) is True


def test_solve_stops_at_the_first_check_that_passes():
    H, g, lam = _random_problem(12)
    Q, P, rho, tol, every = 2, 2, 4.0, 1e-3, 7
    m, n = H.shape
    v, hist, st = O.solve(H, g, Q, P, rho, lam, 400, tol=tol, check_every=every)
    k = len(hist)
    assert 0 < k < 400 and k % every == 0
    # replay the same iterations: the rule holds at iteration k and fails at
    # every earlier multiple of check_every
    ro, co = O.split_offsets(m, Q), O.split_offsets(n, P)
    blocks = O.setup(H, ro, co, rho)
    s2 = O.State.zeros(m, n, Q, P)
    for it in range(1, k + 1):
        s2, rp2, rd2 = O.step(H, g, ro, co, rho, lam, blocks, s2)
        if it % every == 0:
            assert O.converged(s2, rp2, rd2, rho, tol) is (it == k)
    assert np.array_equal(s2.v, v)


# --------------------------------------------------------------------------
# push-through form of the x-update against the literal one
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m,n,Q,P,rho,ro", [
    (48, 160, 1, 1, 1.0, None),       # unsplit, wide
    (48, 160, 4, 1, 1.0, None),       # consensus
    (48, 160, 1, 3, 6.0, None),       # sectioning
    (48, 160, 3, 2, 4.0, None),       # combined
    (60, 40, 2, 2, 8.0, None),        # tall blocks 30 x 20 (direct factor)
    (50, 90, 2, 3, 9.0, [0, 35, 50]), # uneven rows: 35 x 30 tall beside 15 x 30 wide
])
def test_push_through_form_matches_literal(m, n, Q, P, rho, ro):
    H, g, lam = _random_problem(13, m=m, n=n)
    v1, h1, s1 = O.solve(H, g, Q, P, rho, lam, 40, row_off=ro)
    v2, h2, s2 = O.solve(H, g, Q, P, rho, lam, 40, row_off=ro, form="push_through")
    scale = max(1.0, np.linalg.norm(v1))
    assert np.linalg.norm(v2 - v1) <= 1e-12 * scale
    assert np.linalg.norm(s2.s - s1.s) <= 1e-12 * max(1.0, np.linalg.norm(s1.s))
    assert np.linalg.norm(s2.ghat - s1.ghat) <= 1e-12 * max(1.0, np.linalg.norm(s1.ghat))
    np.testing.assert_allclose(h2, h1, rtol=1e-9, atol=1e-24)
